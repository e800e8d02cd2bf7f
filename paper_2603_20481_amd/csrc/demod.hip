// demod stage: max-log LLRs, one thread per (frame, user, symbol, subcarrier);
// consecutive threads write consecutive LLR groups.  The body is
// demk::demod_elem (frames are contiguous, so the frame index folds into the
// user index).
#include "demod_core.h"

namespace rxphy {
namespace {

using namespace demk;

template <int Q>
__global__ void __launch_bounds__(256)
demod_kernel(const float2* __restrict__ xt, const float* __restrict__ nu, float* __restrict__ llr,
             int64_t total, int D, int n_sc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  demod_elem<Q>(xt, nu, llr, idx, D, n_sc);
}

}  // namespace

rxphy_status launch_demod(const rxphy_frame& fr, int32_t nf, const float2* xt, const float* nu,
                          float* llr, hipStream_t s) {
  const int D = fr.n_sym - 1;
  const int64_t total = (int64_t)nf * fr.K * D * fr.n_sc;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return fail(RXPHY_EUNSUPPORTED, "demod grid too large");
  switch (fr.qam_bits) {
    case 2: hipLaunchKernelGGL(demod_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, xt, nu, llr, total, D, fr.n_sc); break;
    case 4: hipLaunchKernelGGL(demod_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, s, xt, nu, llr, total, D, fr.n_sc); break;
    case 6: hipLaunchKernelGGL(demod_kernel<6>, dim3((unsigned)blocks), dim3(256), 0, s, xt, nu, llr, total, D, fr.n_sc); break;
    default: return fail(RXPHY_EINVAL, "qam_bits = %d", fr.qam_bits);
  }
  return launch_status("demod kernel");
}

}  // namespace rxphy
