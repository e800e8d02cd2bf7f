// csi stage: least-squares channel estimate from comb pilots, held over the
// pilot group.  One thread per (frame, antenna, user, subcarrier); threads of a
// wave cover consecutive subcarriers, so the H write is fully coalesced and the
// gathered symbol-0 reads of a group hit the same cache line.
#include "common.h"

namespace rxphy {
namespace {

__global__ void __launch_bounds__(256)
csi_kernel(const float2* __restrict__ yf, const float2* __restrict__ pil, float2* __restrict__ h,
           int M, int K, int S, int n_sc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_sc) return;
  const int mu = blockIdx.y;            // m * K + u
  const int f = blockIdx.z;
  const int m = mu / K, u = mu - m * K;
  const int G = n_sc / K;
  const int g = min(i / K, G - 1);
  const int q = g * K + u;
  const float2 y = yf[((int64_t)(f * M + m) * S) * n_sc + q];
  const float2 p = pil[(int64_t)f * n_sc + q];
  const float pp = p.x * p.x + p.y * p.y;
  // y * conj(p) / |p|^2 ; a zero pilot gives 0/0 = NaN, flagged downstream
  const float2 e = make_float2((y.x * p.x + y.y * p.y) / pp, (y.y * p.x - y.x * p.y) / pp);
  h[((int64_t)(f * M + m) * K + u) * n_sc + i] = e;
}

}  // namespace

rxphy_status launch_csi(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                        float2* h, hipStream_t s) {
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  dim3 grid((fr.n_sc + 255) / 256, fr.M * fr.K, nf);
  hipLaunchKernelGGL(csi_kernel, grid, dim3(256), 0, s, yf, pil, h, fr.M, fr.K, fr.n_sym, fr.n_sc);
  return launch_status("csi kernel");
}

}  // namespace rxphy
