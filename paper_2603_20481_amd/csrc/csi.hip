// csi stage: one launch over every (frame, antenna, 512-subcarrier tile); the
// estimate itself is csik::csi_tile.
#include "csi_core.h"

namespace rxphy {
namespace {

using namespace csik;

__global__ void __launch_bounds__(CSI_WG)
csi_kernel(const float2* __restrict__ yf, const float2* __restrict__ pil, float2* __restrict__ h,
           int M, int K, int S, int n_sc) {
  __shared__ float2 ls[CSI_LDS];
  const int m = blockIdx.y;
  const int f = blockIdx.z;
  csi_tile(yf + ((int64_t)(f * M + m) * S) * n_sc, pil + (int64_t)f * n_sc,
           h + ((int64_t)(f * M + m) * K) * n_sc, K, n_sc, blockIdx.x * CSI_TILE, ls);
}

}  // namespace

rxphy_status launch_csi(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                        float2* h, hipStream_t s) {
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  dim3 grid((fr.n_sc + CSI_TILE - 1) / CSI_TILE, fr.M, nf);
  hipLaunchKernelGGL(csi_kernel, grid, dim3(CSI_WG), 0, s, yf, pil, h, fr.M, fr.K, fr.n_sym, fr.n_sc);
  return launch_status("csi kernel");
}

}  // namespace rxphy
