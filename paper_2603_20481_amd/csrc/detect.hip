// equal stage: per-subcarrier ZF / MMSE detection for gfx950 (phase 1 and the
// factorisation live in detect_core.h).  The forward kernel adds the MMSE
// unbiasing x_tilde = x_hat / mu, the noise variances, the flags and the
// erasures, and writes x_tilde [F][K][D][n_sc], nu [F][K][n_sc], flags [F][n_sc].
#include "detect_core.h"

namespace rxphy {
namespace {

using namespace det;

template <int KP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
detect_fp32_kernel(const float2* __restrict__ H, const float2* __restrict__ Yf,
                   float2* __restrict__ xt, float* __restrict__ nu, uint8_t* __restrict__ flags,
                   int M, int K, int S, int n_sc, float n0, int mmse) {
  __shared__ float2 smem[SMEM];
  __shared__ int nonfin[TS];
  const int f = blockIdx.y;
  const int i0 = blockIdx.x * TS;
  const int D = S - 1;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  if (tid < TS) nonfin[tid] = 0;
  __syncthreads();

  f32x4 gr[4], gi[4], zr[4], zi[4];
  gram_mf(H + (int64_t)f * M * K * n_sc, Yf + (int64_t)f * M * S * n_sc, M, K, S, n_sc, i0, smem,
          nonfin, gr, gi, zr, zi);

  // ---- phase 2
  float2* P = smem + w * 4 * PMAT;
  const int col = l & 15, g4 = (l >> 4) * 4;      // MFMA output: rows g4 + r, column col
  const int scl = l >> 4, row = l & 15;           // phase-2 lane: subcarrier scl, index row
  float2* Pm = P + scl * PMAT;
  float2 z[16], v[16];
  float inv[16], dl;
  bool ok;
  factor_solve<KP>(P, Pm, gr, gi, zr, zi, K, n0, mmse, row, col, g4, z, v, inv, dl, ok);
  if (mmse) unbias_all<KP>(Seq16{}, dl, n0, K, z);

  const bool mu_bad = mmse && row < K && !(1.0f - n0 * dl > 0.f);
  const uint64_t bal = __ballot(mu_bad);
  if ((bal >> (16 * scl)) & 0xffffull) ok = false;

  const int i = i0 + 4 * w + scl;
  if (i >= n_sc) return;
  const bool nf = nonfin[4 * w + scl] != 0;
  const bool erase = nf || !ok;
  if (row < D) {
#pragma unroll
    for (int uu = 0; uu < 16; ++uu) {
      if (uu < K) {
        float2 x = z[uu];
        if (erase) x = make_float2(0.f, 0.f);
        xt[((int64_t)(f * K + uu) * D + row) * n_sc + i] = x;
      }
    }
  }
  if (row < K) {
    float nv;
    if (mmse) {
      // (1 - mu) / mu with 1 - mu = N0 d formed directly: subtracting mu from 1
      // would cancel most digits for strong users (mu close to 1)
      nv = n0 * dl * __builtin_amdgcn_rcpf(1.0f - n0 * dl);
    } else {
      nv = n0 * dl;
    }
    nu[(int64_t)(f * K + row) * n_sc + i] = erase ? INFINITY : nv;
  }
  if (row == 0 && flags) flags[(int64_t)f * n_sc + i] = nf ? RXPHY_FLAG_NONFINITE : (ok ? 0 : RXPHY_FLAG_BREAKDOWN);
}

}  // namespace

rxphy_status launch_detect(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf,
                           float2* xt, float* nu, uint8_t* flags, rxphy_precision prec, float thr,
                           hipStream_t s) {
  (void)thr;
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  if (prec != RXPHY_FP32) return fail(RXPHY_EUNSUPPORTED, "precision %d not built yet", (int)prec);
  dim3 grid((fr.n_sc + TS - 1) / TS, nf);
  const int mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
  if (fr.K <= 4)
    hipLaunchKernelGGL(detect_fp32_kernel<4>, grid, dim3(256), 0, s, h, yf, xt, nu, flags, fr.M, fr.K,
                       fr.n_sym, fr.n_sc, fr.n0, mmse);
  else if (fr.K <= 8)
    hipLaunchKernelGGL(detect_fp32_kernel<8>, grid, dim3(256), 0, s, h, yf, xt, nu, flags, fr.M, fr.K,
                       fr.n_sym, fr.n_sc, fr.n0, mmse);
  else
    hipLaunchKernelGGL(detect_fp32_kernel<16>, grid, dim3(256), 0, s, h, yf, xt, nu, flags, fr.M, fr.K,
                       fr.n_sym, fr.n_sc, fr.n0, mmse);
  return launch_status("detect kernel");
}

}  // namespace rxphy
