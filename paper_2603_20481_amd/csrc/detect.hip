// equal stage: per-subcarrier ZF / MMSE detection for gfx950 (phase 1 and the
// factorisation live in detect_core.h).  The forward kernel adds the MMSE
// unbiasing x_tilde = x_hat / mu, the noise variances, the flags and the
// erasures, and writes x_tilde [F][K][D][n_sc], nu [F][K][n_sc], flags [F][n_sc].
// K is padded to KP in {4, 8, 16} (an identity block: same solution,
// straight-line phase 2).
#include "demod_core.h"
#include "detect_core.h"

namespace rxphy {
namespace {

using namespace det;

constexpr int TPB = 1;   // tiles per workgroup

// FU: fused CSI (H formed from the pilot symbol of Yf and the pilots pil).
template <int KP, int P, bool FU>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
detect_kernel(const float2* __restrict__ H, const float2* __restrict__ Yf,
              const float2* __restrict__ pil, float2* __restrict__ xt, float* __restrict__ nu,
              uint8_t* __restrict__ flags, int M, int K, int S, int n_sc, float n0, int mmse, float thr,
              uint32_t* __restrict__ rlist) {
  __shared__ float2 smem[SMEM_ALL];
  __shared__ int nonfin[TS];
  const int64_t f = blockIdx.y;
  // TPB consecutive tiles per workgroup: the first chunk of the next tile is
  // loaded while the current tile is being factored and solved
  const int nt = (n_sc + TS - 1) / TS;
  const int t0 = blockIdx.x * TPB;
  const int t1 = min(t0 + TPB, nt);
  float2 hv[8], yv[8], pv;
  bool have0 = false;
  for (int t = t0; t < t1; ++t) {
    if (t > t0) __syncthreads();
    detect_tile<KP, P, FU>(FU ? nullptr : H + f * M * K * n_sc, Yf + f * M * S * n_sc,
                           xt + f * K * (S - 1) * n_sc, nu + f * K * n_sc,
                           flags ? flags + f * n_sc : nullptr, M, K, S, n_sc, n0, mmse, thr, rlist,
                           (uint32_t)(f * n_sc), t * TS, smem, nonfin, hv, yv, pv, have0,
                           t + 1 < t1 ? (t + 1) * TS : -1, nullptr, nullptr,
                           FU ? pil + f * n_sc : nullptr);
  }
}

__global__ void clear_count_kernel(uint32_t* rlist) {
  if (threadIdx.x == 0) rlist[0] = 0u;
}

// ------------------------------------------------------------ FP64 refinement
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dmulcj(double2 a, double2 b) {   // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsc(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 d2(float2 v) { return make_double2((double)v.x, (double)v.y); }

constexpr int RP = 17;   // row pitch (double2) of the 16 x 16 work matrices

// One wavefront per listed subcarrier (grid-stride over the list): A and
// b = H^H y are re-formed in FP64 from the FP32 inputs, A = L L^H in FP64,
// refinement x <- x + A^{-1} (b - A x) from the low-precision x0, and
// d = diag(A^{-1}) from the FP64 factor; then the unbiasing, nu and flags.
// A subcarrier with a non-finite channel or data value is erased and flagged
// NONFINITE.  A start that is not finite (the low-precision factor broke down) becomes
// x0 = 0.  Two steps are taken: one step leaves a relative error of about
// kappa * eps64 times that of x0, and x0 carries no correct digit once
// kappa * u exceeds 1 (u = 2^-8 for BF16 operands, 2^-11 for FP16), which the
// refined subcarriers come close to or pass by construction; the second
// step brings every subcarrier with kappa * eps64 << 1 to FP64 accuracy.
//
// x0 may be null (start from 0); xt is written when not null; Q > 0 writes
// the max-log LLRs of the refined symbols into llr as the demod stage does.
template <int Q>
__global__ void __launch_bounds__(64)
refine_kernel(const float2* __restrict__ H, const float2* __restrict__ Yf,
              const float2* __restrict__ pil, const float2* __restrict__ x0, float2* __restrict__ xt,
              float* __restrict__ nu, uint8_t* __restrict__ flags, float* __restrict__ llr,
              const uint32_t* __restrict__ rlist, int M, int K, int S, int n_sc, float n0f, int mmse) {
  __shared__ double2 Hs[64 * 16];
  __shared__ double2 Ys[64 * 16];
  __shared__ double2 A[16 * RP];    // A, kept for the residuals
  __shared__ double2 Lf[16 * RP];   // its FP64 Cholesky factor
  __shared__ double2 Bv[16 * RP];   // b = H^H Y
  __shared__ double2 R[16 * RP];
  __shared__ double2 X[16 * RP];
  __shared__ double2 V[16 * RP];
  __shared__ double dd[16];
  __shared__ float nvs[16];
  __shared__ int bad, nfin;
  const int D = S - 1;
  const int tid = threadIdx.x;
  const double n0 = (double)n0f;
  const uint32_t count = rlist[0];
  for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
    const uint32_t sub = rlist[RL_OFF + e];
    const int f = (int)(sub / (uint32_t)n_sc), i = (int)(sub - (uint32_t)f * n_sc);
    if (tid == 0) nfin = 0;
    __syncthreads();
    // every lane's loads issued before the first is used: 16 channel and 16
    // data values at most per lane (M K <= 1024, M D <= 1024)
    {
      float2 hv[16], yv[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int q = tid + 64 * t;
        hv[t] = yv[t] = make_float2(0.f, 0.f);
        if (q < M * K) {
          const int m = q / K, u = q - m * K;
          if (pil) {                              // fused CSI: the LS estimate, as the CSI stage forms it
            const int G = n_sc / K, qq = min(i / K, G - 1) * K + u;
            hv[t] = ls_estimate(Yf[((int64_t)(f * M + m) * S) * n_sc + qq], pil[(int64_t)f * n_sc + qq]);
          } else {
            hv[t] = H[((int64_t)(f * M + m) * K + u) * n_sc + i];
          }
        }
        if (q < M * D) {
          const int m = q / D, s = q - m * D;
          yv[t] = Yf[((int64_t)(f * M + m) * S + 1 + s) * n_sc + i];
        }
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int q = tid + 64 * t;
        if (q < M * K) {
          if (!(isfinite(hv[t].x) && isfinite(hv[t].y))) nfin = 1;
          Hs[(q / K) * 16 + (q - (q / K) * K)] = d2(hv[t]);
        }
        if (q < M * D) {
          if (!(isfinite(yv[t].x) && isfinite(yv[t].y))) nfin = 1;
          Ys[(q / D) * 16 + (q - (q / D) * D)] = d2(yv[t]);
        }
      }
    }
    for (int q = tid; q < K * D; q += 64) {     // x0; a non-finite start becomes 0
      const int u = q / D, s = q - u * D;
      const float2 v = x0 ? x0[((int64_t)(f * K + u) * D + s) * n_sc + i] : make_float2(0.f, 0.f);
      X[u * RP + s] = (isfinite(v.x) && isfinite(v.y)) ? d2(v) : make_double2(0.0, 0.0);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int q = tid; q < K * K; q += 64) {                       // A = H^H H (+ N0 I)
      const int r = q / K, c = q - r * K;
      double2 acc = make_double2(0.0, 0.0);
      for (int m = 0; m < M; ++m) acc = dadd(acc, dmulcj(Hs[m * 16 + r], Hs[m * 16 + c]));
      if (r == c && mmse) acc.x += n0;
      A[r * RP + c] = acc;
      Lf[r * RP + c] = acc;
    }
    for (int q = tid; q < K * D; q += 64) {                       // b = H^H Y
      const int r = q / D, s = q - r * D;
      double2 acc = make_double2(0.0, 0.0);
      for (int m = 0; m < M; ++m) acc = dadd(acc, dmulcj(Hs[m * 16 + r], Ys[m * 16 + s]));
      Bv[r * RP + s] = acc;
    }
    __syncthreads();
    for (int j = 0; j < K; ++j) {                                 // Lf = L, A = L L^H
      if (tid == 0) {
        const double dj = Lf[j * RP + j].x;
        if (!(dj > 0.0) || !isfinite(dj)) bad = 1;
        Lf[j * RP + j] = make_double2(sqrt(dj), 0.0);
      }
      __syncthreads();
      const double ljj = Lf[j * RP + j].x;
      for (int r = j + 1 + tid; r < K; r += 64) Lf[r * RP + j] = dsc(Lf[r * RP + j], 1.0 / ljj);
      __syncthreads();
      const int w2 = K - j - 1;
      for (int q = tid; q < w2 * w2; q += 64) {
        const int r = j + 1 + q / w2, c = j + 1 + q % w2;
        if (c <= r) Lf[r * RP + c] = dsub(Lf[r * RP + c], dmul(Lf[r * RP + j], make_double2(Lf[c * RP + j].x, -Lf[c * RP + j].y)));
      }
      __syncthreads();
    }
    for (int step = 0; step < 2; ++step) {
      for (int q = tid; q < K * D; q += 64) {                     // residual b - A x
        const int r = q / D, s = q - r * D;
        double2 acc = Bv[r * RP + s];
        for (int k = 0; k < K; ++k) acc = dsub(acc, dmul(A[r * RP + k], X[k * RP + s]));
        R[r * RP + s] = acc;
      }
      __syncthreads();
      if (tid < D) {                                              // x += A^{-1} residual, per column
        const int s = tid;
        for (int r = 0; r < K; ++r) {
          double2 acc = R[r * RP + s];
          for (int k = 0; k < r; ++k) acc = dsub(acc, dmul(Lf[r * RP + k], R[k * RP + s]));
          R[r * RP + s] = dsc(acc, 1.0 / Lf[r * RP + r].x);
        }
        for (int r = K - 1; r >= 0; --r) {
          double2 acc = R[r * RP + s];
          for (int k = r + 1; k < K; ++k) acc = dsub(acc, dmulcj(Lf[k * RP + r], R[k * RP + s]));
          R[r * RP + s] = dsc(acc, 1.0 / Lf[r * RP + r].x);
          X[r * RP + s] = dadd(X[r * RP + s], R[r * RP + s]);
        }
      } else if (step == 0 && tid >= 32 && tid - 32 < K) {        // column u of L^{-1}: d_u
        const int u = tid - 32;
        double acc2 = 0.0;
        for (int r = 0; r < K; ++r) {
          double2 acc = make_double2(r == u ? 1.0 : 0.0, 0.0);
          for (int k = u; k < r; ++k) acc = dsub(acc, dmul(Lf[r * RP + k], V[k * RP + u]));
          const double2 vr = r < u ? make_double2(0.0, 0.0) : dsc(acc, 1.0 / Lf[r * RP + r].x);
          V[r * RP + u] = vr;
          acc2 += vr.x * vr.x + vr.y * vr.y;
        }
        dd[u] = acc2;
        if (mmse && !(1.0 - n0 * acc2 > 0.0)) bad = 1;
      }
      __syncthreads();
    }
    const bool erase = bad != 0 || nfin != 0;
    for (int u = tid; u < K; u += 64) {
      const double d = dd[u];
      const double nv = mmse ? n0 * d / (1.0 - n0 * d) : n0 * d;
      const float v = erase ? INFINITY : (float)nv;
      nvs[u] = v;
      nu[(int64_t)(f * K + u) * n_sc + i] = v;
    }
    __syncthreads();
    for (int q = tid; q < K * D; q += 64) {
      const int u = q / D, s = q - u * D;
      double2 x = X[u * RP + s];
      if (mmse) x = dsc(x, 1.0 / (1.0 - n0 * dd[u]));
      const float2 xf = erase ? make_float2(0.f, 0.f) : make_float2((float)x.x, (float)x.y);
      const int64_t e = ((int64_t)(f * K + u) * D + s) * n_sc + i;
      if (xt) xt[e] = xf;
      if constexpr (Q > 0) demk::demod_point<Q>(xf, nvs[u], llr + e * Q);
    }
    if (tid == 0 && flags)
      flags[(int64_t)f * n_sc + i] = nfin ? RXPHY_FLAG_NONFINITE : erase ? RXPHY_FLAG_BREAKDOWN : RXPHY_FLAG_REFINED;
    __syncthreads();
  }
}

// The 16-user fused path's refinement: one workgroup per listed pilot group
// (a 16-subcarrier tile, grid-stride over the list), whose subcarriers share
// one channel estimate.  H = the LS estimate of the group (FP64 from the FP32
// pilot symbol), A = H^H H (+ N0 I), its FP64 Cholesky factor and d =
// diag(A^{-1}) are formed once for the tile.  Every (subcarrier, symbol)
// right-hand side is then taken by 16 lanes, lane u holding row u, 32 of
// them at a time (two data symbols of the tile per round): b = H^H y,
// and from x = 0 two steps x <- x + A^{-1} (b - A x) (the steps of
// refine_kernel), the triangular solves column by column with the solved
// entry broadcast to the group.  The unbiased symbols wait in LDS until the
// tile's non-finite data values are known; then x_tilde, the LLRs (as the
// demod stage forms them), nu and the flags are written.  A non-finite
// estimate erases the tile; a non-finite data value erases its subcarrier
// (NONFINITE).
constexpr int RG_SYM = 2;                      // data symbols per round
constexpr int RG_THREADS = RG_SYM * 256;
template <int Q>
__global__ void __launch_bounds__(RG_THREADS)
refine_group_kernel(const float2* __restrict__ Yf, const float2* __restrict__ pil, float2* __restrict__ xt,
                    float* __restrict__ nu, uint8_t* __restrict__ flags, float* __restrict__ llr,
                    const uint32_t* __restrict__ rlist, int M, int S, int n_sc, float n0f, int mmse) {
  __shared__ double2 Hs[64 * 16];
  __shared__ double2 A[16 * RP];
  __shared__ double2 Lf[16 * RP];
  __shared__ double2 V[16 * RP];
  __shared__ float2 Xf[16 * 16 * 16];         // [subcarrier][symbol][user], unbiased
  __shared__ float2 Ys[RG_SYM * 64 * 16];     // the round's data: [symbol][antenna][subcarrier]
  __shared__ double dd[16];
  __shared__ int bad, hnf;
  __shared__ int snf[16];
  const int D = S - 1;
  const int tid = threadIdx.x, u = tid & 15, grp = tid >> 4;
  const double n0 = (double)n0f;
  const int nt = (n_sc + 15) / 16, G = n_sc / 16;
  const uint32_t count = rlist[0];
  for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t tile = rlist[RL_OFF + it];
    const int f = (int)(tile / (uint32_t)nt), tt = (int)(tile - (uint32_t)f * nt);
    const int i0 = tt * 16, cnt = min(16, n_sc - i0), g = min(tt, G - 1);
    if (tid == 0) { bad = 0; hnf = 0; }
    if (tid < 16) snf[tid] = 0;
    __syncthreads();
    for (int q = tid; q < M * 16; q += RG_THREADS) {     // the group's LS estimate
      const int m = q >> 4, uu = q & 15, qq = g * 16 + uu;
      const float2 hv = ls_estimate(Yf[((int64_t)(f * M + m) * S) * n_sc + qq], pil[(int64_t)f * n_sc + qq]);
      if (!(isfinite(hv.x) && isfinite(hv.y))) hnf = 1;
      Hs[m * 16 + uu] = d2(hv);
    }
    __syncthreads();
    if (tid < 256) {                                     // A = H^H H (+ N0 I), one entry per thread
      const int r = tid >> 4, c = tid & 15;
      double2 acc = make_double2(0.0, 0.0);
      for (int m = 0; m < M; ++m) acc = dadd(acc, dmulcj(Hs[m * 16 + r], Hs[m * 16 + c]));
      if (r == c && mmse) acc.x += n0;
      A[r * RP + c] = acc;
      Lf[r * RP + c] = acc;
    }
    __syncthreads();
    for (int j = 0; j < 16; ++j) {                       // Lf = L, A = L L^H
      if (tid == 0) {
        const double dj = Lf[j * RP + j].x;
        if (!(dj > 0.0) || !isfinite(dj)) bad = 1;
        Lf[j * RP + j] = make_double2(sqrt(dj), 0.0);
      }
      __syncthreads();
      const double ljj = Lf[j * RP + j].x;
      if (tid > j && tid < 16) Lf[tid * RP + j] = dsc(Lf[tid * RP + j], 1.0 / ljj);
      __syncthreads();
      const int w2 = 15 - j;
      if (tid < w2 * w2) {
        const int r = j + 1 + tid / w2, c = j + 1 + tid % w2;
        if (c <= r)
          Lf[r * RP + c] = dsub(Lf[r * RP + c], dmul(Lf[r * RP + j], make_double2(Lf[c * RP + j].x, -Lf[c * RP + j].y)));
      }
      __syncthreads();
    }
    if (tid < 16) {                                      // column u of L^{-1}: d_u
      double acc2 = 0.0;
      for (int r = 0; r < 16; ++r) {
        double2 acc = make_double2(r == tid ? 1.0 : 0.0, 0.0);
        for (int k = tid; k < r; ++k) acc = dsub(acc, dmul(Lf[r * RP + k], V[k * RP + tid]));
        const double2 vr = r < tid ? make_double2(0.0, 0.0) : dsc(acc, 1.0 / Lf[r * RP + r].x);
        V[r * RP + tid] = vr;
        acc2 += vr.x * vr.x + vr.y * vr.y;
      }
      dd[tid] = acc2;
      if (mmse && !(1.0 - n0 * acc2 > 0.0)) bad = 1;
    }
    __syncthreads();
    // right-hand sides: round s0 takes symbols s0 .. s0 + RG_SYM - 1; group grp the
    // subcarrier e = grp % 16 of symbol s0 + grp / 16; lane u = row u
    const double linv = 1.0 / Lf[u * RP + u].x;
    const double ub = mmse ? 1.0 / (1.0 - n0 * dd[u]) : 1.0;
    const int e = grp & 15, sl = grp >> 4;
    for (int s0 = 0; s0 < D; s0 += RG_SYM) {
      // the round's data into LDS, every load issued at once (consecutive
      // threads, consecutive subcarriers)
      {
        float2 yv[2 * RG_SYM];
#pragma unroll
        for (int t = 0; t < 2 * RG_SYM; ++t) {
          const int q = t * RG_THREADS + tid;            // [symbol][antenna][subcarrier]
          const int m = (q >> 4) & 63, ee = q & 15, s = s0 + (q >> 10);
          yv[t] = (s < D && m < M && ee < cnt) ? Yf[((int64_t)(f * M + m) * S + 1 + s) * n_sc + i0 + ee]
                                               : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int t = 0; t < 2 * RG_SYM; ++t) {
          if (!(isfinite(yv[t].x) && isfinite(yv[t].y))) snf[tid & 15] = 1;
          Ys[t * RG_THREADS + tid] = yv[t];
        }
      }
      __syncthreads();
      double2 b = make_double2(0.0, 0.0);
      for (int m = 0; m < M; ++m) b = dadd(b, dmulcj(Hs[m * 16 + u], d2(Ys[(sl * 64 + m) * 16 + e])));
      __syncthreads();                                   // Ys is rewritten by the next round
      const int s = s0 + sl;
      if (s >= D || e >= cnt) continue;                  // the group's 16 lanes together
      double2 x = make_double2(0.0, 0.0);
      for (int step = 0; step < 2; ++step) {
        double2 r = b;                                   // b - A x
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
          const double2 xk = make_double2(__shfl(x.x, k, 16), __shfl(x.y, k, 16));
          r = dsub(r, dmul(A[u * RP + k], xk));
        }
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {                   // L^-1, column k: entry k final, then eliminated below
          if (u == k) r = dsc(r, linv);
          const double2 rk = make_double2(__shfl(r.x, k, 16), __shfl(r.y, k, 16));
          if (u > k) r = dsub(r, dmul(Lf[u * RP + k], rk));
        }
#pragma unroll 4
        for (int k = 15; k >= 0; --k) {                  // L^-H, column k of L^H = conj of row k of L
          if (u == k) r = dsc(r, linv);
          const double2 rk = make_double2(__shfl(r.x, k, 16), __shfl(r.y, k, 16));
          if (u < k) r = dsub(r, dmulcj(Lf[k * RP + u], rk));
        }
        x = dadd(x, r);
      }
      const double2 xv = dsc(x, ub);
      Xf[(e * 16 + s) * 16 + u] = make_float2((float)xv.x, (float)xv.y);
    }
    __syncthreads();                                     // Xf, snf complete
    {
      const int ee = tid & 15;                           // consecutive lanes, consecutive subcarriers
      if (ee < cnt) {
        const int i = i0 + ee;
        const bool sub_nf = hnf != 0 || snf[ee] != 0;
        const bool erase = bad != 0 || sub_nf;
        for (int q = grp; q < 16 * D; q += RG_THREADS / 16) {
          const int uu = q / D, s = q - uu * D;
          const double d = dd[uu];
          const float nv = erase ? INFINITY : (float)(mmse ? n0 * d / (1.0 - n0 * d) : n0 * d);
          const float2 xf = erase ? make_float2(0.f, 0.f) : Xf[(ee * 16 + s) * 16 + uu];
          const int64_t ex = ((int64_t)(f * 16 + uu) * D + s) * n_sc + i;
          if (xt) xt[ex] = xf;
          if constexpr (Q > 0) demk::demod_point<Q>(xf, nv, llr + ex * Q);
        }
        if (grp < 16) {
          const int uu = grp;
          const double d = dd[uu];
          nu[(int64_t)(f * 16 + uu) * n_sc + i] = erase ? INFINITY : (float)(mmse ? n0 * d / (1.0 - n0 * d) : n0 * d);
        }
        if (grp == 0 && flags)
          flags[(int64_t)f * n_sc + i] = sub_nf ? RXPHY_FLAG_NONFINITE : erase ? RXPHY_FLAG_BREAKDOWN
                                                                              : RXPHY_FLAG_REFINED;
      }
    }
    __syncthreads();
  }
}

template <int KP, int P, bool FU>
void launch_one(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf, const float2* pil,
                float2* xt, float* nu, uint8_t* flags, float thr, uint32_t* rl, hipStream_t s) {
  dim3 grid(((fr.n_sc + TS - 1) / TS + TPB - 1) / TPB, nf);
  hipLaunchKernelGGL((detect_kernel<KP, P, FU>), grid, dim3(256), 0, s, h, yf, pil, xt, nu, flags, fr.M,
                     fr.K, fr.n_sym, fr.n_sc, fr.n0, fr.detector == RXPHY_MMSE ? 1 : 0, thr, rl);
}

template <int P, bool FU>
void launch_k(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf, const float2* pil,
              float2* xt, float* nu, uint8_t* flags, float thr, uint32_t* rl, hipStream_t s) {
  if (fr.K <= 4) launch_one<4, P, FU>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
  else if (fr.K <= 8) launch_one<8, P, FU>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
  else launch_one<16, P, FU>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
}

template <int P>
void launch_p(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf, const float2* pil,
              float2* xt, float* nu, uint8_t* flags, float thr, uint32_t* rl, hipStream_t s) {
  if (pil) launch_k<P, true>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
  else launch_k<P, false>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
}

}  // namespace

bool group_path(const rxphy_frame& fr, rxphy_precision) { return fr.K == 16; }

size_t csi_detect_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec) {
  if (group_path(fr, prec)) return group_workspace_bytes(fr, nf, prec);
  return detect_workspace_bytes(fr, nf, prec);
}

size_t csi_detect_demod_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec) {
  if (group_path(fr, prec)) return group_workspace_bytes(fr, nf, prec);
  const size_t a = (detect_workspace_bytes(fr, nf, prec) + 255) & ~(size_t)255;
  return a + (size_t)nf * fr.K * (fr.n_sym - 1) * fr.n_sc * 8;
}

size_t detect_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec) {
  if (prec == RXPHY_FP32) return 0;
  return (size_t)RL_OFF * 4 + (size_t)nf * fr.n_sc * 4;
}

rxphy_status launch_detect(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf,
                           const float2* pil, float2* xt, float* nu, uint8_t* flags, rxphy_precision prec,
                           float thr, void* ws, hipStream_t s) {
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  if (pil && group_path(fr, prec))
    return launch_detect_group(fr, nf, yf, pil, xt, nu, flags, nullptr, prec, thr, ws, s);
  if (prec == RXPHY_FP32) {
    launch_p<P_FP32>(fr, nf, h, yf, pil, xt, nu, flags, thr, nullptr, s);
    return launch_status("detect kernel");
  }
  uint32_t* rl = (uint32_t*)ws;
  hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(64), 0, s, rl);
  if (prec == RXPHY_BF16) launch_p<P_BF16>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
  else launch_p<P_FP16>(fr, nf, h, yf, pil, xt, nu, flags, thr, rl, s);
  rxphy_status st = launch_status("detect kernel");
  if (st) return st;
  return launch_refine(fr, nf, h, yf, pil, xt, xt, nu, flags, nullptr, rl, s);
}

rxphy_status launch_refine_group(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                 float2* xt, float* nu, uint8_t* flags, float* llr, const uint32_t* rl,
                                 hipStream_t s) {
  const int64_t n_tiles = (int64_t)nf * ((fr.n_sc + 15) / 16);
  const unsigned blocks = (unsigned)(n_tiles < 2048 ? n_tiles : 2048);
  const int mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
  const int q = llr ? fr.qam_bits : 0;
#define RXPHY_REFINE_G(QQ)                                                                                    \
  hipLaunchKernelGGL(refine_group_kernel<QQ>, dim3(blocks), dim3(RG_THREADS), 0, s, yf, pil, xt, nu, flags, llr, rl, \
                     fr.M, fr.n_sym, fr.n_sc, fr.n0, mmse)
  switch (q) {
    case 0: RXPHY_REFINE_G(0); break;
    case 2: RXPHY_REFINE_G(2); break;
    case 4: RXPHY_REFINE_G(4); break;
    default: RXPHY_REFINE_G(6); break;
  }
#undef RXPHY_REFINE_G
  return launch_status("group refine kernel");
}

rxphy_status launch_refine(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf,
                           const float2* pil, const float2* x0, float2* xt, float* nu, uint8_t* flags,
                           float* llr, const uint32_t* rl, hipStream_t s) {
  const int64_t n_sub = (int64_t)nf * fr.n_sc;
  const unsigned blocks = (unsigned)(n_sub < 4096 ? n_sub : 4096);
  const int mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
  const int q = llr ? fr.qam_bits : 0;
#define RXPHY_REFINE(QQ)                                                                                      \
  hipLaunchKernelGGL(refine_kernel<QQ>, dim3(blocks), dim3(64), 0, s, h, yf, pil, x0, xt, nu, flags, llr, rl, \
                     fr.M, fr.K, fr.n_sym, fr.n_sc, fr.n0, mmse)
  switch (q) {
    case 0: RXPHY_REFINE(0); break;
    case 2: RXPHY_REFINE(2); break;
    case 4: RXPHY_REFINE(4); break;
    default: RXPHY_REFINE(6); break;
  }
#undef RXPHY_REFINE
  return launch_status("refine kernel");
}

}  // namespace rxphy
