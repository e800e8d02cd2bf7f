// Adjoint of the receiver map x -> LLR (FP32), and workspace sizing.
//
// Gradients use PyTorch's complex convention g = dL/dRe + j dL/dIm.  The
// backward pass recomputes the forward quantities it needs (the Cholesky
// factors are recomputed per subcarrier, never stored) and runs, in order:
//   demod adjoint   dLLR_j/dx = 2 (l0 - l1) / nu on the bit's axis (l_b the
//                   nearest level with bit b, ties to the lowest point index),
//                   dLLR_j/dnu = -LLR_j / nu;
//   detect adjoint  with A = H^H H (+ N0 I), X_hat = A^{-1} H^H Y,
//                   G_hat = dL/dX_hat (MMSE: dL/dx_tilde / mu), e_u the weight
//                   of d_u = [A^{-1}]_uu (ZF: N0 dL/dnu_u; MMSE:
//                   N0 (Re sum_s conj(g_su) x_hat_su + dL/dnu_u) / mu_u^2),
//                   V = A^{-1} G_hat and C = X_hat V^H + V X_hat^H + 2 A^{-1} E A^{-1}:
//                   dL/dY = H V,  dL/dH = Y V^H - H C;
//   csi adjoint     dL/dYf0[q] = p[q] / |p[q]|^2 * sum over the pilot group of
//                   dL/dH[m][u][i] (q = g K + u; 0 past the last full group
//                   and where the pilot is zero);
//   fft adjoint     the unscaled inverse-direction DFT of the used-bin gradient
//                   (zero-padded grid), cyclic-prefix samples get 0.
#include <cstring>

#include "abi_checks.h"
#include "detect_core.h"

namespace rxphy {
namespace {

using namespace det;

// ----------------------------------------------------------------- demod adjoint
template <int Q>
__device__ __forceinline__ float lvl(int code) {
  constexpr int B = Q / 2;
  if constexpr (B == 1) {
    return (code & 1) ? -0.70710678118654752f : 0.70710678118654752f;
  } else if constexpr (B == 2) {
    const float s0 = (code & 2) ? -1.f : 1.f, s1 = (code & 1) ? -1.f : 1.f;
    return s0 * (2.f - s1) * 0.31622776601683793f;
  } else {
    const float s0 = (code & 4) ? -1.f : 1.f, s1 = (code & 2) ? -1.f : 1.f, s2 = (code & 1) ? -1.f : 1.f;
    return s0 * (4.f - s1 * (2.f - s2)) * 0.15430334996209191f;
  }
}

// Nearest levels with bit t = 0 / 1 on one axis (strict < keeps the lowest code).
template <int Q>
__device__ __forceinline__ void axis_argmin(float x, float* l0, float* l1) {
  constexpr int B = Q / 2;
  float d0[B], d1[B];
#pragma unroll
  for (int t = 0; t < B; ++t) { d0[t] = d1[t] = INFINITY; l0[t] = l1[t] = 0.f; }
#pragma unroll
  for (int code = 0; code < (1 << B); ++code) {
    const float lv = lvl<Q>(code);
    const float d = (x - lv) * (x - lv);
#pragma unroll
    for (int t = 0; t < B; ++t) {
      if ((code >> (B - 1 - t)) & 1) { if (d < d1[t]) { d1[t] = d; l1[t] = lv; } }
      else                           { if (d < d0[t]) { d0[t] = d; l0[t] = lv; } }
    }
  }
}

template <int Q>
__global__ void __launch_bounds__(256)
demod_adjoint_kernel(const float2* __restrict__ xt, const float* __restrict__ nu,
                     const float* __restrict__ dllr, float2* __restrict__ gxt,
                     float* __restrict__ gnu, int64_t n_fu, int D, int n_sc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (f, u, i)
  if (idx >= n_fu * n_sc) return;
  const int64_t fu = idx / n_sc;
  const int i = (int)(idx - fu * n_sc);
  const float v = nu[idx];
  const bool erased = __builtin_isinf(v);
  const float inv = erased ? 0.f : 1.0f / v;
  float gn = 0.f;
  for (int s = 0; s < D; ++s) {
    const int64_t e = (fu * D + s) * n_sc + i;
    const float2 x = xt[e];
    const float* dl = dllr + e * Q;
    float re0[Q / 2], re1[Q / 2], im0[Q / 2], im1[Q / 2];
    axis_argmin<Q>(x.x, re0, re1);
    axis_argmin<Q>(x.y, im0, im1);
    float gr = 0.f, gi = 0.f;
#pragma unroll
    for (int t = 0; t < Q / 2; ++t) {
      const float a = dl[2 * t], b = dl[2 * t + 1];
      const float lr = (re0[t] - re1[t]) * (2.f * x.x - re0[t] - re1[t]) * inv;
      const float li = (im0[t] - im1[t]) * (2.f * x.y - im0[t] - im1[t]) * inv;
      gr += a * 2.f * (re0[t] - re1[t]) * inv;
      gi += b * 2.f * (im0[t] - im1[t]) * inv;
      gn -= (a * lr + b * li) * inv;
    }
    gxt[e] = erased ? make_float2(0.f, 0.f) : make_float2(gr, gi);
  }
  gnu[idx] = erased ? 0.f : gn;
}

// ---------------------------------------------------------------- detect adjoint
// MMSE gains of every user in every lane of the row; padded users (U >= K)
// get 1 so that their zero rows stay exactly zero.
template <int U>
__device__ __forceinline__ void gather_mu(float dl, float n0, int mmse, int K, float* mu) {
  const float m = 1.0f - n0 * bc<U>(dl);
  mu[U] = (mmse && U < K) ? m : 1.0f;
}
template <int... Us>
__device__ __forceinline__ void gather_mu_all(Seq<Us...>, float dl, float n0, int mmse, int K, float* mu) {
  (gather_mu<Us>(dl, n0, mmse, K, mu), ...);
}
template <int U>
__device__ __forceinline__ void gather_e(float e, float* ek) { ek[U] = bc<U>(e); }
template <int... Us>
__device__ __forceinline__ void gather_e_all(Seq<Us...>, float e, float* ek) { (gather_e<Us>(e, ek), ...); }

// Per subcarrier (one 16-lane row of a wave each): recompute the factor and
// X_hat, then solve V = A^{-1} G_hat (lane = data symbol) and A^{-1} (lane =
// column).  Writes X_hat and V [F][n_sc][K][D], A^{-1} [F][n_sc][K][K] and the
// weights e [F][n_sc][K]; all zero for erased subcarriers.
template <int KP>
__global__ void __launch_bounds__(256)
detect_adjoint_kernel(const float2* __restrict__ H, const float2* __restrict__ Yf,
                      const float2* __restrict__ gxt, const float* __restrict__ gnu,
                      float2* __restrict__ Xw, float2* __restrict__ Vw, float2* __restrict__ Aw,
                      float* __restrict__ Ew, int M, int K, int S, int n_sc, float n0, int mmse) {
  __shared__ float2 smem[SMEM];
  __shared__ int nonfin[TS];
  const int f = blockIdx.y;
  const int i0 = blockIdx.x * TS;
  const int D = S - 1;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  if (tid < TS) nonfin[tid] = 0;
  __syncthreads();

  f32x4 gr[4], gi[4], zr[4], zi[4];
  float2 hv[8], yv[8], pv;
  gram_mf(H + (int64_t)f * M * K * n_sc, Yf + (int64_t)f * M * S * n_sc, M, K, S, n_sc, i0, smem,
          nonfin, gr, gi, zr, zi, hv, yv, pv);
  float2* P = smem + w * 4 * PMAT;
  const int col = l & 15, g4 = (l >> 4) * 4;
  const int scl = l >> 4, row = l & 15;
  float2* Pm = P + scl * PMAT;                       // holds L after factor_solve
  float2 x[16], v[16];
  float inv[16], dl;
  bool ok;
  factor_solve<KP>(P, Pm, gr, gi, zr, zi, K, n0, mmse, row, col, g4, x, v, inv, dl, ok);

  const int i = i0 + 4 * w + scl;
  const bool in_i = i < n_sc;
  float mu[16];
  gather_mu_all(Seq16{}, dl, n0, mmse, K, mu);
  const bool mu_bad = mmse && row < K && !(1.0f - n0 * dl > 0.f);
  const uint64_t bal = __ballot(mu_bad);
  if ((bal >> (16 * scl)) & 0xffffull) ok = false;
  const bool erase = !in_i || nonfin[4 * w + scl] != 0 || !ok;
  const int64_t sub = (int64_t)f * n_sc + i;

  // incoming gradients: lane `row` = symbol s holds column s of dL/dx_tilde
  float2 g[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    g[u] = (!erase && row < D && u < K) ? gxt[((int64_t)(f * K + u) * D + row) * n_sc + i]
                                       : make_float2(0.f, 0.f);
    if (erase) x[u] = make_float2(0.f, 0.f);
  }
  const float gn = (!erase && row < K) ? gnu[(int64_t)(f * K + row) * n_sc + i] : 0.f;

  // e_row, the weight of d_row, and G_hat
  float e;
  if (mmse) {
    float mine = 0.f, mr = 1.f;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const float t = row_sum(g[u].x * x[u].x + g[u].y * x[u].y);   // sum_s Re(conj(g_su) x_su)
      if (u == row) { mine = t; mr = mu[u]; }
    }
    e = n0 * (mine + gn) / (mr * mr);
#pragma unroll
    for (int u = 0; u < 16; ++u) g[u] = cscale(g[u], 1.0f / mu[u]);
  } else {
    e = n0 * gn;
  }
  if (in_i && row < D) {
#pragma unroll
    for (int u = 0; u < KP; ++u) if (u < K) Xw[(sub * K + u) * D + row] = x[u];
  }
  if (in_i && row < K) Ew[sub * K + row] = erase ? 0.f : e;

  fwd_all<KP>(Seq16{}, Pm, inv, g);                // V column s = A^{-1} G_hat column s
  bwd_all<KP>(Seq16{}, Pm, inv, g);
  bwd_all<KP>(Seq16{}, Pm, inv, v);                // column `row` of A^{-1} = L^{-H} L^{-1} e_row
  if (!in_i) return;
  if (row < D) {
#pragma unroll
    for (int u = 0; u < KP; ++u) if (u < K) Vw[(sub * K + u) * D + row] = erase ? make_float2(0.f, 0.f) : g[u];
  }
  if (row < K) {
#pragma unroll
    for (int k = 0; k < KP; ++k) if (k < K) Aw[(sub * K + k) * K + row] = erase ? make_float2(0.f, 0.f) : v[k];
  }
}

// C = X_hat V^H + V X_hat^H + 2 A^{-1} diag(e) A^{-1} per (frame, subcarrier)
// entry (i, j).  A workgroup stages the X_hat, V, A^{-1} and e of c_ns(K, D)
// consecutive subcarriers in LDS (they are contiguous in the workspace, so
// the loads coalesce) and its threads take the ns K^2 entries in turn: up to
// 1024 entries and 2048 X_hat / V values per workgroup, so that each one
// moves enough bytes to keep the loads of a CU's few workgroups in flight.
// Cw: [F][n_sc][K][K].
constexpr int C_NS_MAX = 64;
constexpr int C_XV = 2048;       // X_hat (and V) values staged per workgroup
constexpr int C_ENT = 1024;      // C entries per workgroup
inline __host__ __device__ int c_ns(int K, int D) {
  int ns = C_NS_MAX;
  ns = ns < C_ENT / (K * K) ? ns : C_ENT / (K * K);
  ns = ns < C_XV / (K * D) ? ns : C_XV / (K * D);
  return ns > 0 ? ns : 1;
}
__global__ void __launch_bounds__(256)
detect_adjoint_c_kernel(const float2* __restrict__ Xw, const float2* __restrict__ Vw,
                        const float2* __restrict__ Aw, const float* __restrict__ Ew,
                        float2* __restrict__ Cw, int64_t n_sub, int K, int D) {
  __shared__ float2 sx[C_XV], sv[C_XV], sa[C_ENT];
  __shared__ float se[C_ENT];
  const int KK = K * K;
  const int NS = c_ns(K, D);
  const int64_t s0 = (int64_t)blockIdx.x * NS;
  const int ns = (int)min((int64_t)NS, n_sub - s0);
  const int tid = threadIdx.x;
  {
    // every load of the workgroup issued before the first LDS store
    const int nxv = ns * K * D, na = ns * KK, ne = ns * K;
    float2 rx[C_XV / 256], rv[C_XV / 256], ra[C_ENT / 256];
    float re[C_ENT / 256];
#pragma unroll
    for (int k = 0; k < C_XV / 256; ++k) {
      const int e = tid + k * 256;
      rx[k] = e < nxv ? Xw[s0 * K * D + e] : make_float2(0.f, 0.f);
      rv[k] = e < nxv ? Vw[s0 * K * D + e] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < C_ENT / 256; ++k) {
      const int e = tid + k * 256;
      ra[k] = e < na ? Aw[s0 * KK + e] : make_float2(0.f, 0.f);
      re[k] = e < ne ? Ew[s0 * K + e] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < C_XV / 256; ++k) {
      const int e = tid + k * 256;
      if (e < nxv) {
        sx[e] = rx[k];
        sv[e] = rv[k];
      }
    }
#pragma unroll
    for (int k = 0; k < C_ENT / 256; ++k) {
      const int e = tid + k * 256;
      if (e < na) sa[e] = ra[k];
      if (e < ne) se[e] = re[k];
    }
  }
  __syncthreads();
  for (int t = tid; t < ns * KK; t += 256) {
    const int sl = t / KK, r = t - sl * KK;
    const int ii = r / K, j = r - ii * K;
    const float2* X = sx + sl * K * D;
    const float2* V = sv + sl * K * D;
    const float2* A = sa + sl * KK;
    const float* E = se + sl * K;
    float2 acc = make_float2(0.f, 0.f);
    for (int s = 0; s < D; ++s) {
      acc = cms_bc(acc, X[ii * D + s], make_float2(-V[j * D + s].x, -V[j * D + s].y));  // + x[ii][s] conj(v[j][s])
      acc = cms_bc(acc, V[ii * D + s], make_float2(-X[j * D + s].x, -X[j * D + s].y));  // + v[ii][s] conj(x[j][s])
    }
    for (int k = 0; k < K; ++k) {
      const float2 a = A[k * K + ii];
      acc = cms_ac(acc, make_float2(-a.x, -a.y), cscale(A[k * K + j], 2.f * E[k]));  // + conj(A[k][ii]) 2 e_k A[k][j]
    }
    Cw[(s0 + sl) * KK + r] = acc;
  }
}

// dL/dY = H V into the data symbols of gyf, dL/dH = Y V^H - H C into gh.
// Workgroup: 16 subcarriers x 32 antennas of one frame, V and C of the 16
// subcarriers staged in LDS; each thread takes one subcarrier and two
// antennas (m and m + 16), so that every V and C value read from LDS serves
// two antennas.  The staged V and C are zero past K users and D symbols (and
// H and Y past them read as zero), so the products run over the compile-time
// bounds KP and DP (DP = 13 for the 14-symbol slot, else 16) with no run-time
// branch between a load and its use: the compiler's memory waits then count
// down the loads in flight instead of draining them (and the stores) at
// every branch join.
template <int KP, int DP>
__global__ void __launch_bounds__(256)
detect_adjoint_apply_kernel(const float2* __restrict__ H, const float2* __restrict__ Yf,
                            const float2* __restrict__ Vw, const float2* __restrict__ Cw,
                            float2* __restrict__ gyf, float2* __restrict__ gh, int M, int K,
                            int S, int n_sc) {
  // per-subcarrier pitches padded by one float2: the 16 subcarrier lanes of a
  // wave then read 16 different bank pairs
  constexpr int VP = KP * DP + 1, CP = KP * KP + 1;
  __shared__ float2 sv[16 * VP];
  __shared__ float2 sc[16 * CP];
  const int D = S - 1;
  const int f = blockIdx.z;
  const int i0 = blockIdx.x * 16, m0 = blockIdx.y * 32;
  const int il = threadIdx.x & 15, ml = threadIdx.x >> 4;
  const int ntile = min(16, n_sc - i0);
  for (int e = threadIdx.x; e < 16 * KP * DP; e += 256) {
    const int t = e / (KP * DP), r = e - t * (KP * DP);
    const int u = r / DP, s2 = r - u * DP;
    sv[t * VP + r] = (t < ntile && u < K && s2 < D) ? Vw[((int64_t)f * n_sc + i0 + t) * K * D + u * D + s2]
                                                     : make_float2(0.f, 0.f);
  }
  for (int e = threadIdx.x; e < 16 * KP * KP; e += 256) {
    const int t = e / (KP * KP), r = e - t * (KP * KP);
    const int a = r / KP, b = r - a * KP;
    sc[t * CP + r] = (t < ntile && a < K && b < K) ? Cw[((int64_t)f * n_sc + i0 + t) * K * K + a * K + b]
                                                    : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int i = i0 + il;
  if (i >= n_sc || m0 + ml >= M) return;
  const bool two = m0 + ml + 16 < M;
  float2 h[2][KP], y[2][DP];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int m = m0 + ml + 16 * a;
    const bool in = a == 0 || two;
#pragma unroll
    for (int u = 0; u < KP; ++u)
      h[a][u] = (in && u < K) ? H[((int64_t)(f * M + m) * K + u) * n_sc + i] : make_float2(0.f, 0.f);
#pragma unroll
    for (int s2 = 0; s2 < DP; ++s2)
      y[a][s2] = (in && s2 < D) ? Yf[((int64_t)(f * M + m) * S + 1 + s2) * n_sc + i] : make_float2(0.f, 0.f);
  }
  const float2* V = sv + il * VP;
  const float2* C = sc + il * CP;
  float2* gy0 = gyf + ((int64_t)(f * M + m0 + ml) * S + 1) * n_sc + i;
  float2* gy1 = gy0 + (int64_t)16 * S * n_sc;
#pragma unroll
  for (int s2 = 0; s2 < DP; ++s2) {
    float2 acc0 = make_float2(0.f, 0.f), acc1 = acc0;
#pragma unroll
    for (int u = 0; u < KP; ++u) {
      const float2 nv = make_float2(-V[u * DP + s2].x, -V[u * DP + s2].y);
      acc0 = cms(acc0, h[0][u], nv);
      acc1 = cms(acc1, h[1][u], nv);
    }
    if (s2 < D) {
      gy0[(int64_t)s2 * n_sc] = acc0;
      if (two) gy1[(int64_t)s2 * n_sc] = acc1;
    }
  }
  float2* gh0 = gh + ((int64_t)(f * M + m0 + ml) * K) * n_sc + i;
  float2* gh1 = gh0 + (int64_t)16 * K * n_sc;
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    float2 acc0 = make_float2(0.f, 0.f), acc1 = acc0;
#pragma unroll
    for (int s2 = 0; s2 < DP; ++s2) {
      const float2 nv = make_float2(-V[u * DP + s2].x, -V[u * DP + s2].y);
      acc0 = cms_bc(acc0, y[0][s2], nv);                                    // + y conj(V)
      acc1 = cms_bc(acc1, y[1][s2], nv);
    }
#pragma unroll
    for (int v2 = 0; v2 < KP; ++v2) {
      const float2 c = C[v2 * KP + u];
      acc0 = cms(acc0, h[0][v2], c);                                        // - H C
      acc1 = cms(acc1, h[1][v2], c);
    }
    if (u < K) {
      gh0[(int64_t)u * n_sc] = acc0;
      if (two) gh1[(int64_t)u * n_sc] = acc1;
    }
  }
}

// ------------------------------------------------------------------ csi adjoint
__global__ void __launch_bounds__(256)
csi_adjoint_kernel(const float2* __restrict__ gh, const float2* __restrict__ pil,
                   float2* __restrict__ gyf, int M, int K, int S, int n_sc) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_sc) return;
  const int m = blockIdx.y, f = blockIdx.z;
  const int G = n_sc / K;
  float2 out = make_float2(0.f, 0.f);
  if (q < G * K) {
    const int g = q / K, u = q - g * K;
    const int lo = g * K, hi = (g == G - 1) ? n_sc : lo + K;
    const float2* row = gh + ((int64_t)(f * M + m) * K + u) * n_sc;
    float2 acc = make_float2(0.f, 0.f);
    for (int i = lo; i < hi; ++i) acc = cadd(acc, row[i]);
    const float2 p = pil[(int64_t)f * n_sc + q];
    const float pp = p.x * p.x + p.y * p.y;
    if (pp > 0.f) out = cmul(acc, make_float2(p.x / pp, p.y / pp));
  }
  gyf[((int64_t)(f * M + m) * S) * n_sc + q] = out;
}

// Sum over each aligned group of 2^LK lanes, returned in every lane of the
// group: an xor butterfly on DPP (quad permutations [1,0,3,2] and [2,3,0,1],
// then the half-row and row mirrors, which pair each 4- / 8-lane block with
// the other one of its 8- / 16-lane group).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int LK>
__device__ __forceinline__ float seg_sum(float v) {
  if constexpr (LK >= 1) v += dpp_f<0xB1>(v);
  if constexpr (LK >= 2) v += dpp_f<0x4E>(v);
  if constexpr (LK >= 3) v += dpp_f<0x141>(v);
  if constexpr (LK >= 4) v += dpp_f<0x140>(v);
  return v;
}

// The CSI adjoint for K = 2^LK users: the pilot groups are aligned blocks of
// K lanes (a workgroup's 256 subcarriers hold whole groups), so thread i
// reads subcarrier i of every user's row (each load a contiguous 512-byte
// wavefront segment), the group sums come from the butterfly, and lane
// i = g K + u keeps user u's; the last group also takes the subcarriers past
// G K, as csi_adjoint_kernel does.
template <int LK>
__global__ void __launch_bounds__(256)
csi_adjoint_pow2_kernel(const float2* __restrict__ gh, const float2* __restrict__ pil,
                        float2* __restrict__ gyf, int M, int S, int n_sc) {
  constexpr int K = 1 << LK;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int m = blockIdx.y, f = blockIdx.z;
  const int G = n_sc / K;
  const int u_me = i & (K - 1);
  const float2* rows = gh + (int64_t)(f * M + m) * K * n_sc;
  float2 v[K];
#pragma unroll
  for (int u = 0; u < K; ++u) v[u] = i < n_sc ? rows[(int64_t)u * n_sc + i] : make_float2(0.f, 0.f);
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const float2 g = make_float2(seg_sum<LK>(v[u].x), seg_sum<LK>(v[u].y));
    if (u == u_me) acc = g;
  }
  if (i >= n_sc) return;
  float2 out = make_float2(0.f, 0.f);
  if (i < G * K) {
    if (i >= (G - 1) * K)
      for (int j = G * K; j < n_sc; ++j) acc = cadd(acc, rows[(int64_t)u_me * n_sc + j]);
    const float2 p = pil[(int64_t)f * n_sc + i];
    const float pp = p.x * p.x + p.y * p.y;
    if (pp > 0.f) out = cmul(acc, make_float2(p.x / pp, p.y / pp));
  }
  gyf[((int64_t)(f * M + m) * S) * n_sc + i] = out;
}

constexpr size_t ALIGN = 256;
inline size_t up(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

struct BwdLayout {
  size_t yf, h, xt, nu, flags, gxt, gnu, xh, v, a, e, c, gyf, gh, total;
};

BwdLayout layout(const rxphy_frame& f, int32_t F) {
  const size_t n = (size_t)F, M = f.M, K = f.K, S = f.n_sym, D = f.n_sym - 1, sc = f.n_sc;
  BwdLayout L{};
  size_t o = 0;
  L.yf = o; o += up(n * M * S * sc * 8);
  L.h = o; o += up(n * M * K * sc * 8);
  L.xt = o; o += up(n * K * D * sc * 8);
  L.nu = o; o += up(n * K * sc * 4);
  L.flags = o; o += up(n * sc);
  L.gxt = o; o += up(n * K * D * sc * 8);
  L.gnu = o; o += up(n * K * sc * 4);
  L.xh = o; o += up(n * sc * K * D * 8);
  L.v = o; o += up(n * sc * K * D * 8);
  L.a = o; o += up(n * sc * K * K * 8);
  L.e = o; o += up(n * sc * K * 4);
  L.c = o; o += up(n * sc * K * K * 8);
  L.gyf = o; o += up(n * M * S * sc * 8);
  L.gh = o; o += up(n * M * K * sc * 8);
  L.total = o;
  return L;
}

}  // namespace
}  // namespace rxphy

using namespace rxphy;

extern "C" {

size_t rxphy_workspace_bytes(const rxphy_frame* frame, int32_t n_frames, int32_t which,
                             int32_t precision_in) {
  if (!valid_precision(precision_in) || check_frame(frame, n_frames) != RXPHY_OK) return 0;
  const rxphy_precision precision = (rxphy_precision)precision_in;
  if (which == RXPHY_WS_DETECT) return detect_workspace_bytes(*frame, n_frames, precision);
  if (which == RXPHY_WS_CSI_DETECT) return csi_detect_workspace_bytes(*frame, n_frames, precision);
  if (which == RXPHY_WS_CSI_DETECT_DEMOD) return csi_detect_demod_workspace_bytes(*frame, n_frames, precision);
  if (which == RXPHY_WS_PRECODE) return frame->K == 16 ? group_workspace_bytes(*frame, n_frames, RXPHY_FP32) : 0;
  if (which == RXPHY_WS_BACKWARD) return layout(*frame, n_frames).total;
  return 0;
}

rxphy_status rxphy_backward(const rxphy_frame* frame, int32_t n_frames, const void* x,
                            const void* pilots, const rxphy_saved* saved, const float* dllr,
                            void* dx, void* dh, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(x, "x")) || (st = check_ptr(pilots, "pilots")) || (st = check_ptr(dllr, "dllr")) ||
      (st = check_ptr(dx, "dx")))
    return st;
  if (n_frames > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", n_frames);
  const rxphy_frame& fr = *frame;
  const BwdLayout L = layout(fr, n_frames);
  if (!ws || ws_bytes < L.total)
    return fail(RXPHY_EWORKSPACE, "backward needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  char* w = (char*)ws;
  const float2* yf = (saved && saved->yf) ? (const float2*)saved->yf : (const float2*)(w + L.yf);
  const float2* h = (saved && saved->h) ? (const float2*)saved->h : (const float2*)(w + L.h);
  const bool have_xt = saved && saved->xt && saved->nu;
  const float2* xt = have_xt ? (const float2*)saved->xt : (const float2*)(w + L.xt);
  const float* nu = have_xt ? saved->nu : (const float*)(w + L.nu);
  uint8_t* flags = (uint8_t*)(w + L.flags);
  float2* gxt = (float2*)(w + L.gxt);
  float* gnu = (float*)(w + L.gnu);
  float2* Xw = (float2*)(w + L.xh);
  float2* Vw = (float2*)(w + L.v);
  float2* Aw = (float2*)(w + L.a);
  float* Ew = (float*)(w + L.e);
  float2* Cw = (float2*)(w + L.c);
  float2* gyf = (float2*)(w + L.gyf);
  float2* gh = dh ? (float2*)dh : (float2*)(w + L.gh);
  const int64_t n_tr = (int64_t)n_frames * fr.M * fr.n_sym;

  if (!(saved && saved->yf))
    if ((st = launch_fft(fr, n_tr, (const float2*)x, (float2*)(w + L.yf), false, stream))) return st;
  if (!(saved && saved->h))
    if ((st = launch_csi(fr, n_frames, yf, (const float2*)pilots, (float2*)(w + L.h), stream))) return st;
  if (!have_xt)
    if ((st = launch_detect(fr, n_frames, h, yf, nullptr, (float2*)(w + L.xt), (float*)(w + L.nu), flags,
                            RXPHY_FP32, 0.f, nullptr, stream)))
      return st;

  const int D = fr.n_sym - 1;
  const int64_t n_fu = (int64_t)n_frames * fr.K;
  const unsigned blocks = (unsigned)((n_fu * fr.n_sc + 255) / 256);
  switch (fr.qam_bits) {
    case 2: hipLaunchKernelGGL(demod_adjoint_kernel<2>, dim3(blocks), dim3(256), 0, stream, xt, nu, dllr, gxt, gnu, n_fu, D, fr.n_sc); break;
    case 4: hipLaunchKernelGGL(demod_adjoint_kernel<4>, dim3(blocks), dim3(256), 0, stream, xt, nu, dllr, gxt, gnu, n_fu, D, fr.n_sc); break;
    default: hipLaunchKernelGGL(demod_adjoint_kernel<6>, dim3(blocks), dim3(256), 0, stream, xt, nu, dllr, gxt, gnu, n_fu, D, fr.n_sc); break;
  }
  if ((st = launch_status("demod adjoint kernel"))) return st;

  const int mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
  dim3 g1((fr.n_sc + TS - 1) / TS, n_frames);
  dim3 g2((fr.n_sc + 15) / 16, (fr.M + 31) / 32, n_frames);
  const int64_t n_sub = (int64_t)n_frames * fr.n_sc;
  const int cns = c_ns(fr.K, D);
  const unsigned gc = (unsigned)((n_sub + cns - 1) / cns);
#define RXPHY_ADJ(KP)                                                                               \
  hipLaunchKernelGGL(detect_adjoint_kernel<KP>, g1, dim3(256), 0, stream, h, yf, gxt, gnu, Xw, Vw,  \
                     Aw, Ew, fr.M, fr.K, fr.n_sym, fr.n_sc, fr.n0, mmse);                          \
  if ((st = launch_status("detect adjoint kernel"))) return st;                                     \
  hipLaunchKernelGGL(detect_adjoint_c_kernel, dim3(gc), dim3(256), 0, stream, Xw, Vw, Aw, Ew, Cw,   \
                     n_sub, fr.K, D);                                                              \
  if ((st = launch_status("detect adjoint c kernel"))) return st;                                   \
  if (D == 13)                                                                                      \
    hipLaunchKernelGGL((detect_adjoint_apply_kernel<KP, 13>), g2, dim3(256), 0, stream, h, yf, Vw, Cw, \
                       gyf, gh, fr.M, fr.K, fr.n_sym, fr.n_sc);                                       \
  else                                                                                              \
    hipLaunchKernelGGL((detect_adjoint_apply_kernel<KP, 16>), g2, dim3(256), 0, stream, h, yf, Vw, Cw, \
                       gyf, gh, fr.M, fr.K, fr.n_sym, fr.n_sc);
  if (fr.K <= 4) { RXPHY_ADJ(4) } else if (fr.K <= 8) { RXPHY_ADJ(8) } else { RXPHY_ADJ(16) }
#undef RXPHY_ADJ
  if ((st = launch_status("detect adjoint apply kernel"))) return st;

  dim3 g3((fr.n_sc + 255) / 256, fr.M, n_frames);
  const float2* pl = (const float2*)pilots;
  switch (fr.K) {
    case 1: hipLaunchKernelGGL(csi_adjoint_pow2_kernel<0>, g3, dim3(256), 0, stream, gh, pl, gyf, fr.M, fr.n_sym, fr.n_sc); break;
    case 2: hipLaunchKernelGGL(csi_adjoint_pow2_kernel<1>, g3, dim3(256), 0, stream, gh, pl, gyf, fr.M, fr.n_sym, fr.n_sc); break;
    case 4: hipLaunchKernelGGL(csi_adjoint_pow2_kernel<2>, g3, dim3(256), 0, stream, gh, pl, gyf, fr.M, fr.n_sym, fr.n_sc); break;
    case 8: hipLaunchKernelGGL(csi_adjoint_pow2_kernel<3>, g3, dim3(256), 0, stream, gh, pl, gyf, fr.M, fr.n_sym, fr.n_sc); break;
    case 16: hipLaunchKernelGGL(csi_adjoint_pow2_kernel<4>, g3, dim3(256), 0, stream, gh, pl, gyf, fr.M, fr.n_sym, fr.n_sc); break;
    default: hipLaunchKernelGGL(csi_adjoint_kernel, g3, dim3(256), 0, stream, gh, pl, gyf, fr.M, fr.K, fr.n_sym, fr.n_sc);
  }
  if ((st = launch_status("csi adjoint kernel"))) return st;
  return launch_fft(fr, n_tr, gyf, (float2*)dx, true, stream);
}

}  // extern "C"
