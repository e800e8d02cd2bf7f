// equal stage: per-subcarrier ZF / MMSE detection for gfx950.
//
// Workgroup = 4 wavefronts = a tile of 16 consecutive subcarriers of one
// frame; each wavefront owns 4 of them.
//
// Phase 1 (products on MFMA).  H and the data symbols are streamed through
// LDS in chunks of 8 antennas: 16 threads load the 16 subcarriers of one
// (antenna, user) or (antenna, symbol) row as one 128-byte coalesced segment.
// Per subcarrier the wave accumulates, with v_mfma_f32_16x16x4_f32 and the
// antenna index as the reduction axis (4 antennas per instruction),
//   Re G = A^T A + B^T B,   Im G = A^T B - B^T A        (H = A + jB)
//   Re Z = A^T C + B^T D,   Im Z = A^T D - B^T C        (Y = C + jD)
// i.e. the Gram matrix G = H^H H and the matched filter Z = H^H Y, each lane
// supplying one (antenna, user) channel value and one (antenna, symbol) data
// value per step; both operands of the Gram come from the same register.
//
// Phase 2 (small dense algebra on VALU).  G and Z go through a wave-private
// LDS slab so that, for each subcarrier, lane t of its 16-lane row holds row t
// of A (= G, or G + N0 I) and column t of Z.  A Cholesky-Crout factorisation
// runs column by column with the row of L being used broadcast by DPP
// row_newbcast; forward substitution solves L W = Z and L V = I together (V
// is L^{-1}, whose squared column norms are d = diag(A^{-1})), then back
// substitution solves L^H X = W.
#include "common.h"

namespace rxphy {
namespace {

constexpr int TS = 16;              // subcarriers per workgroup tile
constexpr int MC = 8;               // antennas per staged chunk
constexpr int PITCH = TS + 1;       // float2 per staged row (bank spread)
constexpr int ROWS = MC * 16;       // staged rows per tensor (K, D <= 16)
constexpr int PP = 17;              // float2 per row of a 16x16 matrix in the slab
constexpr int PMAT = 16 * PP;       // float2 per matrix
constexpr int SMEM = 2 * ROWS * PITCH;
static_assert(16 * PMAT <= SMEM, "post-phase slab must fit in the staging area");

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int L>
__device__ __forceinline__ float bc(float v) {   // lane L of each 16-lane row, to the whole row
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + L, 0xF, 0xF, false));
}
template <int L>
__device__ __forceinline__ float2 bc2(float2 v) { return make_float2(bc<L>(v.x), bc<L>(v.y)); }

__device__ __forceinline__ float2 cmul_cj(float2 a, float2 b) {   // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ bool finite2(float2 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Cholesky-Crout of the row-distributed A (lane `row` holds a[c] = A[row][c]).
// On exit a[c] = L[row][c] for c <= row and inv[j] = 1 / L[j][j] in every lane.
template <int J>
__device__ __forceinline__ void crout_step(float2* a, float* inv, int row, int K, bool& ok) {
  if (J >= K) return;
  float2 s = a[J];
#pragma unroll
  for (int k = 0; k < J; ++k) s = csub(s, cmulc(a[k], bc2<J>(a[k])));   // - L[row][k] conj(L[J][k])
  const float d = bc<J>(s.x);                                            // pivot from lane J
  ok = ok && (d > 0.f) && __builtin_isfinite(d);
  const float ljj = sqrtf(d);
  const float iv = 1.0f / ljj;
  inv[J] = iv;
  a[J] = row == J ? make_float2(ljj, 0.f) : (row > J ? cscale(s, iv) : a[J]);
}

// Forward substitution of two right-hand sides held per lane (w, v).
template <int I>
__device__ __forceinline__ void fwd_step(const float2* a, const float* inv, float2* w, float2* v, int K) {
  if (I >= K) return;
  float2 sw = w[I], sv = v[I];
#pragma unroll
  for (int k = 0; k < I; ++k) {
    const float2 lik = bc2<I>(a[k]);                                     // L[I][k]
    sw = csub(sw, cmul(lik, w[k]));
    sv = csub(sv, cmul(lik, v[k]));
  }
  w[I] = cscale(sw, inv[I]);
  v[I] = cscale(sv, inv[I]);
}

template <int... Js>
struct Seq {};
using Seq16 = Seq<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15>;

// Back substitution L^H x = w (in place): x[I] = (w[I] - sum_{k>I} conj(L[k][I]) x[k]) / L[I][I].
template <int I, int KK>
__device__ __forceinline__ void bwd_term(const float2* a, const float2* w, float2& sx, int K) {
  if constexpr (KK > I) {
    if (KK < K) sx = csub(sx, cmul_cj(bc2<KK>(a[I]), w[KK]));
  }
}
template <int I, int... Ks>
__device__ __forceinline__ void bwd_terms(Seq<Ks...>, const float2* a, const float2* w, float2& sx, int K) {
  (bwd_term<I, Ks>(a, w, sx, K), ...);
}
template <int I>
__device__ __forceinline__ void bwd_step(const float2* a, const float* inv, float2* w, int K) {
  if (I >= K) return;
  float2 sx = w[I];
  bwd_terms<I>(Seq16{}, a, w, sx, K);
  w[I] = cscale(sx, inv[I]);
}

template <int... Js>
__device__ __forceinline__ void crout_all(Seq<Js...>, float2* a, float* inv, int row, int K, bool& ok) {
  (crout_step<Js>(a, inv, row, K, ok), ...);
}
template <int... Is>
__device__ __forceinline__ void fwd_all(Seq<Is...>, const float2* a, const float* inv, float2* w, float2* v, int K) {
  (fwd_step<Is>(a, inv, w, v, K), ...);
}
template <int... Is>
__device__ __forceinline__ void bwd_all(Seq<Is...>, const float2* a, const float* inv, float2* w, int K) {
  (bwd_step<15 - Is>(a, inv, w, K), ...);
}
template <int U>
__device__ __forceinline__ void bcast_mu(float dl, float n0, float* mu) { mu[U] = 1.0f - n0 * bc<U>(dl); }
template <int... Us>
__device__ __forceinline__ void bcast_mu_all(Seq<Us...>, float dl, float n0, float* mu) {
  (bcast_mu<Us>(dl, n0, mu), ...);
}

__global__ void __launch_bounds__(256)
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
#pragma unroll
  for (int t = 0; t < 4; ++t) gr[t] = gi[t] = zr[t] = zi[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  float2* Hs = smem;
  float2* Ys = smem + ROWS * PITCH;
  const float2* Hf = H + (int64_t)f * M * K * n_sc;
  const float2* Yff = Yf + (int64_t)f * M * S * n_sc;
  const int c16 = tid & 15;
  const int ic = i0 + c16;
  const bool in_range = ic < n_sc;
  const int u = l & 15, kq = l >> 4;

  // chunk loads go to registers first (all issued back to back) and the next
  // chunk is prefetched while the current one feeds the MFMAs
  float2 hv[8], yv[8];
  auto load_chunk = [&](int m0) {
    const int mc = min(MC, M - m0);
    const int rh = mc * K, ry = mc * D;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int r = (tid >> 4) + 16 * it;
      hv[it] = (in_range && r < rh) ? Hf[(int64_t)(m0 * K + r) * n_sc + ic] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int r = (tid >> 4) + 16 * it;
      const int ml = r / D, s = r - ml * D;
      yv[it] = (in_range && r < ry) ? Yff[(int64_t)((m0 + ml) * S + 1 + s) * n_sc + ic]
                                    : make_float2(0.f, 0.f);
    }
  };
  load_chunk(0);
  for (int m0 = 0; m0 < M; m0 += MC) {
    const int mc = min(MC, M - m0);
    bool bad = false;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int r = (tid >> 4) + 16 * it;
      bad |= !finite2(hv[it]) || !finite2(yv[it]);
      if (r < ROWS) {
        Hs[r * PITCH + c16] = hv[it];
        Ys[r * PITCH + c16] = yv[it];
      }
    }
    if (bad) nonfin[c16] = 1;
    __syncthreads();
    if (m0 + MC < M) load_chunk(m0 + MC);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (4 * a < mc) {
        const int ml = 4 * a + kq;
        const bool okh = ml < mc && u < K;
        const bool oky = ml < mc && u < D;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int sc = 4 * w + t;
          const float2 h = okh ? Hs[(ml * K + u) * PITCH + sc] : make_float2(0.f, 0.f);
          const float2 y = oky ? Ys[(ml * D + u) * PITCH + sc] : make_float2(0.f, 0.f);
          gr[t] = mfma(h.x, h.x, gr[t]);
          gr[t] = mfma(h.y, h.y, gr[t]);
          gi[t] = mfma(h.x, h.y, gi[t]);
          gi[t] = mfma(-h.y, h.x, gi[t]);
          zr[t] = mfma(h.x, y.x, zr[t]);
          zr[t] = mfma(h.y, y.y, zr[t]);
          zi[t] = mfma(h.x, y.y, zi[t]);
          zi[t] = mfma(-h.y, y.x, zi[t]);
        }
      }
    }
    __syncthreads();
  }

  // ---- phase 2: G and Z of this wave's 4 subcarriers through its LDS slab
  float2* P = smem + w * 4 * PMAT;
  const int col = l & 15, g4 = (l >> 4) * 4;      // MFMA output: rows g4 + r, column col
  const int scl = l >> 4, row = l & 15;           // phase-2 lane: subcarrier scl, index row
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[t * PMAT + (g4 + r) * PP + col] = make_float2(gr[t][r], gi[t][r]);
  __syncthreads();
  float2 a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = P[scl * PMAT + row * PP + c];
    if (mmse && c == row) a[c].x += n0;
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[t * PMAT + (g4 + r) * PP + col] = make_float2(zr[t][r], zi[t][r]);
  __syncthreads();
  float2 z[16], v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    z[k] = P[scl * PMAT + k * PP + row];          // column `row` of Z
    v[k] = make_float2(k == row ? 1.f : 0.f, 0.f);  // column `row` of I
  }

  bool ok = true;
  float inv[16];
  crout_all(Seq16{}, a, inv, row, K, ok);
  fwd_all(Seq16{}, a, inv, z, v, K);
  bwd_all(Seq16{}, a, inv, z, K);
  float dl = 0.f;                                  // d_row = sum_k |L^{-1}[k][row]|^2
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < K) dl += v[k].x * v[k].x + v[k].y * v[k].y;

  float mu[16];
  bcast_mu_all(Seq16{}, dl, n0, mu);
  bool mu_bad = mmse && row < K && !(1.0f - n0 * dl > 0.f);
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
        if (mmse) x = cscale(x, 1.0f / mu[uu]);
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
      nv = n0 * dl / (1.0f - n0 * dl);
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
  hipLaunchKernelGGL(detect_fp32_kernel, grid, dim3(256), 0, s, h, yf, xt, nu, flags, fr.M, fr.K,
                     fr.n_sym, fr.n_sc, fr.n0, fr.detector == RXPHY_MMSE ? 1 : 0);
  return launch_status("detect kernel");
}

}  // namespace rxphy
