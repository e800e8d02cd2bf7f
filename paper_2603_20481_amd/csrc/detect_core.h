// Device code shared by the detector and its adjoint.
//
// Phase 1 (products on MFMA).  A workgroup of 4 wavefronts owns a tile of 16
// consecutive subcarriers of one frame, each wavefront 4 of them.  H and the
// data symbols stream through LDS in chunks of 8 antennas: 16 threads load the
// 16 subcarriers of one (antenna, user) or (antenna, symbol) row as one
// 128-byte segment, into registers first (all loads issued back to back) with
// the next chunk prefetched while the current one feeds the MFMAs.  Per
// subcarrier the wave accumulates, with v_mfma_f32_16x16x4_f32 and the antenna
// as the reduction axis (4 antennas per instruction),
//   Re G = A^T A + B^T B,   Im G = A^T B - B^T A        (H = A + jB)
//   Re Z = A^T C + B^T D,   Im Z = A^T D - B^T C        (Y = C + jD)
// i.e. the Gram matrix G = H^H H and the matched filter Z = H^H Y; each lane
// supplies one (antenna, user) channel value and one (antenna, symbol) data
// value per step, and both operands of the Gram come from the same register.
//
// Phase 2 (small dense algebra on VALU).  G and Z pass through a wave-private
// LDS slab so that, for each subcarrier, lane t of its 16-lane row holds row t
// of A (= G, or G + N0 I).  A Cholesky-Crout factorisation runs column by
// column with the current row of L broadcast by DPP row_newbcast; the solve
// L V = I is folded into the same steps (V = L^{-1}; its squared column norms
// are d = diag(A^{-1})).  L then replaces Z in the slab and the forward and
// back substitutions for column t of Z read it as LDS broadcasts.  K is padded
// to KP in {4, 8, 16} with an identity block, which leaves the solution of the
// K x K system unchanged and keeps phase 2 free of runtime bounds.
#pragma once

#include "common.h"

namespace rxphy {
namespace det {

constexpr int TS = 16;              // subcarriers per workgroup tile
constexpr int MC = 8;               // antennas per staged chunk
constexpr int PITCH = TS + 1;       // float2 per staged row (bank spread)
constexpr int ROWS = MC * 16;       // staged rows per tensor (K, D <= 16)
constexpr int PP = 17;              // float2 per row of a 16x16 matrix in the slab
constexpr int PMAT = 16 * PP + 4;   // float2 per matrix (the 4 matrices of a wave land on distinct banks)
constexpr int SMEM = (2 * ROWS * PITCH > 16 * PMAT) ? 2 * ROWS * PITCH : 16 * PMAT;

// LDS of the shared-factor path (tiles whose 16 subcarriers carry one
// channel matrix): the four waves' partial Gram matrices, the one factor L,
// 1 / L_kk, d_k = [A^-1]_kk and the tile's flags.
struct SharedFactor {
  float2 part[4][16 * PP];
  float2 L[16 * PP];
  float inv[16];
  float dl[16];
  float afro2;          // ||A||_F^2 (the condition estimate of the mixed precisions)
  int ok;
  int uniform;
};
constexpr int SMEM_ALL = SMEM + (int)((sizeof(SharedFactor) + sizeof(float2) - 1) / sizeof(float2));

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int L>
__device__ __forceinline__ float bc(float v) {   // lane L of each 16-lane row, to the whole row
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + L, 0xF, 0xF, true));
}
template <int L>
__device__ __forceinline__ float2 bc2(float2 v) { return make_float2(bc<L>(v.x), bc<L>(v.y)); }

// Sum of v over the 16 lanes of each DPP row, returned in every lane of the row.
__device__ __forceinline__ float row_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x111, 0xF, 0xF, true));  // row_shr:1
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x112, 0xF, 0xF, true));  // row_shr:2
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x114, 0xF, 0xF, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x118, 0xF, 0xF, true));  // row_shr:8
  return bc<15>(v);
}

// Condition estimate of the mixed precisions: kappa_est = ||A||_F tr(A^{-1})
// from the squared Frobenius norm of A and d_k = [A^{-1}]_kk.  Since
// ||A||_F >= lambda_max and tr(A^{-1}) >= 1 / lambda_min it never falls below
// kappa_2(A), and it exceeds it by at most K^1.5.
__device__ __forceinline__ float cond_estimate(float afro2, float trace_inv) {
  return __builtin_sqrtf(afro2) * trace_inv;
}

// Complex multiply-subtract kernels written as four FMAs each.
__device__ __forceinline__ float2 cms(float2 s, float2 a, float2 b) {      // s - a b
  s.x = fmaf(-a.x, b.x, s.x); s.x = fmaf(a.y, b.y, s.x);
  s.y = fmaf(-a.x, b.y, s.y); s.y = fmaf(-a.y, b.x, s.y);
  return s;
}
__device__ __forceinline__ float2 cms_bc(float2 s, float2 a, float2 b) {   // s - a conj(b)
  s.x = fmaf(-a.x, b.x, s.x); s.x = fmaf(-a.y, b.y, s.x);
  s.y = fmaf(-a.y, b.x, s.y); s.y = fmaf(a.x, b.y, s.y);
  return s;
}
__device__ __forceinline__ float2 cms_ac(float2 s, float2 a, float2 b) {   // s - conj(a) b
  s.x = fmaf(-a.x, b.x, s.x); s.x = fmaf(-a.y, b.y, s.x);
  s.y = fmaf(-a.x, b.y, s.y); s.y = fmaf(a.y, b.x, s.y);
  return s;
}

__device__ __forceinline__ bool finite2(float2 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Operand precision of the phase-1 products.
enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP16 = 2 };

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// 16x16x16 product with 4 operand values per lane (k = 4 (lane / 16) + v),
// operands rounded to nearest even from FP32, FP32 accumulation.
template <int P>
__device__ __forceinline__ f32x4 mfma_lp(float a0, float a1, float a2, float a3, float b0, float b1,
                                         float b2, float b3, f32x4 c) {
  if constexpr (P == P_BF16) {
    const bf16x4 a = {(__bf16)a0, (__bf16)a1, (__bf16)a2, (__bf16)a3};
    const bf16x4 b = {(__bf16)b0, (__bf16)b1, (__bf16)b2, (__bf16)b3};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                     __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
  } else {
    const f16x4 a = {(_Float16)a0, (_Float16)a1, (_Float16)a2, (_Float16)a3};
    const f16x4 b = {(_Float16)b0, (_Float16)b1, (_Float16)b2, (_Float16)b3};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
}

// Cholesky-Crout of the row-distributed A (lane `row` holds a[c] = A[row][c]).
// On exit a[c] = L[row][c] for c < row and inv[j] = 1 / L[j][j] in every lane.
// Step J also advances L V = I by one row: row J of L (k < J) is final after
// step J-1 and is already being broadcast, so v[J] = (v[J] - sum_k L[J][k] v[k]) / L[J][J].
template <int J, int KP>
__device__ __forceinline__ void crout_step(float2* a, float2* v, float* inv, int row, bool& ok) {
  if constexpr (J < KP) {
    float2 s = a[J], sv = v[J];
#pragma unroll
    for (int k = 0; k < J; ++k) {
      const float2 ljk = bc2<J>(a[k]);                                   // L[J][k]
      s = cms_bc(s, a[k], ljk);                                          // - L[row][k] conj(L[J][k])
      sv = cms(sv, ljk, v[k]);
    }
    const float d = bc<J>(s.x);                                          // pivot from lane J
    ok = ok && (d > 0.f) && __builtin_isfinite(d);
    const float iv = __builtin_amdgcn_rsqf(d);                           // 1 / L[J][J]
    inv[J] = iv;
    // every lane scales: rows above J produce upper-triangle values and the
    // diagonal lane gets ~(L[J][J], 0); neither is ever read (solves use inv[])
    a[J] = cscale(s, iv);
    v[J] = cscale(sv, iv);
    // pin each step's results to its step: left free, the compiler may sink
    // the arithmetic to the last use and keep every row of L alive at once
    asm volatile("" : "+v"(a[J].x), "+v"(a[J].y), "+v"(v[J].x), "+v"(v[J].y));
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Forward substitution L W = Z for the right-hand side held by this lane; row
// I of L is read from the wave's LDS slab (the 16 lanes of a row read the same
// address, a broadcast).
template <int I, int KP>
__device__ __forceinline__ void fwd_step(const float2* Lm, const float* inv, float2* w) {
  if constexpr (I >= KP) return;
  float2 sw = w[I];
#pragma unroll
  for (int k = 0; k < I; ++k) sw = cms(sw, Lm[I * PP + k], w[k]);      // - L[I][k] w[k]
  w[I] = cscale(sw, inv[I]);
  asm volatile("" : "+v"(w[I].x), "+v"(w[I].y));                        // pinned, see crout_step
  __builtin_amdgcn_sched_barrier(0);
}

template <int... Js>
struct Seq {};
using Seq16 = Seq<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15>;

// Back substitution L^H x = w (in place): x[I] = (w[I] - sum_{k>I} conj(L[k][I]) x[k]) / L[I][I].
template <int I, int KP>
__device__ __forceinline__ void bwd_step(const float2* Lm, const float* inv, float2* w) {
  if constexpr (I >= KP) return;
  float2 sx = w[I];
#pragma unroll
  for (int k = I + 1; k < KP; ++k) sx = cms_ac(sx, Lm[k * PP + I], w[k]);
  w[I] = cscale(sx, inv[I]);
  asm volatile("" : "+v"(w[I].x), "+v"(w[I].y));                        // pinned, see crout_step
  __builtin_amdgcn_sched_barrier(0);
}

template <int KP, int... Js>
__device__ __forceinline__ void crout_all(Seq<Js...>, float2* a, float2* v, float* inv, int row, bool& ok) {
  (crout_step<Js, KP>(a, v, inv, row, ok), ...);
}
template <int KP, int... Is>
__device__ __forceinline__ void fwd_all(Seq<Is...>, const float2* Lm, const float* inv, float2* w) {
  (fwd_step<Is, KP>(Lm, inv, w), ...);
}
template <int KP, int... Is>
__device__ __forceinline__ void bwd_all(Seq<Is...>, const float2* Lm, const float* inv, float2* w) {
  (bwd_step<15 - Is, KP>(Lm, inv, w), ...);
}
// MMSE: x_tilde_u = x_hat_u / mu_u with mu_u = 1 - N0 d_u, d_u held by lane u
// (padded users, u >= K, are left as they are).
template <int U, int KP>
__device__ __forceinline__ void unbias(float dl, float n0, int K, bool keep, float2* z) {
  if constexpr (U < KP) {
    const float r = __builtin_amdgcn_rcpf(1.0f - n0 * bc<U>(dl));   // every lane joins the DPP
    if (U < K && !keep) z[U] = cscale(z[U], r);
  }
}
template <int KP, int... Us>
__device__ __forceinline__ void unbias_all(Seq<Us...>, float dl, float n0, int K, bool keep, float2* z) {
  (unbias<Us, KP>(dl, n0, K, keep, z), ...);
}


// Phase 1 for the tile starting at subcarrier i0 of one frame (Hf, Yff point at
// that frame).  Accumulators: gr/gi = Re/Im G, zr/zi = Re/Im Z, one per
// subcarrier of the wave, in MFMA output layout (lane l: rows 4(l/16)+r,
// column l%16).  nonfin[c] is set for tile subcarriers with non-finite input.
// Byte-offset buffer loads: a lane whose offset is at or past the end of the
// buffer reads zero without touching memory (the hardware range check of a
// raw buffer resource), so absent rows and subcarriers need neither a branch
// nor a select.
constexpr uint32_t OOB = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float2 ld2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Loads 8-antenna chunk m0 of the tile at i0 into registers: lane (rb, c16)
// with rb = tid / 16 gets slot rb of antenna m0 + it for it = 0..7, i.e.
// H[m0 + it][rb][i0 + c16] and Y[m0 + it][1 + rb][i0 + c16]; absent slots,
// antennas and subcarriers read zero.  The byte offsets are a lane constant
// plus it times a uniform stride, and all 16 loads are issued back to back.
// FU (fused CSI): instead of H, hv gets the pilot-symbol value Y[m][0][q] of
// the lane's pilot subcarrier q = g(i) K + rb and pv its pilot p[q]; the LS
// estimate is formed when the chunk is staged (stage_h), after the loads have
// landed.
template <bool FU>
__device__ __forceinline__ void load_chunk(const float2* __restrict__ Hf, const float2* __restrict__ Yff,
                                           const float2* __restrict__ pil, int M, int K, int S, int n_sc,
                                           int i0, int m0, float2* hv, float2* yv, float2& pv) {
  const int tid = tid_x();
  const int rb = tid >> 4, ic = i0 + (tid & 15);
  const int D = S - 1;
  const __amdgpu_buffer_rsrc_t yrs = rsrc(Yff, (uint32_t)M * S * n_sc * 8u);
  const bool in_range = ic < n_sc;
  const uint32_t y_lane = in_range && rb < D ? (uint32_t)((1 + rb) * n_sc + ic) * 8u : OOB;
  const uint32_t y_ant = (uint32_t)S * n_sc * 8u;
  const int mc = min(MC, M - m0);
  if constexpr (!FU) {
    const __amdgpu_buffer_rsrc_t hrs = rsrc(Hf, (uint32_t)M * K * n_sc * 8u);
    const uint32_t h_lane = in_range && rb < K ? (uint32_t)(rb * n_sc + ic) * 8u : OOB;
    const uint32_t h_ant = (uint32_t)K * n_sc * 8u;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const uint32_t a = (uint32_t)(m0 + it);
      hv[it] = ld2(hrs, it < mc ? h_lane + a * h_ant : OOB);
      yv[it] = ld2(yrs, it < mc ? y_lane + a * y_ant : OOB);
    }
  } else {
    const int G = n_sc / K;
    const int q = min(ic / K, G - 1) * K + rb;
    const bool hok = in_range && rb < K;
    const uint32_t q_lane = hok ? (uint32_t)q * 8u : OOB;
    if (m0 == 0) pv = ld2(rsrc(pil, (uint32_t)n_sc * 8u), q_lane);
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const uint32_t a = (uint32_t)(m0 + it);
      hv[it] = ld2(yrs, it < mc ? q_lane + a * y_ant : OOB);
      yv[it] = ld2(yrs, it < mc ? y_lane + a * y_ant : OOB);
    }
  }
}

// The channel value a lane stages for (antenna m0 + it, its user slot): the
// loaded H, or with FU the LS estimate from the loaded pilot-symbol value
// (zero for absent users, antennas and subcarriers).
template <bool FU>
__device__ __forceinline__ float2 stage_h(float2 h, float2 pv, int it, int M, int K, int n_sc, int i0,
                                          int m0) {
  if constexpr (!FU) {
    return h;
  } else {
    const int tid = tid_x();
    const bool ok = (tid >> 4) < K && i0 + (tid & 15) < n_sc && it < min(MC, M - m0);
    return ok ? ls_estimate(h, pv) : make_float2(0.f, 0.f);
  }
}

// Phase 1: Gram matrix and matched filter of the tile's 16 subcarriers.
// H and the data symbols are staged per 8-antenna chunk as [antenna][16 slots]
// rows (slot = user for H, data symbol for Y; absent slots, antennas and
// subcarriers hold zero), so the MFMA loop reads them unmasked.  A
// subcarrier with a non-finite input gets nonfin[c] = 1.
template <int P = P_FP32, bool FU = false>
__device__ __forceinline__ void gram_mf(const float2* __restrict__ Hf, const float2* __restrict__ Yff,
                                        int M, int K, int S, int n_sc, int i0, float2* smem,
                                        int* nonfin, f32x4* gr, f32x4* gi, f32x4* zr, f32x4* zi,
                                        float2* hv, float2* yv, float2& pv, const float2* pil = nullptr,
                                        bool have0 = false, int i0n = -1, const float2* Hn = nullptr,
                                        const float2* Yn = nullptr, const float2* pn = nullptr) {
#pragma unroll
  for (int t = 0; t < 4; ++t) gr[t] = gi[t] = zr[t] = zi[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int tid = tid_x(), w = tid >> 6, l = tid & 63;
  float2* Hs = smem;
  float2* Ys = smem + ROWS * PITCH;
  const int c16 = tid & 15;
  const int u = l & 15, kq = l >> 4;
  const int rb = tid >> 4;
  // chunk 0 may already be in hv/yv (prefetched by the previous tile); the
  // next chunk is loaded while the current one feeds the MFMAs (its loads
  // issued as soon as this wave has staged the current one, before the
  // barrier), and after the last chunk the first chunk of tile i0n (if >= 0)
  // is prefetched
  float probe = 0.f;
  if (!have0) load_chunk<FU>(Hf, Yff, pil, M, K, S, n_sc, i0, 0, hv, yv, pv);
  for (int m0 = 0; m0 < M; m0 += MC) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int r = rb + 16 * it;
      const float2 h = stage_h<FU>(hv[it], pv, it, M, K, n_sc, i0, m0);
      probe = __builtin_fmaf(h.x, 0.f, probe);
      probe = __builtin_fmaf(h.y, 0.f, probe);
      probe = __builtin_fmaf(yv[it].x, 0.f, probe);
      probe = __builtin_fmaf(yv[it].y, 0.f, probe);
      Hs[r * PITCH + c16] = h;
      Ys[r * PITCH + c16] = yv[it];
    }
    if (m0 + MC < M) load_chunk<FU>(Hf, Yff, pil, M, K, S, n_sc, i0, m0 + MC, hv, yv, pv);
    else if (i0n >= 0)
      load_chunk<FU>(Hn ? Hn : Hf, Yn ? Yn : Yff, pn ? pn : pil, M, K, S, n_sc, i0n, 0, hv, yv, pv);
    __syncthreads();
    if constexpr (P == P_FP32) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int row = (4 * a + kq) * 16 + u;     // antenna 4a + kq, slot u
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int sc = 4 * w + t;
          const float2 hr = Hs[row * PITCH + sc];
          const float2 yr = Ys[row * PITCH + sc];
          gr[t] = mfma(hr.x, hr.x, gr[t]);
          gr[t] = mfma(hr.y, hr.y, gr[t]);
          gi[t] = mfma(hr.x, hr.y, gi[t]);
          gi[t] = mfma(-hr.y, hr.x, gi[t]);
          zr[t] = mfma(hr.x, yr.x, zr[t]);
          zr[t] = mfma(hr.y, yr.y, zr[t]);
          zi[t] = mfma(hr.x, yr.y, zi[t]);
          zi[t] = mfma(-hr.y, yr.x, zi[t]);
        }
      }
    } else {
      // one 16x16x16 instruction per product covers the whole 8-antenna chunk:
      // lane (kq, u) supplies antennas 2 kq and 2 kq + 1 as (re, im, re, im);
      // Re G = X^T X, Im G = X^T X', Re Z = X^T Y, Im Z = X^T Y' with
      // X' = (b, -a) and Y' = (d, -c) per antenna.
      const int r0 = (2 * kq) * 16 + u, r1 = (2 * kq + 1) * 16 + u;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int sc = 4 * w + t;
        const float2 a0 = Hs[r0 * PITCH + sc], a1 = Hs[r1 * PITCH + sc];
        const float2 c0 = Ys[r0 * PITCH + sc], c1 = Ys[r1 * PITCH + sc];
        gr[t] = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, a0.x, a0.y, a1.x, a1.y, gr[t]);
        gi[t] = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, a0.y, -a0.x, a1.y, -a1.x, gi[t]);
        zr[t] = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, c0.x, c0.y, c1.x, c1.y, zr[t]);
        zi[t] = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, c0.y, -c0.x, c1.y, -c1.x, zi[t]);
      }
    }
    __syncthreads();
  }
  if (!(probe == 0.f)) nonfin[c16] = 1;
  __syncthreads();
}

// Phase 2 up to the ZF/MMSE solution: consumes the accumulators of gram_mf.
// On exit (lane `row` of subcarrier row `scl`): x[k] = column `row` of
// X_hat = A^{-1} Z (before the MMSE unbiasing), v[k] = column `row` of L^{-1},
// inv[k] = 1 / L[k][k], dl = d_row = [A^{-1}]_{row,row}, ok = factorisation
// succeeded; the subcarrier's slab Pm holds L row by row.
template <int KP, bool NORM = false>
__device__ __forceinline__ void factor_solve(float2* P, float2* Pm, const f32x4* gr, const f32x4* gi,
                                             const f32x4* zr, const f32x4* zi, int K, float n0,
                                             int mmse, int row, int col, int g4, float2* x, float2* v,
                                             float* inv, float& dl, bool& ok, float* afro2 = nullptr) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[t * PMAT + (g4 + r) * PP + col] = make_float2(gr[t][r], gi[t][r]);
  __syncthreads();
  float2 a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = Pm[row * PP + c];                       // row `row` of A
    if (c == row) a[c].x = row < K ? a[c].x + (mmse ? n0 : 0.f) : 1.0f;
  }
  if constexpr (NORM) {                            // ||A||_F^2 over the K x K block
    float s2 = 0.f;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < K) s2 += a[c].x * a[c].x + a[c].y * a[c].y;
    *afro2 = row_sum(row < K ? s2 : 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[t * PMAT + (g4 + r) * PP + col] = make_float2(zr[t][r], zi[t][r]);

  ok = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = make_float2(k == row ? 1.f : 0.f, 0.f);
  crout_all<KP>(Seq16{}, a, v, inv, row, ok);     // a[c] = L[row][c] for c < row
  dl = 0.f;
#pragma unroll
  for (int k = 0; k < KP; ++k) dl += v[k].x * v[k].x + v[k].y * v[k].y;

  __syncthreads();                                 // Z is in the slab
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = Pm[k * PP + row];   // column `row` of Z
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 16; ++c) Pm[row * PP + c] = a[c];   // L, row by row
  __syncthreads();
  fwd_all<KP>(Seq16{}, Pm, inv, x);                // L W = Z
  bwd_all<KP>(Seq16{}, Pm, inv, x);                // L^H X = W
}

// P: operand precision of the phase-1 products (detect_core.h).  For BF16 and
// FP16, subcarriers whose condition estimate ||A||_F tr(A^{-1}) exceeds the
// threshold, or whose low-precision factorisation breaks down,
// are handed to the FP64 refinement kernel: their x_hat (before the MMSE
// unbiasing) is written to xt and the subcarrier is appended to a device-side
// list (rlist[0] = count, entries from rlist[RL_OFF]).
// Phase 1 of the shared-factor path.  Same staging as gram_mf; the matched
// filter is accumulated for every subcarrier, the Gram matrix only once: for
// the tile's first subcarrier, each wave over every fourth 8-antenna chunk
// (g0r/g0i, a partial sum).  Every in-range H value is compared with the
// tile's first subcarrier (DPP broadcast of lane 0 of each 16-lane row); any
// difference, including a NaN, clears sf->uniform and the caller falls back
// to the per-subcarrier path.
template <int P = P_FP32, bool FU = false>
__device__ __forceinline__ void gram_mf_shared(const float2* __restrict__ Hf, const float2* __restrict__ Yff,
                                               const float2* __restrict__ pil, int M, int K, int S,
                                               int n_sc, int i0, float2* smem, int* nonfin,
                                               SharedFactor* sf, f32x4* zr, f32x4* zi, f32x4& g0r,
                                               f32x4& g0i, float2* hv, float2* yv, float2& pv,
                                               bool have0) {
  // matched filter with three real products per complex one: for h = a + jb,
  // y = c + jd, conj(h) y = (k1 + b (c + d)) + j (k1 + a (d - c)), k1 = (a - b) c
  f32x4 zk[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) zr[t] = zi[t] = zk[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  g0r = g0i = f32x4{0.f, 0.f, 0.f, 0.f};
  const int tid = tid_x(), w = tid >> 6, l = tid & 63;
  float2* Hs = smem;
  float2* Ys = smem + ROWS * PITCH;
  const int c16 = tid & 15;
  const int ic = i0 + c16;
  const int u = l & 15, kq = l >> 4;
  const int rb = tid >> 4;
  const bool in_range = ic < n_sc;
  float probe = 0.f;
  bool differ = false;
  if (!have0) load_chunk<FU>(Hf, Yff, pil, M, K, S, n_sc, i0, 0, hv, yv, pv);
  for (int m0 = 0; m0 < M; m0 += MC) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int r = rb + 16 * it;
      const float2 h = stage_h<FU>(hv[it], pv, it, M, K, n_sc, i0, m0);
      probe = __builtin_fmaf(h.x, 0.f, probe);
      probe = __builtin_fmaf(h.y, 0.f, probe);
      probe = __builtin_fmaf(yv[it].x, 0.f, probe);
      probe = __builtin_fmaf(yv[it].y, 0.f, probe);
      const float fx = bc<0>(h.x), fy = bc<0>(h.y);
      differ |= in_range && (h.x != fx || h.y != fy);
      Hs[r * PITCH + c16] = h;
      Ys[r * PITCH + c16] = yv[it];
    }
    if (m0 + MC < M) load_chunk<FU>(Hf, Yff, pil, M, K, S, n_sc, i0, m0 + MC, hv, yv, pv);
    __syncthreads();
    const bool gram_here = ((m0 / MC) & 3) == w;
    if constexpr (P == P_FP32) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int row = (4 * a + kq) * 16 + u;
        if (gram_here) {
          const float2 h0 = Hs[row * PITCH];
          g0r = mfma(h0.x, h0.x, g0r);
          g0r = mfma(h0.y, h0.y, g0r);
          g0i = mfma(h0.x, h0.y, g0i);
          g0i = mfma(-h0.y, h0.x, g0i);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int sc = 4 * w + t;
          const float2 hr = Hs[row * PITCH + sc];
          const float2 yr = Ys[row * PITCH + sc];
          zk[t] = mfma(hr.x - hr.y, yr.x, zk[t]);
          zr[t] = mfma(hr.y, yr.x + yr.y, zr[t]);
          zi[t] = mfma(hr.x, yr.y - yr.x, zi[t]);
        }
      }
    } else {
      // low precision: one 16x16x16 product per term covers the chunk (as in
      // gram_mf), the Gram matrix once per tile from its first subcarrier
      const int r0 = (2 * kq) * 16 + u, r1 = (2 * kq + 1) * 16 + u;
      if (gram_here) {
        const float2 a0 = Hs[r0 * PITCH], a1 = Hs[r1 * PITCH];
        g0r = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, a0.x, a0.y, a1.x, a1.y, g0r);
        g0i = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, a0.y, -a0.x, a1.y, -a1.x, g0i);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int sc = 4 * w + t;
        const float2 a0 = Hs[r0 * PITCH + sc], a1 = Hs[r1 * PITCH + sc];
        const float2 c0 = Ys[r0 * PITCH + sc], c1 = Ys[r1 * PITCH + sc];
        zr[t] = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, c0.x, c0.y, c1.x, c1.y, zr[t]);
        zi[t] = mfma_lp<P>(a0.x, a0.y, a1.x, a1.y, c0.y, -c0.x, c1.y, -c1.x, zi[t]);
      }
    }
    __syncthreads();
  }
  if constexpr (P == P_FP32) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      zr[t] += zk[t];
      zi[t] += zk[t];
    }
  }
  if (!(probe == 0.f)) nonfin[c16] = 1;
  if (differ) sf->uniform = 0;
  __syncthreads();
}

// Phase 2 of the shared-factor path: wave wf sums the partial Gram matrices,
// factors A once and publishes L, 1 / L_kk, d and ok; every wave then solves
// for its own subcarriers with that L.  Outputs as factor_solve; prefetch()
// is called once by every wave, with no register of the factorisation live.  (Wave w of
// every workgroup sits on SIMD w, so callers rotate wf from tile to tile to
// spread the factorisations over the four SIMDs.)
template <int KP, bool NORM, class Prefetch>
__device__ __forceinline__ void factor_solve_shared(float2* Pw, float2* Pm, SharedFactor* sf, int w, int wf,
                                                    const f32x4& g0r, const f32x4& g0i, const f32x4* zr,
                                                    const f32x4* zi, int K, float n0, int mmse, int row,
                                                    int col, int g4, float2* x, float* inv, float& dl,
                                                    bool& ok, float* afro2, Prefetch prefetch) {
#pragma unroll
  for (int r = 0; r < 4; ++r) sf->part[w][(g4 + r) * PP + col] = make_float2(g0r[r], g0i[r]);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) Pw[t * PMAT + (g4 + r) * PP + col] = make_float2(zr[t][r], zi[t][r]);
  __syncthreads();
  if (w == wf) {
    float2 a[16], v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float2 s = sf->part[0][row * PP + c];
      s = cadd(s, sf->part[1][row * PP + c]);
      s = cadd(s, sf->part[2][row * PP + c]);
      s = cadd(s, sf->part[3][row * PP + c]);
      if (c == row) s.x = row < K ? s.x + (mmse ? n0 : 0.f) : 1.0f;
      a[c] = s;
    }
    float s2 = 0.f;
    if constexpr (NORM) {                                // ||A||_F^2 over the K x K block
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < K) s2 += a[c].x * a[c].x + a[c].y * a[c].y;
      s2 = row_sum(row < K ? s2 : 0.f);
    }
    bool okw = true;
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = make_float2(k == row ? 1.f : 0.f, 0.f);
    crout_all<KP>(Seq16{}, a, v, inv, row, okw);
    float d = 0.f;
#pragma unroll
    for (int k = 0; k < KP; ++k) d += v[k].x * v[k].x + v[k].y * v[k].y;
    if (g4 == 0) {                                       // lanes 0..15: one copy
#pragma unroll
      for (int c = 0; c < 16; ++c) sf->L[row * PP + c] = a[c];
      sf->dl[row] = d;
      sf->inv[row] = inv[row];
      if (row == 0) {
        sf->ok = okw ? 1 : 0;
        if constexpr (NORM) sf->afro2 = s2;
      }
    }
  }
  // the next tile's first chunk: the factoring wave after its factorisation,
  // the others right away, so the loads fly during the wait and the solves
  prefetch();
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = Pm[k * PP + row];   // column `row` of Z
#pragma unroll
  for (int k = 0; k < 16; ++k) inv[k] = sf->inv[k];
  dl = sf->dl[row];
  ok = sf->ok != 0;
  if constexpr (NORM) *afro2 = sf->afro2;
  fwd_all<KP>(Seq16{}, sf->L, inv, x);                  // L W = Z
  bwd_all<KP>(Seq16{}, sf->L, inv, x);                  // L^H X = W
}

constexpr int RL_OFF = 64;

// One tile of TS subcarriers from i0 of one frame (H [M][K][n_sc], Yf
// [M][S][n_sc], xt [K][D][n_sc], nu [K][n_sc], flags [n_sc] of that frame);
// 256 threads; smem holds SMEM_ALL slots, nonfin TS.  A refined subcarrier i is
// listed as sub_base + i.  With FU the channel is not read from H: it is the
// LS estimate from the pilot symbol of Yf and the pilots pil (exactly the CSI
// stage's value).  hv/yv/pv carry chunk 0 of this tile in when have0 is
// set; if i0n >= 0 they carry chunk 0 of the tile at i0n out (of the frame at
// Hn/Yn, default this one), with have0 set, so that its loads fly during this
// tile's phase 2.  The caller synchronises before reusing smem.
// xl: x_tilde is not written to xt but left in LDS for the caller (the
// batched kernel's fused demapping), in the slab of each lane's subcarrier:
// tile subcarrier e = 4 w + scl at smem + e * PMAT, x_tilde[u][s] at
// [16 u + s] and nu[u] at [256 + u].x (the values the global outputs would
// hold; nu is written to its output as well).  The caller reads them after a
// barrier, before smem is reused.
static_assert(PMAT >= 256 + 16, "slab too small for a subcarrier's x_tilde and nu");
template <int KP, int P, bool FU = false>
__device__ __forceinline__ void detect_tile(const float2* __restrict__ H, const float2* __restrict__ Yf,
                                            float2* __restrict__ xt, float* __restrict__ nu,
                                            uint8_t* __restrict__ flags, int M, int K, int S, int n_sc,
                                            float n0, int mmse, float thr, uint32_t* __restrict__ rlist,
                                            uint32_t sub_base, int i0, float2* smem, int* nonfin,
                                            float2* hv, float2* yv, float2& pv, bool& have0, int i0n,
                                            const float2* Hn = nullptr, const float2* Yn = nullptr,
                                            const float2* pil = nullptr, const float2* pn = nullptr,
                                            bool xl = false) {
  const int D = S - 1;
  const int tid = tid_x(), w = tid >> 6, l = tid & 63;
  SharedFactor* sf = reinterpret_cast<SharedFactor*>(smem + SMEM);
  if (tid < TS) nonfin[tid] = 0;
  if (tid == 0) sf->uniform = 1;
  __syncthreads();

  float2* Pw = smem + w * 4 * PMAT;
  const int col = l & 15, g4 = (l >> 4) * 4;      // MFMA output: rows g4 + r, column col
  const int scl = l >> 4, row = l & 15;           // phase-2 lane: subcarrier scl, index row
  float2* Pm = Pw + scl * PMAT;
  float2 z[16];
  float inv[16], dl, afro2 = 0.f;
  bool ok;
  constexpr bool NORM = P != P_FP32;
  // The CSI stage holds the estimate constant over each pilot group of K
  // subcarriers, so a tile inside one group usually carries one channel
  // matrix: then the Gram matrix is formed once and A is factored once per
  // tile (the result equals the per-subcarrier path up to summation order).
  // (Only a tile of K >= 16 users, or the last pilot group's tile, can lie in
  // one group, so the path is compiled for the K padding of 16 alone.  With
  // BF16 / FP16 operands the shared Gram matrix is formed in that precision
  // too, so the condition estimate and the refinement see the same A.)
  bool shared = false;
  if constexpr (KP == 16) {
    const int G = n_sc / K;
    const int last = min(i0 + TS, n_sc) - 1;
    if (min(i0 / K, G - 1) == min(last / K, G - 1)) {
      f32x4 zr[4], zi[4], g0r, g0i;
      gram_mf_shared<P, FU>(H, Yf, pil, M, K, S, n_sc, i0, smem, nonfin, sf, zr, zi, g0r, g0i, hv, yv, pv,
                            have0);
      have0 = false;
      shared = __builtin_amdgcn_readfirstlane(sf->uniform) != 0;
      if (shared) {
        factor_solve_shared<KP, NORM>(Pw, Pm, sf, w, (i0 / TS) & 3, g0r, g0i, zr, zi, K, n0, mmse, row, col,
                                      g4, z, inv, dl, ok, &afro2, [&]() {
                                  if (i0n >= 0)
                                    load_chunk<FU>(Hn ? Hn : H, Yn ? Yn : Yf, pn ? pn : pil, M, K, S, n_sc,
                                                   i0n, 0, hv, yv, pv);
                                });
        have0 = i0n >= 0;
      }
    }
  }
  if (!shared) {
    // with K padded to 16 this path is the rare fallback and holds no
    // prefetch across its phase 2 (registers)
    constexpr bool PREF = KP != 16;
    f32x4 gr[4], gi[4], zr[4], zi[4];
    gram_mf<P, FU>(H, Yf, M, K, S, n_sc, i0, smem, nonfin, gr, gi, zr, zi, hv, yv, pv, pil, have0,
                   PREF ? i0n : -1, Hn, Yn, pn);
    have0 = PREF && i0n >= 0;
    float2 v[16];
    factor_solve<KP, NORM>(Pw, Pm, gr, gi, zr, zi, K, n0, mmse, row, col, g4, z, v, inv, dl, ok, &afro2);
  }

  const bool mu_bad = mmse && row < K && !(1.0f - n0 * dl > 0.f);
  const uint64_t bal = __ballot(mu_bad);
  if ((bal >> (16 * scl)) & 0xffffull) ok = false;
  const int i = i0 + 4 * w + scl;
  const bool nf = nonfin[4 * w + scl] != 0;
  bool refine = false;
  if constexpr (P != P_FP32) {
    const float kest = cond_estimate(afro2, row_sum(row < K ? dl : 0.f));
    refine = !nf && (!ok || !(kest <= thr));
  }
  if (mmse) unbias_all<KP>(Seq16{}, dl, n0, K, refine, z);
  if (i >= n_sc) return;

  if (refine) {                                   // finished in FP64 by refine_kernel
    if (row == 0) {
      const uint32_t slot = atomicAdd(rlist, 1u);
      rlist[RL_OFF + slot] = sub_base + (uint32_t)i;
    }
    // a low-precision breakdown leaves z non-finite: start the FP64 step from
    // x0 = 0 instead, which makes it a full FP64 solve
    if (row < D) {
#pragma unroll
      for (int uu = 0; uu < 16; ++uu)
        if (uu < K) xt[((int64_t)uu * D + row) * n_sc + i] = ok ? z[uu] : make_float2(0.f, 0.f);
    }
    return;
  }
  const bool erase = nf || !ok;
  if (row < D) {
#pragma unroll
    for (int uu = 0; uu < 16; ++uu) {
      if (uu < K) {
        float2 x = z[uu];
        if (erase) x = make_float2(0.f, 0.f);
        if (xl) Pm[16 * uu + row] = x;             // this wave's solves are done with Pm
        else xt[((int64_t)uu * D + row) * n_sc + i] = x;
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
    nu[(int64_t)row * n_sc + i] = erase ? INFINITY : nv;
    if (xl) Pm[256 + row] = make_float2(erase ? INFINITY : nv, 0.f);
  }
  if (row == 0 && flags) flags[i] = nf ? RXPHY_FLAG_NONFINITE : (ok ? 0 : RXPHY_FLAG_BREAKDOWN);
}

}  // namespace det
}  // namespace rxphy
