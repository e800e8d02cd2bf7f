// Fused CSI + ZF / MMSE detector for K = 16 users, FP32: the comb-pilot
// least-squares channel estimate and textbook linear (zero-forcing / MMSE)
// detection, the stages named csi and equal in the paper's preamble.
//
// With 16 users a pilot group spans exactly one 16-subcarrier tile, and the
// LS estimate is held over the group, so every subcarrier of a tile sees the
// same channel matrix H (64 x 16).  Per tile the work is
//   G = H^H H (+ N0 I) once, its Cholesky factor and A^-1 once, and
//   Z = H^H Y for 16 subcarriers x D data symbols, then X = A^-1 Z.
// Two kernels, so that the short serial factorisation never holds up the
// streaming part:
//
//  group_factor_kernel  two tiles per wavefront: loads each tile's
//    pilot-symbol row and pilots, forms H (LS), the Gram matrix on MFMA, and
//    factors A = G (+ N0 I) (Cholesky-Crout with V = L^-1, one tile per
//    16-lane row), then A^-1 = V^H V on MFMA; writes A^-1, d_k = [A^-1]_kk
//    and flags into a 2.25 KiB record per tile.  Many independent
//    wavefronts per SIMD hide each one's serial latency.
//  detect_group_kernel  one workgroup per tile: the data operands are loaded
//    straight from HBM into the lanes that use them (lane (kq, u) of
//    v_mfma_f32_16x16x4_f32: B = Y[4s + kq][1 + d][i0 + u], 16 lanes per
//    128-byte row segment), all of a wave's loads issued at once, no LDS
//    staging.  Wave w owns data symbols d = w, w + 4, w + 8, w + 12 and runs
//    all 64 antennas for them (16 steps of 4 antennas); H is formed again
//    (LS) into LDS as the A operand.  X = A^-1 Z is formed from the same
//    accumulator lanes with the record's A^-1 rows on MFMA (no transposition
//    and no substitution chain), then unbiased, stored and (Q > 0) demapped.
//
// The Gram products, the factorisation, d_k, nu and the flags are the steps
// the general detector (detect_core.h, shared-factor path) performs on the
// same values in the same order, so they are bit-identical to rxphy_csi +
// rxphy_detect; x_tilde comes from the explicit inverse instead of the two
// triangular solves and agrees with it to rounding.
#include <type_traits>

#include "demod_core.h"
#include "detect_core.h"

namespace rxphy {

// Per-tile factor record (workspace of the fused path).
struct alignas(256) GroupRec {
  float2 B[16 * 16];     // A^-1 = V^H V (V = L^-1), row-major
  float dl[16];          // d_k = [A^-1]_kk as the factorisation forms it
  int ok;                // factorisation succeeded
  int hbad;              // a non-finite channel value
  int refine;            // BF16 / FP16: the tile is finished by the FP64 refinement
  int pad;
};

namespace {

using namespace det;

constexpr int GWAVES = 4;     // waves per workgroup
constexpr int FTPW = 2;       // tiles per wavefront of the factor kernel
typedef float float4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// 16x16x32 products of gfx950 with 8 operand values per lane (lane l supplies
// A[l % 16][8 (l / 16) + t] and B[8 (l / 16) + t][l % 16], t = 0..7): BF16 or
// FP16 operands (rounded to nearest even from FP32), FP32 accumulation.
template <int P>
struct LowP;
template <>
struct LowP<P_BF16> {
  typedef bf16x8 vec;
  typedef __bf16 elem;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct LowP<P_FP16> {
  typedef f16x8 vec;
  typedef _Float16 elem;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ float2 ldg2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// One transmit point: Q = 0 reads a complex64 symbol; Q = 2, 4, 6 reads the
// point's Q bit bytes (b0 first, non-zero = one) and maps them as
// rxphy_modulate does (axis codes b0 b2 b4 / b1 b3 b5, most significant
// first).  `e` is the point's element index (or past the range).
template <int Q>
__device__ __forceinline__ float2 load_point(__amdgpu_buffer_rsrc_t r, uint32_t e) {
  if constexpr (Q == 0) {
    return ldg2(r, e * 8u);
  } else {
    uint32_t b = 0;                              // byte t of the point at bits 8t .. 8t+7
    if constexpr (Q == 2) {
      b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(e * 2u), 0, 0);
    } else if constexpr (Q == 4) {
      b = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(e * 4u), 0, 0);
    }
    int ci = 0, cq = 0;
    if constexpr (Q == 6) {
      const uint32_t h0 = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(e * 6u), 0, 0);
      const uint32_t h1 = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(e * 6u + 2u), 0, 0);
      const uint32_t h2 = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(e * 6u + 4u), 0, 0);
      const uint32_t by[6] = {h0 & 255u, h0 >> 8, h1 & 255u, h1 >> 8, h2 & 255u, h2 >> 8};
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        ci = 2 * ci + (by[2 * t] != 0);
        cq = 2 * cq + (by[2 * t + 1] != 0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < Q / 2; ++t) {
        ci = 2 * ci + (((b >> (16 * t)) & 255u) != 0);
        cq = 2 * cq + (((b >> (16 * t + 8)) & 255u) != 0);
      }
    }
    return make_float2(demk::axis_level<Q>(ci), demk::axis_level<Q>(cq));
  }
}

// Byte offsets are a lane part plus a wave-uniform part, formed next to each
// load (the empty asm keeps the compiler from precomputing all of them into
// registers).  The frame's buffer resource ends after antenna M - 1, so
// antennas at or past M read zero by the hardware range check; a subcarrier
// past n_sc moves the lane part past the end (OOB, which no uniform part can
// wrap).
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// ------------------------------------------------------------- factorisation
// H[4 s + kq][u] (s = 0..15) of tile tix for this lane (the MFMA A / B operand
// layout): the pilot-symbol values and the user's pilot; a tile past the end
// reads zero without touching memory.
__device__ __forceinline__ void factor_loads(const float2* Yf, const float2* pil, int tix, int T, int nt, int M,
                                             int S, int n_sc, int kq, int u, float2* hv, float2& pv) {
  const bool in = tix < T;
  const int f = in ? tix / nt : 0;
  const int tt = tix - f * nt;
  const int q = min(tt, n_sc / 16 - 1) * 16 + u;
  const __amdgpu_buffer_rsrc_t yr = rsrc(Yf + (int64_t)f * M * S * n_sc, (uint32_t)M * S * n_sc * 8u);
  const uint32_t ant = (uint32_t)S * n_sc * 32u;
  uint32_t row = opaque(in ? (uint32_t)(kq * S * n_sc + q) * 8u : OOB);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    hv[s] = ldg2(yr, row);
    row = opaque(row + ant);
  }
  pv = ldg2(rsrc(pil + (int64_t)f * n_sc, (uint32_t)n_sc * 8u), in ? (uint32_t)q * 8u : OOB);
}

// LS estimate, non-finite check and A = sum of the four partial Gram matrices
// (8-antenna chunks c and c + 4, in order, summed in order) into t as rows
// of pitch PP; returns whether a channel value is non-finite.
// BF16 / FP16 (P): the Gram matrix from operands rounded to that precision,
// 32 antennas per product: element t of lane (kq, u) is antenna
// 4 (8 c + t) + kq of user u, in both operands.
template <int P>
__device__ __forceinline__ bool factor_gram(float2* hv, float2 pv, int M, int kq, int u, float2* t) {
  float probe = 0.f;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    hv[s] = 4 * s + kq < M ? ls_estimate(hv[s], pv) : make_float2(0.f, 0.f);
    probe = __builtin_fmaf(hv[s].x, 0.f, probe);
    probe = __builtin_fmaf(hv[s].y, 0.f, probe);
  }
  if constexpr (P != P_FP32) {
    using LP = LowP<P>;
    using E = typename LP::elem;
    f32x4 gr = {0.f, 0.f, 0.f, 0.f}, gi = gr;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (32 * c < M) {
        typename LP::vec ar, ai;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ar[e] = (E)hv[8 * c + e].x;
          ai[e] = (E)hv[8 * c + e].y;
        }
        gr = LP::mma(ar, ar, gr);
        gr = LP::mma(ai, ai, gr);
        gi = LP::mma(ar, ai, gi);
        gi = LP::mma(-ai, ar, gi);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) t[(4 * kq + r) * PP + u] = make_float2(gr[r], gi[r]);
    return __ballot(!(probe == 0.f)) != 0ull;
  }
  f32x4 pr[4], pi[4];
#pragma unroll
  for (int wp = 0; wp < 4; ++wp) {
    pr[wp] = pi[wp] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = wp + 4 * b;
      if (c * MC < M) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const float2 h = hv[2 * c + a];
          pr[wp] = mfma(h.x, h.x, pr[wp]);
          pr[wp] = mfma(h.y, h.y, pr[wp]);
          pi[wp] = mfma(h.x, h.y, pi[wp]);
          pi[wp] = mfma(-h.y, h.x, pi[wp]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float2 g = make_float2(pr[0][r], pi[0][r]);
    g = cadd(g, make_float2(pr[1][r], pi[1][r]));
    g = cadd(g, make_float2(pr[2][r], pi[2][r]));
    g = cadd(g, make_float2(pr[3][r], pi[3][r]));
    t[(4 * kq + r) * PP + u] = g;
  }
  return __ballot(!(probe == 0.f)) != 0ull;
}

// Each wavefront factors TPW tiles: all of their loads issued at once, their
// Gram matrices one after the other on MFMA, then one Crout pass in which
// 16-lane row k works on tile k % TPW (the factorisation's broadcasts stay
// within a row).  Two tiles per wavefront keep four wavefronts per SIMD.
//
// BF16 / FP16 (P): the Gram matrix from low-precision operands, the Cholesky
// factor in FP32, and tiles whose condition estimate ||A||_F tr(A^-1) exceeds
// thr (or whose factorisation broke down) are marked in their record and
// appended to the refinement list rl (one entry per tile, frame * tiles +
// tile), which the FP64 group refinement works through.
template <int TPW, int P = P_FP32>
__global__ void __launch_bounds__(256)
group_factor_kernel(const float2* __restrict__ Yf, const float2* __restrict__ pil, GroupRec* __restrict__ rec,
                    int T, int nt, int M, int S, int n_sc, float n0, int mmse, float thr = 0.f,
                    uint32_t* __restrict__ rl = nullptr) {
  __shared__ float2 tp[GWAVES][TPW][16 * PP];
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int u = l & 15, kq = l >> 4;
  const int base = (blockIdx.x * GWAVES + w) * TPW;           // tiles base .. base + TPW - 1
  if (base >= T) return;                                       // a whole wave; no barrier below

  float2 hv[TPW][16], pv[TPW];
  bool bad[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) factor_loads(Yf, pil, base + t, T, nt, M, S, n_sc, kq, u, hv[t], pv[t]);
#pragma unroll
  for (int t = 0; t < TPW; ++t) bad[t] = factor_gram<P>(hv[t], pv[t], M, kq, u, tp[w][t]);

  // row kq of the wave factors tile base + kq % TPW; lane `row` holds A[row][:]
  const int tk = kq % TPW;
  const int row = u;
  float2 a[16], v[16];
  float inv[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    float2 g = tp[w][tk][row * PP + c];
    if (c == row) g.x = g.x + (mmse ? n0 : 0.f);
    a[c] = g;
  }
  float afro2 = 0.f;                             // ||A||_F^2 (mixed precisions)
  if constexpr (P != P_FP32) {
#pragma unroll
    for (int c = 0; c < 16; ++c) afro2 += a[c].x * a[c].x + a[c].y * a[c].y;
    afro2 = row_sum(afro2);
  }
  bool okw = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = make_float2(k == row ? 1.f : 0.f, 0.f);
  crout_all<16>(Seq16{}, a, v, inv, row, okw);
  float d = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) d += v[k].x * v[k].x + v[k].y * v[k].y;
  // V = L^-1 (lane `row` holds its column `row`) over A in LDS, then
  // B = V^H V per tile: the Gram product again, V[4 s + kq][u] as both operands
  if (kq < TPW) {
#pragma unroll
    for (int k = 0; k < 16; ++k) tp[w][tk][k * PP + row] = v[k];
  }
#pragma unroll
  for (int g = 0; g < TPW; ++g) {
    f32x4 br = {0.f, 0.f, 0.f, 0.f}, bi = br;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float2 x = tp[w][g][(4 * s + kq) * PP + u];
      br = mfma(x.x, x.x, br);
      br = mfma(x.y, x.y, br);
      bi = mfma(x.x, x.y, bi);
      bi = mfma(-x.y, x.x, bi);
    }
    if (base + g < T) {
      GroupRec& R = rec[base + g];
#pragma unroll
      for (int r = 0; r < 4; ++r) R.B[(4 * kq + r) * 16 + u] = make_float2(br[r], bi[r]);
    }
  }
  const int tix = base + tk;
  bool hb = bad[0];
#pragma unroll
  for (int t = 1; t < TPW; ++t)
    if (tk == t) hb = bad[t];
  bool refine = false;
  if constexpr (P != P_FP32) {
    const float kest = cond_estimate(afro2, row_sum(d));
    refine = !hb && (!okw || !(kest <= thr));     // the same in every lane of the row
  }
  if (kq < TPW && tix < T) {
    GroupRec& R = rec[tix];
    R.dl[row] = d;
    if (row == 0) {
      R.ok = okw ? 1 : 0;                        // the same in every lane of the row
      R.hbad = hb ? 1 : 0;
      R.refine = refine ? 1 : 0;
      if (refine) rl[RL_OFF + atomicAdd(rl, 1u)] = (uint32_t)tix;   // the tile into the list
    }
  }
}

// ------------------------------------------------------------------ detector
// Z = H^H Y over the 16 antenna steps, in order, for symbol slot J, three
// real products per complex one: for h = a + jb, y = c + jd,
// conj(h) y = (k1 + b (c + d)) + j (k1 + a (d - c)), k1 = (a - b) c; then
// X = A^-1 Z from the same lanes: step r of the product takes the users
// 4 kq + r, which this lane already holds (Z rows 4 kq + r, column u), against
// B[u][4 kq + r]; (a + jb)(c + jd) = (k1 - b (c + d)) + j (k1 + a (d - c)),
// k1 = (a + b) c.  x gets X rows 4 kq + r, column u.
template <int J, bool FULLM>
__device__ __forceinline__ void z_slot(const float2* hs, const float2 (*y)[3], const float2* brow, float& probe,
                                       int kq, int u, int M, f32x4& xr, f32x4& xi) {
  f32x4 zk = {0.f, 0.f, 0.f, 0.f}, zr = zk, zi = zk;
#pragma unroll
  for (int s = 0; s < 16; ++s) {                // antennas 4 s .. 4 s + 3
    if (FULLM || (s >> 1) * MC < M) {           // else an absent 8-antenna chunk
      const float2 h = hs[(4 * s + kq) * 16 + u];
      const float2 yv = y[s][J];
      probe = __builtin_fmaf(yv.x, 0.f, probe);
      probe = __builtin_fmaf(yv.y, 0.f, probe);
      zk = mfma(h.x - h.y, yv.x, zk);
      zr = mfma(h.y, yv.x + yv.y, zr);
      zi = mfma(h.x, yv.y - yv.x, zi);
    }
  }
  zr += zk;
  zi += zk;
  f32x4 xk = {0.f, 0.f, 0.f, 0.f};
  xr = xi = xk;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float2 b = brow[r];
    xk = mfma(b.x + b.y, zr[r], xk);
    xr = mfma(b.y, zr[r] + zi[r], xr);
    xi = mfma(b.x, zi[r] - zr[r], xi);
  }
  xr = xk - xr;
  xi = xk + xi;
}

// BF16 / FP16 (P): Z = H^H Y from operands rounded to that precision, four
// real products per complex one over 32 antennas at a time (element t of lane
// (kq, u) is antenna 4 (8 c + t) + kq: user u's channel in the first operand,
// subcarrier u's data in the second), then X = A^-1 Z in FP32 as z_slot does.
template <int J, bool FULLM, int P>
__device__ __forceinline__ void z_slot_lp(const float2* hs, const float2 (*y)[3], const float2* brow, float& probe,
                                          int kq, int u, int M, f32x4& xr, f32x4& xi) {
  using LP = LowP<P>;
  using E = typename LP::elem;
  f32x4 zr = {0.f, 0.f, 0.f, 0.f}, zi = zr;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (FULLM || 32 * c < M) {
      typename LP::vec hr, hi, yr, yi;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int s = 8 * c + e;
        const float2 h = hs[(4 * s + kq) * 16 + u];
        const float2 yv = y[s][J];
        probe = __builtin_fmaf(yv.x, 0.f, probe);
        probe = __builtin_fmaf(yv.y, 0.f, probe);
        hr[e] = (E)h.x;
        hi[e] = (E)h.y;
        yr[e] = (E)yv.x;
        yi[e] = (E)yv.y;
      }
      zr = LP::mma(hr, yr, zr);
      zr = LP::mma(hi, yi, zr);
      zi = LP::mma(hr, yi, zi);
      zi = LP::mma(-hi, yr, zi);
    }
  }
  f32x4 xk = {0.f, 0.f, 0.f, 0.f};
  xr = xi = xk;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float2 b = brow[r];
    xk = mfma(b.x + b.y, zr[r], xk);
    xr = mfma(b.y, zr[r] + zi[r], xr);
    xi = mfma(b.x, zi[r] - zr[r], xi);
  }
  xr = xk - xr;
  xi = xk + xi;
}

// Symbol slot j (d = w + 4 j) of this lane's data into register slot R:
// y[s][R] = Y[4 s + kq][1 + d][i0 + u]; a slot the wave does not own reads
// zero without touching memory, so every wave issues the same loads.
template <int R>
__device__ __forceinline__ void load_slot(float2 (*y)[3], __amdgpu_buffer_rsrc_t yr, uint32_t lane, int j, int nj,
                                          uint32_t ant, uint32_t sym) {
  uint32_t row = opaque(j < nj ? lane + (uint32_t)j * sym : OOB);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    y[s][R] = ldg2(yr, row);
    row = opaque(row + ant);
  }
}

// One workgroup per (tile, frame): blockIdx.x = tile, blockIdx.y = frame.
// Q > 0: the demod stage follows in the same kernel (max-log LLRs of every
// equalised symbol into llr, as demod_kernel computes them from x_tilde and
// nu); xt may then be null (not written).
//
// BF16 / FP16 (P): the matched filter from low-precision operands (z_slot_lp);
// a tile whose record is marked for refinement writes nothing (the FP64
// refinement kernel writes all of its outputs).
// Three workgroups per CU for FP32 (168 registers), two for BF16 / FP16
// (their operand conversions need 187 registers; at 168 they spill).
template <int Q, int P = P_FP32>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == P_FP32 ? 3 : 2)))
detect_group_kernel(const float2* __restrict__ Yf, const float2* __restrict__ pil,
                    const GroupRec* __restrict__ rec, float2* __restrict__ xt, float* __restrict__ nu,
                    uint8_t* __restrict__ flags, float* __restrict__ llr, int M, int S, int n_sc, float n0,
                    int mmse) {
  __shared__ float2 hs[64 * 16];                // H of the tile: [antenna][user]
  __shared__ uint32_t nfmask[GWAVES];           // subcarriers with a non-finite data value
  __shared__ float4v utab[16];                  // per user: 1 / mu (MMSE), nu, 1 / nu
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar branches
  const int u = l & 15, kq = l >> 4;
  const int D = S - 1;
  const int64_t f = blockIdx.y;
  const int tt = blockIdx.x;
  const int i0 = tt * 16;
  const int g = min(tt, n_sc / 16 - 1);        // the tile's pilot group
  // symbols of this wave: d = w + 4 j for j < nj
  const int nj = D > w ? (D - w + 3) >> 2 : 0;

  // ---- loads, oldest first: this lane's part of the tile's record (row u of
  // A^-1, columns 4 kq .. 4 kq + 3; d_k of its users; the flags), this wave's
  // 16 antennas of the pilot-symbol row and the pilots, then all of its data
  // (a fixed count of loads per wave, so that each use waits for exactly its
  // own; slots the wave does not own read zero without touching memory)
  const GroupRec* R = rec + (f * gridDim.x + tt);
  const __amdgpu_buffer_rsrc_t rr = rsrc(R, (uint32_t)sizeof(GroupRec));
  float2 brow[4];
  {
    const uint32_t o = opaque((uint32_t)(u * 16 + 4 * kq) * 8u);
    const float4v b01 = __builtin_bit_cast(float4v, __builtin_amdgcn_raw_buffer_load_b128(rr, (int)o, 0, 0));
    const float4v b23 = __builtin_bit_cast(float4v, __builtin_amdgcn_raw_buffer_load_b128(rr, (int)(o + 16u), 0, 0));
    brow[0] = make_float2(b01.x, b01.y);
    brow[1] = make_float2(b01.z, b01.w);
    brow[2] = make_float2(b23.x, b23.y);
    brow[3] = make_float2(b23.z, b23.w);
  }
  const float4v dl4 = __builtin_bit_cast(
      float4v, __builtin_amdgcn_raw_buffer_load_b128(rr, (int)opaque(2048u + 16u * kq), 0, 0));
  const float2 okh = ldg2(rr, opaque(2048u + 64u));
  float2 rfp = make_float2(0.f, 0.f);
  if constexpr (P != P_FP32) rfp = ldg2(rr, opaque(2048u + 72u));
  const __amdgpu_buffer_rsrc_t yr = rsrc(Yf + f * M * S * n_sc, (uint32_t)M * S * n_sc * 8u);
  const uint32_t ant = (uint32_t)S * n_sc * 32u;             // 4 antennas
  const uint32_t sym = (uint32_t)n_sc * 32u;                 // 4 symbols
  float2 hv[4], pv;
  {
    const int q = g * 16 + u;
    uint32_t row = opaque((uint32_t)((16 * w + kq) * S * n_sc + q) * 8u);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      hv[a] = ldg2(yr, row);
      row = opaque(row + ant);
    }
    pv = ldg2(rsrc(pil + f * n_sc, (uint32_t)n_sc * 8u), opaque((uint32_t)q * 8u));
  }
  // three symbol slots in registers at a time: the fourth (only wave 0 has
  // one with 13 data symbols) is loaded into slot 0's registers as soon as
  // slot 0 has been consumed
  float2 y[16][3];
  const uint32_t lane = i0 + u < n_sc ? (uint32_t)((kq * S + 1 + w) * n_sc + i0 + u) * 8u : OOB;
  load_slot<0>(y, yr, lane, 0, nj, ant, sym);
  load_slot<1>(y, yr, lane, 1, nj, ant, sym);
  load_slot<2>(y, yr, lane, 2, nj, ant, sym);
  if constexpr (P != P_FP32)
    if (__builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, rfp.x)) != 0) return;   // the whole workgroup

  // ---- H = LS estimate (absent antennas zero) into LDS
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int m = 16 * w + 4 * a + kq;
    hs[m * 16 + u] = m < M ? ls_estimate(hv[a], pv) : make_float2(0.f, 0.f);
  }
  // every user's MMSE gain and noise variance, the same for all 16 subcarriers
  // (one factor per tile): formed once here, as the demod stage forms 1 / nu
  // from the stored nu
  if (w == 0 && u == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float dk = dl4[r];
      const float nv = mmse ? n0 * dk * __builtin_amdgcn_rcpf(1.0f - n0 * dk) : n0 * dk;
      utab[4 * kq + r] = float4v{__builtin_amdgcn_rcpf(1.0f - n0 * dk), nv, 1.0f / nv, 0.f};
    }
  }
  __syncthreads();

  // ---- per-subcarrier factor state: every user's mu counts (the four rows
  // of lanes with the same u hold the 16 users)
  const int i = i0 + u;
  bool ok = __builtin_bit_cast(int, okh.x) != 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) ok = ok && (!mmse || 1.0f - n0 * dl4[r] > 0.f);
  {
    const uint64_t okb = __ballot(ok);
    ok = ((okb | (okb >> 16) | (okb >> 32) | (okb >> 48)) & 0xffffull) == 0xffffull;
  }
  float2* xo = xt ? xt + f * 16 * D * n_sc : nullptr;
  float* lo = llr + f * 16 * D * n_sc * Q;
  const bool col = i < n_sc;

  // ---- X = A^-1 H^H Y for this wave's symbols, stored as each is done
  // (a subcarrier found non-finite below is cleared afterwards)
  float probe = 0.f;
  auto emit = [&](int j, const f32x4& xr, const f32x4& xi) {
    if (!col) return;
    const int d = w + 4 * j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float4v ut = utab[4 * kq + r];
      float2 x = make_float2(xr[r], xi[r]);
      if (mmse) x = cscale(x, ut.x);
      if (!ok) x = make_float2(0.f, 0.f);
      const int64_t e = ((int64_t)(4 * kq + r) * D + d) * n_sc + i;
      if (xo) xo[e] = x;
      if constexpr (Q > 0) {
        demk::demod_point_inv<Q, true>(x, !ok || __builtin_isinf(ut.y), ut.z, lo + e * Q);
        __builtin_amdgcn_sched_barrier(0);       // one point at a time (registers)
      }
    }
  };
  f32x4 xr, xi;
  auto zs = [&](auto jc, auto fm) {
    constexpr int J = decltype(jc)::value;
    constexpr bool FM = decltype(fm)::value;
    if constexpr (P == P_FP32) z_slot<J, FM>(hs, y, brow, probe, kq, u, M, xr, xi);
    else z_slot_lp<J, FM, P>(hs, y, brow, probe, kq, u, M, xr, xi);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  if (M == 64) {
    using FM = std::true_type;
    if (nj > 0) { zs(I0{}, FM{}); emit(0, xr, xi); }
    load_slot<0>(y, yr, lane, 3, nj, ant, sym);
    if (nj > 1) { zs(I1{}, FM{}); emit(1, xr, xi); }
    if (nj > 2) { zs(I2{}, FM{}); emit(2, xr, xi); }
    if (nj > 3) { zs(I0{}, FM{}); emit(3, xr, xi); }
  } else {
    using FM = std::false_type;
    if (nj > 0) { zs(I0{}, FM{}); emit(0, xr, xi); }
    load_slot<0>(y, yr, lane, 3, nj, ant, sym);
    if (nj > 1) { zs(I1{}, FM{}); emit(1, xr, xi); }
    if (nj > 2) { zs(I2{}, FM{}); emit(2, xr, xi); }
    if (nj > 3) { zs(I0{}, FM{}); emit(3, xr, xi); }
  }
  {
    const uint64_t bad = __ballot(!(probe == 0.f));
    const uint32_t m16 = (uint32_t)(bad | (bad >> 16) | (bad >> 32) | (bad >> 48)) & 0xffffu;
    if (l == 0) nfmask[w] = m16;
  }
  __syncthreads();

  // ---- non-finite inputs: the subcarrier is erased (same lane, same
  // addresses, so the zeros land after the values above); noise variances
  // and flags
  const uint32_t nfm = nfmask[0] | nfmask[1] | nfmask[2] | nfmask[3];
  const bool hb = __builtin_bit_cast(int, okh.y) != 0;
  const bool nf_i = hb || ((nfm >> u) & 1u);
  if (col && nf_i) {
    for (int j = 0; j < nj; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t e = ((int64_t)(4 * kq + r) * D + w + 4 * j) * n_sc + i;
        if (xo) xo[e] = make_float2(0.f, 0.f);
        if constexpr (Q > 0) demk::demod_point<Q, true>(make_float2(0.f, 0.f), INFINITY, lo + e * Q);
      }
    }
  }
  const bool erase = nf_i || !ok;
  if (col && w == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) nu[(f * 16 + 4 * kq + r) * n_sc + i] = erase ? INFINITY : utab[4 * kq + r].y;
    if (kq == 0 && flags) flags[f * n_sc + i] = nf_i ? RXPHY_FLAG_NONFINITE : (ok ? 0 : RXPHY_FLAG_BREAKDOWN);
  }
}

// ------------------------------------------------------------------ precoder
// Downlink zero-forcing precoding with the uplink estimate (reciprocity):
// per tile X = H A^-1 S for the 16 users' symbols S [F][16][D][n_sc], i.e.
// W = A^-1 S from the factor record (step r of the product takes users
// 4 kq + r of S, which this lane loads, against B[u][4 kq + r]), then
// X = H W for each block of 16 antennas (step r takes H[16 b + u][4 kq + r]
// from LDS against W[4 kq + r][u], which this lane holds); both with three
// real products per complex one.  A tile whose factorisation broke down, or
// whose channel is not finite, transmits nothing (X = 0) and is flagged.
// One workgroup per (tile, frame); wave w owns the symbols d = w + 4 j.
template <int Q>
__global__ void __launch_bounds__(256)
precode_group_kernel(const float2* __restrict__ Yf, const float2* __restrict__ pil,
                     const GroupRec* __restrict__ rec, const void* __restrict__ src, float2* __restrict__ xf,
                     uint8_t* __restrict__ flags, int M, int S, int n_sc) {
  __shared__ float2 hs[64 * 16];                // H of the tile: [antenna][user]
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int u = l & 15, kq = l >> 4;
  const int D = S - 1;
  const int64_t f = blockIdx.y;
  const int tt = blockIdx.x;
  const int i0 = tt * 16;
  const int g = min(tt, n_sc / 16 - 1);
  const int nj = D > w ? (D - w + 3) >> 2 : 0;

  const GroupRec* R = rec + (f * gridDim.x + tt);
  const __amdgpu_buffer_rsrc_t rr = rsrc(R, (uint32_t)sizeof(GroupRec));
  float2 brow[4];
  {
    const uint32_t o = opaque((uint32_t)(u * 16 + 4 * kq) * 8u);
    const float4v b01 = __builtin_bit_cast(float4v, __builtin_amdgcn_raw_buffer_load_b128(rr, (int)o, 0, 0));
    const float4v b23 = __builtin_bit_cast(float4v, __builtin_amdgcn_raw_buffer_load_b128(rr, (int)(o + 16u), 0, 0));
    brow[0] = make_float2(b01.x, b01.y);
    brow[1] = make_float2(b01.z, b01.w);
    brow[2] = make_float2(b23.x, b23.y);
    brow[3] = make_float2(b23.z, b23.w);
  }
  const float2 okh = ldg2(rr, opaque(2048u + 64u));
  const __amdgpu_buffer_rsrc_t yr = rsrc(Yf + f * M * S * n_sc, (uint32_t)M * S * n_sc * 8u);
  const uint32_t ant = (uint32_t)S * n_sc * 32u;
  float2 hv[4], pv;
  {
    const int q = g * 16 + u;
    uint32_t row = opaque((uint32_t)((16 * w + kq) * S * n_sc + q) * 8u);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      hv[a] = ldg2(yr, row);
      row = opaque(row + ant);
    }
    pv = ldg2(rsrc(pil + f * n_sc, (uint32_t)n_sc * 8u), opaque((uint32_t)q * 8u));
  }
  // S[4 kq + r][d][i0 + u] for the wave's symbols (absent ones read zero)
  float2 sv[4][4];
  {
    constexpr uint32_t PB = Q ? Q : 8;           // bytes per point
    const __amdgpu_buffer_rsrc_t sr =
        rsrc((const uint8_t*)src + f * 16 * D * n_sc * PB, (uint32_t)16 * D * n_sc * PB);
    const uint32_t OOBE = OOB / 8u;              // an element index whose byte offset is past any range
    const uint32_t lane = i0 + u < n_sc ? (uint32_t)((4 * kq * D + w) * n_sc + i0 + u) : OOBE;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t row = opaque(j < nj ? lane + (uint32_t)j * 4u * n_sc : OOBE);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sv[j][r] = load_point<Q>(sr, row);
        row = opaque(row + (uint32_t)D * n_sc);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int m = 16 * w + 4 * a + kq;
    hs[m * 16 + u] = m < M ? ls_estimate(hv[a], pv) : make_float2(0.f, 0.f);
  }
  __syncthreads();

  const bool hb = __builtin_bit_cast(int, okh.y) != 0;
  const bool ok = __builtin_bit_cast(int, okh.x) != 0;
  const bool erase = hb || !ok;
  const int i = i0 + u;
  float2* xo = xf + f * M * D * n_sc;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j >= nj) break;
    const int d = w + 4 * j;
    // W = A^-1 S
    f32x4 wk = {0.f, 0.f, 0.f, 0.f}, wr = wk, wi = wk;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float2 b = brow[r], sr2 = sv[j][r];
      wk = mfma(b.x + b.y, sr2.x, wk);
      wr = mfma(b.y, sr2.x + sr2.y, wr);
      wi = mfma(b.x, sr2.y - sr2.x, wi);
    }
    const f32x4 Wr = wk - wr, Wi = wk + wi;
    // X = H W, 16 antennas at a time
#pragma unroll
    for (int bl = 0; bl < 4; ++bl) {
      if (16 * bl >= M) break;
      f32x4 xk = {0.f, 0.f, 0.f, 0.f}, xr = xk, xi = xk;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float2 h = hs[(16 * bl + u) * 16 + 4 * kq + r];
        xk = mfma(h.x + h.y, Wr[r], xk);
        xr = mfma(h.y, Wr[r] + Wi[r], xr);
        xi = mfma(h.x, Wi[r] - Wr[r], xi);
      }
      if (i < n_sc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = 16 * bl + 4 * kq + r;
          if (m < M)
            xo[((int64_t)m * D + d) * n_sc + i] =
                erase ? make_float2(0.f, 0.f) : make_float2(xk[r] - xr[r], xk[r] + xi[r]);
        }
      }
    }
  }
  if (w == 0 && kq == 0 && i < n_sc && flags)
    flags[f * n_sc + i] = hb ? RXPHY_FLAG_NONFINITE : (ok ? 0 : RXPHY_FLAG_BREAKDOWN);
}

}  // namespace

rxphy_status launch_precode(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                            const void* src, int src_bits, float2* xf, uint8_t* flags, void* ws, bool reuse,
                            hipStream_t s) {
  if (nf == 0) return RXPHY_OK;
  if (fr.K != 16) return fail(RXPHY_EUNSUPPORTED, "precode: K = %d (the precoder is built for 16 users)", fr.K);
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  if (!ws || ((uintptr_t)ws & 7u)) return fail(RXPHY_EWORKSPACE, "precode workspace must be 8-byte aligned");
  const int nt = (fr.n_sc + 15) / 16;
  const int64_t T = (int64_t)nf * nt;
  GroupRec* rec = (GroupRec*)ws;
  if (!reuse) {                                  // else: the uplink's records for these frames are in ws
    hipLaunchKernelGGL((group_factor_kernel<FTPW, P_FP32>), dim3((unsigned)((T + FTPW * GWAVES - 1) / (FTPW * GWAVES))),
                       dim3(256), 0, s, yf, pil, rec, (int)T, nt, fr.M, fr.n_sym, fr.n_sc, fr.n0,
                       fr.detector == RXPHY_MMSE ? 1 : 0, 0.f, (uint32_t*)nullptr);
    rxphy_status st = launch_status("group factor kernel");
    if (st) return st;
  }
  const dim3 grid(nt, nf);
  switch (src_bits) {
    case 0: hipLaunchKernelGGL(precode_group_kernel<0>, grid, dim3(256), 0, s, yf, pil, rec, src, xf, flags, fr.M, fr.n_sym, fr.n_sc); break;
    case 2: hipLaunchKernelGGL(precode_group_kernel<2>, grid, dim3(256), 0, s, yf, pil, rec, src, xf, flags, fr.M, fr.n_sym, fr.n_sc); break;
    case 4: hipLaunchKernelGGL(precode_group_kernel<4>, grid, dim3(256), 0, s, yf, pil, rec, src, xf, flags, fr.M, fr.n_sym, fr.n_sc); break;
    case 6: hipLaunchKernelGGL(precode_group_kernel<6>, grid, dim3(256), 0, s, yf, pil, rec, src, xf, flags, fr.M, fr.n_sym, fr.n_sc); break;
    default: return fail(RXPHY_EINVAL, "qam_bits = %d", src_bits);
  }
  return launch_status("precode kernel");
}

size_t group_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec) {
  const size_t recs = (size_t)nf * ((fr.n_sc + 15) / 16) * sizeof(GroupRec);
  if (prec == RXPHY_FP32) return recs;
  return recs + (size_t)RL_OFF * 4 + (size_t)nf * fr.n_sc * 4;      // + the refinement list (tiles)
}

namespace {
__global__ void clear_list_kernel(uint32_t* rl) {
  if (threadIdx.x == 0) rl[0] = 0u;
}

template <int P>
rxphy_status launch_group_p(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                            float2* xt, float* nu, uint8_t* flags, float* llr, float thr, GroupRec* rec,
                            uint32_t* rl, hipStream_t s) {
  const int nt = (fr.n_sc + 15) / 16;
  const int64_t T = (int64_t)nf * nt;
  const int mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
  hipLaunchKernelGGL((group_factor_kernel<FTPW, P>), dim3((unsigned)((T + FTPW * GWAVES - 1) / (FTPW * GWAVES))), dim3(256),
                     0, s, yf, pil, rec, (int)T, nt, fr.M, fr.n_sym, fr.n_sc, fr.n0, mmse, thr, rl);
  rxphy_status st = launch_status("group factor kernel");
  if (st) return st;
  const dim3 grid(nt, nf);
  const int q = llr ? fr.qam_bits : 0;
#define RXPHY_GROUP_LAUNCH(QQ)                                                                                   \
  hipLaunchKernelGGL((detect_group_kernel<QQ, P>), grid, dim3(256), 0, s, yf, pil, rec, xt, nu, flags, llr, fr.M, \
                     fr.n_sym, fr.n_sc, fr.n0, mmse)
  switch (q) {
    case 0: RXPHY_GROUP_LAUNCH(0); break;
    case 2: RXPHY_GROUP_LAUNCH(2); break;
    case 4: RXPHY_GROUP_LAUNCH(4); break;
    case 6: RXPHY_GROUP_LAUNCH(6); break;
    default: return fail(RXPHY_EINVAL, "qam_bits = %d", fr.qam_bits);
  }
#undef RXPHY_GROUP_LAUNCH
  return launch_status("detect group kernel");
}
}  // namespace

rxphy_status launch_detect_group(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                 float2* xt, float* nu, uint8_t* flags, float* llr, rxphy_precision prec,
                                 float thr, void* ws, hipStream_t s) {
  if (nf == 0) return RXPHY_OK;
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);   // grid y
  if (!ws || ((uintptr_t)ws & 7u)) return fail(RXPHY_EWORKSPACE, "csi_detect workspace must be 8-byte aligned");
  GroupRec* rec = (GroupRec*)ws;
  if (prec == RXPHY_FP32) return launch_group_p<P_FP32>(fr, nf, yf, pil, xt, nu, flags, llr, 0.f, rec, nullptr, s);
  uint32_t* rl = (uint32_t*)((char*)ws + group_workspace_bytes(fr, nf, RXPHY_FP32));
  hipLaunchKernelGGL(clear_list_kernel, dim3(1), dim3(64), 0, s, rl);
  rxphy_status st = launch_status("clear list kernel");
  if (st) return st;
  st = prec == RXPHY_BF16 ? launch_group_p<P_BF16>(fr, nf, yf, pil, xt, nu, flags, llr, thr, rec, rl, s)
                          : launch_group_p<P_FP16>(fr, nf, yf, pil, xt, nu, flags, llr, thr, rec, rl, s);
  if (st) return st;
  return launch_refine_group(fr, nf, yf, pil, xt, nu, flags, llr, rl, s);
}

}  // namespace rxphy
