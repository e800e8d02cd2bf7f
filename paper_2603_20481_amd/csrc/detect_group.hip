// Fused CSI + ZF / MMSE detector for K = 16 users, FP32 (Sec. III-B LS
// estimate with the comb pilots, Sec. III-C equaliser, Eq. (4)-(6)).
//
// With 16 users a pilot group spans exactly one 16-subcarrier tile, and the
// LS estimate is held over the group, so every subcarrier of a tile sees the
// same channel matrix H (64 x 16).  Per tile the work is
//   G = H^H H (+ N0 I) once, its Cholesky factor once, and
//   Z = H^H Y for 16 subcarriers x D data symbols, then L L^H X = Z.
// This kernel is built around that shape instead of staging H per subcarrier:
//
//  * The data operands are loaded straight from HBM into the lanes that use
//    them (lane (kq, u) of v_mfma_f32_16x16x4_f32: B = Y[4s + kq][1 + d][i0 + u],
//    16 lanes per 128-byte row segment), all of a wave's loads issued at
//    once, no LDS staging.  Wave w owns data symbols d = w, w + 4, w + 8,
//    w + 12 and runs all 64 antennas for them (16 steps of 4 antennas).
//  * H is formed once per tile (each wave 16 antennas: the pilot-symbol row
//    and the pilots, LS) into LDS, read by every wave as the A operand.
//  * The partial Gram matrices meet in LDS; one wave (rotating over the
//    waves with the fewest symbols) factors A; each wave transposes its own
//    Z through a wave-private LDS slab and solves its own right-hand sides
//    (lane = (symbol, subcarrier)).  Two workgroups share a CU, so one's
//    loads and products overlap the other's factorisation and solves.
//
// Every product, sum and factorisation step is the one the general detector
// (detect_core.h, shared-factor path) performs on the same values in the
// same order, so the results are bit-identical to rxphy_csi + rxphy_detect.
#include "detect_core.h"

namespace rxphy {
namespace {

using namespace det;

constexpr int GWAVES = 4;     // waves per workgroup
constexpr int NJ = 4;         // symbol slots per wave: d = w + 4 j
constexpr int ZP = 17;        // float2 pitch of a slab row (bank spread)

struct GroupLds {
  float2 h[64 * 16];                    // H of the tile: [antenna][user]
  float2 part[GWAVES][16 * PP];         // per-wave partial Gram matrices
  float2 L[16 * PP];                    // Cholesky factor, row by row
  float inv[16];                        // 1 / L_kk
  float dl[16];                         // d_k = [A^-1]_kk
  int ok;
  int hbad[GWAVES];                     // a non-finite H value (per storing wave)
  uint32_t nfmask[GWAVES];              // subcarriers with a non-finite data value
  float2 slab[GWAVES][NJ * 16 * ZP];    // per wave: Z as [slot j][user k][subcarrier]
};

__device__ __forceinline__ float2 ldg2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
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

// Z = H^H Y over the 16 antenna steps, in order, for symbol slot J, three
// real products per complex one: for h = a + jb, y = c + jd,
// conj(h) y = (k1 + b (c + d)) + j (k1 + a (d - c)), k1 = (a - b) c.
template <int J, bool FULLM>
__device__ __forceinline__ void z_slot(const float2* hs, const float2 (*y)[NJ], f32x4& zr, f32x4& zi,
                                       float& probe, int kq, int u, int M) {
  f32x4 zk = {0.f, 0.f, 0.f, 0.f};
  zr = zi = zk;
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
}

template <bool FULLM>
__device__ __forceinline__ void z_all(const float2* hs, const float2 (*y)[NJ], f32x4* zr, f32x4* zi,
                                      float& probe, int nj, int kq, int u, int M) {
  if (nj > 0) z_slot<0, FULLM>(hs, y, zr[0], zi[0], probe, kq, u, M);
  if (nj > 1) z_slot<1, FULLM>(hs, y, zr[1], zi[1], probe, kq, u, M);
  if (nj > 2) z_slot<2, FULLM>(hs, y, zr[2], zi[2], probe, kq, u, M);
  if (nj > 3) z_slot<3, FULLM>(hs, y, zr[3], zi[3], probe, kq, u, M);
}

// One workgroup per (tile, frame): blockIdx.x = tile, blockIdx.y = frame.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
detect_group_kernel(const float2* __restrict__ Yf, const float2* __restrict__ pil, float2* __restrict__ xt,
                    float* __restrict__ nu, uint8_t* __restrict__ flags, int M, int S, int n_sc, float n0,
                    int mmse) {
  __shared__ GroupLds sh;
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

  const __amdgpu_buffer_rsrc_t yr = rsrc(Yf + f * M * S * n_sc, (uint32_t)M * S * n_sc * 8u);
  const uint32_t ant = (uint32_t)S * n_sc * 32u;             // 4 antennas
  const uint32_t sym = (uint32_t)n_sc * 32u;                 // 4 symbols

  // ---- loads: this wave's 16 antennas of the pilot-symbol row and the
  // pilots, then all of its data, symbol slot by symbol slot
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
  float2 y[16][NJ];
  {
    const uint32_t lane = i0 + u < n_sc ? (uint32_t)((kq * S + 1 + w) * n_sc + i0 + u) * 8u : OOB;
    // (a fixed count of loads, so that each use waits for exactly its own:
    // the slots this wave does not own read zero without touching memory)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      uint32_t row = opaque(j < nj ? lane + (uint32_t)j * sym : OOB);
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        y[s][j] = ldg2(yr, row);
        row = opaque(row + ant);
      }
    }
  }

  // ---- H = LS estimate (absent antennas zero), non-finite check
  {
    float probe = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int m = 16 * w + 4 * a + kq;
      const float2 h = m < M ? ls_estimate(hv[a], pv) : make_float2(0.f, 0.f);
      probe = __builtin_fmaf(h.x, 0.f, probe);
      probe = __builtin_fmaf(h.y, 0.f, probe);
      sh.h[m * 16 + u] = h;
    }
    const bool bad = __ballot(!(probe == 0.f)) != 0ull;
    if (l == 0) sh.hbad[w] = bad ? 1 : 0;
  }
  __syncthreads();

  // ---- phase 1: Z for this wave's symbols, the partial Gram matrix over
  // the 8-antenna chunks w and w + 4
  {
    f32x4 zr[NJ], zi[NJ];
    float probe = 0.f;
    if (M == 64) z_all<true>(sh.h, y, zr, zi, probe, nj, kq, u, M);
    else z_all<false>(sh.h, y, zr, zi, probe, nj, kq, u, M);
    float2* slab = sh.slab[w];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      if (j < nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) slab[(j * 16 + 4 * kq + r) * ZP + u] = make_float2(zr[j][r], zi[j][r]);
    const uint64_t bad = __ballot(!(probe == 0.f));
    const uint32_t m16 = (uint32_t)(bad | (bad >> 16) | (bad >> 32) | (bad >> 48)) & 0xffffu;
    if (l == 0) sh.nfmask[w] = m16;
  }
  {
    f32x4 g0r = {0.f, 0.f, 0.f, 0.f}, g0i = g0r;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = w + 4 * b;                  // chunk c: antennas 8 c .. 8 c + 7
      if (c * MC < M) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const float2 h = sh.h[(8 * c + 4 * a + kq) * 16 + u];
          g0r = mfma(h.x, h.x, g0r);
          g0r = mfma(h.y, h.y, g0r);
          g0i = mfma(h.x, h.y, g0i);
          g0i = mfma(-h.y, h.x, g0i);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.part[w][(4 * kq + r) * PP + u] = make_float2(g0r[r], g0i[r]);
  }
  __syncthreads();

  // ---- factorisation: one of the waves with the fewest symbols
  const int e0 = D & 3;
  const int wf = e0 ? e0 + (int)(tt % (4 - e0)) : (tt & 3);
  if (w == wf) {
    const int row = u;
    float2 a[16], v[16];
    float inv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float2 s = sh.part[0][row * PP + c];
      s = cadd(s, sh.part[1][row * PP + c]);
      s = cadd(s, sh.part[2][row * PP + c]);
      s = cadd(s, sh.part[3][row * PP + c]);
      if (c == row) s.x = s.x + (mmse ? n0 : 0.f);
      a[c] = s;
    }
    bool okw = true;
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = make_float2(k == row ? 1.f : 0.f, 0.f);
    crout_all<16>(Seq16{}, a, v, inv, row, okw);
    float d = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) d += v[k].x * v[k].x + v[k].y * v[k].y;
    if (kq == 0) {
#pragma unroll
      for (int c = 0; c < 16; ++c) sh.L[row * PP + c] = a[c];
      sh.dl[row] = d;
      sh.inv[row] = inv[row];
      if (row == 0) sh.ok = okw ? 1 : 0;
    }
  }
  __syncthreads();

  // ---- solves: lane (kq, u) = symbol slot kq, subcarrier u of this wave
  const int d = w + 4 * kq;
  const int i = i0 + u;
  const uint32_t nfm = sh.nfmask[0] | sh.nfmask[1] | sh.nfmask[2] | sh.nfmask[3];
  const bool hb = (sh.hbad[0] | sh.hbad[1] | sh.hbad[2] | sh.hbad[3]) != 0;
  const bool nf_i = hb || ((nfm >> u) & 1u);
  bool ok = sh.ok != 0;
  if (mmse) {
#pragma unroll
    for (int k = 0; k < 16; ++k) ok = ok && (1.0f - n0 * sh.dl[k] > 0.f);
  }
  const bool erase = nf_i || !ok;
  if (d < D) {
    float2 z[16];
    float inv[16];
    const float2* slab = sh.slab[w];
#pragma unroll
    for (int k = 0; k < 16; ++k) z[k] = slab[(kq * 16 + k) * ZP + u];
#pragma unroll
    for (int k = 0; k < 16; ++k) inv[k] = sh.inv[k];
    fwd_all<16>(Seq16{}, sh.L, inv, z);          // L W = Z
    bwd_all<16>(Seq16{}, sh.L, inv, z);          // L^H X = W
    if (mmse) {
#pragma unroll
      for (int k = 0; k < 16; ++k) z[k] = cscale(z[k], __builtin_amdgcn_rcpf(1.0f - n0 * sh.dl[k]));
    }
    if (i < n_sc) {
      float2* xo = xt + f * 16 * D * n_sc;
#pragma unroll
      for (int k = 0; k < 16; ++k) xo[((int64_t)k * D + d) * n_sc + i] = erase ? make_float2(0.f, 0.f) : z[k];
    }
  }
  if (i < n_sc) {
    const int k = 4 * w + kq;
    const float dk = sh.dl[k];
    const float nv = mmse ? n0 * dk * __builtin_amdgcn_rcpf(1.0f - n0 * dk) : n0 * dk;
    nu[(f * 16 + k) * n_sc + i] = erase ? INFINITY : nv;
    if (w == 0 && kq == 0 && flags)
      flags[f * n_sc + i] = nf_i ? RXPHY_FLAG_NONFINITE : (ok ? 0 : RXPHY_FLAG_BREAKDOWN);
  }
}

}  // namespace

rxphy_status launch_detect_group(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                 float2* xt, float* nu, uint8_t* flags, hipStream_t s) {
  if (nf == 0) return RXPHY_OK;
  const dim3 grid((fr.n_sc + 15) / 16, nf);
  hipLaunchKernelGGL(detect_group_kernel, grid, dim3(256), 0, s, yf, pil, xt, nu, flags, fr.M, fr.n_sym,
                     fr.n_sc, fr.n0, fr.detector == RXPHY_MMSE ? 1 : 0);
  return launch_status("detect group kernel");
}

}  // namespace rxphy
