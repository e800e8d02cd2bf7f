// Batched segment FFT (Section III-A1: a non-overlapping N_FFT-point FFT per
// segment; Section IV-D: time-parallel across segments) for gfx950.
//
// One transform per segment (antenna, OFDM symbol).  Each thread owns 8
// points; the transform runs as Stockham auto-sort passes (radix 8, then a
// final radix 2, 4 or 8) whose exchanges go through LDS with one padding slot
// per 8 complex values.  The first pass reads the segment straight from HBM
// (coalesced, the cyclic prefix skipped by offset) and the last pass writes
// straight to HBM, keeping only the used bins.  The inverse-direction variant
// (used by the adjoint) gathers the used-bin vector into a zero-padded grid on
// the way in and writes every time sample (zeros over the cyclic prefix).
#include "common.h"

namespace rxphy {
namespace {

__device__ __forceinline__ int padi(int i) { return i + (i >> 3); }

template <bool INV>
__device__ __forceinline__ float2 mul_mj(float2 a) {  // * -j (forward) or * +j (inverse)
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ float2 twid(float2 a, float2 w) {
  return INV ? cmulc(a, w) : cmul(a, w);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& c0, float2& c1, float2& c2, float2& c3) {
  float2 e0 = cadd(c0, c2), e1 = csub(c0, c2);
  float2 o0 = cadd(c1, c3), o1 = mul_mj<INV>(csub(c1, c3));
  c0 = cadd(e0, o0);
  c2 = csub(e0, o0);
  c1 = cadd(e1, o1);
  c3 = csub(e1, o1);
}

template <bool INV>
__device__ __forceinline__ void dft4v(float2* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }

// 8-point DFT in registers: split into even/odd output halves.
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  const float h = 0.70710678118654752440f;
  float2 a0 = cadd(v[0], v[4]), a1 = cadd(v[1], v[5]), a2 = cadd(v[2], v[6]), a3 = cadd(v[3], v[7]);
  float2 b0 = csub(v[0], v[4]), b1 = csub(v[1], v[5]), b2 = csub(v[2], v[6]), b3 = csub(v[3], v[7]);
  // b_r *= W8^r with W8 = exp(-j pi/4) (forward) or exp(+j pi/4) (inverse)
  b1 = INV ? make_float2(h * (b1.x - b1.y), h * (b1.x + b1.y))
           : make_float2(h * (b1.x + b1.y), h * (b1.y - b1.x));
  b2 = mul_mj<INV>(b2);
  b3 = INV ? make_float2(-h * (b3.x + b3.y), h * (b3.x - b3.y))
           : make_float2(h * (b3.y - b3.x), -h * (b3.x + b3.y));
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 4) dft4v<INV>(v);
  else dft2<INV>(v);
}

constexpr int n_radix8(int n) { return n % 8 == 0 ? 1 + n_radix8(n / 8) : 0; }
constexpr int ipow8(int p) { return p == 0 ? 1 : 8 * ipow8(p - 1); }

template <int N>
struct Geom {
  static constexpr int T = N / 8;                    // threads per transform
  static constexpr int WG = T < 256 ? 256 : T;       // workgroup size
  static constexpr int TPW = WG / T;                 // transforms per workgroup
  static constexpr int LDSN = N + N / 8;             // padded LDS slots per transform
  static constexpr int N8 = n_radix8(N);             // radix-8 factors
  static constexpr int REM = N / ipow8(N8);          // 1, 2 or 4
  static constexpr int LAST_R = REM == 1 ? 8 : REM;  // radix of the last pass
  static constexpr int NMID = REM == 1 ? N8 - 2 : N8 - 1;  // LDS-to-LDS radix-8 passes
};

// Each workgroup runs PER_WG transforms per transform slot in a loop: the
// twiddles a thread needs are the same for every transform, so they are
// loaded into registers once, and the next segment's input is fetched while
// the current one moves through LDS.
constexpr int PER_WG = 8;

template <int N, bool INV>
__device__ __forceinline__ void load_input(const float2* __restrict__ in, int64_t tr, bool active,
                                           int tid, int sym_len, int cp, int n_sc, float2* v) {
  constexpr int T = N / 8;
  const int half = n_sc >> 1;
  if (!INV) {
    const float2* src = in + (active ? tr : 0) * sym_len + cp;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = active ? src[tid + r * T] : make_float2(0.f, 0.f);
  } else {
    const float2* src = in + (active ? tr : 0) * n_sc;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i = (tid + r * T + half) & (N - 1);
      v[r] = (active && i < n_sc) ? src[i] : make_float2(0.f, 0.f);
    }
  }
}

template <int N, bool INV>
__global__ void __launch_bounds__(Geom<N>::WG)
fft_kernel(const float2* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ tw,
           int64_t n_tr, int sym_len, int cp, int n_sc) {
  using G = Geom<N>;
  constexpr int T = G::T;
  constexpr int R = G::LAST_R;
  constexpr int NS = N / R;
  constexpr int NMID = G::NMID;
  __shared__ float2 lds[G::TPW * G::LDSN];
  const int sub = threadIdx.x / T;
  const int tid = threadIdx.x - sub * T;
  float2* buf = lds + sub * G::LDSN;
  const int half = n_sc >> 1;

  // twiddles of this thread: middle passes (Ns = 8, 64, ...) and the last pass
  float2 twm[NMID > 0 ? NMID : 1][7];
  float2 twl[8 / R][R - 1];
  {
    int Ns = 8;
#pragma unroll
    for (int p = 0; p < NMID; ++p) {
      const int k = tid & (Ns - 1);
      const int step = 4096 / (Ns * 8);
#pragma unroll
      for (int r = 1; r < 8; ++r) twm[p][r - 1] = tw[r * k * step];
      Ns *= 8;
    }
#pragma unroll
    for (int b = 0; b < 8 / R; ++b) {
      const int j = tid + b * T;
#pragma unroll
      for (int r = 1; r < R; ++r) twl[b][r - 1] = tw[r * j * (4096 / N)];
    }
  }

  const int64_t base = (int64_t)blockIdx.x * G::TPW * PER_WG + sub;
  float2 v[8], vn[8];
  load_input<N, INV>(in, base, base < n_tr, tid, sym_len, cp, n_sc, v);
  for (int it = 0; it < PER_WG; ++it) {
    const int64_t tr = base + (int64_t)it * G::TPW;
    const bool active = tr < n_tr;
    // pass 0: radix 8, Ns = 1 (no twiddles); input element tid + r T
    dft8<INV>(v);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[padi(tid * 8 + r)] = v[r];
    __syncthreads();
    if (it + 1 < PER_WG) {
      const int64_t tn = tr + G::TPW;
      load_input<N, INV>(in, tn, tn < n_tr, tid, sym_len, cp, n_sc, vn);
    }
    // middle radix-8 passes, Ns = 8, 64, ...
    int Ns = 8;
#pragma unroll
    for (int p = 0; p < NMID; ++p) {
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = buf[padi(tid + r * (N / 8))];
      const int k = tid & (Ns - 1);
#pragma unroll
      for (int r = 1; r < 8; ++r) v[r] = twid<INV>(v[r], twm[p][r - 1]);
      dft8<INV>(v);
      __syncthreads();
      const int o = (tid - k) * 8 + k;  // (tid / Ns) * Ns * 8 + k
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[padi(o + r * Ns)] = v[r];
      __syncthreads();
      Ns *= 8;
    }
    // last pass: radix R, Ns = N / R; each thread does 8 / R butterflies j
#pragma unroll
    for (int b = 0; b < 8 / R; ++b) {
      const int j = tid + b * T;
      float2 w[R];
#pragma unroll
      for (int r = 0; r < R; ++r) w[r] = buf[padi(j + r * NS)];
#pragma unroll
      for (int r = 1; r < R; ++r) w[r] = twid<INV>(w[r], twl[b][r - 1]);
      dftR<R, INV>(w);
      if (active) {
        if (!INV) {
          float2* dst = out + tr * n_sc;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int i = (j + r * NS + half) & (N - 1);
            if (i < n_sc) dst[i] = w[r];
          }
        } else {
          float2* dst = out + tr * sym_len + cp;
#pragma unroll
          for (int r = 0; r < R; ++r) dst[j + r * NS] = w[r];
        }
      }
    }
    if (INV && active) {
      float2* dst = out + tr * sym_len;
      for (int n = tid; n < cp; n += T) dst[n] = make_float2(0.f, 0.f);
    }
    __syncthreads();   // the next transform's pass 0 overwrites this LDS slab
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = vn[r];
  }
}

template <int N, bool INV>
rxphy_status run(int64_t n_tr, const float2* in, float2* out, const float2* tw, int sym_len,
                 int cp, int n_sc, hipStream_t s) {
  using G = Geom<N>;
  const int64_t per = (int64_t)G::TPW * PER_WG;
  int64_t blocks = (n_tr + per - 1) / per;
  if (blocks > 0x7fffffff) return fail(RXPHY_EUNSUPPORTED, "too many transforms (%lld)", (long long)n_tr);
  hipLaunchKernelGGL((fft_kernel<N, INV>), dim3((unsigned)blocks), dim3(G::WG), 0, s, in, out, tw,
                     n_tr, sym_len, cp, n_sc);
  return launch_status("fft kernel");
}

}  // namespace

rxphy_status launch_fft(const rxphy_frame& fr, int64_t n_tr, const float2* in, float2* out,
                        bool inverse, hipStream_t s) {
  const float2* tw = nullptr;
  rxphy_status st = ensure_device_tables(&tw);
  if (st) return st;
  const int L = (int)sym_len(fr);
#define RXPHY_FFT_CASE(NN)                                                                  \
  case NN:                                                                                  \
    return inverse ? run<NN, true>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, s)              \
                   : run<NN, false>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, s);
  switch (fr.n_fft) {
    RXPHY_FFT_CASE(512)
    RXPHY_FFT_CASE(1024)
    RXPHY_FFT_CASE(2048)
    RXPHY_FFT_CASE(4096)
  }
#undef RXPHY_FFT_CASE
  return fail(RXPHY_EUNSUPPORTED, "n_fft = %d", fr.n_fft);
}

}  // namespace rxphy
