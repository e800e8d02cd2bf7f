// Segment FFT tile body (Section III-A1: a non-overlapping N_FFT-point FFT per
// segment; Section IV-D: time-parallel across segments), shared by the
// per-stage FFT kernels and the persistent batched kernel.
//
// A workgroup has 256 threads.  A transform is owned by N/8 virtual threads of
// 8 points each; for N <= 2048 a thread is one virtual thread and a workgroup
// holds 256/(N/8) transforms side by side, for N = 4096 each thread plays two
// virtual threads.  The transform runs as Stockham auto-sort passes (radix 8,
// then a last radix 2, 4 or 8) whose exchanges go through LDS with one padding
// slot per 8 complex values.  The first pass reads the segment straight from
// HBM (coalesced, the cyclic prefix skipped by offset) and the last pass writes
// straight to HBM, keeping only the used bins.  The inverse-direction variant
// (used by the adjoint) gathers the used-bin vector into a zero-padded grid on
// the way in and writes every time sample (zeros over the cyclic prefix).
#pragma once

#include <type_traits>

#include "common.h"

namespace rxphy {
namespace fftk {

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

constexpr int WG = 256;                              // threads per workgroup

template <int N>
struct Geom {
  static constexpr int T = N / 8;                    // virtual threads per transform
  static constexpr int VT = T > WG ? T / WG : 1;     // virtual threads per thread
  static constexpr int TT = T / VT;                  // threads per transform
  static constexpr int TPW = WG / TT;                // transforms per workgroup pass
  static constexpr int LDSN = N + N / 8;             // padded LDS slots per transform
  static constexpr int LDS = TPW * LDSN;             // LDS slots per workgroup
  static constexpr int N8 = n_radix8(N);             // radix-8 factors
  static constexpr int REM = N / ipow8(N8);          // 1, 2 or 4
  static constexpr int LAST_R = REM == 1 ? 8 : REM;  // radix of the last pass
  static constexpr int NMID = REM == 1 ? N8 - 2 : N8 - 1;  // LDS-to-LDS radix-8 passes
  static_assert(WG % TT == 0 && T % VT == 0, "bad FFT geometry");
};

constexpr int LDS_MAX = Geom<4096>::LDS;             // largest LDS need of any size

// Samples are complex64, or 16-bit fixed-point I/Q pairs (short2): value =
// integer * scale.  A 16-bit pair is loaded as one raw 32-bit word (kept in
// the .x slot) and converted only where the transform first uses it, so the
// eight loads of a transform stay in flight together.
__device__ __forceinline__ float2 to_f2(float2 v, float) { return v; }
__device__ __forceinline__ float2 to_f2(short2 v, float) {
  return make_float2(__builtin_bit_cast(float, v), 0.f);
}

template <typename IN_T>
__device__ __forceinline__ void finish_input(float2* v, float scale) {
  if constexpr (!std::is_same<IN_T, float2>::value) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const short2 s = __builtin_bit_cast(short2, v[r].x);
      v[r] = make_float2((float)s.x * scale, (float)s.y * scale);
    }
  }
}

template <int N, bool INV, typename IN_T = float2>
__device__ __forceinline__ void load_input(const IN_T* __restrict__ in, int64_t tr, bool active,
                                           int vt, int sym_len, int cp, int n_sc, float2* v,
                                           float scale = 1.f) {
  constexpr int T = N / 8;
  const int half = n_sc >> 1;
  if constexpr (!INV) {
    const IN_T* src = in + (active ? tr : 0) * sym_len + cp;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = active ? to_f2(src[vt + r * T], scale) : make_float2(0.f, 0.f);
  } else {
    const float2* src = in + (active ? tr : 0) * n_sc;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i = (vt + r * T + half) & (N - 1);
      v[r] = (active && i < n_sc) ? src[i] : make_float2(0.f, 0.f);
    }
  }
}

// Transforms first, first + TPW, ..., first + (iters - 1) TPW of the thread's
// transform slot (first = workgroup base + slot); transforms >= n_tr are
// skipped.  The twiddles a thread needs are the same for every transform, so
// they are loaded into registers once.  `lds` holds Geom<N>::LDS
// slots; the caller synchronises before reusing it.
// Inverse output as 16-bit I/Q (the transmit fronthaul format): each
// component times out_scale, rounded to nearest even and saturated.
__device__ __forceinline__ short2 to_sc16(float2 v, float s) {
  const int a = min(max(__float2int_rn(v.x * s), -32768), 32767);
  const int b = min(max(__float2int_rn(v.y * s), -32768), 32767);
  return make_short2((short)a, (short)b);
}

template <int N, bool INV, bool MAG = false, typename IN_T = float2, bool OUT16 = false>
__device__ __forceinline__ void fft_tile(const IN_T* __restrict__ in, float2* __restrict__ out,
                                         const float2* __restrict__ tw, int64_t n_tr, int64_t base,
                                         int iters, int sym_len, int cp, int n_sc, float2* lds,
                                         bool cp_tail = false, float in_scale = 1.f, float out_scale = 1.f) {
  using G = Geom<N>;
  constexpr int T = G::T;
  constexpr int VT = G::VT;
  constexpr int R = G::LAST_R;
  constexpr int NS = N / R;
  constexpr int NMID = G::NMID;
  const int tx = tid_x();
  const int sub = tx / G::TT;
  const int tid = tx - sub * G::TT;
  float2* buf = lds + sub * G::LDSN;
  const int half = n_sc >> 1;

  // twiddles: the middle passes (Ns = 8, 64, ...) depend on vt mod Ns, which is
  // the same for every virtual thread of a thread (Ns divides 256); the last
  // pass has its own per virtual thread
  float2 twm[NMID > 0 ? NMID : 1][7];
  float2 twl[VT][8 / R][R - 1];
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
    for (int q = 0; q < VT; ++q)
#pragma unroll
      for (int b = 0; b < 8 / R; ++b) {
        const int j = tid + q * G::TT + b * T;
#pragma unroll
        for (int r = 1; r < R; ++r) twl[q][b][r - 1] = tw[r * j * (4096 / N)];
      }
  }

  // With one virtual thread the next segment is prefetched during the current
  // one; with two, the 16 loads per thread already in flight suffice and the
  // registers of a prefetch would cost occupancy.
  constexpr bool PREFETCH = VT == 1;
  base += sub;
  float2 v[VT][8], vn[PREFETCH ? VT : 1][8];
  if (PREFETCH) {
#pragma unroll
    for (int q = 0; q < VT; ++q)
      load_input<N, INV, IN_T>(in, base, base < n_tr, tid + q * G::TT, sym_len, cp, n_sc, v[q], in_scale);
  }
  for (int it = 0; it < iters; ++it) {
    const int64_t tr = base + (int64_t)it * G::TPW;
    const bool active = tr < n_tr;
    if (!PREFETCH) {
#pragma unroll
      for (int q = 0; q < VT; ++q)
        load_input<N, INV, IN_T>(in, tr, active, tid + q * G::TT, sym_len, cp, n_sc, v[q], in_scale);
    }
    // pass 0: radix 8, Ns = 1 (no twiddles); input element vt + r T
#pragma unroll
    for (int q = 0; q < VT; ++q) {
      const int vt = tid + q * G::TT;
      finish_input<IN_T>(v[q], in_scale);
      dft8<INV>(v[q]);
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[vt * 9 + r] = v[q][r];   // padi(8 vt + r)
    }
    __syncthreads();
    if (PREFETCH && it + 1 < iters) {
      const int64_t tn = tr + G::TPW;
#pragma unroll
      for (int q = 0; q < VT; ++q)
        load_input<N, INV, IN_T>(in, tn, tn < n_tr, tid + q * G::TT, sym_len, cp, n_sc, vn[q], in_scale);
    }
    // middle radix-8 passes, Ns = 8, 64, ...
    int Ns = 8;
#pragma unroll
    for (int p = 0; p < NMID; ++p) {
#pragma unroll
      for (int q = 0; q < VT; ++q) {
        const int vt = tid + q * G::TT;
        const float2* src = buf + padi(vt);     // padi(vt + r N/8) = padi(vt) + r (N/8 + N/64)
#pragma unroll
        for (int r = 0; r < 8; ++r) v[q][r] = src[r * (N / 8 + N / 64)];
#pragma unroll
        for (int r = 1; r < 8; ++r) v[q][r] = twid<INV>(v[q][r], twm[p][r - 1]);
        dft8<INV>(v[q]);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < VT; ++q) {
        const int vt = tid + q * G::TT;
        const int k = vt & (Ns - 1);
        const int o = (vt - k) * 8 + k;  // (vt / Ns) * Ns * 8 + k
        float2* dst = buf + padi(o);             // padi(o + r Ns) = padi(o) + r (Ns + Ns/8)
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[r * (Ns + Ns / 8)] = v[q][r];
      }
      __syncthreads();
      Ns *= 8;
    }
    // last pass: radix R, Ns = N / R; each virtual thread does 8 / R butterflies j
#pragma unroll
    for (int q = 0; q < VT; ++q)
#pragma unroll
      for (int b = 0; b < 8 / R; ++b) {
        const int j = tid + q * G::TT + b * T;
        float2 w[R];
        const float2* src = buf + padi(j);      // NS is a multiple of 8
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = src[r * (NS + NS / 8)];
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = twid<INV>(w[r], twl[q][b][r - 1]);
        dftR<R, INV>(w);
        if (active) {
          if constexpr (MAG) {
            // magnitudes of the used bins (a float row of n_sc per transform)
            float* dst = reinterpret_cast<float*>(out) + tr * n_sc;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int i = (j + r * NS + half) & (N - 1);
              if (i < n_sc) dst[i] = sqrtf(w[r].x * w[r].x + w[r].y * w[r].y);
            }
          } else if (!INV) {
            float2* dst = out + tr * n_sc;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int i = (j + r * NS + half) & (N - 1);
              if (i < n_sc) dst[i] = w[r];
            }
          } else if constexpr (OUT16) {
            short2* dst = reinterpret_cast<short2*>(out) + tr * sym_len + cp;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int n = j + r * NS;
              const short2 q = to_sc16(w[r], out_scale);
              dst[n] = q;
              if (n >= N - cp) dst[n - N] = q;       // the cyclic prefix repeats the last cp samples
            }
          } else {
            float2* dst = out + tr * sym_len + cp;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int n = j + r * NS;
              dst[n] = w[r];
              // transmitter: the cyclic prefix repeats the last cp samples
              if (cp_tail && n >= N - cp) dst[n - N] = w[r];
            }
          }
        }
      }
    if (INV && !OUT16 && active && !cp_tail) {      // adjoint: the prefix carries no gradient
      float2* dst = out + tr * sym_len;
      for (int n = tid; n < cp; n += G::TT) dst[n] = make_float2(0.f, 0.f);
    }
    __syncthreads();   // the next transform's pass 0 overwrites this LDS slab
    if (PREFETCH) {
#pragma unroll
      for (int q = 0; q < VT; ++q)
#pragma unroll
        for (int r = 0; r < 8; ++r) v[q][r] = vn[PREFETCH ? q : 0][r];
    }
  }
}

}  // namespace fftk
}  // namespace rxphy
