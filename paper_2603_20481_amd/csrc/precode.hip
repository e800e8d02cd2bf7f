// Downlink precoder for any user count K < 16 (16 users take the pilot-group
// kernels the fused detector uses): X = H A^-1 S per subcarrier with
// A = H^H H (+ N0 I for the regularised form), H the LS estimate held over a
// pilot group of K subcarriers (the trailing n_sc mod K join the last group).
//
// One wave per (frame, pilot group): the group's H goes to LDS, lanes form
// the Gram entries, lane 0 factors A = L L^H (Cholesky, FP32), and every lane
// then takes (data symbol, subcarrier) right-hand sides in turn: forward and
// back substitution with L from LDS, then X = H w written for every antenna
// (consecutive lanes take consecutive subcarriers, so the writes coalesce).
// A pivot <= 0 or not finite erases the group and flags BREAKDOWN; a
// non-finite estimate erases it and flags NONFINITE.
#include "common.h"
#include "demod_core.h"

namespace rxphy {
namespace {

constexpr int PK = 16;
constexpr int PM = 64;

__device__ __forceinline__ float2 cm(float2 a, float2 b) {          // a b
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmc(float2 a, float2 b) {         // conj(a) b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// One transmit point: a complex64 symbol (Q = 0), or Q bit bytes mapped as
// rxphy_modulate maps them (axis codes b0 b2 b4 / b1 b3 b5).
template <int Q>
__device__ __forceinline__ float2 point_at(const void* src, int64_t e) {
  if constexpr (Q == 0) {
    return static_cast<const float2*>(src)[e];
  } else {
    const uint8_t* b = static_cast<const uint8_t*>(src) + e * Q;
    int ci = 0, cq = 0;
#pragma unroll
    for (int t = 0; t < Q / 2; ++t) {
      ci = 2 * ci + (b[2 * t] != 0);
      cq = 2 * cq + (b[2 * t + 1] != 0);
    }
    return make_float2(demk::axis_level<Q>(ci), demk::axis_level<Q>(cq));
  }
}

template <int Q>
__global__ void __launch_bounds__(64)
precode_general_kernel(const float2* __restrict__ yf, const float2* __restrict__ pil, const void* __restrict__ sym,
                       float2* __restrict__ xf, uint8_t* __restrict__ flags, int M, int K, int S, int n_sc,
                       float n0, int mmse) {
  __shared__ float2 H[PM * PK];               // [m][u]
  __shared__ float2 L[PK * PK];               // Gram, then its Cholesky factor (lower)
  __shared__ float dinv[PK];
  __shared__ int state;                       // 0 ok, 1 breakdown, 2 non-finite estimate
  __shared__ float2 vb[64 * (PK + 1)];        // per-lane right-hand sides
  const int tid = threadIdx.x;
  const int64_t f = blockIdx.y;
  const int g = blockIdx.x, G = n_sc / K;
  const int i0 = g * K, i1 = g == G - 1 ? n_sc : i0 + K;
  const int D = S - 1;
  const float2* y0 = yf + f * M * S * n_sc;
  const float2* p = pil + f * n_sc;
  int bad = 0;
  for (int e = tid; e < M * K; e += 64) {
    const int m = e / K, u = e - m * K;
    const float2 h = ls_estimate(y0[(int64_t)m * S * n_sc + i0 + u], p[i0 + u]);
    H[m * PK + u] = h;
    bad |= !(isfinite(h.x) && isfinite(h.y));
  }
  bad = __syncthreads_or(bad);
  for (int e = tid; e < K * K; e += 64) {
    const int a = e / K, b = e - a * K;
    float2 acc = make_float2(0.f, 0.f);
    for (int m = 0; m < M; ++m) {
      const float2 t = cmc(H[m * PK + a], H[m * PK + b]);
      acc.x += t.x;
      acc.y += t.y;
    }
    if (a == b && mmse) acc.x += n0;
    L[a * PK + b] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    int st = bad ? 2 : 0;
    for (int j = 0; j < K && st == 0; ++j) {
      float d = L[j * PK + j].x;
      for (int k = 0; k < j; ++k) {
        const float2 l = L[j * PK + k];
        d -= l.x * l.x + l.y * l.y;
      }
      if (!(d > 0.f) || !isfinite(d)) {
        st = 1;
        break;
      }
      const float r = sqrtf(d);
      L[j * PK + j] = make_float2(r, 0.f);
      dinv[j] = 1.f / r;
      for (int i = j + 1; i < K; ++i) {
        float2 s = L[i * PK + j];
        for (int k = 0; k < j; ++k) {
          const float2 t = cm(L[i * PK + k], make_float2(L[j * PK + k].x, -L[j * PK + k].y));
          s.x -= t.x;
          s.y -= t.y;
        }
        L[i * PK + j] = make_float2(s.x * dinv[j], s.y * dinv[j]);
      }
    }
    state = st;
  }
  __syncthreads();
  const int st = state;
  const int w = i1 - i0;                      // <= 2K - 1 < 64
  if (flags && tid < w) flags[f * n_sc + i0 + tid] = st == 2 ? RXPHY_FLAG_NONFINITE : (st ? RXPHY_FLAG_BREAKDOWN : 0);
  float2* xo = xf + f * M * D * n_sc;
  const int64_t so = f * K * D * n_sc;          // first point of the frame
  for (int r = tid; r < D * w; r += 64) {
    const int d = r / w, i = i0 + (r - d * w);
    if (st) {
      for (int m = 0; m < M; ++m) xo[((int64_t)m * D + d) * n_sc + i] = make_float2(0.f, 0.f);
      continue;
    }
    float2* v = vb + tid * (PK + 1);               // this lane's right-hand side (odd stride: no bank clash)
    for (int u = 0; u < K; ++u) v[u] = point_at<Q>(sym, so + ((int64_t)u * D + d) * n_sc + i);
    for (int a = 0; a < K; ++a) {                  // L y = s
      float2 t = v[a];
      for (int b = 0; b < a; ++b) {
        const float2 q = cm(L[a * PK + b], v[b]);
        t.x -= q.x;
        t.y -= q.y;
      }
      v[a] = make_float2(t.x * dinv[a], t.y * dinv[a]);
    }
    for (int a = K - 1; a >= 0; --a) {             // L^H w = y
      float2 t = v[a];
      for (int b = a + 1; b < K; ++b) {
        const float2 q = cmc(L[b * PK + a], v[b]);
        t.x -= q.x;
        t.y -= q.y;
      }
      v[a] = make_float2(t.x * dinv[a], t.y * dinv[a]);
    }
    for (int m = 0; m < M; ++m) {
      float2 acc = make_float2(0.f, 0.f);
      for (int u = 0; u < K; ++u) {
        const float2 q = cm(H[m * PK + u], v[u]);
        acc.x += q.x;
        acc.y += q.y;
      }
      xo[((int64_t)m * D + d) * n_sc + i] = acc;
    }
  }
}

}  // namespace

rxphy_status launch_precode_general(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                    const void* src, int src_bits, float2* xf, uint8_t* flags, hipStream_t s) {
  if (nf == 0) return RXPHY_OK;
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  const dim3 grid(fr.n_sc / fr.K, nf);
  const int mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
#define RXPHY_PRECODE_GENERAL(QQ)                                                                               \
  hipLaunchKernelGGL(precode_general_kernel<QQ>, grid, dim3(64), 0, s, yf, pil, src, xf, flags, fr.M, fr.K, \
                     fr.n_sym, fr.n_sc, fr.n0, mmse)
  switch (src_bits) {
    case 0: RXPHY_PRECODE_GENERAL(0); break;
    case 2: RXPHY_PRECODE_GENERAL(2); break;
    case 4: RXPHY_PRECODE_GENERAL(4); break;
    case 6: RXPHY_PRECODE_GENERAL(6); break;
    default: return fail(RXPHY_EINVAL, "qam_bits = %d", src_bits);
  }
#undef RXPHY_PRECODE_GENERAL
  return launch_status("precode kernel (general K)");
}

}  // namespace rxphy
