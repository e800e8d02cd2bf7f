// Spectrum-sensing pipeline (Section III-A1: TF plot of segment FFT
// magnitudes; Section IV-B: PSD, Savitzky-Golay, noise floor, PSD pruning,
// column Otsu, morphological operations, 4-connected components and boxes;
// Section III-A: detection metrics on the host).
//
// Kernels, all batched over plots (grid y / z = plot):
//   fft_kernel<F, false, MAG>  magnitudes of the centred bins (fft.hip)
//   colstat_kernel   column sum (PSD), min and max; 64 columns per workgroup,
//                    16 waves over the rows
//   floor_kernel     Savitzky-Golay smoothing, lowest local minimum, theta
//   otsu_kernel      per retained column: LDS histogram, exact integer Otsu,
//                    mask written in a second pass over the column strip
//   morph_kernel     64x64 tile + halo as 128-bit row masks, the six
//                    erosions / dilations as shifts and ANDs / ORs,
//                    then the tile's components labelled in LDS from row
//                    runs (bit operations on the row masks); mask and
//                    labels (each pixel's local root) written
//   merge_kernel     lock-free unions across tile borders (smaller index wins)
//   flatten_kernel   every label to its root; roots counted per 1024 pixels
//   scan_kernel      per-plot exclusive scan of the counts; box records reset
//   assign_kernel    each root gets its ordinal (raster order of roots)
//   boxes_kernel     per tile: each local component's box (from the tile
//                    list the morphology kernel wrote) folded into its
//                    component's box; overflowed tiles read pixel by pixel
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace rxphy {
namespace {

constexpr int SG_MAX = 63;

// Per 64x64 tile: its local components (after the morphology), each with its
// root (the component's first pixel, a plot-local index) and its bounding box
// inside the tile, in plot coordinates.  n = -1: more than TL_CAP components,
// the box kernel then reads the tile's pixels instead.
constexpr int TL_CAP = 64;
struct TileEntry {
  int32_t root;
  int16_t t0, f0, t1, f1;
};
struct TileList {
  int32_t n, pad[3];
  TileEntry e[TL_CAP];
};

struct SgCoef {
  float c[SG_MAX];
  int h;
};

__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

// ------------------------------------------------------------ column stats
// Column kernels: 64 columns per workgroup (lane = column, 256-byte row
// loads), CW waves over the rows.
constexpr int CW = 16;
constexpr int OU = 8;                         // rows per wave whose loads the Otsu passes issue together

__global__ void __launch_bounds__(64 * CW)
colstat_kernel(const float* __restrict__ tf, float* __restrict__ psd, float* __restrict__ lo,
               float* __restrict__ hi, int T, int F) {
  __shared__ float ss[CW][64], smn[CW][64], smx[CW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int64_t p = blockIdx.y;
  const float* col = tf + p * T * F + c;
  float s = 0.f, mn = INFINITY, mx = -INFINITY;
  for (int t0 = w; t0 < T; t0 += CW * OU) {      // OU loads in flight; summed in row order as they arrive
    float v[OU];
#pragma unroll
    for (int u = 0; u < OU; ++u) v[u] = col[(int64_t)min(t0 + u * CW, T - 1) * F];
#pragma unroll
    for (int u = 0; u < OU; ++u) {
      if (t0 + u * CW < T) {
        s += v[u];
        mn = fminf(mn, v[u]);
        mx = fmaxf(mx, v[u]);
      }
    }
  }
  ss[w][lane] = s;
  smn[w][lane] = mn;
  smx[w][lane] = mx;
  __syncthreads();
  if (w == 0) {
    float a = ss[0][lane], l = smn[0][lane], h = smx[0][lane];
    for (int i = 1; i < CW; ++i) {               // fixed order: the same sum on every run
      a += ss[i][lane];
      l = fminf(l, smn[i][lane]);
      h = fmaxf(h, smx[i][lane]);
    }
    psd[p * F + c] = a;
    lo[p * F + c] = l;
    hi[p * F + c] = h;
  }
}

// ------------------------------------------------------ noise floor, theta
__global__ void __launch_bounds__(1024)
floor_kernel(const float* __restrict__ psd, float* __restrict__ psd_s, float* __restrict__ flo, SgCoef sg,
             float factor, int F) {
  __shared__ float sp[4096], sm[4096];
  __shared__ float red[2][16];
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x;
  for (int j = tid; j < F; j += 1024) sp[j] = psd[p * F + j];
  __syncthreads();
  const int h = sg.h;
  for (int j = tid; j < F; j += 1024) {
    float acc = 0.f;
    for (int k = -h; k <= h; ++k) {
      int q = j + k;
      q = q < 0 ? -q : (q >= F ? 2 * (F - 1) - q : q);      // mirror about the end samples
      acc += sg.c[k + h] * sp[q];
    }
    sm[j] = acc;
    psd_s[p * F + j] = acc;
  }
  __syncthreads();
  float best = INFINITY, all = INFINITY;                   // lowest local minimum, lowest value
  for (int j = tid; j < F; j += 1024) {
    const float v = sm[j];
    all = fminf(all, v);
    if (j > 0 && j < F - 1 && v <= sm[j - 1] && v <= sm[j + 1]) best = fminf(best, v);
  }
  best = wave_min(best);
  all = wave_min(all);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = best;
    red[1][tid >> 6] = all;
  }
  __syncthreads();
  if (tid == 0) {
    float b = INFINITY, a = INFINITY;
    for (int i = 0; i < 16; ++i) {
      b = fminf(b, red[0][i]);
      a = fminf(a, red[1][i]);
    }
    const float n0 = b < INFINITY ? b : a;       // no interior local minimum: the lowest value
    flo[2 * p] = n0;
    flo[2 * p + 1] = factor * n0;
  }
}

// ------------------------------------------------------------------ Otsu
__device__ __forceinline__ int value_bin(float v, float lo, float scale, int bins) {
  const int b = (int)((v - lo) * scale);         // truncation = floor for v >= lo
  return b < 0 ? 0 : (b < bins - 1 ? b : bins - 1);
}

// Otsu's threshold: the bin k (class 0 = bins <= k) maximising
// (N m0 - M w0)^2 / (w0 w1) (between-class variance times N^2), ties to the
// smallest k, -1 if no k leaves both classes non-empty.  Exact: |N m0 - M w0|
// <= N * N * (bins - 1), whose square fits 64 bits for N <= 4096 and
// bins <= 256; the cross products are compared in 128 bits.
struct OtsuBest {
  uint64_t num, den;
  int k;
};

__device__ __forceinline__ bool better(uint64_t num, uint64_t den, const OtsuBest& b) {
  return b.k < 0 || (unsigned __int128)num * b.den > (unsigned __int128)b.num * den;
}

// Histogram counts are 16-bit halves of LDS words: bin b of a column is half
// (b & 1) of word (b >> 1).  A column has at most 4096 values, so a half never
// carries into the other.
__device__ __forceinline__ uint32_t hcount(const uint32_t* h, int b) {
  return (h[b >> 1] >> ((b & 1) * 16)) & 0xffffu;
}

__global__ void __launch_bounds__(64 * CW)
otsu_kernel(const float* __restrict__ tf, const float* __restrict__ psd, const float* __restrict__ lo_,
            const float* __restrict__ hi_, const float* __restrict__ flo, int32_t* __restrict__ kbin,
            uint8_t* __restrict__ mask, int T, int F, int bins) {
  __shared__ uint32_t hist[64 * 129];
  __shared__ int64_t qw[CW][64], qm[CW][64];
  __shared__ OtsuBest qb[CW][64];
  __shared__ int kk[64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int64_t p = blockIdx.y;
  const int stride = (bins + 1) / 2 + 1;        // words per column, odd: the 64 columns hit different banks
  for (int i = tid; i < 64 * stride; i += 64 * CW) hist[i] = 0u;
  const bool keep = psd[p * F + c] >= flo[2 * p + 1];
  const float lo = lo_[p * F + c], hi = hi_[p * F + c];
  const bool spread = hi > lo;
  const float scale = spread ? __fdiv_rn((float)bins, hi - lo) : 0.f;
  const float* col = tf + p * T * F + c;
  const uint32_t* hc = hist + lane * stride;
  __syncthreads();
  if (keep) {
    for (int t0 = w; t0 < T; t0 += CW * OU) {    // OU loads in flight per wave before their bins
      float v[OU];
#pragma unroll
      for (int u = 0; u < OU; ++u) {
        const int t = t0 + u * CW;
        v[u] = t < T ? col[(int64_t)t * F] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < OU; ++u) {
        if (t0 + u * CW < T) {
          const int b = value_bin(v[u], lo, scale, bins);
          atomicAdd(hist + lane * stride + (b >> 1), 1u << ((b & 1) * 16));
        }
      }
    }
  }
  __syncthreads();
  // wave w scans candidate thresholds k in [w q, (w + 1) q), q = ceil((bins - 1) / CW)
  const int q = (bins - 1 + CW - 1) / CW;
  const int k0 = w * q, k1 = min(bins - 1, k0 + q);
  {
    int64_t sw = 0, sm = 0;
    for (int b = k0; b < k1; ++b) {
      const uint32_t v = hcount(hc, b);
      sw += v;
      sm += (int64_t)b * v;
    }
    qw[w][lane] = sw;
    qm[w][lane] = sm;
  }
  __syncthreads();
  {
    int64_t w0 = 0, m0 = 0, M = 0;
    for (int i = 0; i < CW; ++i) {
      if (i < w) {
        w0 += qw[i][lane];
        m0 += qm[i][lane];
      }
      M += qm[i][lane];
    }
    M += (int64_t)(bins - 1) * hcount(hc, bins - 1);    // the last bin is never in class 0
    const int64_t N = T;
    OtsuBest best{0, 1, -1};
    if (keep) {
      for (int k = k0; k < k1; ++k) {
        const uint32_t v = hcount(hc, k);
        w0 += v;
        m0 += (int64_t)k * v;
        const int64_t w1 = N - w0;
        if (w0 == 0 || w1 == 0) continue;
        const int64_t d = N * m0 - M * w0;
        const uint64_t a = (uint64_t)(d < 0 ? -d : d);
        const uint64_t num = a * a, den = (uint64_t)(w0 * w1);
        if (better(num, den, best)) best = OtsuBest{num, den, k};
      }
    }
    qb[w][lane] = best;
  }
  __syncthreads();
  if (w == 0) {
    OtsuBest best = qb[0][lane];
    for (int i = 1; i < CW; ++i) {                 // strictly better only: ties keep the smaller k
      const OtsuBest& o = qb[i][lane];
      if (o.k >= 0 && better(o.num, o.den, best)) best = o;
    }
    kk[lane] = best.k;
    kbin[p * F + c] = best.k;
  }
  __syncthreads();
  const int k = kk[lane];
  uint8_t* mc = mask + p * T * F + c;
  for (int t0 = w; t0 < T; t0 += CW * OU) {
    float v[OU];
#pragma unroll
    for (int u = 0; u < OU; ++u) {
      const int t = t0 + u * CW;
      v[u] = t < T && k >= 0 ? col[(int64_t)t * F] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < OU; ++u) {
      const int t = t0 + u * CW;
      if (t < T) mc[(int64_t)t * F] = (k >= 0 && value_bin(v[u], lo, scale, bins) > k) ? 1 : 0;
    }
  }
}

// ------------------------------------------------------------ morphology
// A 64x64 core with a halo of 4 rows (four 3x3 operations) and 6 columns
// (six operations 3 wide): MR x MC region rows held as 128-bit masks (bit c =
// region column c), with a second mask of the pixels inside the plot.
// Dilation ORs the shifted rows of the foreground (outside = 0); erosion ANDs
// them with the outside set to 1; both clear the outside again.  Rows and
// columns beyond the region use neutral values; the error this makes moves
// one pixel per operation and never reaches the core.
constexpr int MR = 64 + 8, MC = 64 + 12;
constexpr uint64_t HI_VALID = (1ull << (MC - 64)) - 1;   // region columns 64 .. MC-1

struct Row {
  uint64_t lo, hi;
};

__device__ __forceinline__ Row shl1(Row x, uint64_t fill) {   // column c -> c + 1
  return Row{(x.lo << 1) | fill, ((x.hi << 1) | (x.lo >> 63)) & HI_VALID};
}
__device__ __forceinline__ Row shr1(Row x, uint64_t fill) {   // column c -> c - 1
  return Row{(x.lo >> 1) | (x.hi << 63), (x.hi >> 1) | (fill << (MC - 65))};
}

template <bool DIL, bool VERT>
__device__ __forceinline__ void row_op(Row (*cur)[MR], Row (*nxt)[MR], Row* hb, const Row* inm) {
  const int r = threadIdx.x;
  Row h{0, 0};
  if (r < MR) {
    const Row x = (*cur)[r], in = inm[r];
    if (DIL) {
      const Row a = shl1(x, 0), b = shr1(x, 0);
      h = Row{x.lo | a.lo | b.lo, x.hi | a.hi | b.hi};
    } else {
      const Row y{x.lo | ~in.lo, (x.hi | ~in.hi) & HI_VALID};
      const Row a = shl1(y, 1), b = shr1(y, 1);
      h = Row{y.lo & a.lo & b.lo, y.hi & a.hi & b.hi};
    }
    if (VERT) hb[r] = h;
  }
  if (VERT) __syncthreads();
  if (r < MR) {
    Row v = h;
    if (VERT) {
      const Row n0 = DIL ? Row{0, 0} : Row{~0ull, HI_VALID};
      const Row u = r > 0 ? hb[r - 1] : n0, d = r < MR - 1 ? hb[r + 1] : n0;
      v = DIL ? Row{u.lo | h.lo | d.lo, u.hi | h.hi | d.hi} : Row{u.lo & h.lo & d.lo, u.hi & h.hi & d.hi};
    }
    const Row in = inm[r];
    (*nxt)[r] = Row{v.lo & in.lo, v.hi & in.hi};
  }
  __syncthreads();
}

// Union-find inside one 64x64 tile in LDS (same rule as the global one: the
// larger root is linked under the smaller, so a local root is the smallest
// pixel of its local component, which is also its smallest global index).
// Path splitting: every node passed is pointed at its grandparent.  Parents
// only ever move to smaller indices of the same set, so the plain stores never
// undo a link that a concurrent atomic min made.
__device__ __forceinline__ int lfind(volatile int* lab, int x) {
  for (;;) {
    const int y = lab[x];
    if (y == x) return x;
    const int z = lab[y];
    if (z == y) return y;
    lab[x] = z;
    x = y;
  }
}

__device__ __forceinline__ uint64_t lowmask(int n) { return n >= 64 ? ~0ull : (1ull << n) - 1; }

__device__ void lunite(volatile int* lab, int a, int b) {
  for (;;) {
    a = lfind(lab, a);
    b = lfind(lab, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin((int*)lab + b, a);
    if (old == b) return;
    b = old;
  }
}

// After the morphology the tile's components are labelled in LDS (union-find
// over row runs); a pixel's global label is its local root's global index
// (-1: background), written for the tile's border pixels and roots (for every
// pixel if the tile's list overflows); only unions across tile borders are
// left for the global pass.
__global__ void __launch_bounds__(256)
morph_kernel(const uint8_t* __restrict__ mask, uint8_t* __restrict__ out, int32_t* __restrict__ lab,
             TileList* __restrict__ tl, int T, int F) {
  // the four morphology row buffers; once the core rows are in crow, their
  // 4608 bytes hold idof: the list position of a local root (255: past the
  // list), one byte per core pixel (fewer LDS bytes per workgroup: seven
  // workgroups per CU instead of six)
  __shared__ Row mb[4][MR];
  static_assert(sizeof(mb) >= 64 * 64, "idof must fit in the row buffers");
  Row* const bufA = mb[0];
  Row* const inm = mb[3];
  Row* const hb = mb[2];
  uint8_t* const idof = reinterpret_cast<uint8_t*>(&mb[0][0]);
  __shared__ uint64_t crow[64];
  __shared__ int loc[64 * 64];
  __shared__ int bb[TL_CAP][4];                 // local box: min row, min column, max row, max column
  __shared__ int16_t rootof[TL_CAP];
  __shared__ int nroots;
  const int f0 = blockIdx.x * 64, t0 = blockIdx.y * 64;
  const int64_t p = blockIdx.z;
  const uint8_t* m = mask + p * T * F;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // region row w + 4 j per wave step j, two ballots each; every load of the
  // wave is issued before the first ballot
  constexpr int RW = MR / 4;
  uint8_t va[RW], vb[RW];
  const int fa = f0 - 6 + lane, fb = f0 - 6 + 64 + lane;
  const bool ca = fa >= 0 && fa < F, cb = lane < MC - 64 && fb >= 0 && fb < F;
  const int fa_c = min(max(fa, 0), F - 1), fb_c = min(max(fb, 0), F - 1);   // in-plot addresses: no branches
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const int t = min(max(t0 - 4 + w + 4 * j, 0), T - 1);
    va[j] = m[(int64_t)t * F + fa_c];
    vb[j] = m[(int64_t)t * F + fb_c];
  }
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const int r = w + 4 * j, t = t0 - 4 + r;
    const bool trow = t >= 0 && t < T;
    const uint64_t ba = __ballot(trow && ca && va[j] != 0), bb = __ballot(trow && cb && vb[j] != 0);
    const uint64_t ia = __ballot(trow && ca), ib = __ballot(trow && cb);
    if (lane == 0) {
      bufA[r] = Row{ba, bb};
      inm[r] = Row{ia, ib};
    }
  }
  __syncthreads();
  Row(*A)[MR] = &mb[0];
  Row(*B)[MR] = &mb[1];
  row_op<true, true>(A, B, hb, inm);               // closing 3x3
  row_op<false, true>(B, A, hb, inm);
  row_op<false, true>(A, B, hb, inm);              // opening 3x3
  row_op<true, true>(B, A, hb, inm);
  row_op<false, false>(A, B, hb, inm);             // opening 1x3 along frequency (leaves a 3x3 opening unchanged)
  row_op<true, false>(B, A, hb, inm);
  // The tile's components from its row runs: a run's first pixel stands for
  // it; thread (row r, quarter q) unites each run of core row r that starts
  // in columns 16 q .. 16 q + 15 with every run of row r - 1 it overlaps,
  // found with bit operations on the row masks (the four waves take the four
  // quarters, so every run is handled by exactly one thread).
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    const Row x = (*A)[r + 4];
    crow[r] = t0 + r < T ? ((x.lo >> 6) | (x.hi << 58)) : 0ull;   // core columns 0..63
  }
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) loc[idx] = -1;
  __syncthreads();
  volatile int* vl = loc;
  const int rr = threadIdx.x & 63;                 // this thread's core row
  const uint64_t quarter = 0xffffull << (16 * (threadIdx.x >> 6));
  {
    uint64_t st = crow[rr] & ~(crow[rr] << 1) & quarter;     // run starts
    while (st) {
      const int c = __builtin_ctzll(st);
      st &= st - 1;
      vl[rr * 64 + c] = rr * 64 + c;
    }
  }
  __syncthreads();
  if (rr > 0) {
    const int r = rr;
    const uint64_t row = crow[r], prow = crow[r - 1];
    const uint64_t pst = prow & ~(prow << 1);
    uint64_t st = row & ~(row << 1) & quarter;
    while (st) {
      const int c0 = __builtin_ctzll(st);
      st &= st - 1;
      const uint64_t inv = ~(row >> c0);
      const int len = inv ? __builtin_ctzll(inv) : 64 - c0;
      const uint64_t span = lowmask(len) << c0;
      const uint64_t ov = prow & span;
      if (!ov) continue;
      const int b = __builtin_ctzll(ov);
      const int ps = 63 - __builtin_clzll(pst & lowmask(b + 1));   // start of the run holding bit b
      lunite(vl, r * 64 + c0, (r - 1) * 64 + ps);
      uint64_t more = pst & span & ~lowmask(b + 1);                // further runs that start in the span
      while (more) {
        const int q = __builtin_ctzll(more);
        more &= more - 1;
        lunite(vl, r * 64 + c0, (r - 1) * 64 + q);
      }
    }
  }
  __syncthreads();
  // the tile's component list: roots numbered in any order, boxes reduced per
  // row run with LDS atomics
  if (threadIdx.x == 0) nroots = 0;
  for (int i = threadIdx.x; i < TL_CAP; i += 256) {
    bb[i][0] = INT_MAX;
    bb[i][1] = INT_MAX;
    bb[i][2] = -1;
    bb[i][3] = -1;
  }
  __syncthreads();
  {
    const int r = rr;
    uint64_t st = crow[r] & ~(crow[r] << 1) & quarter;
    while (st) {
      const int c = __builtin_ctzll(st);
      st &= st - 1;
      const int x = r * 64 + c;
      if (lfind(vl, x) == x) {
        const int id = atomicAdd(&nroots, 1);
        idof[x] = id < TL_CAP ? (uint8_t)id : 255;
        if (id < TL_CAP) rootof[id] = (int16_t)x;
      }
    }
  }
  __syncthreads();
  {
    const int r = rr;
    const uint64_t row = crow[r];
    uint64_t st = row & ~(row << 1) & quarter;
    while (st) {
      const int c0 = __builtin_ctzll(st);
      st &= st - 1;
      const uint64_t inv = ~(row >> c0);
      const int c1 = c0 + (inv ? __builtin_ctzll(inv) : 64 - c0) - 1;
      const int id = idof[lfind(vl, r * 64 + c0)];
      if (id != 255) {
        atomicMin(&bb[id][0], r);
        atomicMin(&bb[id][1], c0);
        atomicMax(&bb[id][2], r);
        atomicMax(&bb[id][3], c1);
      }
    }
  }
  __syncthreads();
  // Labels: the tile's border pixels (the merge reads them) and, below, its
  // listed roots; every pixel when the list overflows (the later passes then
  // read the tile pixel by pixel).  Interior labels of a listed tile are never
  // read.
  const int n = nroots;
  const bool all_px = n > TL_CAP;
  uint8_t* o = out + p * T * F;
  int32_t* L = lab + p * T * F;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int r = idx >> 6, c = idx & 63;
    const int t = t0 + r, f = f0 + c;
    if (t < T) {
      const uint64_t row = crow[r];
      const bool fg = ((row >> c) & 1ull) != 0;
      o[(int64_t)t * F + f] = fg ? 1 : 0;
      if (all_px || r == 0 || r == 63 || c == 0 || c == 63) {
        int g = -1;
        if (fg) {
          const uint64_t st = row & ~(row << 1) & lowmask(c + 1);
          const int root = lfind(vl, r * 64 + 63 - __builtin_clzll(st));
          g = (t0 + (root >> 6)) * F + f0 + (root & 63);
        }
        L[(int64_t)t * F + f] = g;
      }
    }
  }
  TileList& out_l = tl[(p * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x];
  if (threadIdx.x == 0) out_l.n = n <= TL_CAP ? n : -1;
  if (n <= TL_CAP) {
    for (int e = threadIdx.x; e < n; e += 256) {
      const int x = rootof[e];
      TileEntry te;
      te.root = (t0 + (x >> 6)) * F + f0 + (x & 63);
      te.t0 = (int16_t)(t0 + bb[e][0]);
      te.f0 = (int16_t)(f0 + bb[e][1]);
      te.t1 = (int16_t)(t0 + bb[e][2]);
      te.f1 = (int16_t)(f0 + bb[e][3]);
      out_l.e[e] = te;
      L[te.root] = te.root;
    }
  }
}

// ------------------------------------------------------------------ CCL
__device__ __forceinline__ int find_root(const int* L, int x) {
  int y = ld_agent(L + x);
  while (y != x) {
    x = y;
    y = ld_agent(L + x);
  }
  return x;
}

// Links the sets of a and b: the larger root is pointed at the smaller one
// with an atomic min; if that root gained another parent meanwhile, the
// union continues from that parent.
__device__ void unite(int* L, int a, int b) {
  for (;;) {
    a = find_root(L, a);
    b = find_root(L, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(L + b, a);
    if (old == b) return;
    b = old;
  }
}

// Unions across tile borders: thread i < 64 takes the tile's top row pixel i
// and the pixel above it, thread 64 + i the left column pixel i and the pixel
// to its left.  Only the first pixel of each run of such pairs along the
// border unites: its neighbour along the border pairs pixels of the same two
// local components (one row or column run on each side).
__global__ void __launch_bounds__(128)
merge_kernel(const uint8_t* __restrict__ mask, int32_t* __restrict__ lab, int T, int F) {
  const int f0 = blockIdx.x * 64, t0 = blockIdx.y * 64;
  const int64_t p = blockIdx.z;
  const int n = T * F;
  const uint8_t* m = mask + p * n;
  int* L = lab + p * n;
  const int i = threadIdx.x & 63;
  int q = 0, nb = 0;
  bool pair = false;
  if (threadIdx.x < 64) {
    q = t0 * F + f0 + i;
    nb = q - F;
    pair = t0 > 0 && m[q] && m[nb];
  } else {
    const int t = t0 + i;
    q = t * F + f0;
    nb = q - 1;
    pair = f0 > 0 && t < T && m[q] && m[nb];
  }
  const uint64_t pb = __ballot(pair);
  if (pair && (i == 0 || !((pb >> (i - 1)) & 1ull))) unite(L, q, nb);
}

// Global roots are counted per (row, tile column): in that order the counts
// follow the raster order of the roots, so their prefix sum gives each root
// its raster ordinal.  One wave per 64x64 tile.  A tile with a component list
// resolves only its listed local roots (every other pixel of the tile still
// points at its local root, which the box kernel follows); a tile whose list
// overflowed resolves every labelled pixel.  A root is the component's first
// pixel, so it sits in the tile that holds it and is counted there once.
__global__ void __launch_bounds__(64)
flatten_kernel(int32_t* __restrict__ lab, const TileList* __restrict__ tl, int32_t* __restrict__ cnt, int T, int F) {
  __shared__ int rc[64];
  const int64_t p = blockIdx.z;
  const int t0 = blockIdx.y * 64, f0 = blockIdx.x * 64;
  const int TX = gridDim.x;
  int* L = lab + p * T * F;
  int32_t* C = cnt + p * T * TX;
  const int lane = threadIdx.x;
  const int n = tl[(p * gridDim.y + blockIdx.y) * TX + blockIdx.x].n;
  if (n >= 0) {
    const TileEntry* te = tl[(p * gridDim.y + blockIdx.y) * TX + blockIdx.x].e;
    rc[lane] = 0;
    __syncthreads();
    if (lane < n) {
      const int x = te[lane].root;
      const int r = find_root(L, x);
      if (r != x)
        L[x] = r;
      else
        atomicAdd(&rc[x / F - t0], 1);
    }
    __syncthreads();
    if (t0 + lane < T) C[(t0 + lane) * TX + blockIdx.x] = rc[lane];
    return;
  }
  for (int r = 0; r < 64 && t0 + r < T; ++r) {
    const int q = (t0 + r) * F + f0 + lane;
    const int l = L[q];
    bool root = false;
    if (l >= 0) {
      const int g = find_root(L, q);
      if (g != q) L[q] = g;
      root = g == q;
    }
    const uint64_t rb = __ballot(root);
    if (lane == 0) C[(t0 + r) * TX + blockIdx.x] = __builtin_popcountll(rb);
  }
}

// Exclusive prefix sum of a plot's counts (n a multiple of 4, 16-byte
// aligned): 4096 counts per pass, four per thread, wave scans by shuffles and
// one LDS exchange of the 16 wave totals; four passes' loads are issued
// before their sums.  Also sets the plot's box count and clears its boxes.
__global__ void __launch_bounds__(1024)
scan_kernel(const int32_t* __restrict__ cnt, int32_t* __restrict__ off, int32_t* __restrict__ n_boxes,
            int32_t* __restrict__ boxes, int max_boxes, int ncnt) {
  __shared__ int wsum[2][16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t p = blockIdx.x;
  const int4* c4 = reinterpret_cast<const int4*>(cnt + p * ncnt);
  int4* o4 = reinterpret_cast<int4*>(off + p * ncnt);
  const int n4 = ncnt / 4;
  int carry = 0, buf = 0;
  for (int c0 = 0; c0 < n4; c0 += 4 * 1024) {
    int4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = c0 + k * 1024 + tid;
      v[k] = i < n4 ? c4[i] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = c0 + k * 1024 + tid;
      const int s4 = v[k].x + v[k].y + v[k].z + v[k].w;
      int inc = s4;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
      }
      if (lane == 63) wsum[buf][w] = inc;
      __syncthreads();
      int below = 0, total = 0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int ws = wsum[buf][j];
        below += j < w ? ws : 0;
        total += ws;
      }
      buf ^= 1;                                   // the next pass writes the other half: one barrier per pass
      const int ex = carry + below + inc - s4;
      if (i < n4) o4[i] = make_int4(ex, ex + v[k].x, ex + v[k].x + v[k].y, ex + v[k].x + v[k].y + v[k].z);
      carry += total;
    }
  }
  if (tid == 0) n_boxes[p] = carry;
  for (int i = tid; i < max_boxes; i += 1024) {
    int32_t* bx = boxes + (p * max_boxes + i) * 4;
    bx[0] = INT_MAX;
    bx[1] = INT_MAX;
    bx[2] = -1;
    bx[3] = -1;
  }
}

// Each global root of the tile takes -2 - its raster ordinal: the prefix of
// its (row, tile column) count plus the tile's roots left of it in its row.
__global__ void __launch_bounds__(64)
assign_kernel(int32_t* __restrict__ lab, const TileList* __restrict__ tl, const int32_t* __restrict__ off, int T,
              int F) {
  __shared__ int key[TL_CAP];                   // row * 64 + column of a global root, -1 for the others
  const int64_t p = blockIdx.z;
  const int t0 = blockIdx.y * 64, f0 = blockIdx.x * 64;
  const int TX = gridDim.x;
  int* L = lab + p * T * F;
  const int32_t* O = off + p * T * TX;
  const int lane = threadIdx.x;
  const TileList& tile = tl[(p * gridDim.y + blockIdx.y) * TX + blockIdx.x];
  const int n = tile.n;
  if (n >= 0) {
    int x = -1, k = -1;
    if (lane < n) {
      x = tile.e[lane].root;
      if (L[x] == x) k = (x / F - t0) * 64 + (x % F - f0);
    }
    key[lane] = k;
    __syncthreads();
    if (k >= 0) {
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const int kj = key[j];
        rank += kj >= 0 && (kj >> 6) == (k >> 6) && kj < k;
      }
      L[x] = -2 - (O[(t0 + (k >> 6)) * TX + blockIdx.x] + rank);
    }
    return;
  }
  for (int r = 0; r < 64 && t0 + r < T; ++r) {
    const int q = (t0 + r) * F + f0 + lane;
    const bool root = L[q] == q;
    const uint64_t rb = __ballot(root);
    if (root) {
      const int rank = __builtin_popcountll(rb & ((1ull << lane) - 1ull));
      L[q] = -2 - (O[(t0 + r) * TX + blockIdx.x] + rank);
    }
  }
}

__device__ __forceinline__ void flush_run(int32_t* boxes, int max_boxes, int ord, int t, int fa, int fb) {
  if (ord < 0 || ord >= max_boxes) return;
  int32_t* bx = boxes + (int64_t)ord * 4;
  atomicMin(bx + 0, t);
  atomicMin(bx + 1, fa);
  atomicMax(bx + 2, t);
  atomicMax(bx + 3, fb);
}

// One workgroup per 64x64 tile.  A tile with a component list folds each
// local component's box into its component's box (four atomic min / max per
// local component); a tile whose list overflowed is read pixel by pixel: each
// wave takes rows of the tile, finds the runs of one component with a shuffle
// and a ballot, and folds each run.
__global__ void __launch_bounds__(256)
boxes_kernel(const uint8_t* __restrict__ mask, const int32_t* __restrict__ lab, const TileList* __restrict__ tl,
             int32_t* __restrict__ boxes, int max_boxes, int T, int F) {
  const int64_t p = blockIdx.z;
  const int t0 = blockIdx.y * 64, f0 = blockIdx.x * 64;
  const int n_px = T * F;
  const int* L = lab + p * n_px;
  int32_t* bx = boxes + p * max_boxes * 4;
  const TileList& tlst = tl[(p * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x];
  const int n = tlst.n;
  if (n >= 0) {
    for (int e = threadIdx.x; e < n; e += 256) {
      const TileEntry te = tlst.e[e];
      const int l = L[te.root];
      const int ord = l < -1 ? -2 - l : -2 - L[l];
      if (ord < max_boxes) {
        int32_t* b = bx + (int64_t)ord * 4;
        atomicMin(b + 0, (int)te.t0);
        atomicMin(b + 1, (int)te.f0);
        atomicMax(b + 2, (int)te.t1);
        atomicMax(b + 3, (int)te.f1);
      }
    }
    return;
  }
  const uint8_t* m = mask + p * n_px;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = w; r < 64 && t0 + r < T; r += 4) {
    const int t = t0 + r;
    const int q = t * F + f0 + lane;
    int ord = -1;
    if (m[q]) {
      const int l = L[q];
      ord = l < -1 ? -2 - l : -2 - L[l];
    }
    const int prev = __shfl_up(ord, 1, 64);
    const bool start = lane == 0 || ord != prev;
    const uint64_t starts = __ballot(start);
    if (start && ord >= 0) {
      const uint64_t nxt = lane == 63 ? 0ull : starts >> (lane + 1);
      const int last = nxt ? lane + __builtin_ctzll(nxt) : 63;
      flush_run(bx, max_boxes, ord, t, f0 + lane, f0 + last);
    }
  }
}

// ------------------------------------------------------------------ host
bool config_ok(const rxphy_sense_config* c) {
  if (!c) return false;
  const int F = c->n_fft;
  return (F == 512 || F == 1024 || F == 2048 || F == 4096) && c->n_rows >= 3 && c->n_rows <= 4096 &&
         c->sg_window >= 3 && c->sg_window <= SG_MAX && (c->sg_window & 1) && c->sg_window <= F &&
         c->sg_order >= 0 && c->sg_order <= 6 && c->sg_order < c->sg_window && std::isfinite(c->psd_factor) &&
         c->psd_factor > 0.f && c->bins >= 2 && c->bins <= 256;
}

// Savitzky-Golay smoothing weights: the value at 0 of the least-squares
// polynomial of degree `order` over offsets -h..h, c = V (V^T V)^-1 e0 with
// V[k][q] = (k/h)^q (scaled for conditioning; same column space), by Gaussian
// elimination with partial pivoting in double.
SgCoef sg_coeffs(int window, int order) {
  const int h = window / 2, n = order + 1;
  double G[7][8] = {};
  for (int k = -h; k <= h; ++k) {
    double pw[7];
    pw[0] = 1.0;
    for (int q = 1; q < n; ++q) pw[q] = pw[q - 1] * ((double)k / h);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) G[a][b] += pw[a] * pw[b];
  }
  for (int a = 0; a < n; ++a) G[a][n] = a == 0 ? 1.0 : 0.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(G[r][col]) > std::fabs(G[piv][col])) piv = r;
    for (int j = 0; j <= n; ++j) std::swap(G[col][j], G[piv][j]);
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double fct = G[r][col] / G[col][col];
      for (int j = col; j <= n; ++j) G[r][j] -= fct * G[col][j];
    }
  }
  double z[7];
  for (int a = 0; a < n; ++a) z[a] = G[a][n] / G[a][a];
  SgCoef s;
  std::memset(&s, 0, sizeof(s));
  s.h = h;
  for (int k = -h; k <= h; ++k) {
    double v = 0.0, pw = 1.0;
    for (int q = 0; q < n; ++q) {
      v += pw * z[q];
      pw *= (double)k / h;
    }
    s.c[k + h] = (float)v;
  }
  return s;
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

struct SenseLayout {
  size_t tf, psd, psd_s, flo, kbin, lo, hi, mask, mask_mo, lab, cnt, off, tl, total;
};

SenseLayout layout(const rxphy_sense_config& c, int32_t P) {
  const size_t TF = (size_t)c.n_rows * c.n_fft, F = c.n_fft;
  const size_t ncnt = (size_t)c.n_rows * (c.n_fft / 64);   // root counts per (row, tile column)
  SenseLayout L{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t at = o;
    o += al(bytes);
    return at;
  };
  L.tf = put(P * TF * 4);
  L.psd = put(P * F * 4);
  L.psd_s = put(P * F * 4);
  L.flo = put(P * 2 * 4);
  L.kbin = put(P * F * 4);
  L.lo = put(P * F * 4);
  L.hi = put(P * F * 4);
  L.mask = put(P * TF);
  L.mask_mo = put(P * TF);
  L.lab = put(P * TF * 4);
  L.cnt = put(P * ncnt * 4);
  L.off = put(P * ncnt * 4);
  L.tl = put(P * (size_t)(c.n_fft / 64) * ((c.n_rows + 63) / 64) * sizeof(TileList));
  L.total = o;
  return L;
}

}  // namespace
}  // namespace rxphy

extern "C" {

size_t rxphy_sense_workspace_bytes(const rxphy_sense_config* cfg, int32_t n_plots) {
  if (!rxphy::config_ok(cfg) || n_plots < 1) return 0;
  return rxphy::layout(*cfg, n_plots).total;
}

rxphy_status rxphy_sense(const rxphy_sense_config* cfg, int32_t n_plots, const void* x,
                         const rxphy_sense_outputs* out, int32_t* n_boxes, int32_t* boxes, int32_t max_boxes,
                         void* ws, size_t ws_bytes, hipStream_t stream) {
  using namespace rxphy;
  clear_error();
  if (!config_ok(cfg))
    return fail(RXPHY_EINVAL, "sense config: n_fft in {512..4096}, 3 <= n_rows <= 4096, odd sg_window 3..63, "
                              "sg_order 0..6 below the window, psd_factor > 0, bins 2..256");
  if (n_plots < 1 || n_plots > 65535) return fail(RXPHY_EINVAL, "n_plots = %d (1 .. 65535)", n_plots);
  if (max_boxes < 0) return fail(RXPHY_EINVAL, "max_boxes = %d", max_boxes);
  if (!x || !n_boxes || (max_boxes > 0 && !boxes)) return fail(RXPHY_EINVAL, "x, n_boxes or boxes is NULL");
  const SenseLayout Lo = layout(*cfg, n_plots);
  if (!ws || ws_bytes < Lo.total) return fail(RXPHY_EWORKSPACE, "sense needs %zu workspace bytes, got %zu", Lo.total, ws_bytes);
  if ((uintptr_t)ws & 255u) return fail(RXPHY_EWORKSPACE, "sense workspace must be 256-byte aligned");
  const rxphy_sense_config& c = *cfg;
  const int T = c.n_rows, F = c.n_fft, P = n_plots;
  const int64_t TF = (int64_t)T * F;
  const int ncnt = T * (F / 64);
  char* w = (char*)ws;
  rxphy_sense_outputs o{};
  if (out) o = *out;
  float* tf = o.tf ? o.tf : (float*)(w + Lo.tf);
  float* psd = o.psd ? o.psd : (float*)(w + Lo.psd);
  float* psd_s = o.psd_smooth ? o.psd_smooth : (float*)(w + Lo.psd_s);
  float* flo = o.floor ? o.floor : (float*)(w + Lo.flo);
  int32_t* kbin = o.otsu_bin ? o.otsu_bin : (int32_t*)(w + Lo.kbin);
  uint8_t* mask = o.mask ? o.mask : (uint8_t*)(w + Lo.mask);
  uint8_t* mask_mo = o.mask_mo ? o.mask_mo : (uint8_t*)(w + Lo.mask_mo);
  float* lo = (float*)(w + Lo.lo);
  float* hi = (float*)(w + Lo.hi);
  int32_t* lab = (int32_t*)(w + Lo.lab);
  int32_t* cnt = (int32_t*)(w + Lo.cnt);
  int32_t* off = (int32_t*)(w + Lo.off);
  const SgCoef sg = sg_coeffs(c.sg_window, c.sg_order);

  rxphy_status st = launch_fft_mag(F, (int64_t)P * T, (const float2*)x, tf, stream);
  if (st) return st;
  const unsigned strips = (unsigned)(F / 64);
  hipLaunchKernelGGL(colstat_kernel, dim3(strips, P), dim3(64 * CW), 0, stream, tf, psd, lo, hi, T, F);
  if ((st = launch_status("colstat kernel"))) return st;
  hipLaunchKernelGGL(floor_kernel, dim3(P), dim3(1024), 0, stream, psd, psd_s, flo, sg, c.psd_factor, F);
  if ((st = launch_status("floor kernel"))) return st;
  hipLaunchKernelGGL(otsu_kernel, dim3(strips, P), dim3(64 * CW), 0, stream, tf, psd, lo, hi, flo, kbin, mask, T, F,
                     c.bins);
  if ((st = launch_status("otsu kernel"))) return st;
  TileList* tl = (TileList*)(w + Lo.tl);
  hipLaunchKernelGGL(morph_kernel, dim3(strips, (T + 63) / 64, P), dim3(256), 0, stream, mask, mask_mo, lab, tl, T,
                     F);
  if ((st = launch_status("morph kernel"))) return st;
  hipLaunchKernelGGL(merge_kernel, dim3(strips, (T + 63) / 64, P), dim3(128), 0, stream, mask_mo, lab, T, F);
  if ((st = launch_status("merge kernel"))) return st;
  hipLaunchKernelGGL(flatten_kernel, dim3(strips, (T + 63) / 64, P), dim3(64), 0, stream, lab, tl, cnt, T, F);
  if ((st = launch_status("flatten kernel"))) return st;
  hipLaunchKernelGGL(scan_kernel, dim3(P), dim3(1024), 0, stream, cnt, off, n_boxes, boxes, max_boxes, ncnt);
  if ((st = launch_status("scan kernel"))) return st;
  hipLaunchKernelGGL(assign_kernel, dim3(strips, (T + 63) / 64, P), dim3(64), 0, stream, lab, tl, off, T, F);
  if ((st = launch_status("assign kernel"))) return st;
  if (max_boxes > 0) {
    hipLaunchKernelGGL(boxes_kernel, dim3(strips, (T + 63) / 64, P), dim3(256), 0, stream, mask_mo, lab, tl, boxes,
                       max_boxes, T, F);
    if ((st = launch_status("boxes kernel"))) return st;
  }
  return RXPHY_OK;
}

rxphy_status rxphy_savgol_weights(int32_t window, int32_t order, float* weights) {
  using namespace rxphy;
  clear_error();
  if (!weights) return fail(RXPHY_EINVAL, "weights is NULL");
  if (window < 3 || window > SG_MAX || !(window & 1) || order < 0 || order > 6 || order >= window)
    return fail(RXPHY_EINVAL, "window = %d, order = %d (odd window 3 .. %d, 0 <= order <= 6, order < window)",
                window, order, SG_MAX);
  const SgCoef sg = sg_coeffs(window, order);
  for (int k = 0; k < window; ++k) weights[k] = sg.c[k];
  return RXPHY_OK;
}

rxphy_status rxphy_box_metrics(const int32_t* gt, int32_t n_gt, const int32_t* det, int32_t n_det,
                               double theta_iou, double* iou, rxphy_detection_metrics* out) {
  using namespace rxphy;
  clear_error();
  if (!out || n_gt < 0 || n_det < 0 || (n_gt && !gt) || (n_det && !det)) return fail(RXPHY_EINVAL, "bad arguments");
  auto area = [](const int32_t* b) { return (double)(b[2] - b[0] + 1) * (double)(b[3] - b[1] + 1); };
  std::vector<double> best_gt(n_gt, 0.0), best_det(n_det, 0.0);
  for (int i = 0; i < n_gt; ++i)
    for (int j = 0; j < n_det; ++j) {
      const int32_t *a = gt + 4 * i, *b = det + 4 * j;
      const int it = std::min(a[2], b[2]) - std::max(a[0], b[0]) + 1;
      const int jf = std::min(a[3], b[3]) - std::max(a[1], b[1]) + 1;
      const double inter = (double)std::max(it, 0) * (double)std::max(jf, 0);
      const double v = inter / (area(a) + area(b) - inter);
      if (iou) iou[(int64_t)i * n_det + j] = v;
      best_gt[i] = std::max(best_gt[i], v);
      best_det[j] = std::max(best_det[j], v);
    }
  int nt = 0, nf = 0;
  double sum = 0.0;
  for (int i = 0; i < n_gt; ++i) {
    nt += n_det > 0 && best_gt[i] > theta_iou;
    sum += best_gt[i];
  }
  for (int j = 0; j < n_det; ++j) nf += n_gt == 0 || best_det[j] < theta_iou;
  out->n_t = nt;
  out->n_f = nf;
  out->p_d = n_gt ? (double)nt / n_gt : NAN;
  out->p_fa = n_det ? (double)nf / n_det : NAN;
  out->mean_iou = n_gt && n_det ? sum / n_gt : 0.0;
  return RXPHY_OK;
}

}  // extern "C"
