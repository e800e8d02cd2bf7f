// dec stage: layered normalised min-sum decoding of quasi-cyclic LDPC codes
// (the channel decoder the paper's preamble names beside its LDPC notation:
// lifting size Z_c, code-block size K_cb, code rate R), for gfx950.
//
// One workgroup per codeword, one thread per check row of a layer (block
// row).  The posterior LLRs of the whole codeword live in LDS (up to 38400
// values, 150 KB); the check-to-bit messages of every check are kept
// compressed in the workspace as the two scaled minima and one word of
// message signs plus the argmin (12 bytes per check, the form from which each
// message is rebuilt exactly), and the next layer's are loaded while the
// current layer is processed.  Per check (bits v_k of the layer's non-zero
// blocks, block columns in increasing order):
//   Q_k = L_{v_k} - R_k,  a1 = alpha * min_k |Q_k|,  a2 = alpha * (second min),
//   R_k = +-(k == argmin ? a2 : a1), negative iff the product of the signs of
//   all Q is negative XOR Q_k < 0,  L_{v_k} = Q_k + R_k,
// each an FP32 operation rounded once (no fused multiply-add), so the result
// is the definition evaluated in FP32.  The syndrome of the hard decisions
// (bit 1 iff L < 0) is tested before the first iteration and after each one;
// the decoder stops at the first zero syndrome.
#include <vector>

#include "common.h"

struct rxphy_ldpc_code {
  int32_t mb, nb, z, n_edges, max_deg;
  uint32_t* d_tab;      // [mb + 1] layer offsets, then [n_edges] ((z - shift) << 16 | column z + shift)
  std::vector<int16_t> base;
  int device;
};

namespace rxphy {
namespace {

constexpr int LDPC_ZMAX = 384;
constexpr int LDPC_DMAX = 27;          // message signs in bits 0..26, argmin in bits 27..31
constexpr int LDPC_NMAX = 38400;       // posterior LLRs held in LDS (150 KB; the edge table takes 7 KB more)
constexpr int LDPC_MBMAX = 64;

// Bit of check row r for the block (column c, shift s): c z + (r + s) mod z.
// A table entry holds lo = c z + s in its low half and hi = z - s in its high
// half, so that the bit is lo + r, less z once r + s wraps (r >= hi); the
// padding entry (column 0, shift 0) is z << 16.
__device__ __forceinline__ int bit_of(uint32_t e, int r, int z) {
  const int lo = (int)(e & 0xffffu), hi = (int)(e >> 16);
  return lo + r - (r >= hi ? z : 0);
}

constexpr int LDPC_PF = 4;             // layers of compressed messages in flight
// Edge slots per lane in one chunk of table and posterior reads, with S lanes
// per check row: a chunk covers CH * S edges of the row (10 for S = 2, 12 for
// S = 4, about one layer of a code with 8 - 12 edges per check), so that few
// slots past the row's degree are processed; DPAD = the slots of all chunks.
template <int S>
struct LdpcChunk {
  static constexpr int CH = S == 2 ? 5 : 3;
  static constexpr int SPAN = CH * S;
  static constexpr int DPAD = (LDPC_DMAX + SPAN - 1) / SPAN * SPAN;
  static constexpr int J = DPAD / S;
};
constexpr int LDPC_PADMAX = 12;        // the widest chunk's span: table padding past the last layer
// layer offsets, edges, and padding for the widest chunk (entries of column 0, shift 0)
constexpr int LDPC_TABMAX = LDPC_MBMAX + 1 + LDPC_MBMAX * LDPC_DMAX + LDPC_PADMAX;
static_assert(LdpcChunk<2>::SPAN <= LDPC_PADMAX && LdpcChunk<4>::SPAN <= LDPC_PADMAX, "table padding");

// S lanes (adjacent, within one quad) share a check row: lane part h takes
// the row's edges k = h, h + S, h + 2S, ...; the parts' partial results are
// combined through DPP quad permutes.  More waves per codeword hide the
// latency of the per-edge dependency chains, at no cost in LDS.
template <int OFF>
__device__ __forceinline__ uint32_t quad_xor_u(uint32_t v) {
  // quad_perm [1,0,3,2] for OFF = 1, [2,3,0,1] for OFF = 2
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, OFF == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int OFF>
__device__ __forceinline__ float quad_xor_f(float v) {
  return __uint_as_float(quad_xor_u<OFF>(__float_as_uint(v)));
}

// Syndrome test on the posteriors in LDS: does any check (all layers) see an
// odd number of hard ones?  T is the edge table in LDS.
template <int S>
__device__ __forceinline__ bool any_check_unsatisfied(const float* L, const uint32_t* T, int mb, int z) {
  const int tid = threadIdx.x, r = tid / S, h = tid % S;
  const bool row = r < z;
  int bad = 0;
  for (int i = 0; i < mb; ++i) {
    const int e0 = __builtin_amdgcn_readfirstlane((int)T[i]);
    const int d = __builtin_amdgcn_readfirstlane((int)T[i + 1]) - e0;
    const uint32_t* E = T + mb + 1 + e0;
    uint32_t par = 0;
    if (row) {
      using C = LdpcChunk<S>;
#pragma unroll
      for (int c = 0; c < C::DPAD / C::SPAN; ++c) {
        if (c * C::SPAN < d) {
          float lv[C::CH];
#pragma unroll
          for (int t = 0; t < C::CH; ++t) lv[t] = L[bit_of(E[(c * C::CH + t) * S + h], r, z)];
#pragma unroll
          for (int t = 0; t < C::CH; ++t) par ^= ((c * C::CH + t) * S + h < d && lv[t] < 0.f) ? 1u : 0u;
        }
      }
    }
    par ^= quad_xor_u<1>(par);
    if constexpr (S == 4) par ^= quad_xor_u<2>(par);
    bad |= (int)par;
  }
  return __syncthreads_or(row ? bad : 0) != 0;
}

// The two smallest magnitudes of the union of this part's and the partner's,
// the first argmin, the parity of the negative signs.
template <int OFF>
__device__ __forceinline__ void combine_parts(float& m1, float& m2, int& idx, uint32_t& neg) {
  const float p1 = quad_xor_f<OFF>(m1), p2 = quad_xor_f<OFF>(m2);
  const int pidx = (int)quad_xor_u<OFF>((uint32_t)idx);
  const uint32_t pneg = quad_xor_u<OFF>(neg);
  const float n2 = fminf(fmaxf(m1, p1), fminf(m2, p2));
  idx = (p1 < m1 || (p1 == m1 && pidx < idx)) ? pidx : idx;
  m1 = fminf(m1, p1);
  m2 = n2;
  neg ^= pneg;
}

// One layer (block row i) for check row r (lane part h): the old messages of
// its check come in compressed (o1, o2, om); the lane's edges are read in
// chunks of LdpcChunk<S>::CH, each chunk's table entries and posteriors requested
// together; slots past the layer's degree read padding or the next layer's
// entries (valid addresses) and take Q = +inf, which changes no minimum and
// no sign.  Writes the new posteriors to L (a slot past the degree writes
// the spare word L[spare] instead, so that no store needs a branch) and
// (part 0) the new compressed messages.  The minimum, second minimum and
// argmin are tracked with selects, not branches.
template <int S>
__device__ __forceinline__ void layer_update(float* L, const uint32_t* T, float* A1, float* A2, uint32_t* MT,
                                             int mb, int z, int i, int r, int h, bool row, float o1, float o2,
                                             uint32_t om, float alpha, int spare) {
  using C = LdpcChunk<S>;
  constexpr int J = C::J;                        // edge slots per lane
  const int e0 = __builtin_amdgcn_readfirstlane((int)T[i]);
  const int d = __builtin_amdgcn_readfirstlane((int)T[i + 1]) - e0;
  const uint32_t* E = T + mb + 1 + e0;
  const int oidx = (int)(om >> 27);
  float q[J];
  int vv[J];
  float m1 = INFINITY, m2 = INFINITY;
  int idx = 0;
  uint32_t neg = 0u;
  if (row) {
#pragma unroll
    for (int c = 0; c < J / C::CH; ++c) {
      if (c * C::SPAN < d) {
        float lv[C::CH];
#pragma unroll
        for (int t = 0; t < C::CH; ++t) {
          const int j = c * C::CH + t;
          vv[j] = bit_of(E[j * S + h], r, z);
          lv[t] = L[vv[j]];
        }
#pragma unroll
        for (int t = 0; t < C::CH; ++t) {
          const int j = c * C::CH + t, k = j * S + h;
          const float mag = k == oidx ? o2 : o1;
          const float r_old = ((om >> k) & 1u) ? -mag : mag;
          const float qk = k < d ? lv[t] - r_old : INFINITY;
          q[j] = qk;
          const float a = __builtin_fabsf(qk);
          // the two smallest magnitudes and the first argmin, without branches:
          // a < m1 -> (a, m1, k); else (m1, min(m2, a), idx)
          const bool lt = a < m1;
          m2 = lt ? m1 : __builtin_fminf(m2, a);
          m1 = lt ? a : m1;
          idx = lt ? k : idx;
          neg ^= qk < 0.f ? 1u : 0u;
        }
      }
    }
  }
  // combine the parts: the two smallest of the union, the first argmin, the parity of the signs
  combine_parts<1>(m1, m2, idx, neg);
  if constexpr (S == 4) combine_parts<2>(m1, m2, idx, neg);
  if (!row) return;
  const float a1 = alpha * m1;
  const float a2 = alpha * m2;
  uint32_t sg = 0u;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = j * S + h;
    if (j * S < d) {                             // the same in every lane; k < d is not:
      const bool in = k < d;                     // a slot past the degree writes the spare word
      const uint32_t sk = neg ^ (q[j] < 0.f ? 1u : 0u);
      const float mag = k == idx ? a2 : a1;
      L[in ? vv[j] : spare] = q[j] + (sk ? -mag : mag);
      sg |= (in ? sk : 0u) << k;
    }
  }
  sg |= quad_xor_u<1>(sg);
  if constexpr (S == 4) sg |= quad_xor_u<2>(sg);
  if (h == 0) {
    const int64_t x = (int64_t)i * z + r;
    A1[x] = a1;
    A2[x] = a2;
    MT[x] = sg | ((uint32_t)idx << 27);
  }
}

template <int NMAX, int S>
__global__ void __launch_bounds__(S == 2 ? 2 * LDPC_ZMAX : 1024)
ldpc_decode_kernel(const uint32_t* __restrict__ tab, int mb, int nb, int z, const float* __restrict__ llr,
                   int max_iter, float alpha, float* __restrict__ post, uint8_t* __restrict__ bits,
                   int32_t* __restrict__ iters, float* __restrict__ msg) {
  __shared__ float L[NMAX + 1];                 // posteriors, and a spare word that masked slots write
  __shared__ uint32_t T[LDPC_TABMAX];
  const int N = nb * z;
  const int64_t cw = blockIdx.x;
  const int tid = threadIdx.x;
  const float* in = llr + cw * N;
  for (int v = tid; v < N; v += blockDim.x) L[v] = in[v];
  const int tlen = mb + 1 + (int)tab[mb];
  for (int t = tid; t < tlen + LdpcChunk<S>::SPAN; t += blockDim.x) T[t] = t < tlen ? tab[t] : (uint32_t)z << 16;
  // compressed messages of this codeword: a1 [mb][z], a2 [mb][z], meta [mb][z]
  float* A1 = msg + cw * 3 * (int64_t)mb * z;
  float* A2 = A1 + (int64_t)mb * z;
  uint32_t* MT = reinterpret_cast<uint32_t*>(A2 + (int64_t)mb * z);
  __syncthreads();

  int it = 0;
  bool more = any_check_unsatisfied<S>(L, T, mb, z);
  const int r = tid / S, h = tid % S;
  const bool row = r < z;
  const int trow = row ? r : z - 1;            // message address of this lane (in range)
  while (more && it < max_iter) {
    ++it;
    const bool first = it == 1;
    // the compressed messages of the next LDPC_PF layers in flight, one
    // register slot per layer (zero messages in the first iteration); the
    // layer loop is unrolled by LDPC_PF so that every slot is a fixed
    // register and each load is waited for only when its layer starts (the
    // loads are unconditional, at clamped addresses, and their values are
    // discarded at the use when not wanted: a load under a branch would be
    // waited for at the branch's end)
    float s1[LDPC_PF], s2[LDPC_PF];
    uint32_t sm[LDPC_PF];
#pragma unroll
    for (int u = 0; u < LDPC_PF; ++u) {
      const int64_t x = (int64_t)min(u, mb - 1) * z + trow;
      s1[u] = A1[x]; s2[u] = A2[x]; sm[u] = MT[x];
    }
    for (int i0 = 0; i0 < mb; i0 += LDPC_PF) {
#pragma unroll
      for (int u = 0; u < LDPC_PF; ++u) {
        const int i = i0 + u;
        const float o1 = first ? 0.f : s1[u], o2 = first ? 0.f : s2[u];
        const uint32_t om = first ? 0u : sm[u];
        const int64_t x = (int64_t)min(i + LDPC_PF, mb - 1) * z + trow;   // layer i + LDPC_PF
        s1[u] = A1[x]; s2[u] = A2[x]; sm[u] = MT[x];
        if (i < mb) {
          layer_update<S>(L, T, A1, A2, MT, mb, z, i, r, h, row, o1, o2, om, alpha, NMAX);
          __syncthreads();                       // the next layer reads this one's L
        }
      }
    }
    more = any_check_unsatisfied<S>(L, T, mb, z);
  }
  float* out = post + cw * N;
  uint8_t* hb = bits ? bits + cw * N : nullptr;
  for (int v = tid; v < N; v += blockDim.x) {
    const float l = L[v];
    out[v] = l;
    if (hb) hb[v] = l < 0.f ? 1 : 0;
  }
  if (tid == 0 && iters) iters[cw] = it;
}

template <int NMAX>
void launch_ldpc(const rxphy_ldpc_code& c, int32_t n_cw, const float* llr, int max_iter, float alpha,
                 float* post, uint8_t* bits, int32_t* iters, float* msg, hipStream_t s) {
  // two lanes per check row above z = 256, four up to it (at most 1024 threads)
  if (c.z > 256) {
    const int threads = (2 * c.z + 63) / 64 * 64;
    hipLaunchKernelGGL((ldpc_decode_kernel<NMAX, 2>), dim3((unsigned)n_cw), dim3(threads), 0, s, c.d_tab, c.mb,
                       c.nb, c.z, llr, max_iter, alpha, post, bits, iters, msg);
  } else {
    const int threads = (4 * c.z + 63) / 64 * 64;
    hipLaunchKernelGGL((ldpc_decode_kernel<NMAX, 4>), dim3((unsigned)n_cw), dim3(threads), 0, s, c.d_tab, c.mb,
                       c.nb, c.z, llr, max_iter, alpha, post, bits, iters, msg);
  }
}

}  // namespace
}  // namespace rxphy

using namespace rxphy;

extern "C" {

rxphy_status rxphy_ldpc_code_create(const int16_t* base, int32_t mb, int32_t nb, int32_t z,
                                    rxphy_ldpc_code** code) {
  clear_error();
  if (!code) return fail(RXPHY_EINVAL, "code is NULL");
  *code = nullptr;
  if (!base) return fail(RXPHY_EINVAL, "base is NULL");
  if (z < 1 || z > LDPC_ZMAX) return fail(z < 1 ? RXPHY_EINVAL : RXPHY_EUNSUPPORTED, "z = %d outside [1, %d]", z, LDPC_ZMAX);
  if (mb < 1 || nb <= mb) return fail(RXPHY_EINVAL, "mb = %d, nb = %d (need 1 <= mb < nb)", mb, nb);
  if (mb > LDPC_MBMAX) return fail(RXPHY_EUNSUPPORTED, "mb = %d > %d", mb, LDPC_MBMAX);
  if ((int64_t)nb * z > LDPC_NMAX) return fail(RXPHY_EUNSUPPORTED, "nb z = %lld > %d", (long long)nb * z, LDPC_NMAX);
  std::vector<uint32_t> tab(mb + 1);
  std::vector<uint32_t> edges;
  int max_deg = 0;
  for (int i = 0; i < mb; ++i) {
    tab[i] = (uint32_t)edges.size();
    int deg = 0;
    for (int j = 0; j < nb; ++j) {
      const int s = base[(int64_t)i * nb + j];
      if (s < -1 || s >= z) return fail(RXPHY_EINVAL, "base[%d][%d] = %d outside [-1, z)", i, j, s);
      if (s >= 0) {
        edges.push_back(((uint32_t)(z - s) << 16) | (uint32_t)(j * z + s));   // see bit_of
        ++deg;
      }
    }
    if (deg < 2) return fail(RXPHY_EINVAL, "row %d of the base matrix has %d non-zero blocks (need >= 2)", i, deg);
    if (deg > LDPC_DMAX) return fail(RXPHY_EUNSUPPORTED, "row %d has %d non-zero blocks (> %d)", i, deg, LDPC_DMAX);
    if (deg > max_deg) max_deg = deg;
  }
  tab[mb] = (uint32_t)edges.size();
  tab.insert(tab.end(), edges.begin(), edges.end());
  rxphy_ldpc_code* c = new rxphy_ldpc_code();
  c->mb = mb;
  c->nb = nb;
  c->z = z;
  c->n_edges = (int32_t)edges.size();
  c->max_deg = max_deg;
  c->base.assign(base, base + (int64_t)mb * nb);
  c->d_tab = nullptr;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(RXPHY_EHIP, "hipGetDevice failed");
  }
  hipError_t e = hipMalloc((void**)&c->d_tab, tab.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpy(c->d_tab, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (c->d_tab) (void)hipFree(c->d_tab);
    delete c;
    return fail(RXPHY_EHIP, "ldpc code table: %s", hipGetErrorString(e));
  }
  *code = c;
  return RXPHY_OK;
}

void rxphy_ldpc_code_destroy(rxphy_ldpc_code* code) {
  if (!code) return;
  if (code->d_tab) (void)hipFree(code->d_tab);
  delete code;
}

size_t rxphy_ldpc_workspace_bytes(const rxphy_ldpc_code* code, int32_t n_cw) {
  if (!code || n_cw < 0) return 0;
  return (size_t)n_cw * code->mb * code->z * 12;
}

rxphy_status rxphy_ldpc_decode(const rxphy_ldpc_code* code, int32_t n_cw, const float* llr, int32_t max_iter,
                               float alpha, float* post, uint8_t* bits, int32_t* iters, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  clear_error();
  if (!code) return fail(RXPHY_EINVAL, "code is NULL");
  if (n_cw < 0) return fail(RXPHY_EINVAL, "n_cw = %d < 0", n_cw);
  if (max_iter < 0) return fail(RXPHY_EINVAL, "max_iter = %d < 0", max_iter);
  if (!(alpha > 0.f) || !(alpha < INFINITY)) return fail(RXPHY_EINVAL, "alpha = %g must be finite and > 0", alpha);
  const size_t need = rxphy_ldpc_workspace_bytes(code, n_cw);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 3u))
    return fail(RXPHY_EWORKSPACE, "ldpc_decode needs %zu workspace bytes (4-byte aligned), got %zu", need, ws_bytes);
  if (n_cw == 0) return RXPHY_OK;
  rxphy_status st;
  if ((st = check_ptr(llr, "llr")) || (st = check_ptr(post, "post"))) return st;
  const rxphy_ldpc_code& c = *code;
  const int64_t N = (int64_t)c.nb * c.z;
  float* msg = (float*)ws;
  if (N <= 4096) launch_ldpc<4096>(c, n_cw, llr, max_iter, alpha, post, bits, iters, msg, stream);
  else if (N <= 12288) launch_ldpc<12288>(c, n_cw, llr, max_iter, alpha, post, bits, iters, msg, stream);
  else launch_ldpc<LDPC_NMAX>(c, n_cw, llr, max_iter, alpha, post, bits, iters, msg, stream);
  return launch_status("ldpc decode kernel");
}

}  // extern "C"
