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
  uint32_t* d_tab;      // [mb + 1] layer offsets, then [n_edges] (column << 16 | shift)
  std::vector<int16_t> base;
  int device;
};

namespace rxphy {
namespace {

constexpr int LDPC_ZMAX = 384;
constexpr int LDPC_DMAX = 27;          // message signs in bits 0..26, argmin in bits 27..31
constexpr int LDPC_NMAX = 38400;       // posterior LLRs held in LDS (150 KB)
constexpr int LDPC_MBMAX = 64;

// Bit of check row r for the block (column c, shift s): c z + (r + s) mod z.
__device__ __forceinline__ int bit_of(uint32_t e, int r, int z) {
  const int c = (int)(e >> 16), s = (int)(e & 0xffffu);
  const int t = r + s;
  return c * z + (t < z ? t : t - z);
}

// Syndrome test: does any check (all layers) see an odd number of hard ones?
__device__ bool any_check_unsatisfied(const float* L, const uint32_t* tab, int mb, int z, int* flag) {
  const int tid = threadIdx.x;
  if (tid == 0) *flag = 0;
  __syncthreads();
  int bad = 0;
  if (tid < z) {
    for (int i = 0; i < mb; ++i) {
      const int o0 = (int)tab[i], o1 = (int)tab[i + 1];
      int par = 0;
      for (int k = o0; k < o1; ++k) par ^= L[bit_of(tab[mb + 1 + k], tid, z)] < 0.f ? 1 : 0;
      bad |= par;
    }
  }
  if (bad) *flag = 1;
  __syncthreads();
  const bool any = *flag != 0;
  __syncthreads();
  return any;
}

template <int NMAX>
__global__ void __launch_bounds__(LDPC_ZMAX)
ldpc_decode_kernel(const uint32_t* __restrict__ tab, int mb, int nb, int z, const float* __restrict__ llr,
                   int max_iter, float alpha, float* __restrict__ post, uint8_t* __restrict__ bits,
                   int32_t* __restrict__ iters, float* __restrict__ msg) {
  __shared__ float L[NMAX];
  __shared__ int flag;
  const int N = nb * z;
  const int64_t cw = blockIdx.x;
  const int tid = threadIdx.x;
  const float* in = llr + cw * N;
  for (int v = tid; v < N; v += blockDim.x) L[v] = in[v];
  // compressed messages of this codeword: a1 [mb][z], a2 [mb][z], meta [mb][z]
  float* A1 = msg + cw * 3 * (int64_t)mb * z;
  float* A2 = A1 + (int64_t)mb * z;
  uint32_t* MT = reinterpret_cast<uint32_t*>(A2 + (int64_t)mb * z);
  __syncthreads();

  int it = 0;
  bool more = any_check_unsatisfied(L, tab, mb, z, &flag);
  const bool row = tid < z;
  while (more && it < max_iter) {
    ++it;
    const bool first = it == 1;
    // this thread's compressed messages of layer 0 (zero messages in the first iteration)
    float n1 = 0.f, n2 = 0.f;
    uint32_t nm = 0u;
    if (row && !first) { n1 = A1[tid]; n2 = A2[tid]; nm = MT[tid]; }
    for (int i = 0; i < mb; ++i) {
      const float o1 = n1, o2 = n2;
      const uint32_t om = nm;
      if (row && !first && i + 1 < mb) {       // the next layer's, in flight during this one
        const int64_t x = (int64_t)(i + 1) * z + tid;
        n1 = A1[x]; n2 = A2[x]; nm = MT[x];
      }
      const int e0 = (int)tab[i], d = (int)tab[i + 1] - e0;
      if (row) {
        const uint32_t* E = tab + mb + 1 + e0;
        const int oidx = (int)(om >> 27);
        float q[LDPC_DMAX];
        float m1 = INFINITY, m2 = INFINITY;
        int idx = 0;
        uint32_t neg = 0u;
#pragma unroll
        for (int k = 0; k < LDPC_DMAX; ++k) {
          if (k < d) {
            const int v = bit_of(E[k], tid, z);
            float r_old = k == oidx ? o2 : o1;
            if ((om >> k) & 1u) r_old = -r_old;
            const float qk = L[v] - r_old;
            q[k] = qk;
            const float a = __builtin_fabsf(qk);
            if (a < m1) { m2 = m1; m1 = a; idx = k; }
            else if (a < m2) { m2 = a; }
            neg ^= qk < 0.f ? 1u : 0u;
          }
        }
        const float a1 = alpha * m1;
        const float a2 = alpha * m2;
        uint32_t sg = 0u;
#pragma unroll
        for (int k = 0; k < LDPC_DMAX; ++k) {
          if (k < d) {
            const int v = bit_of(E[k], tid, z);
            const uint32_t sk = neg ^ (q[k] < 0.f ? 1u : 0u);
            float rk = k == idx ? a2 : a1;
            if (sk) rk = -rk;
            L[v] = q[k] + rk;
            sg |= sk << k;
          }
        }
        const int64_t x = (int64_t)i * z + tid;
        A1[x] = a1;
        A2[x] = a2;
        MT[x] = sg | ((uint32_t)idx << 27);
      }
      __syncthreads();                          // the next layer reads this one's L
    }
    more = any_check_unsatisfied(L, tab, mb, z, &flag);
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
  const int threads = (c.z + 63) / 64 * 64;
  hipLaunchKernelGGL(ldpc_decode_kernel<NMAX>, dim3((unsigned)n_cw), dim3(threads), 0, s, c.d_tab, c.mb, c.nb, c.z,
                     llr, max_iter, alpha, post, bits, iters, msg);
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
        edges.push_back(((uint32_t)j << 16) | (uint32_t)s);
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
