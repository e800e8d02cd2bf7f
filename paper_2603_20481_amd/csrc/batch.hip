// Batched uneven frames: one persistent launch runs the four forward stages of
// every frame of a plan.
//
// Work list.  The host cuts every frame's stages into work items and lists
// them stage-major (all FFT items of all frames, then all CSI items, ...).  A
// fixed grid of 256-thread workgroups pops item indices from a device counter;
// an item of stage s > 0 of frame f first waits until frame f's stage s-1
// counter reaches that stage's item count, runs the same tile body as the
// single-frame kernel of its stage, and then bumps frame f's stage-s counter.
// Because every item depends only on items listed before it, and a popped item
// is always held by a running workgroup, the lowest unfinished item can always
// run: the launch cannot deadlock whatever the grid.  A wait that exceeds the
// spin limit sets a status bit and gives up instead of hanging.
//
// Memory ordering.  Each XCD has its own L2, so a producer publishes with an
// agent-scope release (its stores complete and its L2 is written back before
// the counter moves) and a consumer acquires at agent scope (its L1 and L2
// copies are invalidated) before it reads the producer's data.  Releases are
// batched per workgroup (see publish below): an L2 writeback per item would
// cost more than the items themselves.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "csi_core.h"
#include "demod_core.h"
#include "detect_core.h"
#include "fft_core.h"

namespace rxphy {
namespace {

constexpr int WGS = 256;
constexpr int POOL = fftk::LDS_MAX > det::SMEM_ALL ? fftk::LDS_MAX : det::SMEM_ALL;
static_assert(POOL >= csik::CSI_LDS, "LDS pool too small");

// Device descriptor of one frame.  Offsets count elements of the tensor's type.
struct BFrame {
  int32_t M, K, n_fft, n_sc, n_sym, cp_len, qam_bits, mmse;
  float n0;
  int32_t kp, fft_iters, csi_tiles, det_tiles, dem_groups;
  int32_t need[4];          // items of each stage (0 for a stage that is not run)
  int64_t x, pil, yf, h, xt, nu, flags, llr;
};

// control block: [0] next item, [1] status, [CTL_DONE + 4 f + s] finished items
constexpr int CTL_DONE = 64;

inline uint32_t item_code(int stage, int f, int tile) {
  return ((uint32_t)stage << 30) | ((uint32_t)f << 16) | (uint32_t)tile;
}

template <int N>
__device__ __forceinline__ void run_fft(const BFrame& d, int tile, const float2* x, float2* yf,
                                        const float2* tw, float2* pool) {
  using G = fftk::Geom<N>;
  const int64_t n_tr = (int64_t)d.M * d.n_sym;
  fftk::fft_tile<N, false>(x + d.x, yf + d.yf, tw, n_tr, (int64_t)tile * G::TPW * d.fft_iters,
                           d.fft_iters, d.cp_len + N, d.cp_len, d.n_sc, pool);
}

__device__ __forceinline__ void run_csi(const BFrame& d, int tile, const float2* yf,
                                        const float2* pil, float2* h, float2* pool) {
  const int nt = (d.n_sc + csik::CSI_TILE - 1) / csik::CSI_TILE;
  const int p0 = tile * d.csi_tiles;
  const int p1 = min(p0 + d.csi_tiles, d.M * nt);
  // the next tile's loads are issued before the current tile is finished
  csik::CsiIn cur, nxt;
  if (p0 < p1) {
    const int m = p0 / nt, t = p0 - m * nt;
    csik::csi_load(yf + d.yf + (int64_t)m * d.n_sym * d.n_sc, pil + d.pil, d.K, d.n_sc,
                   t * csik::CSI_TILE, cur);
  }
  for (int p = p0; p < p1; ++p) {
    const int m = p / nt, t = p - m * nt;
    if (p + 1 < p1) {
      const int mn = (p + 1) / nt, tn = (p + 1) - mn * nt;
      csik::csi_load(yf + d.yf + (int64_t)mn * d.n_sym * d.n_sc, pil + d.pil, d.K, d.n_sc,
                     tn * csik::CSI_TILE, nxt);
    }
    if (p > p0) __syncthreads();
    csik::csi_finish(h + d.h + (int64_t)m * d.K * d.n_sc, d.K, d.n_sc, t * csik::CSI_TILE, cur, pool);
    cur = nxt;
  }
}

// The demapping of one detector tile from the x_tilde and nu detect_tile left
// in LDS: thread (user u, tile subcarrier e) takes every data symbol of
// (u, i0 + e), as the demod stage's column loop does (the same demod_point,
// so the LLRs are bit-identical); consecutive threads write consecutive
// subcarriers' LLRs.
template <int Q>
__device__ __forceinline__ void demod_tile(const BFrame& d, int i0, const float2* pool, float* llr) {
  const int D = d.n_sym - 1;
  const int u = tid_x() >> 4, e = tid_x() & 15, i = i0 + e;
  if (u >= d.K || i >= d.n_sc) return;
  const float2* xs = pool + e * det::PMAT;        // the slab of tile subcarrier e
  const float v = xs[256 + u].x;
  const bool er = __builtin_isinf(v);
  const float inv = er ? 0.f : 1.0f / v;
  float* dst = llr + d.llr + ((int64_t)u * D * d.n_sc + i) * Q;
  for (int s = 0; s < D; ++s) demk::demod_point_inv<Q>(xs[16 * u + s], er, inv, dst + (int64_t)s * d.n_sc * Q);
}

// FU: the CSI stage fused in (the channel is the LS estimate formed from the
// pilot symbol of yf and the pilots, bit-identical to the CSI stage's value).
// DM: the demod stage fused in as well (x_tilde never written).
template <int KP, bool FU, bool DM>
__device__ __forceinline__ void run_detect(const BFrame& d, int tile, const float2* h, const float2* yf,
                                           const float2* pil, float2* xt, float* nu, uint8_t* flags,
                                           float* llr, float2* pool, int* nonfin) {
  const int nt = (d.n_sc + det::TS - 1) / det::TS;
  const int t0 = tile * d.det_tiles;
  const int t1 = min(t0 + d.det_tiles, nt);
  constexpr bool dm = DM;
  float2 hv[8], yv[8], pv;
  bool have0 = false;
  for (int t = t0; t < t1; ++t) {
    if (t > t0) __syncthreads();
    det::detect_tile<KP, det::P_FP32, FU>(FU ? nullptr : h + d.h, yf + d.yf, dm ? nullptr : xt + d.xt, nu + d.nu,
                                          flags ? flags + d.flags : nullptr, d.M, d.K, d.n_sym, d.n_sc,
                                          d.n0, d.mmse, 0.f, nullptr, 0u, t * det::TS, pool, nonfin, hv, yv,
                                          pv, have0, t + 1 < t1 ? (t + 1) * det::TS : -1, nullptr, nullptr,
                                          FU ? pil + d.pil : nullptr, nullptr, dm);
    if constexpr (DM) {
      __syncthreads();                              // every wave's slab written
      switch (d.qam_bits) {
        case 2: demod_tile<2>(d, t * det::TS, pool, llr); break;
        case 4: demod_tile<4>(d, t * det::TS, pool, llr); break;
        default: demod_tile<6>(d, t * det::TS, pool, llr); break;
      }
    }
  }
}

template <int Q>
__device__ __forceinline__ void run_demod(const BFrame& d, int tile, const float2* xt, const float* nu,
                                          float* llr) {
  const int D = d.n_sym - 1;
  const int total = d.K * d.n_sc;                 // (user, subcarrier) columns
  const int base = tile * d.dem_groups * WGS;
  for (int g = 0; g < d.dem_groups; ++g) {
    const int c = base + g * WGS + tid_x();
    if (c < total) {
      const int u = c / d.n_sc, i = c - u * d.n_sc;
      const uint32_t o = (uint32_t)(u * D) * (uint32_t)d.n_sc + (uint32_t)i;
      demk::demod_column<Q>(xt + d.xt + o, nu[d.nu + c], llr + d.llr + (int64_t)o * Q, D, d.n_sc);
    }
  }
}

// Run header in device memory: the plan's tables (written at creation) and the
// buffers of the current run (written by the reset kernel).  The persistent
// kernel takes only a pointer to it, which keeps the values live across its
// item loop (SGPRs) few; every stage body still has to fit in the register
// budget of 3 waves per SIMD next to them.
template <class T>
using gptr = __attribute__((address_space(1))) T*;   // pointer known to be global memory

struct Header {
  gptr<const BFrame> frames;
  gptr<const uint32_t> items;
  gptr<const float2> tw;
  uint32_t n_items, spin_limit;
  gptr<const float2> x;
  gptr<const float2> pil;
  gptr<float2> yf;
  gptr<float2> h;
  gptr<float2> xt;
  gptr<float> nu;
  gptr<uint8_t> flags;
  gptr<float> llr;
};

__global__ void __launch_bounds__(WGS)
reset_kernel(Header* __restrict__ hdr, uint32_t* __restrict__ ctl, int n, const float2* x,
             const float2* pil, float2* yf, float2* h, float2* xt, float* nu, uint8_t* flags, float* llr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->x = (gptr<const float2>)x; hdr->pil = (gptr<const float2>)pil; hdr->yf = (gptr<float2>)yf;
    hdr->h = (gptr<float2>)h; hdr->xt = (gptr<float2>)xt; hdr->nu = (gptr<float>)nu;
    hdr->flags = (gptr<uint8_t>)flags; hdr->llr = (gptr<float>)llr;
  }
  for (int i = blockIdx.x * WGS + threadIdx.x; i < n; i += gridDim.x * WGS) ctl[i] = 0u;
}

// Publishing finished items.  A workgroup does not bump a frame's stage
// counter after every item: it keeps its finished (frame, stage) counts in LDS
// and publishes them together, with one agent-scope release (one L2
// writeback), when it moves on to an item of another stage, before it would
// block on a dependency, when the list is full, and at exit.  Because the list
// is stage-major, nobody can be waiting for a stage-s count before the first
// stage-(s+1) item is popped, and every holder of stage-s counts publishes as
// soon as its current item ends; a workgroup never blocks while holding
// unpublished counts, so the no-deadlock argument above still holds.
constexpr int PEND = 64;

struct Pending {
  uint32_t slot[PEND];      // CTL_DONE + 4 f + s
  uint32_t count[PEND];
  int n, stage;
};

// All threads call this (uniform); on return the counts are published.
__device__ __forceinline__ void publish(Pending& pd, uint32_t* __restrict__ ctl) {
  __builtin_amdgcn_s_waitcnt(0);                   // this wave's stores have reached L2
  __syncthreads();
  const int n = pd.n;
  if (n > 0 && threadIdx.x < 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");    // L2 written back
    for (int e = threadIdx.x; e < n; e += 64)
      __hip_atomic_fetch_add(&ctl[pd.slot[e]], pd.count[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (threadIdx.x == 0) pd.n = 0;
  __syncthreads();
}

// FUSE: the plan forms the channel estimate inside the detector items; DM:
// the detector items demap their tiles (one instantiation per dataflow, so
// that each carries only its own detector bodies and their register needs).
template <bool FUSE, bool DM>
__global__ void __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(3)))
batch_kernel(const Header* __restrict__ hdr, uint32_t* __restrict__ ctl) {
  __shared__ float2 pool[POOL];
  __shared__ int nonfin[det::TS];
  __shared__ uint32_t s_item;
  __shared__ int s_ready;
  __shared__ Pending pd;
  if (threadIdx.x == 0) { pd.n = 0; pd.stage = -1; }
  for (;;) {
    // reload the header per item (it is small), through a pointer the compiler
    // cannot hoist loads across, so that its fields do not stay live in SGPRs
    gptr<const Header> hp = (gptr<const Header>)hdr;
    asm volatile("" : "+s"(hp));
    __syncthreads();                               // the previous item is done with LDS
    if (threadIdx.x == 0)
      s_item = __hip_atomic_fetch_add(&ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t q = __builtin_amdgcn_readfirstlane(s_item);
    if (q >= hp->n_items) {
      publish(pd, ctl);
      break;
    }
    const uint32_t code = hp->items[q];
    const int stage = (int)(code >> 30), f = (int)((code >> 16) & 0x3fffu), tile = (int)(code & 0xffffu);
    const BFrame& d = *(const BFrame*)(hp->frames + f);
    if (__builtin_amdgcn_readfirstlane(pd.n) > 0 && __builtin_amdgcn_readfirstlane(pd.stage) != stage)
      publish(pd, ctl);
    if (stage > 0) {
      // the stage this item waits for: the previous one, or the FFT for a
      // detector item that forms the channel estimate itself
      const int dep = (stage == 2 && FUSE) ? 0 : stage - 1;
      const uint32_t need = (uint32_t)d.need[dep];
      uint32_t* cnt = &ctl[CTL_DONE + 4 * f + dep];
      if (threadIdx.x == 0)
        s_ready = need == 0 || __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
      __syncthreads();
      if (!__builtin_amdgcn_readfirstlane(s_ready)) {
        publish(pd, ctl);                          // never block holding unpublished counts
        if (threadIdx.x == 0) {
          const uint32_t limit = hp->spin_limit;
          uint32_t spins = 0;
          while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (++spins > limit) {
              __hip_atomic_fetch_or(&ctl[1], (uint32_t)RXPHY_PLAN_WAIT_TIMEOUT, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            __builtin_amdgcn_s_sleep(4);
          }
        }
      }
      // acquire: this CU's L1 and this XCD's L2 drop what they may hold of the
      // producers' data (one wave's invalidate serves the whole workgroup)
      if (threadIdx.x < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __syncthreads();
    }
    switch (stage) {
      case 0: {
        const float2* x = (const float2*)hp->x;
        float2* yf = (float2*)hp->yf;
        const float2* tw = (const float2*)hp->tw;
        switch (d.n_fft) {
          case 512: run_fft<512>(d, tile, x, yf, tw, pool); break;
          case 1024: run_fft<1024>(d, tile, x, yf, tw, pool); break;
          case 2048: run_fft<2048>(d, tile, x, yf, tw, pool); break;
          default: run_fft<4096>(d, tile, x, yf, tw, pool); break;
        }
        break;
      }
      case 1: run_csi(d, tile, (const float2*)hp->yf, (const float2*)hp->pil, (float2*)hp->h, pool); break;
      case 2: {
        const float2* h = (const float2*)hp->h;
        const float2* yf = (const float2*)hp->yf;
        const float2* pil = (const float2*)hp->pil;
        float2* xt = (float2*)hp->xt;
        float* nu = (float*)hp->nu;
        uint8_t* flags = (uint8_t*)hp->flags;
        float* llr = (float*)hp->llr;
        switch (d.kp) {
          case 4: run_detect<4, FUSE, DM>(d, tile, h, yf, pil, xt, nu, flags, llr, pool, nonfin); break;
          case 8: run_detect<8, FUSE, DM>(d, tile, h, yf, pil, xt, nu, flags, llr, pool, nonfin); break;
          default: run_detect<16, FUSE, DM>(d, tile, h, yf, pil, xt, nu, flags, llr, pool, nonfin); break;
        }
        break;
      }
      default: {
        if constexpr (!DM) {                       // a plan that demaps in the detector has no demod items
          const float2* xt = (const float2*)hp->xt;
          const float* nu = (const float*)hp->nu;
          float* llr = (float*)hp->llr;
          switch (d.qam_bits) {
            case 2: run_demod<2>(d, tile, xt, nu, llr); break;
            case 4: run_demod<4>(d, tile, xt, nu, llr); break;
            default: run_demod<6>(d, tile, xt, nu, llr); break;
          }
        }
        break;
      }
    }
    // record the finished item; publish when the list is full
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t slot = (uint32_t)(CTL_DONE + 4 * f + stage);
      const int n = pd.n;
      if (n > 0 && pd.slot[n - 1] == slot) {
        pd.count[n - 1] += 1u;
      } else {
        pd.slot[n] = slot;
        pd.count[n] = 1u;
        pd.n = n + 1;
      }
      pd.stage = stage;
      s_ready = pd.n == PEND;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_ready)) publish(pd, ctl);
  }
}

int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// The persistent kernel of a plan's dataflow.
const void* plan_kernel(int fuse_csi, int fuse_demod) {
  if (fuse_csi) return fuse_demod ? (const void*)batch_kernel<true, true> : (const void*)batch_kernel<true, false>;
  return fuse_demod ? (const void*)batch_kernel<false, true> : (const void*)batch_kernel<false, false>;
}

int fft_tpw(int n) { return n <= 2048 ? WGS / (n / 8) : 1; }

}  // namespace
}  // namespace rxphy

using namespace rxphy;

struct rxphy_plan {
  int dev = 0;
  int32_t n_frames = 0;
  std::vector<BFrame> desc;
  std::vector<rxphy_offsets> offs;   // bytes
  rxphy_offsets totals{};
  int64_t counts[4] = {0, 0, 0, 0};
  uint32_t n_items = 0;
  int32_t grid = 0;
  uint32_t spin_limit = 0;
  int fuse_csi = 0, fuse_demod = 0;
  int n_ctl = 0;
  BFrame* d_desc = nullptr;
  uint32_t* d_items = nullptr;
  uint32_t* d_ctl = nullptr;
  Header* d_hdr = nullptr;
  const float2* tw = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(rxphy_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_desc) (void)hipFree(p->d_desc);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_ctl) (void)hipFree(p->d_ctl);
  if (p->d_hdr) (void)hipFree(p->d_hdr);
  delete p;
}

rxphy_status check_batch(const rxphy_plan* p, const rxphy_batch* b) {
  if (!p) return fail(RXPHY_EINVAL, "plan is NULL");
  if (!b) return fail(RXPHY_EINVAL, "buffers is NULL");
  rxphy_status st;
  if ((st = check_ptr(b->x, "x")) || (st = check_ptr(b->pilots, "pilots")) ||
      (st = check_ptr(b->yf, "yf")) || (!p->fuse_csi && (st = check_ptr(b->h, "h"))) ||
      (!p->fuse_demod && (st = check_ptr(b->xt, "xt"))) || (st = check_ptr(b->nu, "nu")) ||
      (st = check_ptr(b->llr, "llr")))
    return st;
  return RXPHY_OK;
}

// argument blocks of the two launches, shared by the direct launch and the graph
struct RunArgs {
  Header* hdr;
  uint32_t* ctl;
  int n_ctl;
  const float2* x;
  const float2* pil;
  float2* yf;
  float2* h;
  float2* xt;
  float* nu;
  uint8_t* flags;
  float* llr;
  void* rptr[11];
  void* bptr[2];
  void** reset_args() {
    rptr[0] = &hdr; rptr[1] = &ctl; rptr[2] = &n_ctl; rptr[3] = &x; rptr[4] = &pil; rptr[5] = &yf;
    rptr[6] = &h; rptr[7] = &xt; rptr[8] = &nu; rptr[9] = &flags; rptr[10] = &llr;
    return rptr;
  }
  void** batch_args() {
    bptr[0] = &hdr; bptr[1] = &ctl;
    return bptr;
  }
};

RunArgs make_args(const rxphy_plan* p, const rxphy_batch* b) {
  RunArgs a;
  a.hdr = p->d_hdr;
  a.ctl = p->d_ctl;
  a.n_ctl = p->n_ctl;
  a.x = (const float2*)b->x;
  a.pil = (const float2*)b->pilots;
  a.yf = (float2*)b->yf;
  a.h = (float2*)b->h;
  a.xt = (float2*)b->xt;
  a.nu = b->nu;
  a.flags = b->flags;
  a.llr = b->llr;
  return a;
}

int reset_blocks(int n_ctl) { return (n_ctl + WGS - 1) / WGS < 64 ? (n_ctl + WGS - 1) / WGS : 64; }

}  // namespace

extern "C" {

rxphy_status rxphy_plan_create(const rxphy_frame* frames, int32_t n_frames, const rxphy_tiles* tiles,
                               const rxphy_plan_options* options, rxphy_plan** plan) {
  clear_error();
  if (!plan) return fail(RXPHY_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (!frames) return fail(RXPHY_EINVAL, "frames is NULL");
  if (n_frames < 1 || n_frames > 16384) return fail(RXPHY_EINVAL, "n_frames = %d outside [1, 16384]", n_frames);
  rxphy_plan_options opt{0, 0, 0u, 0, 0};
  if (options) opt = *options;
  int stages = opt.stages == 0 ? RXPHY_STAGE_ALL : opt.stages;
  if (stages & ~RXPHY_STAGE_ALL) return fail(RXPHY_EINVAL, "stages = %d", opt.stages);
  if (opt.fuse_csi != 0 && opt.fuse_csi != 1) return fail(RXPHY_EINVAL, "fuse_csi = %d", opt.fuse_csi);
  if (opt.fuse_demod != 0 && opt.fuse_demod != 1) return fail(RXPHY_EINVAL, "fuse_demod = %d", opt.fuse_demod);
  if (opt.fuse_csi) stages &= ~RXPHY_STAGE_CSI;        // the detector items form the estimate
  if (opt.fuse_demod) stages &= ~RXPHY_STAGE_DEMOD;    // ... and demap their tiles
  if (opt.grid < 0) return fail(RXPHY_EINVAL, "grid = %d < 0", opt.grid);

  rxphy_plan* p = new rxphy_plan();
  p->n_frames = n_frames;
  p->spin_limit = opt.spin_limit ? opt.spin_limit : (1u << 22);
  p->fuse_csi = opt.fuse_csi;
  p->fuse_demod = opt.fuse_demod;
  p->desc.resize(n_frames);
  p->offs.resize(n_frames);
  std::vector<uint32_t> items[4];
  rxphy_offsets run{0, 0, 0, 0, 0, 0, 0, 0};
  for (int f = 0; f < n_frames; ++f) {
    const rxphy_frame& fr = frames[f];
    rxphy_status st = check_frame(&fr, 1);
    if (st) {
      free_plan(p);
      return fail(st, "frame %d: %s", f, rxphy_last_error());
    }
    rxphy_tiles t{0, 0, 0, 0, 0};
    if (tiles) t = tiles[f];
    if (t.fft_iters < 0 || t.csi_tiles < 0 || t.det_tiles < 0 || t.dem_groups < 0 || t.fft_iters > 64 ||
        t.csi_tiles > 512 || t.det_tiles > 256 || t.dem_groups > 4096) {
      free_plan(p);
      return fail(RXPHY_EINVAL, "frame %d: tile sizes out of range", f);
    }
    const int kp_min = fr.K <= 4 ? 4 : fr.K <= 8 ? 8 : 16;
    if (t.det_kp != 0 && t.det_kp != 4 && t.det_kp != 8 && t.det_kp != 16) {
      free_plan(p);
      return fail(RXPHY_EINVAL, "frame %d: det_kp = %d", f, t.det_kp);
    }
    if (t.det_kp != 0 && t.det_kp < kp_min) {
      free_plan(p);
      return fail(RXPHY_EINVAL, "frame %d: det_kp = %d < K = %d", f, t.det_kp, fr.K);
    }
    BFrame& d = p->desc[f];
    d.M = fr.M; d.K = fr.K; d.n_fft = fr.n_fft; d.n_sc = fr.n_sc; d.n_sym = fr.n_sym;
    d.cp_len = fr.cp_len; d.qam_bits = fr.qam_bits; d.mmse = fr.detector == RXPHY_MMSE ? 1 : 0;
    d.n0 = fr.n0;
    d.kp = t.det_kp ? t.det_kp : kp_min;
    d.fft_iters = t.fft_iters ? t.fft_iters : 4;
    d.csi_tiles = t.csi_tiles ? t.csi_tiles : 2;
    d.det_tiles = t.det_tiles ? t.det_tiles : 1;
    d.dem_groups = t.dem_groups ? t.dem_groups : 4;
    const int64_t D = fr.n_sym - 1;
    const int64_t n_tr = (int64_t)fr.M * fr.n_sym;
    const int64_t per_fft = (int64_t)fft_tpw(fr.n_fft) * d.fft_iters;
    const int64_t nt_csi = (int64_t)fr.M * ((fr.n_sc + csik::CSI_TILE - 1) / csik::CSI_TILE);
    const int64_t nt_det = (fr.n_sc + det::TS - 1) / det::TS;
    const int64_t n_dem = (int64_t)fr.K * fr.n_sc;
    const int64_t need[4] = {(n_tr + per_fft - 1) / per_fft, (nt_csi + d.csi_tiles - 1) / d.csi_tiles,
                             (nt_det + d.det_tiles - 1) / d.det_tiles,
                             (n_dem + (int64_t)d.dem_groups * WGS - 1) / ((int64_t)d.dem_groups * WGS)};
    for (int s = 0; s < 4; ++s) {
      const bool on = (stages >> s) & 1;
      if (need[s] > 0xffff) {
        free_plan(p);
        return fail(RXPHY_EUNSUPPORTED, "frame %d: %lld items in stage %d (max 65535)", f,
                    (long long)need[s], s);
      }
      d.need[s] = on ? (int32_t)need[s] : 0;
      if (on)
        for (int64_t t2 = 0; t2 < need[s]; ++t2) items[s].push_back(item_code(s, f, (int)t2));
      p->counts[s] += d.need[s];
    }
    // packed layout, each tensor of each frame on a 256-byte boundary
    rxphy_offsets& o = p->offs[f];
    const int64_t L = (int64_t)fr.cp_len + fr.n_fft;
    o.x = run.x;         run.x = align256(run.x + (int64_t)fr.M * fr.n_sym * L * 8);
    o.pilots = run.pilots; run.pilots = align256(run.pilots + (int64_t)fr.n_sc * 8);
    o.yf = run.yf;       run.yf = align256(run.yf + (int64_t)fr.M * fr.n_sym * fr.n_sc * 8);
    o.h = run.h;         run.h = align256(run.h + (int64_t)fr.M * fr.K * fr.n_sc * 8);
    o.xt = run.xt;       run.xt = align256(run.xt + (int64_t)fr.K * D * fr.n_sc * 8);
    o.nu = run.nu;       run.nu = align256(run.nu + (int64_t)fr.K * fr.n_sc * 4);
    o.flags = run.flags; run.flags = align256(run.flags + (int64_t)fr.n_sc);
    o.llr = run.llr;     run.llr = align256(run.llr + (int64_t)fr.K * D * fr.n_sc * fr.qam_bits * 4);
    d.x = o.x / 8; d.pil = o.pilots / 8; d.yf = o.yf / 8; d.h = o.h / 8; d.xt = o.xt / 8;
    d.nu = o.nu / 4; d.flags = o.flags; d.llr = o.llr / 4;
  }
  p->totals = run;
  std::vector<uint32_t> all;
  for (int s = 0; s < 4; ++s) all.insert(all.end(), items[s].begin(), items[s].end());
  p->n_items = (uint32_t)all.size();
  p->n_ctl = CTL_DONE + 4 * n_frames;

  rxphy_status st = ensure_device_tables(&p->tw);
  if (st) { free_plan(p); return st; }
  hipError_t e = hipGetDevice(&p->dev);
  if (e == hipSuccess) e = hipMalloc(&p->d_desc, sizeof(BFrame) * n_frames);
  if (e == hipSuccess) e = hipMalloc(&p->d_items, sizeof(uint32_t) * (all.empty() ? 1 : all.size()));
  if (e == hipSuccess) e = hipMalloc(&p->d_ctl, sizeof(uint32_t) * p->n_ctl);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_desc, p->desc.data(), sizeof(BFrame) * n_frames, hipMemcpyHostToDevice);
  if (e == hipSuccess && !all.empty())
    e = hipMemcpy(p->d_items, all.data(), sizeof(uint32_t) * all.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->d_ctl, 0, sizeof(uint32_t) * p->n_ctl);
  if (e == hipSuccess) e = hipMalloc(&p->d_hdr, sizeof(Header));
  if (e == hipSuccess) {
    Header hh{};
    hh.frames = (gptr<const BFrame>)p->d_desc;
    hh.items = (gptr<const uint32_t>)p->d_items;
    hh.tw = (gptr<const float2>)p->tw;
    hh.n_items = p->n_items;
    hh.spin_limit = p->spin_limit;
    e = hipMemcpy(p->d_hdr, &hh, sizeof(Header), hipMemcpyHostToDevice);
  }
  int grid = opt.grid;
  if (e == hipSuccess && grid == 0) {
    int per_cu = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, plan_kernel(p->fuse_csi, p->fuse_demod), WGS, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->dev);
    grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  if (e != hipSuccess) {
    free_plan(p);
    return fail(RXPHY_EHIP, "plan set-up: %s", hipGetErrorString(e));
  }
  p->grid = grid;
  *plan = p;
  return RXPHY_OK;
}

rxphy_status rxphy_plan_layout(const rxphy_plan* plan, rxphy_offsets* per_frame, rxphy_offsets* totals) {
  clear_error();
  if (!plan) return fail(RXPHY_EINVAL, "plan is NULL");
  if (per_frame)
    for (int f = 0; f < plan->n_frames; ++f) per_frame[f] = plan->offs[f];
  if (totals) *totals = plan->totals;
  return RXPHY_OK;
}

rxphy_status rxphy_plan_info(const rxphy_plan* plan, int64_t* counts, int32_t* grid) {
  clear_error();
  if (!plan) return fail(RXPHY_EINVAL, "plan is NULL");
  if (counts)
    for (int s = 0; s < 4; ++s) counts[s] = plan->counts[s];
  if (grid) *grid = plan->grid;
  return RXPHY_OK;
}

rxphy_status rxphy_plan_forward(rxphy_plan* plan, const rxphy_batch* buffers, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_batch(plan, buffers);
  if (st) return st;
  RunArgs a = make_args(plan, buffers);
  hipLaunchKernelGGL(reset_kernel, dim3(reset_blocks(a.n_ctl)), dim3(WGS), 0, stream, a.hdr, a.ctl,
                     a.n_ctl, a.x, a.pil, a.yf, a.h, a.xt, a.nu, a.flags, a.llr);
  if ((st = launch_status("plan reset kernel"))) return st;
  if (plan->n_items == 0) return RXPHY_OK;
  const hipError_t e = hipLaunchKernel(plan_kernel(plan->fuse_csi, plan->fuse_demod), dim3(plan->grid), dim3(WGS),
                                       a.batch_args(), 0, stream);
  if (e != hipSuccess) return fail(RXPHY_EHIP, "batch kernel: %s", hipGetErrorString(e));
  return launch_status("batch kernel");
}

rxphy_status rxphy_plan_graph(rxphy_plan* plan, const rxphy_batch* buffers) {
  clear_error();
  rxphy_status st = check_batch(plan, buffers);
  if (st) return st;
  if (plan->exec) { (void)hipGraphExecDestroy(plan->exec); plan->exec = nullptr; }
  if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
  RunArgs a = make_args(plan, buffers);
  hipKernelNodeParams rp{};
  rp.func = (void*)reset_kernel;
  rp.gridDim = dim3(reset_blocks(a.n_ctl));
  rp.blockDim = dim3(WGS);
  rp.sharedMemBytes = 0;
  rp.kernelParams = a.reset_args();
  rp.extra = nullptr;
  hipKernelNodeParams bp{};
  bp.func = (void*)plan_kernel(plan->fuse_csi, plan->fuse_demod);
  bp.gridDim = dim3(plan->grid);
  bp.blockDim = dim3(WGS);
  bp.sharedMemBytes = 0;
  bp.kernelParams = a.batch_args();
  bp.extra = nullptr;
  hipGraphNode_t nr = nullptr, nb = nullptr;
  hipError_t e = hipGraphCreate(&plan->graph, 0);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nr, plan->graph, nullptr, 0, &rp);
  if (e == hipSuccess && plan->n_items > 0) e = hipGraphAddKernelNode(&nb, plan->graph, &nr, 1, &bp);
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    plan->exec = nullptr;
    return fail(RXPHY_EHIP, "plan graph: %s", hipGetErrorString(e));
  }
  return RXPHY_OK;
}

rxphy_status rxphy_plan_replay(rxphy_plan* plan, hipStream_t stream) {
  clear_error();
  if (!plan) return fail(RXPHY_EINVAL, "plan is NULL");
  if (!plan->exec) return fail(RXPHY_EINVAL, "plan has no graph (call rxphy_plan_graph first)");
  hipError_t e = hipGraphLaunch(plan->exec, stream);
  if (e != hipSuccess) return fail(RXPHY_EHIP, "graph launch: %s", hipGetErrorString(e));
  return RXPHY_OK;
}

rxphy_status rxphy_plan_device_status(rxphy_plan* plan, uint32_t* status) {
  clear_error();
  if (!plan || !status) return fail(RXPHY_EINVAL, "plan or status is NULL");
  hipError_t e = hipMemcpy(status, plan->d_ctl + 1, sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(RXPHY_EHIP, "status read: %s", hipGetErrorString(e));
  return RXPHY_OK;
}

void rxphy_plan_destroy(rxphy_plan* plan) { free_plan(plan); }

}  // extern "C"
