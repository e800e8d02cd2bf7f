// Real-time streaming of receiver tasks (Section III-B's bounded-latency
// rule, Section IV-D's ping-pong buffer): `depth` slots handed out in turn,
// each with its own HIP stream, completion event and buffers; the slot ring
// and its completion thread (stream_ring.h) stamp every task's latency
// against its arrival.  Host code only: a task is the library's own fft +
// csi_detect_demod calls.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "common.h"
#include "stream_ring.h"

namespace {

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;    // recorded after the task's last operation
  void* d_x = nullptr;          // host I/O staging of the inputs
  void* d_p = nullptr;
  void* d_yf = nullptr;         // FFT output (every stream)
  void* d_ws = nullptr;         // csi_detect_demod workspace
  float* d_llr = nullptr;       // host I/O staging of the outputs
  float* d_nu = nullptr;
  uint8_t* d_fl = nullptr;
  void* h_x = nullptr;          // pinned host buffers (host I/O)
  void* h_p = nullptr;
  float* h_llr = nullptr;
  float* h_nu = nullptr;
  uint8_t* h_fl = nullptr;
};

// Completion of a slot's task = its event.  The slots' events are created
// before the completion thread starts and destroyed after it has stopped.
struct HipPoller {
  const std::vector<Slot>* slots = nullptr;
  int device = 0;
  void start() { (void)hipSetDevice(device); }
  rxphy::Poll operator()(int i, char* msg, size_t cap) const {
    const hipError_t e = hipEventQuery((*slots)[(size_t)i].done);
    if (e == hipErrorNotReady) return rxphy::Poll::NotReady;
    if (e == hipSuccess) return rxphy::Poll::Done;
    snprintf(msg, cap, "%s", hipGetErrorString(e));
    return rxphy::Poll::Failed;
  }
};

}  // namespace

struct rxphy_stream {
  rxphy_frame fr{};
  int32_t nf = 0, depth = 0, host_io = 0, device = 0;
  float sc16 = 0.f;                             // > 0: 16-bit I/Q samples with this scale
  size_t bx = 0, bp = 0, byf = 0, bws = 0, bllr = 0, bnu = 0, bfl = 0;
  std::vector<Slot> slots;
  std::unique_ptr<rxphy::SlotRing<HipPoller>> ring;
};

namespace {

using rxphy::fail;
using rxphy::steady_ns;

void free_slot(Slot& sl) {
  if (sl.st) (void)hipStreamDestroy(sl.st);
  if (sl.done) (void)hipEventDestroy(sl.done);
  for (void* p : {sl.d_x, sl.d_p, sl.d_yf, sl.d_ws, (void*)sl.d_llr, (void*)sl.d_nu, (void*)sl.d_fl})
    if (p) (void)hipFree(p);
  for (void* p : {sl.h_x, sl.h_p, (void*)sl.h_llr, (void*)sl.h_nu, (void*)sl.h_fl})
    if (p) (void)hipHostFree(p);
  sl = Slot{};
}

rxphy_status alloc_slot(rxphy_stream* s, Slot& sl) {
  auto dev = [](void** p, size_t n) { return n ? hipMalloc(p, n) : hipSuccess; };
  auto host = [](void** p, size_t n) { return hipHostMalloc(p, n, hipHostMallocDefault); };
  hipError_t e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
  if (e == hipSuccess) e = dev(&sl.d_yf, s->byf);
  if (e == hipSuccess) e = dev(&sl.d_ws, s->bws);
  if (s->host_io) {
    if (e == hipSuccess) e = dev(&sl.d_x, s->bx);
    if (e == hipSuccess) e = dev(&sl.d_p, s->bp);
    if (e == hipSuccess) e = dev((void**)&sl.d_llr, s->bllr);
    if (e == hipSuccess) e = dev((void**)&sl.d_nu, s->bnu);
    if (e == hipSuccess) e = dev((void**)&sl.d_fl, s->bfl);
    if (e == hipSuccess) e = host(&sl.h_x, s->bx);
    if (e == hipSuccess) e = host(&sl.h_p, s->bp);
    if (e == hipSuccess) e = host((void**)&sl.h_llr, s->bllr);
    if (e == hipSuccess) e = host((void**)&sl.h_nu, s->bnu);
    if (e == hipSuccess) e = host((void**)&sl.h_fl, s->bfl);
  }
  if (e != hipSuccess) return fail(RXPHY_EHIP, "stream allocation: %s", hipGetErrorString(e));
  return RXPHY_OK;
}

void destroy_all(rxphy_stream* s) {
  if (s->ring) s->ring->shutdown();             // the completion thread stops before the events go
  for (Slot& sl : s->slots) free_slot(sl);
  delete s;
}

}  // namespace

extern "C" {

int64_t rxphy_clock_ns(void) { return steady_ns(); }

rxphy_status rxphy_stream_create(const rxphy_frame* frame, int32_t n_frames, int32_t depth, int32_t host_io,
                                 float sc16_scale, rxphy_stream** stream) {
  rxphy::clear_error();
  if (!stream) return fail(RXPHY_EINVAL, "stream is NULL");
  *stream = nullptr;
  rxphy_status st = rxphy::check_frame(frame, n_frames);
  if (st) return st;
  if (n_frames < 1 || n_frames > 65535) return fail(RXPHY_EINVAL, "n_frames = %d (1 .. 65535)", n_frames);
  if (depth < 1 || depth > 8) return fail(RXPHY_EINVAL, "depth = %d (1 .. 8)", depth);
  if (host_io != 0 && host_io != 1) return fail(RXPHY_EINVAL, "host_io = %d (0 or 1)", host_io);
  if (!(sc16_scale >= 0.0f) || !std::isfinite(sc16_scale))
    return fail(RXPHY_EINVAL, "sc16_scale = %g (0 or finite > 0)", sc16_scale);
  const rxphy_frame& fr = *frame;
  const size_t F = (size_t)n_frames, D = (size_t)fr.n_sym - 1;
  rxphy_stream* s = new rxphy_stream();
  s->fr = fr;
  s->nf = n_frames;
  s->depth = depth;
  s->host_io = host_io;
  s->sc16 = sc16_scale;
  s->bx = F * fr.M * fr.n_sym * (size_t)(fr.cp_len + fr.n_fft) * (sc16_scale > 0.f ? 4 : 8);
  s->bp = F * fr.n_sc * 8;
  s->byf = F * fr.M * fr.n_sym * (size_t)fr.n_sc * 8;
  s->bws = rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_CSI_DETECT_DEMOD, RXPHY_FP32);
  s->bllr = F * fr.K * D * fr.n_sc * fr.qam_bits * 4;
  s->bnu = F * fr.K * (size_t)fr.n_sc * 4;
  s->bfl = F * fr.n_sc;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return fail(RXPHY_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  s->slots.resize(depth);
  for (Slot& sl : s->slots) {
    if ((st = alloc_slot(s, sl))) {
      destroy_all(s);
      return st;
    }
  }
  s->ring.reset(new rxphy::SlotRing<HipPoller>(depth));
  s->ring->start(HipPoller{&s->slots, s->device});
  *stream = s;
  return RXPHY_OK;
}

rxphy_status rxphy_stream_host_buffers(rxphy_stream* s, int32_t slot, rxphy_stream_host* host) {
  rxphy::clear_error();
  if (!s || !host) return fail(RXPHY_EINVAL, "stream or host is NULL");
  if (!s->host_io) return fail(RXPHY_EINVAL, "device-resident stream has no host buffers");
  if (slot < 0 || slot >= s->depth) return fail(RXPHY_EINVAL, "slot = %d (0 .. %d)", slot, s->depth - 1);
  const Slot& sl = s->slots[slot];
  *host = rxphy_stream_host{sl.h_x, sl.h_p, sl.h_llr, sl.h_nu, sl.h_fl};
  return RXPHY_OK;
}

rxphy_status rxphy_stream_acquire(rxphy_stream* s, int32_t* slot) {
  rxphy::clear_error();
  if (!s || !slot) return fail(RXPHY_EINVAL, "stream or slot is NULL");
  int k = -1;
  if (!s->ring->acquire(&k)) return fail(RXPHY_EINVAL, "the next slot is acquired and not yet submitted");
  *slot = k;
  return RXPHY_OK;
}

rxphy_status rxphy_stream_submit(rxphy_stream* s, int32_t slot, int64_t arrival_ns, const void* x,
                                 const void* pilots, float* llr, float* nu, uint8_t* flags) {
  rxphy::clear_error();
  if (!s) return fail(RXPHY_EINVAL, "stream is NULL");
  if (slot < 0 || slot >= s->depth) return fail(RXPHY_EINVAL, "slot = %d (0 .. %d)", slot, s->depth - 1);
  if (arrival_ns < 0) return fail(RXPHY_EINVAL, "arrival_ns = %lld", (long long)arrival_ns);
  Slot& sl = s->slots[slot];
  if (!s->ring->acquired(slot)) return fail(RXPHY_EINVAL, "slot %d was not acquired", slot);
  if (s->host_io) {
    if (x || pilots || llr || nu || flags)
      return fail(RXPHY_EINVAL, "host I/O stream: x, pilots, llr, nu and flags must be NULL");
    x = sl.d_x;
    pilots = sl.d_p;
    llr = sl.d_llr;
    nu = sl.d_nu;
    flags = sl.d_fl;
  } else if (!x || !pilots || !llr || !nu) {
    return fail(RXPHY_EINVAL, "device-resident stream: x, pilots, llr and nu must be device pointers");
  }
  const int64_t t_sub = steady_ns();
  hipError_t e = hipSuccess;
  if (s->host_io) {
    e = hipMemcpyAsync(sl.d_x, sl.h_x, s->bx, hipMemcpyHostToDevice, sl.st);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.d_p, sl.h_p, s->bp, hipMemcpyHostToDevice, sl.st);
    if (e != hipSuccess) return fail(RXPHY_EHIP, "input copy: %s", hipGetErrorString(e));
  }
  rxphy_status st = s->sc16 > 0.f ? rxphy_fft_sc16(&s->fr, s->nf, (const int16_t*)x, s->sc16, sl.d_yf, sl.st)
                                  : rxphy_fft(&s->fr, s->nf, x, sl.d_yf, sl.st);
  if (!st)
    st = rxphy_csi_detect_demod(&s->fr, s->nf, sl.d_yf, pilots, nullptr, nu, flags, llr, RXPHY_FP32, 0.0f, sl.d_ws,
                                s->bws, sl.st);
  if (st) return st;
  if (s->host_io) {
    e = hipMemcpyAsync(sl.h_llr, sl.d_llr, s->bllr, hipMemcpyDeviceToHost, sl.st);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.h_nu, sl.d_nu, s->bnu, hipMemcpyDeviceToHost, sl.st);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.h_fl, sl.d_fl, s->bfl, hipMemcpyDeviceToHost, sl.st);
    if (e != hipSuccess) return fail(RXPHY_EHIP, "output copy: %s", hipGetErrorString(e));
  }
  e = hipEventRecord(sl.done, sl.st);
  if (e != hipSuccess) return fail(RXPHY_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
  s->ring->commit(slot, arrival_ns ? arrival_ns : t_sub);
  return RXPHY_OK;
}

rxphy_status rxphy_stream_drain(rxphy_stream* s) {
  rxphy::clear_error();
  if (!s) return fail(RXPHY_EINVAL, "stream is NULL");
  char msg[320];
  if (!s->ring->drain(msg, sizeof(msg))) return fail(RXPHY_EHIP, "%s", msg);
  return RXPHY_OK;
}

rxphy_status rxphy_stream_latencies(rxphy_stream* s, double* lat_us, int64_t cap, int64_t* n) {
  rxphy::clear_error();
  if (!s || !n || cap < 0 || (cap > 0 && !lat_us)) return fail(RXPHY_EINVAL, "bad arguments");
  *n = s->ring->latencies(lat_us, cap);
  return RXPHY_OK;
}

rxphy_status rxphy_stream_reset_latencies(rxphy_stream* s) {
  rxphy::clear_error();
  if (!s) return fail(RXPHY_EINVAL, "stream is NULL");
  const int64_t busy = s->ring->reset_latencies();
  if (busy) return fail(RXPHY_EINVAL, "%lld task(s) outstanding", (long long)busy);
  return RXPHY_OK;
}

void rxphy_stream_destroy(rxphy_stream* s) {
  if (!s) return;
  destroy_all(s);                               // waits for outstanding tasks first
}

rxphy_status rxphy_latency_summarize(const double* lat_us, int64_t n, double bound_us, rxphy_latency_summary* out) {
  rxphy::clear_error();
  if (!out || n < 0 || (n > 0 && !lat_us)) return fail(RXPHY_EINVAL, "bad arguments");
  *out = rxphy_latency_summary{};
  if (n == 0) return RXPHY_OK;
  std::vector<double> v(lat_us, lat_us + n);
  for (double t : v)
    if (std::isnan(t)) return fail(RXPHY_EINVAL, "a latency is NaN (task not completed)");
  std::sort(v.begin(), v.end());
  // nearest rank: the ceil(p n / 100)-th smallest, in integer arithmetic
  auto rank = [&](int64_t p) { return v[(size_t)((p * n + 99) / 100 - 1)]; };
  double sum = 0.0;
  int64_t ok = 0;
  for (double t : v) {
    sum += t;
    ok += t <= bound_us;
  }
  out->count = n;
  out->on_time = ok;
  out->meets_99 = 100 * ok >= 99 * n;
  out->p50_us = rank(50);
  out->p99_us = rank(99);
  out->max_us = v.back();
  out->mean_us = sum / (double)n;
  return RXPHY_OK;
}

}  // extern "C"
