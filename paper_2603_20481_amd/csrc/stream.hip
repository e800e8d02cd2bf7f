// Real-time streaming of receiver tasks (Section III-B's bounded-latency
// rule, Section IV-D's ping-pong buffer): `depth` slots handed out in turn,
// each with its own HIP stream, completion event and buffers, and a
// completion thread that stamps every task's latency against its arrival.
// Host code only: a task is the library's own fft + csi_detect_demod calls.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace {

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
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
  bool acquired = false;        // handed out by acquire, not yet submitted
  bool busy = false;            // submitted, completion not yet seen
  int64_t task = -1;
  int64_t arrival = 0;
};

int64_t steady_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct rxphy_stream {
  rxphy_frame fr{};
  int32_t nf = 0, depth = 0, host_io = 0, device = 0;
  float sc16 = 0.f;                             // > 0: 16-bit I/Q samples with this scale
  size_t bx = 0, bp = 0, byf = 0, bws = 0, bllr = 0, bnu = 0, bfl = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::thread watcher;
  bool stop = false;
  int32_t next = 0;             // slot the next acquire hands out
  int64_t outstanding = 0;
  std::vector<double> lat;      // per submitted task, NaN until completed
  rxphy_status async_err = RXPHY_OK;
  char async_msg[256] = {0};
};

namespace {

using rxphy::fail;

// Completion thread: polls the events of busy slots (outside the lock) and
// stamps each completion with the steady clock.  It spins with yields while
// tasks are outstanding (a sleeping poll would add the timer's slack to every
// latency) and waits on the condition variable otherwise.
void watch(rxphy_stream* s) {
  hipSetDevice(s->device);
  std::vector<int> busy;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->outstanding == 0) {
      if (s->stop) return;
      s->cv.wait(lk);
      continue;
    }
    busy.clear();
    for (int i = 0; i < s->depth; ++i)
      if (s->slots[i].busy) busy.push_back(i);
    lk.unlock();
    bool any = false;
    for (int i : busy) {
      const hipError_t e = hipEventQuery(s->slots[i].done);
      if (e == hipErrorNotReady) continue;
      const int64_t t = steady_ns();
      lk.lock();
      Slot& sl = s->slots[i];
      if (e != hipSuccess && s->async_err == RXPHY_OK) {
        s->async_err = RXPHY_EHIP;
        snprintf(s->async_msg, sizeof(s->async_msg), "task %lld: %s", (long long)sl.task, hipGetErrorString(e));
      }
      s->lat[sl.task] = (double)(t - sl.arrival) * 1e-3;
      sl.busy = false;
      --s->outstanding;
      lk.unlock();
      any = true;
    }
    if (any)
      s->cv.notify_all();
    else
      std::this_thread::yield();
    lk.lock();
  }
}

void free_slot(Slot& sl) {
  if (sl.st) hipStreamDestroy(sl.st);
  if (sl.done) hipEventDestroy(sl.done);
  for (void* p : {sl.d_x, sl.d_p, sl.d_yf, sl.d_ws, (void*)sl.d_llr, (void*)sl.d_nu, (void*)sl.d_fl})
    if (p) hipFree(p);
  for (void* p : {sl.h_x, sl.h_p, (void*)sl.h_llr, (void*)sl.h_nu, (void*)sl.h_fl})
    if (p) hipHostFree(p);
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
  s->watcher = std::thread(watch, s);
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
  std::unique_lock<std::mutex> lk(s->mu);
  Slot& sl = s->slots[s->next];
  if (sl.acquired) return fail(RXPHY_EINVAL, "slot %d is acquired and not yet submitted", s->next);
  s->cv.wait(lk, [&] { return !sl.busy; });
  sl.acquired = true;
  *slot = s->next;
  s->next = (s->next + 1) % s->depth;
  return RXPHY_OK;
}

rxphy_status rxphy_stream_submit(rxphy_stream* s, int32_t slot, int64_t arrival_ns, const void* x,
                                 const void* pilots, float* llr, float* nu, uint8_t* flags) {
  rxphy::clear_error();
  if (!s) return fail(RXPHY_EINVAL, "stream is NULL");
  if (slot < 0 || slot >= s->depth) return fail(RXPHY_EINVAL, "slot = %d (0 .. %d)", slot, s->depth - 1);
  if (arrival_ns < 0) return fail(RXPHY_EINVAL, "arrival_ns = %lld", (long long)arrival_ns);
  Slot& sl = s->slots[slot];
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!sl.acquired) return fail(RXPHY_EINVAL, "slot %d was not acquired", slot);
  }
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
  {
    std::lock_guard<std::mutex> lk(s->mu);
    sl.acquired = false;
    sl.busy = true;
    sl.task = (int64_t)s->lat.size();
    sl.arrival = arrival_ns ? arrival_ns : t_sub;
    s->lat.push_back(NAN);
    ++s->outstanding;
  }
  s->cv.notify_all();
  return RXPHY_OK;
}

rxphy_status rxphy_stream_drain(rxphy_stream* s) {
  rxphy::clear_error();
  if (!s) return fail(RXPHY_EINVAL, "stream is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&] { return s->outstanding == 0; });
  if (s->async_err) return fail(s->async_err, "%s", s->async_msg);
  return RXPHY_OK;
}

rxphy_status rxphy_stream_latencies(rxphy_stream* s, double* lat_us, int64_t cap, int64_t* n) {
  rxphy::clear_error();
  if (!s || !n || cap < 0 || (cap > 0 && !lat_us)) return fail(RXPHY_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  const int64_t m = (int64_t)s->lat.size();
  if (cap > 0) std::copy(s->lat.begin(), s->lat.begin() + std::min(cap, m), lat_us);
  *n = m;
  return RXPHY_OK;
}

rxphy_status rxphy_stream_reset_latencies(rxphy_stream* s) {
  rxphy::clear_error();
  if (!s) return fail(RXPHY_EINVAL, "stream is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->outstanding) return fail(RXPHY_EINVAL, "%lld task(s) outstanding", (long long)s->outstanding);
  s->lat.clear();
  return RXPHY_OK;
}

void rxphy_stream_destroy(rxphy_stream* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->outstanding == 0; });
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->watcher.joinable()) s->watcher.join();
  destroy_all(s);
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
