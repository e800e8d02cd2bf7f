// Slot ring and completion thread of the real-time streaming runtime
// (Section III-B's bounded-latency rule, Section IV-D's ping-pong buffer),
// host code only: no HIP here, so the same state machine is built both into
// the library (polling HIP events) and into a host test program (polling a
// simulated device) that runs under ThreadSanitizer and AddressSanitizer.
//
// `depth` slots are handed out in turn by acquire, which blocks while the
// next slot's previous task is still running (back-pressure).  A task is
// committed on its slot after its work has been enqueued; the completion
// thread polls the busy slots outside the lock and stamps each completion
// with the steady clock against the task's arrival time.  Latencies are kept
// per task in commit order (NaN until the task completes).
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>

namespace rxphy {

inline int64_t steady_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// What the poller reports for a busy slot.
enum class Poll { NotReady, Done, Failed };

// Poller: a copyable callable `Poll operator()(int slot, char* msg, size_t cap)`,
// called only by the completion thread, never under the ring's lock; on
// Failed it writes a message.  `void start()` runs once on the completion
// thread before the first poll (e.g. to select the device).
template <class Poller>
class SlotRing {
 public:
  explicit SlotRing(int depth) : st_((size_t)depth), depth_(depth) {}
  SlotRing(const SlotRing&) = delete;
  SlotRing& operator=(const SlotRing&) = delete;
  ~SlotRing() { shutdown(); }

  int depth() const { return depth_; }

  // Starts the completion thread (once).
  void start(Poller poller) {
    watcher_ = std::thread([this, poller]() mutable { watch(poller); });
  }

  // Hands out the next slot in turn, waiting while its previous task runs.
  // Returns false, and changes nothing, if that slot is acquired and not yet
  // committed (the caller must submit it first).  The next slot is looked up
  // again after every wait: with several producers another one may have
  // taken it meanwhile.
  bool acquire(int* slot) {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      State& s = st_[(size_t)next_];
      if (s.acquired) return false;
      if (!s.busy) {
        s.acquired = true;
        *slot = next_;
        next_ = (next_ + 1) % depth_;
        return true;
      }
      cv_.wait(lk);
    }
  }

  bool acquired(int slot) {
    std::lock_guard<std::mutex> lk(mu_);
    return st_[(size_t)slot].acquired;
  }

  // The task on an acquired slot has been enqueued (its completion marker
  // recorded): from now on the completion thread polls it.
  void commit(int slot, int64_t arrival_ns) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      State& s = st_[(size_t)slot];
      s.acquired = false;
      s.busy = true;
      s.task = (int64_t)lat_.size();
      s.arrival = arrival_ns;
      lat_.push_back(NAN);
      ++outstanding_;
    }
    cv_.notify_all();
  }

  // Waits until no task is outstanding; returns false with the first
  // completion error's message if any task failed.
  bool drain(char* msg, size_t cap) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return outstanding_ == 0; });
    if (failed_) snprintf(msg, cap, "%s", err_);
    return !failed_;
  }

  // Copies up to cap latencies (us, commit order); returns how many exist.
  int64_t latencies(double* out, int64_t cap) {
    std::lock_guard<std::mutex> lk(mu_);
    const int64_t m = (int64_t)lat_.size();
    if (cap > 0) std::copy(lat_.begin(), lat_.begin() + std::min(cap, m), out);
    return m;
  }

  // Clears the latencies; refused (returns the count) while tasks are outstanding.
  int64_t reset_latencies() {
    std::lock_guard<std::mutex> lk(mu_);
    if (outstanding_ == 0) lat_.clear();
    return outstanding_;
  }

  // Waits for every outstanding task, then stops and joins the completion thread.
  void shutdown() {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return outstanding_ == 0; });
      stop_ = true;
    }
    cv_.notify_all();
    if (watcher_.joinable()) watcher_.join();
  }

 private:
  struct State {
    bool acquired = false;   // handed out by acquire, not yet committed
    bool busy = false;       // committed, completion not yet seen
    int64_t task = -1;
    int64_t arrival = 0;
  };

  // Spins with yields while tasks are outstanding (a sleeping poll would add
  // the timer's slack to every latency); waits on the condition otherwise.
  void watch(Poller& poll) {
    poll.start();
    std::vector<int> busy;
    char msg[256];
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      if (outstanding_ == 0) {
        if (stop_) return;
        cv_.wait(lk);
        continue;
      }
      busy.clear();
      for (int i = 0; i < depth_; ++i)
        if (st_[(size_t)i].busy) busy.push_back(i);
      lk.unlock();
      bool any = false;
      for (int i : busy) {
        msg[0] = 0;
        const Poll p = poll(i, msg, sizeof(msg));
        if (p == Poll::NotReady) continue;
        const int64_t t = steady_ns();
        lk.lock();
        State& s = st_[(size_t)i];
        if (p == Poll::Failed && !failed_) {
          failed_ = true;
          snprintf(err_, sizeof(err_), "task %lld: %s", (long long)s.task, msg);
        }
        lat_[(size_t)s.task] = (double)(t - s.arrival) * 1e-3;
        s.busy = false;
        --outstanding_;
        lk.unlock();
        any = true;
      }
      if (any)
        cv_.notify_all();
      else
        std::this_thread::yield();
      lk.lock();
    }
  }

  std::vector<State> st_;
  const int depth_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::thread watcher_;
  bool stop_ = false;
  int next_ = 0;
  int64_t outstanding_ = 0;
  std::vector<double> lat_;
  bool failed_ = false;
  char err_[320] = {0};
};

}  // namespace rxphy
