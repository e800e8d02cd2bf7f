// Host stress test of the streaming runtime's slot ring and completion
// thread (paper_2603_20481_amd/csrc/stream_ring.h), built with g++ under
// ThreadSanitizer or AddressSanitizer + UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  The device is simulated: committing a task
// arms its slot with a completion deadline a random few microseconds ahead,
// and the poller reports the task done once the deadline has passed (or
// failed, for tasks the scenario marks as failing).  The scenarios check the
// ring's contract: slots are handed out in turn, a slot is never reused
// while its task runs, every committed task gets exactly one finite,
// non-negative latency, drain waits for all of them, misuse is refused, a
// completion error is reported once, and shutdown with tasks outstanding
// waits for them.  Exit status 0 = every check passed.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_2603_20481_amd/csrc/stream_ring.h"

namespace {

std::atomic<int> failures{0};

#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

// The simulated device: per slot, the deadline of the task running on it
// (0 = idle), whether it fails, and a count of polls that saw it running.
struct Device {
  explicit Device(int depth) : deadline(depth), fail(depth), running(depth) {
    for (int i = 0; i < depth; ++i) {
      deadline[i].store(0);
      fail[i].store(false);
      running[i].store(0);
    }
  }
  std::vector<std::atomic<int64_t>> deadline;
  std::vector<std::atomic<bool>> fail;
  std::vector<std::atomic<int>> running;     // tasks armed on the slot and not yet seen done
  std::atomic<int> starts{0};
};

struct FakePoller {
  Device* dev = nullptr;
  void start() { dev->starts.fetch_add(1); }
  rxphy::Poll operator()(int i, char* msg, size_t cap) const {
    const int64_t t = dev->deadline[(size_t)i].load(std::memory_order_acquire);
    if (t == 0 || rxphy::steady_ns() < t) return rxphy::Poll::NotReady;
    dev->deadline[(size_t)i].store(0, std::memory_order_release);
    dev->running[(size_t)i].fetch_sub(1);
    if (dev->fail[(size_t)i].exchange(false)) {
      std::snprintf(msg, cap, "simulated failure on slot %d", i);
      return rxphy::Poll::Failed;
    }
    return rxphy::Poll::Done;
  }
};

using Ring = rxphy::SlotRing<FakePoller>;

// Enqueues a task on an acquired slot: arms the simulated device, then
// commits (the order of an event record followed by the commit).
void enqueue(Ring& ring, Device& dev, int slot, int64_t arrival, int64_t work_ns, bool fails) {
  CHECK(dev.running[(size_t)slot].load() == 0);        // never reused while running
  dev.running[(size_t)slot].fetch_add(1);
  dev.fail[(size_t)slot].store(fails);
  dev.deadline[(size_t)slot].store(rxphy::steady_ns() + work_ns, std::memory_order_release);
  ring.commit(slot, arrival);
}

void scenario_throughput(int depth, int tasks, unsigned seed) {
  Device dev(depth);
  Ring ring(depth);
  ring.start(FakePoller{&dev});
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> work(0, 20000);
  std::atomic<bool> done{false};
  // a reader polls the latencies while tasks complete
  std::thread reader([&] {
    std::vector<double> buf(64);
    while (!done.load()) {
      const int64_t n = ring.latencies(buf.data(), (int64_t)buf.size());
      CHECK(n >= 0);
      std::this_thread::yield();
    }
  });
  int expect = 0;
  for (int k = 0; k < tasks; ++k) {
    int slot = -1;
    CHECK(ring.acquire(&slot));
    CHECK(slot == expect);                              // handed out in turn
    expect = (expect + 1) % depth;
    const int64_t arrival = rxphy::steady_ns();
    enqueue(ring, dev, slot, arrival, work(rng), false);
  }
  char msg[320];
  CHECK(ring.drain(msg, sizeof(msg)));
  done.store(true);
  reader.join();
  std::vector<double> lat((size_t)tasks);
  CHECK(ring.latencies(lat.data(), tasks) == tasks);
  for (double t : lat) CHECK(std::isfinite(t) && t >= 0.0);
  CHECK(ring.reset_latencies() == 0);
  CHECK(ring.latencies(nullptr, 0) == 0);
  ring.shutdown();
  CHECK(dev.starts.load() == 1);
  for (int i = 0; i < depth; ++i) CHECK(dev.running[(size_t)i].load() == 0);
}

void scenario_misuse_and_failure() {
  Device dev(2);
  Ring ring(2);
  ring.start(FakePoller{&dev});
  int a = -1, b = -1, c = -1;
  CHECK(ring.acquire(&a) && a == 0);
  CHECK(ring.acquired(0) && !ring.acquired(1));
  CHECK(ring.acquire(&b) && b == 1);
  CHECK(!ring.acquire(&c));                             // slot 0 is acquired, not yet committed
  enqueue(ring, dev, a, rxphy::steady_ns(), 50000, true);
  enqueue(ring, dev, b, rxphy::steady_ns(), 1000, false);
  CHECK(ring.reset_latencies() >= 0);                   // refused or done, never torn
  char msg[320] = {0};
  CHECK(!ring.drain(msg, sizeof(msg)));                 // the failure is reported
  CHECK(std::string(msg).find("simulated failure on slot 0") != std::string::npos);
  CHECK(!ring.drain(msg, sizeof(msg)));                 // and stays reported
  std::vector<double> lat(2);
  CHECK(ring.latencies(lat.data(), 2) == 2);
  CHECK(std::isfinite(lat[0]) && std::isfinite(lat[1]));
  ring.shutdown();
}

void scenario_backpressure_and_shutdown() {
  // depth 1: acquire waits for the running task; shutdown with a task
  // outstanding waits for it.
  Device dev(1);
  Ring* ring = new Ring(1);
  ring->start(FakePoller{&dev});
  int s = -1;
  CHECK(ring->acquire(&s) && s == 0);
  enqueue(*ring, dev, s, rxphy::steady_ns(), 200000, false);
  const int64_t t0 = rxphy::steady_ns();
  CHECK(ring->acquire(&s) && s == 0);                   // blocks until the task is done
  CHECK(dev.running[0].load() == 0);
  CHECK(rxphy::steady_ns() - t0 >= 0);
  enqueue(*ring, dev, s, rxphy::steady_ns(), 100000, false);
  delete ring;                                          // shuts down after the outstanding task
  CHECK(dev.running[0].load() == 0);
}

void scenario_producers(int depth, int per_thread, int threads) {
  // several producer threads share one ring (acquire / commit are
  // serialised by the ring; each thread enqueues only slots it acquired)
  Device dev(depth);
  Ring ring(depth);
  ring.start(FakePoller{&dev});
  std::vector<std::thread> ts;
  std::atomic<int> committed{0};
  for (int t = 0; t < threads; ++t) {
    ts.emplace_back([&, t] {
      std::mt19937 rng(1000u + (unsigned)t);
      std::uniform_int_distribution<int> work(0, 5000);
      for (int k = 0; k < per_thread; ++k) {
        int slot = -1;
        while (!ring.acquire(&slot)) std::this_thread::yield();   // another thread holds the next slot
        enqueue(ring, dev, slot, rxphy::steady_ns(), work(rng), false);
        committed.fetch_add(1);
      }
    });
  }
  for (auto& th : ts) th.join();
  char msg[320];
  CHECK(ring.drain(msg, sizeof(msg)));
  std::vector<double> lat((size_t)committed.load());
  CHECK(ring.latencies(lat.data(), (int64_t)lat.size()) == committed.load());
  for (double x : lat) CHECK(std::isfinite(x) && x >= 0.0);
}

}  // namespace

int main() {
  for (int depth = 1; depth <= 4; ++depth) {
    scenario_throughput(depth, 600, 7u * (unsigned)depth);
    std::fprintf(stderr, "throughput, depth %d: done\n", depth);
  }
  scenario_misuse_and_failure();
  std::fprintf(stderr, "misuse and failure: done\n");
  scenario_backpressure_and_shutdown();
  std::fprintf(stderr, "back-pressure and shutdown: done\n");
  scenario_producers(3, 150, 4);
  std::fprintf(stderr, "four producers: done\n");
  if (failures.load()) {
    std::fprintf(stderr, "%d check(s) failed\n", failures.load());
    return 1;
  }
  std::printf("ring stress: all checks passed\n");
  return 0;
}
