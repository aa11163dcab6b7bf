// Host-thread model of the arrival-counter protocol of the XCD-cooperative
// passes (one plane of scratch shared by the G workgroups of an XCD).
//
// Each workgroup is a thread that owns G-th of the plane's rows and of its
// columns.  Per image it writes its rows, arrives on A, waits for G arrivals
// on A (generation nA), reads its columns, arrives on B; per subband pair it
// waits on B (every workgroup done reading), writes its columns, arrives on
// A, waits on A, reads its rows, arrives on B.  Counters only grow; a wait
// is for the G arrivals of one generation and gives up after a bounded number
// of polls, setting the abort word and an error flag, after which every other
// waiter returns at its next wait.  Arrive is a release, a completed wait an
// acquire (on the GPU: the waited-for stores are acknowledged by the L2
// before the arrive, and the reader invalidates its L1 after the wait).
//
// Every value read is checked against the value the current phase wrote, so
// a missing or misplaced wait shows up as a stale or early value.  Random
// yields and short sleeps vary the interleaving.
//
// usage: xcd_protocol_model G images pairs seed dead spin
//   dead >= 0: that workgroup stops arriving after its first phase (a
//   forced give-up); spin: polls per wait before giving up.
// Prints "ok <reads>" or "gave-up" (exit 0), or "mismatch ..." (exit 1).
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr int kLines = 4;   // rows (and columns) owned by each workgroup

struct Shared {
  int G, N;
  std::vector<std::atomic<long long>> plane;   // N x N values
  std::atomic<unsigned> A{0}, B{0}, abort{0};
  std::atomic<int> err{0};
  std::atomic<long long> reads{0};
  std::atomic<int> bad{0};
  explicit Shared(int g) : G(g), N(g * kLines), plane((size_t)g * kLines * g * kLines) {
    for (auto &v : plane) v.store(-1, std::memory_order_relaxed);
  }
};

long long tag(int image, int phase, int r, int c) {
  return (((long long)image * 4096 + phase) * 4096 + r) * 4096 + c;
}

void jitter(std::mt19937 &rng) {
  const unsigned u = rng() % 16;
  if (u == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
  else if (u < 6) std::this_thread::yield();
}

bool wait_for(Shared &s, std::atomic<unsigned> &cnt, unsigned target, long spin) {
  for (long i = 0;; ++i) {
    if (cnt.load(std::memory_order_acquire) >= target) return true;
    if (s.abort.load(std::memory_order_relaxed)) return false;
    if (i >= spin) {
      s.abort.store(1, std::memory_order_relaxed);
      s.err.store(1, std::memory_order_relaxed);
      return false;
    }
    std::this_thread::yield();
  }
}

void arrive(std::atomic<unsigned> &cnt) { cnt.fetch_add(1, std::memory_order_release); }

void workgroup(Shared &s, int w, int images, int pairs, unsigned seed, int dead, long spin) {
  std::mt19937 rng(seed * 7919u + (unsigned)w);
  const int G = s.G, N = s.N;
  unsigned nA = 0, nB = 0;
  auto at = [&](int r, int c) -> std::atomic<long long> & { return s.plane[(size_t)r * N + c]; };
  auto check = [&](int r, int c, long long want) {
    const long long got = at(r, c).load(std::memory_order_relaxed);
    s.reads.fetch_add(1, std::memory_order_relaxed);
    if (got != want) {
      if (s.bad.fetch_add(1) == 0)
        std::printf("mismatch wg %d at (%d, %d): got %lld want %lld\n", w, r, c, got, want);
    }
  };
  for (int b = 0; b < images; ++b) {
    if (!wait_for(s, s.B, (unsigned)G * nB, spin)) return;
    for (int i = 0; i < kLines; ++i) {            // rows of the image
      const int r = w * kLines + i;
      for (int c = 0; c < N; ++c) at(r, c).store(tag(b, 0, r, c), std::memory_order_relaxed);
      jitter(rng);
    }
    if (w == dead) return;                        // never arrives
    arrive(s.A);
    ++nA;
    if (!wait_for(s, s.A, (unsigned)G * nA, spin)) return;
    for (int i = 0; i < kLines; ++i) {            // columns of the spectrum
      const int c = w * kLines + i;
      for (int r = 0; r < N; ++r) check(r, c, tag(b, 0, r, c));
      jitter(rng);
    }
    arrive(s.B);
    ++nB;
    for (int p = 0; p < pairs; ++p) {
      if (!wait_for(s, s.B, (unsigned)G * nB, spin)) return;
      for (int i = 0; i < kLines; ++i) {          // column transforms of pair p
        const int c = w * kLines + i;
        for (int r = 0; r < N; ++r) at(r, c).store(tag(b, 1 + p, r, c), std::memory_order_relaxed);
        jitter(rng);
      }
      arrive(s.A);
      ++nA;
      if (!wait_for(s, s.A, (unsigned)G * nA, spin)) return;
      for (int i = 0; i < kLines; ++i) {          // row transforms of pair p
        const int r = w * kLines + i;
        for (int c = 0; c < N; ++c) check(r, c, tag(b, 1 + p, r, c));
        jitter(rng);
      }
      arrive(s.B);
      ++nB;
    }
  }
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: %s G images pairs seed dead spin\n", argv[0]);
    return 2;
  }
  const int G = std::atoi(argv[1]), images = std::atoi(argv[2]), pairs = std::atoi(argv[3]);
  const unsigned seed = (unsigned)std::atoi(argv[4]);
  const int dead = std::atoi(argv[5]);
  const long spin = std::atol(argv[6]);
  Shared s(G);
  std::vector<std::thread> th;
  for (int w = 0; w < G; ++w) th.emplace_back(workgroup, std::ref(s), w, images, pairs, seed, dead, spin);
  for (auto &t : th) t.join();
  if (s.bad.load()) return 1;
  if (s.err.load()) {
    std::printf("gave-up\n");
    return 0;
  }
  std::printf("ok %lld\n", s.reads.load());
  return 0;
}
