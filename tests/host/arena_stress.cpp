// Host-side stress test of the arena allocator (rtm_arena.h), built with the
// sanitizers by tests/test_host_logic.py.  Checks, against a model of the
// live blocks: 256-byte alignment, no overlap, exact used-byte accounting,
// null on exhaustion, full coalescing after everything is released, and (in
// the threaded mode) the same under concurrent alloc/release.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <cstdlib>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "rtm_arena.h"

static int fail(const char* what, long a = 0, long b = 0) {
  std::fprintf(stderr, "FAIL: %s (%ld, %ld)\n", what, a, b);
  std::exit(1);
}

static int single(size_t arena_size, int ops, unsigned seed) {
  std::vector<char> backing(arena_size + 256);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(backing.data()) + 255) & ~uintptr_t(255));
  rtm::Arena a;
  a.init(base, arena_size);
  std::map<char*, size_t> live;  // pointer -> rounded size
  std::mt19937_64 rng(seed);
  size_t used = 0, nulls = 0;
  for (int i = 0; i < ops; ++i) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      size_t n = 1 + rng() % (arena_size / 16);
      if (rng() % 10 == 0) n = 1 + rng() % 300;  // small blocks too
      char* p = static_cast<char*>(a.alloc(n));
      const size_t r = rtm::align256(n);
      if (!p) {
        ++nulls;
        continue;
      }
      if ((p - base) % 256 != 0) fail("alignment", p - base);
      if (p < base || p + r > base + arena_size) fail("out of range", p - base, r);
      auto nx = live.lower_bound(p);
      if (nx != live.end() && p + r > nx->first) fail("overlap with next", p - base, nx->first - base);
      if (nx != live.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second > p) fail("overlap with previous", pv->first - base, p - base);
      }
      std::memset(p, 0xAB, r);  // ASan: the whole rounded block is ours
      live[p] = r;
      used += r;
    } else {
      auto it = live.begin();
      std::advance(it, rng() % live.size());
      a.release(it->first, it->second);
      used -= it->second;
      live.erase(it);
    }
    if (a.used() != used) fail("used bytes", (long)a.used(), (long)used);
  }
  for (auto& kv : live) a.release(kv.first, kv.second);
  if (a.used() != 0) fail("used after release", (long)a.used());
  // everything coalesced: the whole arena is one free range again
  void* all = a.alloc(arena_size & ~size_t(255));
  if (all != base) fail("no full-size block after release");
  if (a.alloc(1) != nullptr) fail("allocation beyond a full arena");
  a.release(all, arena_size & ~size_t(255));
  std::printf("single: %d ops, %zu exhausted allocations, peak %zu of %zu\n", ops, nulls, a.peak(), arena_size);
  return 0;
}

static int threaded(size_t arena_size, int threads, int ops) {
  std::vector<char> backing(arena_size + 256);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(backing.data()) + 255) & ~uintptr_t(255));
  rtm::Arena a;
  a.init(base, arena_size);
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&, t] {
      std::mt19937_64 rng(1234 + t);
      std::vector<std::pair<char*, size_t>> mine;
      for (int i = 0; i < ops; ++i) {
        if (mine.empty() || rng() % 2) {
          size_t n = 1 + rng() % 4096;
          char* p = static_cast<char*>(a.alloc(n));
          if (p) {
            std::memset(p, t, rtm::align256(n));  // a block owned by two threads would race here
            mine.push_back({p, n});
          }
        } else {
          size_t k = rng() % mine.size();
          a.release(mine[k].first, mine[k].second);
          mine[k] = mine.back();
          mine.pop_back();
        }
      }
      for (auto& m : mine) a.release(m.first, m.second);
    });
  for (auto& t : ts) t.join();
  if (a.used() != 0) fail("threaded: used after release", (long)a.used());
  if (a.alloc(arena_size & ~size_t(255)) != base) fail("threaded: not coalesced");
  std::printf("threaded: %d threads x %d ops, peak %zu\n", threads, ops, a.peak());
  return 0;
}

int main(int argc, char** argv) {
  const bool thr = argc > 1 && std::string(argv[1]) == "threaded";
  if (thr) return threaded(1 << 20, 8, 20000);
  single(1 << 20, 200000, 1);
  single((1 << 20) + 100, 50000, 2);  // size not a multiple of 256
  return 0;
}
