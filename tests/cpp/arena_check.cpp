// Randomised check of the serving loop's best-fit arena allocator (lk_arena.hpp):
// no overlap, alignment, exact accounting, full coalescing, best-fit choice, and failure
// only when no free block is large enough.  Prints "OK" and exits 0 on success.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "lk_arena.hpp"

using lksrv::Arena;

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      exit(1);                                                     \
    }                                                              \
  } while (0)

struct Live {
  uint64_t addr, bytes;
};

static void check_state(const Arena &a, uint64_t base, const std::vector<Live> &live) {
  uint64_t used = 0;
  for (const Live &l : live) used += Arena::round(l.bytes ? l.bytes : 1);
  CHECK(a.used() == used);
  uint64_t free_total = 0, prev_end = 0;
  bool first = true;
  a.for_each_free([&](uint64_t off, uint64_t len) {
    CHECK(len > 0 && off % Arena::kGranule == 0 && len % Arena::kGranule == 0);
    if (!first) CHECK(off > prev_end);  // sorted and never touching: fully coalesced
    first = false;
    prev_end = off + len;
    free_total += len;
    for (const Live &l : live) {  // free blocks never overlap live ones
      const uint64_t lo = l.addr - base, hi = lo + Arena::round(l.bytes ? l.bytes : 1);
      CHECK(hi <= off || lo >= off + len);
    }
  });
  CHECK(prev_end <= a.size());
  CHECK(free_total + used == a.size());
}

int main(int argc, char **argv) {
  const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
  const uint64_t base = 1ull << 40, size = (64ull << 20) + 768;  // not a granule multiple
  Arena a(base, size);
  CHECK(a.size() == size / Arena::kGranule * Arena::kGranule);
  CHECK(a.free_blocks() == 1 && a.largest_free() == a.size());
  std::mt19937_64 rng(seed);
  std::vector<Live> live;
  for (int step = 0; step < 20000; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      // log-uniform sizes 1 B .. 4 MiB, plus exact granule multiples
      const int sh = static_cast<int>(rng() % 23);
      uint64_t bytes = (rng() % 4 == 0) ? ((rng() % 64) + 1) * Arena::kGranule : 1 + rng() % (1ull << sh);
      const uint64_t need = Arena::round(bytes);
      // best fit expected: smallest free length >= need, lowest offset among equals
      uint64_t best_len = 0, best_off = 0;
      a.for_each_free([&](uint64_t off, uint64_t len) {
        if (len >= need && (best_len == 0 || len < best_len)) {
          best_len = len;
          best_off = off;
        }
      });
      uint64_t addr = 0;
      const bool ok = a.alloc(bytes, &addr);
      CHECK(ok == (best_len != 0));
      if (ok) {
        CHECK(addr - base == best_off);
        CHECK(addr % Arena::kGranule == 0 && addr >= base && addr + need <= base + a.size());
        for (const Live &l : live) {
          const uint64_t hi = l.addr + Arena::round(l.bytes);
          CHECK(addr + need <= l.addr || addr >= hi);
        }
        live.push_back({addr, bytes});
      }
    } else {
      const size_t k = rng() % live.size();
      a.release(live[k].addr, live[k].bytes);
      live[k] = live.back();
      live.pop_back();
    }
    if (step % 97 == 0) check_state(a, base, live);
  }
  check_state(a, base, live);
  CHECK(a.peak() >= a.used());
  while (!live.empty()) {
    a.release(live.back().addr, live.back().bytes);
    live.pop_back();
  }
  check_state(a, base, live);
  CHECK(a.free_blocks() == 1 && a.largest_free() == a.size() && a.used() == 0);
  // exhaustion: fill with granules, then one more fails; release every other one and a
  // two-granule request still fails (no two adjacent free granules), a one-granule fits
  Arena b(0, 16 * Arena::kGranule);
  std::vector<uint64_t> g;
  uint64_t x;
  while (b.alloc(1, &x)) g.push_back(x);
  CHECK(g.size() == 16 && !b.alloc(1, &x));
  for (size_t i = 0; i < g.size(); i += 2) b.release(g[i], 1);
  CHECK(b.free_blocks() == 8 && !b.alloc(2 * Arena::kGranule, &x) && b.alloc(Arena::kGranule, &x));
  printf("OK\n");
  return 0;
}
