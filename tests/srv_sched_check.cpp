// Randomised check of the serving engine's arena allocator against a
// brute-force model of the byte range, and of the request footprint layout.
// Built with the host compiler only; prints "OK" on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "srv_sched.h"

using lrnr::srv::Arena;

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);     \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main() {
  std::mt19937_64 rng(12345);
  for (int trial = 0; trial < 50; ++trial) {
    const int64_t size = 256 * (64 + rng() % 4096);
    Arena a(size);
    std::vector<char> owner(size / 256, 0);  // 1 = allocated
    struct Blk { int64_t off, bytes; };
    std::vector<Blk> live;
    for (int op = 0; op < 2000; ++op) {
      if (live.empty() || rng() % 3 != 0) {
        const int64_t bytes = 1 + rng() % (size / 8);
        const int64_t off = a.alloc(bytes);
        const int64_t n = lrnr::srv::align_up(bytes);
        // brute force: does any free aligned run of n bytes exist?
        bool fits = false;
        for (int64_t s = 0, run = 0; s < size / 256 && !fits; ++s) {
          run = owner[s] ? 0 : run + 1;
          fits = run * 256 >= n;
        }
        if (off < 0) {
          CHECK(!fits);
          continue;
        }
        CHECK(off % 256 == 0 && off + n <= size);
        for (int64_t s = off / 256; s < (off + n) / 256; ++s) {
          CHECK(owner[s] == 0);
          owner[s] = 1;
        }
        live.push_back({off, bytes});
      } else {
        const size_t i = rng() % live.size();
        a.release(live[i].off, live[i].bytes);
        const int64_t n = lrnr::srv::align_up(live[i].bytes);
        for (int64_t s = live[i].off / 256; s < (live[i].off + n) / 256; ++s) owner[s] = 0;
        live.erase(live.begin() + i);
      }
      int64_t used = 0;
      for (char c : owner) used += c ? 256 : 0;
      CHECK(a.used() == used);
      CHECK(a.peak() >= a.used());
    }
    for (const Blk& b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0);
    CHECK(a.free_blocks() == 1 && a.largest_free() == a.size());  // fully coalesced
  }
  // footprint: disjoint, aligned, ordered regions covering the total
  for (int64_t n : {0, 1, 255, 256, 1024, 4097, 65536}) {
    const auto f = lrnr::srv::footprint(n, n / 8, n / 8, 27, 292, 25600, 256, 128);
    const int64_t offs[] = {f.xt, f.x0, f.tb, f.s, f.m, f.v, f.mu, f.loss, f.step, f.partials, f.u,
                            f.total};
    for (int i = 0; i + 1 < 12; ++i) CHECK(offs[i] % 256 == 0 && offs[i] < offs[i + 1]);
    CHECK(f.x0 - f.xt >= n * 8 && f.u - f.partials >= (int64_t)f.tiles * 292 * 4);
    CHECK(f.total - f.u >= 25600 * 4);
    CHECK(f.v - f.m == f.m - f.s);
    const int64_t tiles = (n + 255) / 256 + (n / 8 + 255) / 256 + (n / 8 + 127) / 128;
    CHECK(f.tiles == tiles);
  }
  std::printf("OK\n");
  return 0;
}
