// Host check of the serving arena's offset bookkeeping: random alloc / release
// sequences against a brute-force byte map (no overlap, alignment, exact use
// counts, full coalescing once everything is released).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main() {
  using pico::OffsetArena;
  // fixed scenario: fill, free the middle, refill the hole exactly
  {
    OffsetArena a(4096);
    const size_t x = a.alloc(1000), y = a.alloc(1024), z = a.alloc(2048);
    CHECK(x == 0 && y == 1024 && z == 2048);
    CHECK(a.alloc(1) == OffsetArena::kNone);
    CHECK(a.release(y));
    CHECK(!a.release(y));
    CHECK(a.largest_free() == 1024);
    CHECK(a.alloc(1024) == 1024);
    CHECK(a.release(x) && a.release(z) && a.release(1024));
    CHECK(a.used() == 0 && a.free_pieces() == 1 && a.largest_free() == 4096);
  }
  std::mt19937_64 rng(12345);
  for (int trial = 0; trial < 200; ++trial) {
    const size_t cap = 256 * (1 + rng() % 400);
    OffsetArena a(cap);
    std::vector<int> owner(cap / 256, -1);     // brute-force map, one cell per 256 B
    std::vector<std::pair<size_t, size_t>> live;  // (offset, rounded length)
    size_t used = 0;
    for (int step = 0; step < 400; ++step) {
      if (live.empty() || rng() % 3) {
        const size_t want = 1 + rng() % (cap / 4 + 1);
        const size_t off = a.alloc(want);
        const size_t len = OffsetArena::round_up(want);
        // a request fails only if no free run of len bytes exists
        size_t run = 0, best = 0;
        for (size_t c = 0; c < owner.size(); ++c) {
          run = owner[c] < 0 ? run + 256 : 0;
          best = run > best ? run : best;
        }
        if (off == OffsetArena::kNone) {
          CHECK(best < len);
          continue;
        }
        CHECK(off % 256 == 0 && off + len <= cap);
        for (size_t c = off / 256; c < (off + len) / 256; ++c) {
          CHECK(owner[c] < 0);
          owner[c] = (int)live.size();
        }
        live.push_back({off, len});
        used += len;
      } else {
        const size_t i = rng() % live.size();
        CHECK(a.release(live[i].first));
        for (size_t c = live[i].first / 256; c < (live[i].first + live[i].second) / 256; ++c) owner[c] = -1;
        used -= live[i].second;
        live.erase(live.begin() + i);
        for (size_t c = 0; c < owner.size(); ++c) owner[c] = -1;
        for (size_t j = 0; j < live.size(); ++j)
          for (size_t c = live[j].first / 256; c < (live[j].first + live[j].second) / 256; ++c) owner[c] = (int)j;
      }
      CHECK(a.used() == used);
      CHECK(a.live_pieces() == live.size());
    }
    for (auto& l : live) CHECK(a.release(l.first));
    CHECK(a.used() == 0 && a.free_pieces() == 1 && a.largest_free() == a.capacity());
  }
  std::printf("arena ok\n");
  return 0;
}
