// Host-only randomized check of the server's arena allocator: live blocks
// never overlap, stay aligned and inside the arena, the free list stays
// disjoint and merged, and freeing everything restores one free block.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "arena.h"

static int fail(const char *what, unsigned long long a, unsigned long long b) {
  std::printf("FAIL %s %llu %llu\n", what, a, b);
  return 1;
}

int main(int argc, char **argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  std::mt19937_64 rng(seed);
  for (int round = 0; round < 40; ++round) {
    const uint64_t align = 1ull << (rng() % 9);
    const uint64_t size = 1 + rng() % (1ull << 22);
    alnrt::Arena a;
    a.reset(size, align);
    if (a.size() % align || a.size() > size || size - a.size() >= align)
      return fail("size", a.size(), size);
    std::map<uint64_t, uint64_t> live; // off -> rounded length
    for (int step = 0; step < 3000; ++step) {
      if (live.empty() || rng() % 3) {
        const uint64_t want = rng() % 4 ? rng() % 4096 : rng() % (size / 2 + 1);
        uint64_t off = 0;
        const bool could = a.fits(want);
        const bool ok = a.alloc(want, &off);
        if (ok != could) return fail("fits disagrees with alloc", want, ok);
        if (!ok) continue;
        const uint64_t len = a.round_up(want ? want : 1);
        if (off % align) return fail("misaligned", off, align);
        if (off + len > a.size()) return fail("past end", off + len, a.size());
        auto nx = live.lower_bound(off);
        if (nx != live.end() && off + len > nx->first) return fail("overlaps next", off, nx->first);
        if (nx != live.begin()) {
          auto pv = std::prev(nx);
          if (pv->first + pv->second > off) return fail("overlaps previous", pv->first, off);
        }
        live[off] = len;
      } else {
        auto it = live.begin();
        std::advance(it, (long)(rng() % live.size()));
        if (!a.release(it->first)) return fail("release", it->first, 0);
        if (a.release(it->first)) return fail("double release accepted", it->first, 0);
        live.erase(it);
      }
      uint64_t used = 0;
      for (auto &l : live) used += l.second;
      if (used != a.used()) return fail("used", used, a.used());
      if (a.live_blocks() != live.size()) return fail("live blocks", a.live_blocks(), live.size());
      // free list: gaps between live blocks, merged (count = non-empty gaps)
      size_t gaps = 0;
      uint64_t cur = 0, largest = 0;
      for (auto &l : live) {
        if (l.first > cur) { ++gaps; largest = std::max(largest, l.first - cur); }
        cur = l.first + l.second;
      }
      if (a.size() > cur) { ++gaps; largest = std::max(largest, a.size() - cur); }
      if (a.free_blocks() != gaps) return fail("free blocks not merged", a.free_blocks(), gaps);
      if (a.largest_free() != largest) return fail("largest free", a.largest_free(), largest);
    }
    for (auto &l : live) a.release(l.first);
    if (a.used() != 0 || a.free_blocks() != (a.size() ? 1u : 0u))
      return fail("not restored", a.used(), a.free_blocks());
  }
  std::printf("OK\n");
  return 0;
}
