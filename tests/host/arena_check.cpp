// Host-only check of the serving result arena (serve_arena.h): random
// sequences of allocations and releases against a plain per-word occupancy
// map.  Every allocation must be the lowest-offset fit, never overlap a live
// block, and releasing everything must leave one free run of the whole size.
#include <cstdio>
#include <random>
#include <utility>
#include <vector>

#include "serve_arena.h"

using lap::WordArena;

int main() {
    std::mt19937_64 rng(3);
    int bad = 0;
    for (int trial = 0; trial < 200; ++trial) {
        const int64_t size = 1 + (int64_t)(rng() % 4000);
        WordArena a(size);
        std::vector<char> used((size_t)size, 0);
        std::vector<std::pair<int64_t, int64_t>> live;
        for (int op = 0; op < 400; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const int64_t w = 1 + (int64_t)(rng() % (size / 8 + 2));
                // expected: the lowest offset with w free words in a row
                int64_t want = -1;
                for (int64_t o = 0, run = 0; o < size; ++o) {
                    run = used[o] ? 0 : run + 1;
                    if (run == w) {
                        want = o - w + 1;
                        break;
                    }
                }
                const int64_t got = a.alloc(w);
                if (got != want) {
                    std::printf("trial %d: alloc(%ld) gave %ld, want %ld\n", trial, (long)w, (long)got, (long)want);
                    ++bad;
                    break;
                }
                if (got >= 0) {
                    for (int64_t o = got; o < got + w; ++o) used[o] = 1;
                    live.emplace_back(got, w);
                }
            } else {
                const size_t k = rng() % live.size();
                const auto blk = live[k];
                live.erase(live.begin() + k);
                if (!a.release(blk.first, blk.second)) ++bad;
                for (int64_t o = blk.first; o < blk.first + blk.second; ++o) used[o] = 0;
                // a second release of the same block is refused
                if (a.release(blk.first, blk.second)) ++bad;
            }
            int64_t f = 0;
            for (char c : used) f += !c;
            if (f != a.free_words()) {
                std::printf("trial %d: %ld free words, map says %ld\n", trial, (long)a.free_words(), (long)f);
                ++bad;
                break;
            }
        }
        for (auto &blk : live)
            if (!a.release(blk.first, blk.second)) ++bad;
        if (a.runs() != 1 || a.free_words() != size || a.alloc(size) != 0) {
            std::printf("trial %d: not one whole run after releasing everything\n", trial);
            ++bad;
        }
    }
    WordArena e(10);
    bad += e.release(-1, 2) || e.release(9, 2) || e.alloc(0) != -1;
    std::printf("%s (%d mismatches)\n", bad ? "FAIL" : "ok", bad);
    return bad != 0;
}
