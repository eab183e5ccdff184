// Randomized check of the serving arena allocator against a byte map.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1806_04801_amd/csrc/arena.h"

int main(int argc, char** argv) {
    const size_t cap = 1 << 18;
    hsma::Arena a(cap);
    std::vector<int> owner(cap, -1);
    struct Blk { size_t off, size; int id; };
    std::vector<Blk> live;
    unsigned seed = argc > 1 ? (unsigned)atoi(argv[1]) : 1;
    srand(seed);
    int next_id = 0;
    for (int step = 0; step < 8000; ++step) {
        if (live.empty() || rand() % 3 != 0) {
            size_t want = 1 + rand() % 12000;
            size_t off;
            if (a.alloc(want, &off)) {
                size_t rounded = (want + 255) & ~(size_t)255;
                if (off % 256 != 0 || off + rounded > cap) { printf("bad offset\n"); return 1; }
                for (size_t i = off; i < off + rounded; ++i) {
                    if (owner[i] != -1) { printf("overlap at step %d\n", step); return 1; }
                    owner[i] = next_id;
                }
                live.push_back({off, rounded, next_id++});
            } else {
                // must really be full: no free run of the rounded size
                size_t rounded = (want + 255) & ~(size_t)255, run = 0, best = 0;
                for (size_t i = 0; i < cap; ++i) { run = owner[i] == -1 ? run + 1 : 0; best = run > best ? run : best; }
                if (best >= rounded) { printf("refused with a free run of %zu >= %zu\n", best, rounded); return 1; }
            }
        } else {
            size_t k = rand() % live.size();
            Blk b = live[k];
            a.release(b.off);
            for (size_t i = b.off; i < b.off + b.size; ++i) owner[i] = -1;
            live.erase(live.begin() + k);
        }
        size_t used = 0;
        for (auto& b : live) used += b.size;
        if (used != a.used() || a.peak() < used || a.peak() > cap) { printf("accounting\n"); return 1; }
    }
    for (auto& b : live) a.release(b.off);
    size_t off;
    if (a.used() != 0 || !a.alloc(cap, &off) || off != 0) { printf("not coalesced\n"); return 1; }
    printf("ok\n");
    return 0;
}
