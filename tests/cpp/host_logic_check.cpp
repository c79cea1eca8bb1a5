// Host logic of the library checked on the CPU: the serving arena's best-fit
// allocator against a brute-force model of its 256-byte units, and the work
// plan of the reuse passes against the bounds the kernels rely on.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"
#include "chunk_plan.h"

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);   \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static void arena_check() {
    const size_t units = 4096, U = 256;
    tofh::Arena a;
    a.reset(units * U);
    std::vector<int> owner(units, -1);   // brute-force model: which block holds each unit
    struct Blk { size_t off, bytes; int id; };
    std::vector<Blk> live;
    std::mt19937_64 rng(7);
    int next_id = 0;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 3 != 0);
        if (do_alloc) {
            const size_t bytes = 1 + rng() % (64 * U);
            const size_t need = (bytes + U - 1) / U;
            // the best hole in the model: smallest free run of at least `need` units
            size_t best_len = 0, run = 0;
            for (size_t u = 0; u <= units; ++u) {
                if (u < units && owner[u] < 0) {
                    ++run;
                    continue;
                }
                if (run >= need && (best_len == 0 || run < best_len)) best_len = run;
                run = 0;
            }
            size_t off = 0;
            const bool ok = a.alloc(bytes, off);
            CHECK(ok == (best_len > 0));
            if (!ok) continue;
            CHECK(off % U == 0 && off / U + need <= units);
            size_t hole = 0;   // the chosen hole is free in the model and is a best fit
            for (size_t u = off / U; u < off / U + need; ++u) CHECK(owner[u] < 0);
            size_t lo = off / U, hi = off / U;
            while (lo > 0 && owner[lo - 1] < 0) --lo;
            while (hi < units && owner[hi] < 0) ++hi;
            hole = hi - lo;
            CHECK(hole == best_len);
            for (size_t u = off / U; u < off / U + need; ++u) owner[u] = next_id;
            live.push_back({off, bytes, next_id++});
        } else {
            const size_t i = rng() % live.size();
            const Blk b = live[i];
            a.free(b.off, b.bytes);
            for (size_t u = b.off / U; u < b.off / U + (b.bytes + U - 1) / U; ++u) owner[u] = -1;
            live[i] = live.back();
            live.pop_back();
        }
        // the largest hole agrees with the model
        size_t best = 0, run = 0;
        for (size_t u = 0; u <= units; ++u) {
            if (u < units && owner[u] < 0) {
                ++run;
                continue;
            }
            best = run > best ? run : best;
            run = 0;
        }
        CHECK(a.largest() == best * U);
    }
    for (const Blk& b : live) a.free(b.off, b.bytes);
    CHECK(a.largest() == units * U);   // everything coalesced back into one hole
}

static void plan_check() {
    const size_t seg[3] = {4, 2, 2};
    for (size_t P : {(size_t)1, (size_t)4096, (size_t)(40 * 24), (size_t)(128 * 128), (size_t)(512 * 512),
                     (size_t)(1024 * 1024)})
        for (size_t B : {(size_t)1, (size_t)17, (size_t)65, (size_t)257})
            for (int k : {0, 3, 5, 8})
                for (int br : {0, 1, 4}) {
                    const tofh::ChunkPlan p = tofh::plan_chunks(P, B, k, br);
                    const size_t K[3] = {1, (size_t)(k > 1 ? k : 1), 2 * (size_t)(br > 1 ? br : 1)};
                    size_t dense = 0;
                    for (int m = 0; m < (br > 0 ? 3 : 2); ++m) {
                        const size_t d = seg[m] * K[m] * P * B * (K[m] + 1);
                        dense = d > dense ? d : dense;
                    }
                    CHECK(p.rays <= ((size_t)1 << 28));
                    CHECK(p.rays >= (dense < ((size_t)1 << 24) ? dense : ((size_t)1 << 24)) || p.rays == ((size_t)1 << 28));
                    for (int m = 0; m < (br > 0 ? 3 : 2); ++m) {
                        const size_t G = p.grid[m];
                        CHECK(G >= 64 && G <= tofh::kShiftGrid && G % 64 == 0);
                        CHECK(p.vis_grid[m] >= 64 && p.vis_grid[m] <= tofh::kVisGrid && p.vis_grid[m] % 64 == 0);
                        // a chunk is a whole number of grid sweeps: every sub-queue takes ct / 64 tasks at most
                        CHECK(p.ct[m] % (G * 128) == 0);
                        CHECK(p.ci[m] >= 1 && p.ci[m] * (K[m] + 1) <= p.ct[m]);
                        CHECK(p.task_cap >= p.ct[m] && p.term_cap >= K[m] * p.ct[m]);
                        CHECK(p.ray_cap >= seg[m] * K[m] * p.ct[m]);
                        // 32-bit queue slots and pair indices
                        CHECK(p.ray_cap < ((size_t)1 << 32) && K[m] * p.ct[m] < ((size_t)1 << 32));
                        // a pass that fits the ray budget runs as one chunk
                        if (dense <= ((size_t)1 << 24)) CHECK(p.ci[m] >= P * B);
                    }
                    // a lowered budget (test support) still gives whole grid
                    // sweeps and fits the default plan's work space
                    for (size_t rays : {(size_t)1, (size_t)81920, (size_t)1 << 20}) {
                        const tofh::ChunkPlan q = tofh::plan_chunks(P, B, k, br, rays);
                        CHECK(q.task_cap <= p.task_cap && q.term_cap <= p.term_cap && q.ray_cap <= p.ray_cap);
                        for (int m = 0; m < (br > 0 ? 3 : 2); ++m) {
                            CHECK(q.ct[m] % ((size_t)q.grid[m] * 128) == 0 && q.ct[m] <= p.ct[m]);
                            CHECK(q.ci[m] >= 1 && q.ci[m] * (K[m] + 1) <= q.ct[m]);
                        }
                    }
                    // any launch shape within the work space (tof_set_launch_config,
                    // tof_autotune): whole sweeps of its own grid, no chunk larger
                    // than the default plan's, grids within their caps
                    for (unsigned sb : {64u, 192u, 2048u, 4096u, tofh::kShiftGrid})
                        for (unsigned vb : {64u, 4096u, 32768u, 65536u})
                            for (size_t rays : {(size_t)0, (size_t)81920}) {
                                const tofh::ChunkPlan q = tofh::plan_chunks(P, B, k, br, rays, sb, vb, &p);
                                CHECK(q.task_cap <= p.task_cap && q.term_cap <= p.term_cap && q.ray_cap <= p.ray_cap);
                                for (int m = 0; m < (br > 0 ? 3 : 2); ++m) {
                                    CHECK(q.grid[m] >= 64 && q.grid[m] <= sb && q.grid[m] % 64 == 0);
                                    CHECK(q.vis_grid[m] >= 64 && q.vis_grid[m] <= vb && q.vis_grid[m] % 64 == 0);
                                    CHECK(q.ct[m] % ((size_t)q.grid[m] * 128) == 0 && q.ct[m] <= p.ct[m]);
                                    CHECK(q.ci[m] >= 1 && q.ci[m] * (K[m] + 1) <= q.ct[m]);
                                }
                            }
                }
}

int main() {
    arena_check();
    plan_check();
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
