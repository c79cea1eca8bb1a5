// Work plan of the reuse passes (host code).
#pragma once

#include <stddef.h>

#include <algorithm>

namespace tofh {

// Grids of the shift and visibility launches: multiples of the 64 queue
// parts, at most kShiftGrid / kVisGrid blocks of 128 lanes, one lane per
// task or ray when fewer.  The persistent visibility waves beyond the
// resident ones start as others finish, which balances the end of the
// launch (16384 blocks: 5% less visibility time than 8192 on the 512^2
// glossy scene).
constexpr unsigned kShiftGrid = 8192;
constexpr unsigned kVisGrid = 16384;
inline size_t lane_grid(size_t lanes, size_t cap) {
    return std::max<size_t>(64, std::min<size_t>(cap, ((lanes + 127) / 128 + 63) / 64 * 64));
}
inline size_t shift_grid(size_t tasks, unsigned cap = kShiftGrid) { return lane_grid(tasks, cap); }
// Scenes of at least this many triangles trace visibility with persistent
// lanes, smaller ones one ray per lane on at most kShiftGrid blocks (the box
// scenes of the serving mix: p50 latency 32.9 -> 27.7 ms that way).
constexpr int kVisPersistentMinTris = 4096;

// A reuse pass runs over chunks of items whose tasks, terms and queued rays
// fit one workspace: at most `rays` visibility rays per chunk; per mode (0
// temporal, 1 spatial, 2 bin axis) ct tasks and ci = ct / (K + 1) items per
// chunk, the shift kernels on `grid` blocks and the visibility kernel on
// `vis_grid`.
struct ChunkPlan {
    size_t rays = 0, ct[3] = {0, 0, 0}, ci[3] = {0, 0, 0}, task_cap = 0, term_cap = 0, ray_cap = 0;
    unsigned grid[3] = {0, 0, 0}, vis_grid[3] = {0, 0, 0};
};

// ray_budget > 0 lowers the budget (more, smaller chunks); a chunk still
// holds at least one sweep of the smallest grid.  shift_cap and vis_cap
// (multiples of 64; shift_cap at most kShiftGrid when `within` is given) cap
// the grids; `within`, the plan a work space was sized for, clamps every
// chunk to that plan's (a multiple of this grid's sweep, which divides it).
inline ChunkPlan plan_chunks(size_t P, size_t B, int k, int br, size_t ray_budget = 0, unsigned shift_cap = kShiftGrid,
                             unsigned vis_cap = kVisGrid, const ChunkPlan* within = nullptr) {
    ChunkPlan p;
    const int modes = br > 0 ? 3 : 2;
    const size_t K[3] = {1, (size_t)std::max(k, 1), 2 * (size_t)std::max(br, 1)};
    const size_t seg[3] = {4, 2, 2};   // visibility segments per shift: across two frames, within one
    size_t dense = 0;
    for (int m = 0; m < modes; ++m) dense = std::max(dense, seg[m] * K[m] * P * B * (K[m] + 1));
    // a sixteenth of the rays of a pass over fully occupied planes, within
    // [2^24, 2^28] rays (0.5 .. 8.6 GB of queue); a pass that needs fewer
    // than 2^24 rays in all runs as one chunk
    p.rays = std::min<size_t>((size_t)1 << 28, std::max<size_t>(std::min<size_t>(dense, (size_t)1 << 24), dense / 16));
    if (ray_budget) p.rays = std::min(p.rays, ray_budget);
    for (int m = 0; m < modes; ++m) {
        const size_t all = P * B * (K[m] + 1);
        const size_t raw = std::max<size_t>(1, std::min(p.rays / (seg[m] * K[m]), all));
        const size_t G = tofh::shift_grid(raw, shift_cap), Q = G * 128;
        // a pass whose every task fits takes one chunk (rounded up to the
        // grid), else whole grid sweeps within the budget
        p.ct[m] = raw >= all ? (all + Q - 1) / Q * Q : std::max(Q, raw / Q * Q);
        if (within) p.ct[m] = std::max(Q, std::min(p.ct[m], within->ct[m]) / Q * Q);
        p.ci[m] = std::max<size_t>(1, p.ct[m] / (K[m] + 1));
        p.grid[m] = (unsigned)G;
        p.vis_grid[m] = (unsigned)tofh::lane_grid(seg[m] * K[m] * p.ct[m], vis_cap);
        p.task_cap = std::max(p.task_cap, p.ct[m]);
        p.term_cap = std::max(p.term_cap, K[m] * p.ct[m]);
        p.ray_cap = std::max(p.ray_cap, seg[m] * K[m] * p.ct[m]);
    }
    // the shrink mapping with R < 1 runs over chunks of the spatial pass's
    // task count with two shifts, at most 4 segments, per pixel
    p.ray_cap = std::max(p.ray_cap, 4 * p.ct[1]);
    return p;
}

}  // namespace tofh
