// Host-side launchers of the library's kernels (internal; not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "tof_device.h"

namespace tofh {

struct FrameArgs {
    tofd::Sens s;
    tofd::SceneDev S;
    tofd::Frames F;
    uint32_t frame;
    unsigned long long* counters;   // kNumCounters x u64
};

// bvh_host.hip (host code): 4-wide tree topology over axis-aligned boxes (binned SAH,
// then a collapse of the binary tree).  Leaf references are
// 0x80000000 | (count - 1) << 28 | first slot, count <= 8.
struct BvhPrim {
    float lo[3], hi[3];
};
int32_t leaf_ref(int first, int count);
int32_t build_bvh4(const std::vector<BvhPrim>& prims, int leaf_max, int node_base, int slot_base,
                   std::vector<tofd::Node4>& nodes, std::vector<int>& heights, std::vector<int>& order);

// bvh.hip
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
void launch_world_verts(const float4* lv, const int* vobj, const float* xf, float4* wv, int nv, hipStream_t st);
void launch_leaf_gather(const int* leaf_tri, const int4* tv, const float4* wv, int T, float4* leaves,
                        hipStream_t st);
// boxes of the nodes order[level_off[l] .. level_off[l+1]) for l = 0, 1, ...
// (children before parents)
void launch_refit(tofd::Node4* nodes, const uint32_t* order, const std::vector<int>& level_off,
                  const float4* leaves, int T, hipStream_t st);

// render.hip
struct GBufOut {
    int* obj;
    float* xi0;
    float* xi1;
    float4* p;
    float4* n;
};
void launch_gbuffer(const FrameArgs& a, GBufOut out, hipStream_t st);
void launch_initial(const FrameArgs& a, tofd::ResSet can, float* pt, float2* direct, hipStream_t st);
void launch_reproject(const FrameArgs& a, const tofd::ResSet& can, const tofd::ResSet& prev, int* prev_pix,
                      float* M_out, hipStream_t st);
void launch_neighbours(const FrameArgs& a, int round, const tofd::ResSet& in, int* nb, float* M_out,
                       hipStream_t st);
// Work items (pixel, plane | cmask << 16) for every plane non-empty in any of
// the ncand candidates, the index of each item's first task, and one
// (item, candidate) task per non-empty candidate; count[0] = items,
// count[1] = tasks.
void launch_items(const FrameArgs& a, int mode, const tofd::ResSet& first, const tofd::ResSet& second,
                  const int* links, int ncand, uint2* items, uint32_t* task0, uint2* tasks, uint32_t* count,
                  uint32_t* out_mask, hipStream_t st);
// Grids of the shift and visibility launches.  The shift kernels run a
// fixed grid of G blocks of 128 lanes (G a multiple of the 64 queue parts, at
// most kShiftGrid) in a grid-stride loop over chunks of tasks that are
// multiples of G * 128 (the chunk quantum): every sub-queue then receives the
// work of exactly chunk / 64 tasks.  Small passes get a small grid, so that
// their queues stay small.
constexpr unsigned kShiftGrid = 8192;
constexpr unsigned kVisGrid = 8192;
inline size_t chunk_quantum(size_t tasks) {
    const size_t blocks = std::min<size_t>(kShiftGrid, ((tasks + 127) / 128 + 63) / 64 * 64);
    return std::max<size_t>(blocks, 64) * 128;
}

// Shifts of a reuse pass, over a chunk of their index range: the forward
// shifts into q of tasks [t_begin, t_end) (fwd[t], shv[2t..2t+1]), then the MIS
// shifts (task, neighbour) g in [g_begin, g_end) into every neighbour domain
// (term[g]).  Each shift queues its visibility segments in q; launch_vis traces
// them in the frame of `slot` and zeroes kill[owner] for blocked ones.  A
// chunk must not queue more rays than q.cap (at most 4 per shift).
void launch_fwd(const FrameArgs& a, int mode, const tofd::ResSet& A, const tofd::ResSet& Bp, const int* links,
                const uint2* items, const uint2* tasks, const uint32_t* count, size_t t_begin, size_t t_end,
                float4* fwd, float4* shv, const tofd::RayQueue& q, unsigned grid, hipStream_t st);
// MIS shifts of tasks [t_begin, t_end): the pairs (task, neighbour) that need
// one are listed in lq (at most K per task), then shifted.
void launch_mis(const FrameArgs& a, int mode, const tofd::ResSet& A, const tofd::ResSet& Bp, const int* links,
                const uint2* items, const uint2* tasks, const uint32_t* count, size_t t_begin, size_t t_end,
                const float4* fwd, const float4* shv, float* term, const tofd::IdxQueue& lq,
                const tofd::RayQueue& q, unsigned grid, hipStream_t st);
void launch_vis(const FrameArgs& a, int slot, const tofd::RayQueue& q, float* kill, hipStream_t st);
// Weighted reservoir merge of each item's candidates into `out`.
void launch_merge(const FrameArgs& a, int mode, const tofd::ResSet& A, const tofd::ResSet& Bp, const int* links,
                  const uint2* items, const uint32_t* task0, const uint32_t* count, size_t max_items,
                  const float4* fwd, const float* term, const float4* shv, int round, tofd::ResSet out,
                  hipStream_t st);
void launch_splat(const FrameArgs& a, const tofd::ResSet& shown, const float* pt, const float2* direct,
                  float* out_image, float* out_hist, float* out_pt_image, float* out_pt_hist, hipStream_t st);

}  // namespace tofh
