// Host-side launchers of the library's kernels (internal; not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "chunk_plan.h"
#include "tof.h"
#include "tof_device.h"

namespace tofh {

// Contexts whose memory an owner hands over (the serving loop): device memory
// [dev, dev + dev_bytes) and pinned host memory [host, host + host_bytes) that
// the context fills front to back (scene, then sensor; a later re-upload or
// sensor change can reclaim only the group allocated last).  Destroying such
// a context frees nothing and waits for its own frames only, not for the
// device.  dev_bytes from tof_footprint, host_bytes from scene_pinned_bytes.
tof_status create_in_region(tof_ctx** out, int device, void* dev, size_t dev_bytes, void* host, size_t host_bytes,
                            uint64_t seed);
// before recording a frame of tof_render_frame under stream capture: wait for
// the pinned upload slot the frame may reuse (an event recorded on the stream
// being captured cannot be waited for during the capture)
tof_status prepare_frame_capture(tof_ctx* c);
// after launching a graph recorded from tof_render_frame under stream capture:
// record on `st` the events the capture left out (the upload ring's and the
// frame's end), which the context's host waits use, and take the frame's
// splat as having cleared the plain-PT deposits (the next frame skips its fill)
tof_status record_frame_events(tof_ctx* c, hipStream_t st);
size_t scene_pinned_bytes(const tof_scene_desc& d);

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

// bvh_build.hip: the objects' 4-wide trees built on the device (Morton
// order, agglomerative clustering, SAH leaves, the host's collapse rule).
// Mesh object m owns leaf slots [m_slot[m], m_slot[m + 1]) and triangles
// m_tri[m] + 0 .. ; nodes are numbered from node_base; leaf_tri[slot] is
// written on the device.  heights: a refit level per node (children in lower
// levels than their parents).  The workspace (blas_build_bytes) is device
// memory the caller owns; the null stream is used and left idle.
struct BlasResult {
    std::vector<tofd::Node4> nodes;   // child links and counts (boxes are the refit's)
    std::vector<int> heights;
    std::vector<int> roots;           // per mesh object: node or leaf reference, -1 without triangles
    std::vector<float> lbox;          // per mesh object: object-space box lo xyz, hi xyz
    int rounds = 0;                   // clustering rounds
    double build_ms = 0.0;
};
size_t blas_build_bytes(size_t T, size_t M);
tof_status build_blas_device(void* work, size_t work_bytes, const int4* tv, const float4* lv,
                             const std::vector<int>& m_slot, const std::vector<int>& m_tri, int node_base,
                             int* leaf_tri, BlasResult& res);

// bvh.hip
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
// wv = world positions, wr = vertices turned into world orientation about their object's origin
void launch_world_verts(const float4* lv, const int* vobj, const float* xf, float4* wv, float4* wr, int nv,
                        hipStream_t st);
void launch_leaf_gather(const int* leaf_tri, const int4* tv, const float4* wv, int T, float4* leaves,
                        hipStream_t st);
// boxes of the nodes order[level_off[l] .. level_off[l+1]) for l = 0, 1, ...
// (children before parents)
void launch_refit(tofd::Node4* nodes, tofd::NodeQ* nq, const uint32_t* order, const std::vector<int>& level_off,
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
// wide: the wide-gate reservoirs of the shrink mapping with R < 1 (rec only,
// P records), or rec == nullptr
void launch_initial(const FrameArgs& a, tofd::ResSet can, tofd::ResSet wide, float* pt, float2* direct,
                    hipStream_t st);
void launch_reproject(const FrameArgs& a, const tofd::ResSet& can, const tofd::ResSet& prev, int* prev_pix,
                      float* M_out, hipStream_t st);
void launch_neighbours(const FrameArgs& a, int round, const tofd::ResSet& in, int* nb, float* M_out,
                       hipStream_t st);
// Work items (pixel, plane | cmask << 16) for every plane non-empty in any of
// the ncand candidates and the index of each item's first task (one task per
// non-empty candidate); count[0] = items, count[1] = tasks.  Task indices grow
// with the item index.
// wsum: [2P] work space for the per-pixel summaries of non-zero mask words
// of `first` and `second` (the passes over pixels' own planes read only the
// words a candidate holds samples in).
void launch_items(const FrameArgs& a, int mode, const tofd::ResSet& first, const tofd::ResSet& second,
                  const int* links, int ncand, uint2* items, uint32_t* task0, uint32_t* count, uint32_t* out_mask,
                  uint32_t* wsum, hipStream_t st);

// A reuse pass runs over chunks of ci items; the chunk's tasks, forward and
// MIS terms and queued rays live in a workspace sized for the chunk
// (chunk_plan.h).  The shift kernels run a fixed grid of G blocks of 128
// lanes (G a multiple of the 64 queue parts) in a grid-stride loop over at
// most ct tasks, ct a multiple of G * 128, so that every sub-queue receives
// the work of at most ct / 64 tasks.

// Tasks of items [i0, i0 + ci) into tasks[] (chunk-relative), and the
// chunk's window win = (first task, task count).
void launch_tasks(const uint2* items, const uint32_t* task0, const uint32_t* count, size_t i0, size_t ci,
                  uint2* tasks, uint32_t* win, hipStream_t st);
// Forward shifts into q of the chunk's tasks t (fwd[t], shv[2t..2t+1]).  Each
// shift queues its visibility segments in q; launch_vis traces them in the
// frame of `slot` and zeroes kill[owner] for blocked ones.
void launch_fwd(const FrameArgs& a, int mode, const tofd::ResSet& A, const tofd::ResSet& Bp, const int* links,
                const uint2* items, const uint2* tasks, const uint32_t* win, float4* fwd, float4* shv,
                const tofd::RayQueue& q, unsigned grid, hipStream_t st);
// MIS shifts of the chunk's tasks: the pairs (task, neighbour) g = t * K + l
// that need one are listed in lq (at most K per task), then shifted (term[g]).
void launch_mis(const FrameArgs& a, int mode, const tofd::ResSet& A, const tofd::ResSet& Bp, const int* links,
                const uint2* items, const uint2* tasks, const uint32_t* win, const float4* fwd, const float4* shv,
                float* term, const tofd::IdxQueue& lq, const tofd::RayQueue& q, unsigned grid, hipStream_t st);
// waves: the occupancy variant of the persistent visibility kernel (5 or 6 waves per SIMD)
void launch_vis(const FrameArgs& a, int slot, const tofd::RayQueue& q, float* kill, unsigned grid, int waves,
                hipStream_t st);
// Weighted reservoir merge of the candidates of items [i0, i0 + ci) into `out`.
void launch_merge(const FrameArgs& a, int mode, const tofd::ResSet& A, const tofd::ResSet& Bp, const int* links,
                  const uint2* items, const uint2* tasks, const uint32_t* task0, const uint32_t* count, size_t i0,
                  size_t ci,
                  const uint32_t* win, const float4* fwd, const float* term, const float4* shv, int round,
                  tofd::ResSet out, int tile, hipStream_t st);
// Shrink mapping of the gate reservoirs of pixels [p0, p0 + np) (at most 2
// visibility segments each, queued in q) and, after their visibility, the
// emptying of the failed ones.
void launch_shrink(const FrameArgs& a, const tofd::ResSet& can, size_t p0, size_t np, const tofd::RayQueue& q,
                   unsigned grid, hipStream_t st);
void launch_shrink_fin(const FrameArgs& a, const tofd::ResSet& can, hipStream_t st);
// Shrink mapping with R < 1: per pixel of [p0, p0 + np) the expansion of the
// gate sample and the shrink of the wide sample (at most 4 visibility
// segments, owners 4 t and 4 t + 1 in scr as floats), then, after their
// visibility, the GRIS merge of the two into the gate.
void launch_shrink_mix(const FrameArgs& a, const tofd::ResSet& can, const tofd::ResSet& wide, size_t p0, size_t np,
                       const tofd::RayQueue& q, float4* scr, unsigned grid, hipStream_t st);
void launch_shrink_mix_fin(const FrameArgs& a, const tofd::ResSet& can, const tofd::ResSet& wide, size_t p0,
                           size_t np, const float4* scr, hipStream_t st);
// Records and mask bits of plane pl copied from `in` to `out` (the gate plane
// across the bin-axis pass).
void launch_copy_plane(const FrameArgs& a, const tofd::ResSet& in, const tofd::ResSet& out, int pl, hipStream_t st);
// clear_pt: the plain-PT deposits are set back to zero as they are read
void launch_splat(const FrameArgs& a, const tofd::ResSet& shown, float* pt, bool clear_pt, const float2* direct,
                  float* out_image, float* out_hist, float* out_pt_image, float* out_pt_hist, hipStream_t st);

}  // namespace tofh
