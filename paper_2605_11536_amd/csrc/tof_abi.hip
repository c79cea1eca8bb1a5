// C ABI of the ToF ReSTIR library: context, scene upload, sensor set,
// frame driver and statistics.  See include/tof.h for the contract.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "tof.h"
#include "chunk_plan.h"
#include "tof_internal.h"

using namespace tofd;

namespace {

// event counters: one bank of kBank u64 per kernel group, summed by tof_get_stats
constexpr int kBank = 16;
static_assert(kNumCounters <= kBank, "counter bank too small");
constexpr size_t kCounterBytes = (size_t)TOF_K_COUNT * kBank * sizeof(unsigned long long);

struct Alloc {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    size_t off0 = SIZE_MAX;   // in a region: offset of the first allocation
};

struct GeomBuf {
    float* xf = nullptr;
    float* vel = nullptr;        // [6 * objects]: linear and angular velocity (velocity domain)
    float4* wv = nullptr;
    float4* wr = nullptr;        // vertices in world orientation about their object's origin
    Node4* nodes = nullptr;      // [n_nodes]: the tree over the objects, then the objects' trees
    NodeQ* nodesq = nullptr;     // [n_nodes]: the same nodes quantized, as traversal reads them
    uint32_t* order = nullptr;   // refit order: object-tree nodes by height, then the top tree's
    float4* leaves = nullptr;
    std::vector<float> xf_host;
    std::vector<float> vel_host;   // velocity domain: what vel holds
    bool built = false;
};

struct SlotHost {
    bool valid = false;
    int geom = 0;
    float gate_c = 0.f;   // gate centre the frame was rendered with
    V3 cam_pos, cam_fwd, cam_right, cam_up;
    float tan_half = 0, aspect = 1, ohx = 0, ohy = 0;
    V3 light_pos;
    V3 cam_vel, light_vel;
    int* gb_obj = nullptr;
    float* gb_xi0 = nullptr;
    float* gb_xi1 = nullptr;
    float4* gb_p = nullptr;
    float4* gb_n = nullptr;
};

}  // namespace

struct tof_ctx {
    int device = 0;
    size_t budget = 0;
    uint64_t seed = 0;
    Alloc scene_mem, sensor_mem;
    Alloc build_mem;                     // the device tree builder's work space during an upload
    int bvh_builder = TOF_BVH_HOST;
    tof_bvh_info bvh_info = {};
    // scene
    bool has_scene = false;
    int n_obj = 0, n_mat = 0, n_vert = 0, n_tri = 0, n_sph = 0;
    float scale = 1.f;
    std::vector<Obj> h_objs;
    Obj* d_objs = nullptr;
    Mat* d_mats = nullptr;
    TriInfo* d_tri = nullptr;
    int* d_sph = nullptr;
    float4* d_lv = nullptr;
    int* d_vobj = nullptr;
    int4* d_tv = nullptr;
    // acceleration structure: the objects' 4-wide trees (topology built once,
    // boxes refit per frame) under a per-frame tree over the objects
    int* d_leaf_tri = nullptr;         // [T] triangle of each leaf slot
    std::vector<int> mesh_objs;        // objects with triangles
    std::vector<int32_t> blas_root;    // per mesh object: root reference of its tree
    std::vector<float> obj_lbox;       // per mesh object: object-space box lo xyz, hi xyz
    std::vector<int> level_off;        // refit levels of the objects' trees (offsets into order)
    int n_tlas_cap = 0, n_blas = 0, n_nodes = 0;
    size_t pinned_bytes = 0;
    GeomBuf geom[2];
    // sensor
    bool has_sensor = false;
    tof_sensor_desc sd{};
    Sens s{};
    SlotHost slot[2];
    // 0 canonical; 1 and 2: the previous frame's final (fin_prev) and a
    // scratch set.  Once the temporal pass has read the previous final, its
    // set is free, so the later passes alternate between 1 and 2 and the new
    // final ends in one of them.
    ResSet sets[3];
    int fin_prev = 2;
    bool prev_valid = false;
    float* pt = nullptr;
    float2* direct = nullptr;
    int* prev_pix = nullptr;
    uint32_t* wsum = nullptr;  // [2P]: per pixel, the mask words that are non-zero (work-list pass)
    bool pt_zero = false;      // pt holds zeros (the last frame's splat cleared what it read)
    bool pt_zero_pending = false;   // a captured frame's splat: pt_zero once its graph is launched
    int* nb = nullptr;
    uint2* items = nullptr;    // [max_items]
    uint32_t* task0 = nullptr; // [max_items]: first task of each item
    // workspace of one item chunk (sizes in plan)
    uint2* tasks = nullptr;    // [task_cap]
    float4* fwd = nullptr;     // [task_cap]: forward-shift terms per task
    float4* wide = nullptr;    // [kRecF4 P]: wide-gate reservoirs of the shrink mapping with R < 1, else none
    float4* shv = nullptr;     // [2 * task_cap]: fields rewritten by each forward shift
    float* term = nullptr;     // [term_cap]: MIS terms per (task, neighbour)
    float4* rays = nullptr;    // [2 * ray_cap]: queued visibility segments
    uint32_t* ray_count = nullptr;
    uint32_t* mis_list = nullptr;   // [term_cap]: (task, neighbour) pairs of one chunk
    uint32_t* mis_count = nullptr;
    uint32_t* count = nullptr;      // [0] items, [1] tasks, [2..3] window of the current chunk
    size_t max_items = 0;
    tofh::ChunkPlan alloc_plan;   // the plan the chunk work space was sized for
    tofh::ChunkPlan plan;         // the plan the passes run: alloc_plan's chunks or smaller
    // launch shape (tof_set_launch_config): most blocks of the shift kernels
    // and of the visibility kernel
    unsigned shift_blocks = tofh::kShiftGrid, vis_blocks = tofh::kVisGrid;
    int vis_waves = 6, merge_tasks = 2;   // occupancy variant of k_vis, tile of k_merge
    size_t ray_budget = 0;        // a lowered ray budget (test support), 0 = the plan's own
    // a pass that may need more than one chunk reads its item count back and
    // launches only the chunks that hold items (contexts of tof_create; a
    // server context never waits in its dispatch, and launches them all)
    bool sync_counts = false;
    uint32_t* count_host = nullptr;   // pinned: the item count of the current pass
    // misc
    unsigned long long* counters = nullptr;
    float* xf_pinned[2] = {nullptr, nullptr};
    hipEvent_t xf_ev[2] = {nullptr, nullptr};
    int xf_ring = 0;
    uint64_t frames = 0;
    // region mode: device and pinned host memory handed over by the owner,
    // filled front to back (no hipMalloc / hipFree of its own)
    char* rbase = nullptr;
    size_t rsize = 0, rused = 0;
    char* hbase = nullptr;
    size_t hsize = 0;
    hipEvent_t done = nullptr;   // recorded after each frame on its stream
    bool capturing = false;      // the frame being issued is recorded by stream capture
    int xf_pending = -1;         // a captured frame's upload-ring event, for record_frame_events
    bool done_pending = false;   // a captured frame's end event, likewise
    bool has_work = false;
    // kernel timing: event pairs recorded in order, reduced on query
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_kernel;
    std::vector<uint32_t*> item_counts;    // device copies of the work-list sizes
    uint32_t* item_hist = nullptr;         // [2 * max_frames] temporal/spatial counts
    size_t item_slots = 0, item_used = 0;
    double acc_ms[TOF_K_COUNT] = {};
    uint64_t acc_n[TOF_K_COUNT] = {};
    uint64_t acc_items[4] = {};
    unsigned long long work0[TOF_K_COUNT * kBank] = {};   // counters when timing was enabled
};

namespace {

// wait for the context's own last frame (not for other work on the device)
hipError_t quiesce(tof_ctx* c) { return c->has_work ? hipEventSynchronize(c->done) : hipSuccess; }

tof_status dev_alloc(tof_ctx* c, Alloc& a, void** out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (c->budget && c->scene_mem.bytes + c->sensor_mem.bytes + c->build_mem.bytes + bytes > c->budget)
        return TOF_ERR_OUT_OF_MEMORY;
    if (c->rbase) {
        if (c->rused + bytes > c->rsize) return TOF_ERR_OUT_OF_MEMORY;
        if (a.off0 == SIZE_MAX) a.off0 = c->rused;
        *out = c->rbase + c->rused;
        c->rused += bytes;
        a.ptrs.push_back(*out);
        a.bytes += bytes;
        return TOF_OK;
    }
    if (hipMalloc(out, bytes) != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return TOF_ERR_OUT_OF_MEMORY;
    }
    a.ptrs.push_back(*out);
    a.bytes += bytes;
    return TOF_OK;
}

// in a region the space is reclaimed when the group is the last one allocated
void free_all(tof_ctx* c, Alloc& a) {
    if (c->rbase) {
        if (a.off0 != SIZE_MAX && a.off0 + a.bytes == c->rused) c->rused = a.off0;
    } else {
        for (void* p : a.ptrs) (void)hipFree(p);
    }
    a.ptrs.clear();
    a.bytes = 0;
    a.off0 = SIZE_MAX;
}

template <typename T>
tof_status alloc_t(tof_ctx* c, Alloc& a, T** out, size_t count) {
    void* p = nullptr;
    tof_status st = dev_alloc(c, a, &p, sizeof(T) * count);
    *out = (T*)p;
    return st;
}

#define TOF_TRY(expr)                    \
    do {                                 \
        tof_status _st = (expr);         \
        if (_st != TOF_OK) return _st;   \
    } while (0)
#define HIP_TRY(expr)                                    \
    do {                                                 \
        if ((expr) != hipSuccess) {                      \
            (void)hipGetLastError();                     \
            return TOF_ERR_DEVICE;                       \
        }                                                \
    } while (0)

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

V3 hv(float a, float b, float c) { return V3{a, b, c}; }
V3 hnorm(V3 a) {
    float l = std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
    return V3{a.x / l, a.y / l, a.z / l};
}
V3 hcross(V3 a, V3 b) { return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

constexpr size_t kRecBytes = 4 * kRecWords;   // one reservoir record


// path trees whose gate candidates come from the wide gate of the shrink
// mapping (R x M_init), 0 when the shrink mapping is off
int wide_trees(const tof_sensor_desc& d) {
    if (!d.gate_enabled || !(d.shrink_k > 1.f)) return 0;
    return (int)std::lround(std::min(1.0, std::max(0.0, (double)d.shrink_r)) * (double)d.m_init);
}
// R < 1: a wide-gate reservoir per pixel besides the gate's own
bool shrink_mix(const tof_sensor_desc& d) {
    const int w = wide_trees(d);
    return w > 0 && w < d.m_init;
}

size_t sensor_footprint(const tof_sensor_desc& d) {
    size_t P = (size_t)d.width * d.height;
    size_t B = (size_t)d.n_bins + (d.gate_enabled ? 1 : 0);
    size_t words = (B + 31) / 32;
    size_t per_set = P * B * kRecBytes + P * 4 + P * words * 4;
    size_t gbuf = 2 * P * (4 + 4 + 4 + 16 + 16);
    const tofh::ChunkPlan pl = tofh::plan_chunks(P, B, d.spatial_k, d.bin_radius);
    return 3 * per_set + gbuf + P * B * 4 /*pt*/ + P * 8 /*direct*/ + P * 4 /*prev*/ + P * 8 /*word summaries*/ +
           P * 4 * (size_t)std::max(d.spatial_k, 1) + P * B * 8 /*items*/ + P * B * 4 /*first task per item*/ +
           pl.task_cap * (8 + 16 + 32) /*tasks, forward terms, shifted fields*/ +
           pl.term_cap * (4 + 4) /*MIS terms, MIS work list*/ + 32 * pl.ray_cap +
           (shrink_mix(d) ? P * kRecBytes : 0) /*wide-gate reservoirs*/ + 64 * 1024;
}

// pinned staging of one frame: transforms, the tree over the objects and its
// refit order, then the velocities
size_t pinned_slot_bytes(size_t n_obj, size_t n_tlas_cap) {
    return (sizeof(float) * 18 * n_obj + (sizeof(Node4) + sizeof(uint32_t)) * n_tlas_cap + 255) & ~(size_t)255;
}

// upper bound of the device memory tof_scene_upload allocates for a scene
size_t scene_footprint(const tof_scene_desc& d) {
    size_t T = 0, mesh = 0;
    for (int o = 0; o < d.num_objects; ++o)
        if (d.object_type[o] == TOF_OBJ_GRID) {
            T += 2 * (size_t)std::max(d.object_grid[5 * o], 0) * (size_t)std::max(d.object_grid[5 * o + 1], 0);
            ++mesh;
        }
    const size_t V = (size_t)std::max(d.num_vertices, 1), O = (size_t)d.num_objects, N = mesh + T + 1;
    return O * (sizeof(Obj) + 4) + (size_t)d.num_materials * sizeof(Mat) + T * (sizeof(TriInfo) + 16 + 4) +
           V * (16 + 4) + 2 * (72 * O + 32 * V + (sizeof(Node4) + sizeof(NodeQ) + 4) * N + 48 * std::max<size_t>(T, 1)) +
           tofh::blas_build_bytes(T, mesh) + 64 * 1024;
}

tof_status alloc_set(tof_ctx* c, ResSet& r, size_t P, size_t B, size_t words) {
    Alloc& a = c->sensor_mem;
    TOF_TRY(alloc_t(c, a, &r.rec, P * B * kRecF4));
    TOF_TRY(alloc_t(c, a, &r.M, P));
    TOF_TRY(alloc_t(c, a, &r.mask, P * words));
    return TOF_OK;
}

// start/stop of one timed launch group (no-ops unless timing is on)
hipError_t timer_mark(tof_ctx* c, int kernel, hipStream_t st) {
    if (!c->timing) return hipSuccess;
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        c->ev_pool.push_back(e);
        c->ev_kernel.push_back(-1);
    }
    c->ev_kernel[c->ev_used] = kernel;
    return hipEventRecord(c->ev_pool[c->ev_used++], st);
}

void timer_reduce(tof_ctx* c) {
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]) == hipSuccess) {
            int k = c->ev_kernel[i];
            c->acc_ms[k] += ms;
            c->acc_n[k] += 1;
        }
    }
    (void)hipGetLastError();
    c->ev_used = 0;
}

SlotDev slot_dev(const tof_ctx* c, int i) {
    const SlotHost& h = c->slot[i];
    const GeomBuf& g = c->geom[h.geom];
    SlotDev d;
    d.wr = g.wr;
    d.xf = g.xf;
    d.nodes = g.nodesq;
    d.n_nodes = c->n_nodes;
    d.leaves = g.leaves;
    d.n_tri = c->n_tri;
    d.cam_pos = h.cam_pos;
    d.cam_fwd = h.cam_fwd;
    d.cam_right = h.cam_right;
    d.cam_up = h.cam_up;
    d.tan_half = h.tan_half;
    d.aspect = h.aspect;
    d.ohx = h.ohx;
    d.ohy = h.ohy;
    d.light_pos = h.light_pos;
    d.vel = g.vel;
    d.cam_vel = h.cam_vel;
    d.light_vel = h.light_vel;
    d.gate_c = h.gate_c;
    d.gb_obj = h.gb_obj;
    d.gb_xi0 = h.gb_xi0;
    d.gb_xi1 = h.gb_xi1;
    d.gb_p = h.gb_p;
    d.gb_n = h.gb_n;
    return d;
}

}  // namespace

extern "C" {

const char* tof_status_string(tof_status s) {
    switch (s) {
        case TOF_OK: return "ok";
        case TOF_ERR_INVALID_ARG: return "invalid argument";
        case TOF_ERR_OUT_OF_MEMORY: return "out of memory (HBM budget or hipMalloc)";
        case TOF_ERR_INVALID_SCENE: return "invalid scene";
        case TOF_ERR_NOT_READY: return "scene or sensor not set";
        case TOF_ERR_DEVICE: return "HIP device error";
        case TOF_ERR_UNIMPLEMENTED: return "unimplemented";
    }
    return "unknown status";
}

tof_status tof_footprint(const tof_scene_desc* scene, const tof_sensor_desc* sensor, size_t* bytes) {
    if (!scene || !sensor || !bytes || scene->num_objects < 1 || !scene->object_type || !scene->object_grid)
        return TOF_ERR_INVALID_ARG;
    *bytes = scene_footprint(*scene) + sensor_footprint(*sensor);
    return TOF_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// The work space of tof_render_frame_noalloc: one file-scope device array per
// GPU (each device that loads the library holds its own copy until the process
// ends).  Host code never names the array as an address: its device address is
// looked up once per device with hipGetSymbolAddress (at the first tof_create
// on that device, with the device current) and kept in g_scratch.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr unsigned kMaxVisBlocks = 65536;   // most blocks a launch shape may give the visibility kernel
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxScratchDevices] = {};

// the device address of `scratch` on `device`, which must be current
static hipError_t scratch_ptr(int device, void** ptr) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = p;
    }
    *ptr = g_scratch[device];
    return hipSuccess;
}

tof_status make_ctx(tof_ctx** out, int device, size_t budget, uint64_t seed, void* dev, size_t dev_bytes, void* host,
                    size_t host_bytes) {
    if (!out) return TOF_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        (void)hipGetLastError();
        return TOF_ERR_DEVICE;
    }
    if (device < 0 || device >= ndev) return TOF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(device));
    {   // resolve the no-allocation work space of this device once
        void* p = nullptr;
        HIP_TRY(scratch_ptr(device, &p));
    }
    tof_ctx* c = new (std::nothrow) tof_ctx();
    if (!c) return TOF_ERR_OUT_OF_MEMORY;
    c->device = device;
    c->budget = budget;
    c->seed = seed;
    c->rbase = (char*)dev;
    c->rsize = dev_bytes;
    c->hbase = (char*)host;
    c->hsize = host_bytes;
    bool ok = true;
    if (c->rbase) {
        Alloc own;
        ok = dev_alloc(c, own, (void**)&c->counters, kCounterBytes) == TOF_OK;
    } else {
        ok = hipMalloc(&c->counters, kCounterBytes) == hipSuccess;
    }
    // the null-stream fill must be complete before any stream reads the counters
    ok = ok && hipMemset(c->counters, 0, kCounterBytes) == hipSuccess && hipStreamSynchronize(nullptr) == hipSuccess &&
         hipEventCreateWithFlags(&c->done, hipEventDisableTiming) == hipSuccess;
    if (ok && !c->hbase) {
        c->sync_counts = true;
        ok = hipHostMalloc((void**)&c->count_host, 64) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        if (c->counters && !c->rbase) (void)hipFree(c->counters);
        if (c->count_host) (void)hipHostFree(c->count_host);
        if (c->done) (void)hipEventDestroy(c->done);
        delete c;
        return TOF_ERR_DEVICE;
    }
    *out = c;
    return TOF_OK;
}

// the passes' chunk plan for the context's launch shape and a ray budget (0:
// the default), within the work space sized at tof_sensor_set
tofh::ChunkPlan plan_of(const tof_ctx* c, size_t rays) {
    return tofh::plan_chunks((size_t)c->s.P, (size_t)c->s.B, c->s.k, c->s.br, rays, c->shift_blocks, c->vis_blocks,
                             &c->alloc_plan);
}
}  // namespace

namespace tofh {

tof_status create_in_region(tof_ctx** out, int device, void* dev, size_t dev_bytes, void* host, size_t host_bytes,
                            uint64_t seed) {
    if (!dev || !dev_bytes || !host || !host_bytes) return TOF_ERR_INVALID_ARG;
    return make_ctx(out, device, dev_bytes, seed, dev, dev_bytes, host, host_bytes);
}

tof_status prepare_frame_capture(tof_ctx* c) {
    HIP_TRY(hipSetDevice(c->device));
    if (c->xf_ev[c->xf_ring]) HIP_TRY(hipEventSynchronize(c->xf_ev[c->xf_ring]));
    return TOF_OK;
}

tof_status record_frame_events(tof_ctx* c, hipStream_t st) {
    if (c->xf_pending >= 0) {
        HIP_TRY(hipEventRecord(c->xf_ev[c->xf_pending], st));
        c->xf_pending = -1;
    }
    if (c->done_pending) {
        HIP_TRY(hipEventRecord(c->done, st));
        c->done_pending = false;
    }
    if (c->pt_zero_pending) {
        c->pt_zero = true;
        c->pt_zero_pending = false;
    }
    return TOF_OK;
}

size_t scene_pinned_bytes(const tof_scene_desc& d) {
    size_t mesh = 0;
    for (int o = 0; o < d.num_objects; ++o) mesh += d.object_type[o] == TOF_OBJ_GRID ? 1 : 0;
    return 2 * pinned_slot_bytes((size_t)d.num_objects, std::max<size_t>(mesh, 1));
}

}  // namespace tofh

extern "C" {

tof_status tof_create(tof_ctx** out, int device, size_t hbm_budget_bytes, uint64_t seed) {
    return make_ctx(out, device, hbm_budget_bytes, seed, nullptr, 0, nullptr, 0);
}

void tof_destroy(tof_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->rbase) {   // nothing to free: wait for the context's own work only
        (void)quiesce(c);
        for (int i = 0; i < 2; ++i)
            if (c->xf_ev[i]) (void)hipEventSynchronize(c->xf_ev[i]);
    } else {
        (void)hipDeviceSynchronize();
        free_all(c, c->scene_mem);
        free_all(c, c->sensor_mem);
        if (c->counters) (void)hipFree(c->counters);
    }
    for (int i = 0; i < 2; ++i) {
        if (c->xf_pinned[i] && !c->hbase) (void)hipHostFree(c->xf_pinned[i]);
        if (c->xf_ev[i]) (void)hipEventDestroy(c->xf_ev[i]);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->done) (void)hipEventDestroy(c->done);
    if (c->count_host) (void)hipHostFree(c->count_host);
    delete c;
}

tof_status tof_scene_upload(tof_ctx* c, const tof_scene_desc* d) {
    if (!c || !d) return TOF_ERR_INVALID_ARG;
    if (d->num_objects < 1 || d->num_objects > kMaxObjects || d->num_materials < 1 || d->num_vertices < 0 ||
        !d->object_type || !d->object_material || !d->object_grid || !d->object_sphere || !d->material_type ||
        !d->material_params || (d->num_vertices > 0 && !d->vertices))
        return TOF_ERR_INVALID_ARG;
    if (!(std::isfinite(d->scene_scale) && d->scene_scale > 0.f)) return TOF_ERR_INVALID_SCENE;
    for (int v = 0; v < d->num_vertices; ++v)
        if (!finite3(d->vertices + 3 * v)) return TOF_ERR_INVALID_SCENE;
    std::vector<Mat> mats(d->num_materials);
    for (int m = 0; m < d->num_materials; ++m) {
        const float* p = d->material_params + 3 * m;
        mats[m] = Mat{d->material_type[m], p[0], p[1], p[2]};
        bool ok = finite3(p) && (mats[m].type == TOF_MAT_LAMBERT || mats[m].type == TOF_MAT_GGX) &&
                  p[0] >= 0.f && p[0] <= 1.f && (mats[m].type == TOF_MAT_LAMBERT || (p[1] > 0.f && p[2] >= 0.f && p[2] <= 1.f));
        if (!ok) return TOF_ERR_INVALID_SCENE;
    }
    std::vector<Obj> objs(d->num_objects);
    std::vector<TriInfo> tris;
    std::vector<int> sph;
    std::vector<int> vobj(d->num_vertices, -1);
    std::vector<int4> tv;
    for (int o = 0; o < d->num_objects; ++o) {
        Obj ob{};
        ob.type = d->object_type[o];
        ob.material = d->object_material[o];
        if (ob.material < 0 || ob.material >= d->num_materials) return TOF_ERR_INVALID_SCENE;
        const int32_t* g = d->object_grid + 5 * o;
        const float* sp = d->object_sphere + 4 * o;
        ob.tri_base = (int)tris.size();
        if (ob.type == TOF_OBJ_GRID) {
            ob.nu = g[0];
            ob.nv = g[1];
            ob.wrap_u = g[2] ? 1 : 0;
            ob.wrap_v = g[3] ? 1 : 0;
            ob.voff = g[4];
            if (ob.nu < 1 || ob.nv < 1 || ob.nu > 65535 || ob.nv > 65535 || ob.voff < 0) return TOF_ERR_INVALID_SCENE;
            long long nvtx = (long long)(ob.nu + 1) * (ob.nv + 1);
            if (ob.voff + nvtx > d->num_vertices) return TOF_ERR_INVALID_SCENE;
            // leaf references hold a 28-bit first slot
            if ((long long)tris.size() + 2LL * ob.nu * ob.nv >= (1LL << 28)) return TOF_ERR_INVALID_SCENE;
            for (long long q = 0; q < nvtx; ++q) vobj[ob.voff + q] = o;
            int row = ob.nu + 1;
            for (int j = 0; j < ob.nv; ++j)
                for (int i = 0; i < ob.nu; ++i) {
                    int b = ob.voff + j * row + i;
                    tris.push_back(TriInfo{o, i, j, 0});
                    tv.push_back(make_int4(b, b + 1, b + row, 0));
                    tris.push_back(TriInfo{o, i, j, 1});
                    tv.push_back(make_int4(b + row + 1, b + row, b + 1, 0));
                }
        } else if (ob.type == TOF_OBJ_SPHERE) {
            if (!finite3(sp) || !(std::isfinite(sp[3]) && sp[3] > 0.f)) return TOF_ERR_INVALID_SCENE;
            ob.cx = sp[0];
            ob.cy = sp[1];
            ob.cz = sp[2];
            ob.r = sp[3];
            sph.push_back(o);
        } else {
            return TOF_ERR_INVALID_SCENE;
        }
        objs[o] = ob;
    }
    // a vertex referenced by two grids would get two transforms
    for (int o = 0; o < d->num_objects; ++o) {
        const Obj& ob = objs[o];
        if (ob.type != TOF_OBJ_GRID) continue;
        long long nvtx = (long long)(ob.nu + 1) * (ob.nv + 1);
        for (long long q = 0; q < nvtx; ++q)
            if (vobj[ob.voff + q] != o) return TOF_ERR_INVALID_SCENE;
    }
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    free_all(c, c->scene_mem);
    c->has_scene = false;
    c->prev_valid = false;
    c->slot[0].valid = c->slot[1].valid = false;
    for (auto& g : c->geom) g = GeomBuf();
    const int T = (int)tris.size();
    Alloc& a = c->scene_mem;
    TOF_TRY(alloc_t(c, a, &c->d_objs, objs.size()));
    TOF_TRY(alloc_t(c, a, &c->d_mats, mats.size()));
    TOF_TRY(alloc_t(c, a, &c->d_tri, std::max(T, 1)));
    TOF_TRY(alloc_t(c, a, &c->d_tv, std::max(T, 1)));
    TOF_TRY(alloc_t(c, a, &c->d_sph, std::max<size_t>(sph.size(), 1)));
    TOF_TRY(alloc_t(c, a, &c->d_lv, std::max(d->num_vertices, 1)));
    TOF_TRY(alloc_t(c, a, &c->d_vobj, std::max(d->num_vertices, 1)));
    std::vector<float4> lv(d->num_vertices);
    for (int v = 0; v < d->num_vertices; ++v)
        lv[v] = make_float4(d->vertices[3 * v], d->vertices[3 * v + 1], d->vertices[3 * v + 2], 0.f);
    HIP_TRY(hipMemcpy(c->d_objs, objs.data(), sizeof(Obj) * objs.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_mats, mats.data(), sizeof(Mat) * mats.size(), hipMemcpyHostToDevice));
    if (T) {
        HIP_TRY(hipMemcpy(c->d_tri, tris.data(), sizeof(TriInfo) * T, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_tv, tv.data(), sizeof(int4) * T, hipMemcpyHostToDevice));
    }
    if (!sph.empty()) HIP_TRY(hipMemcpy(c->d_sph, sph.data(), sizeof(int) * sph.size(), hipMemcpyHostToDevice));
    if (d->num_vertices) {
        HIP_TRY(hipMemcpy(c->d_lv, lv.data(), sizeof(float4) * lv.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_vobj, vobj.data(), sizeof(int) * vobj.size(), hipMemcpyHostToDevice));
    }
    // objects' trees: binned SAH over each mesh object's triangles in object
    // space, leaves of at most 4 triangles, leaf slots object after object
    c->mesh_objs.clear();
    c->blas_root.clear();
    c->obj_lbox.clear();
    std::vector<Node4> blas;
    std::vector<int> heights, leaf_tri(T), order;
    int n_mesh = 0;
    for (int o = 0; o < d->num_objects; ++o) n_mesh += objs[o].type == TOF_OBJ_GRID ? 1 : 0;
    c->n_tlas_cap = std::max(n_mesh, 1);
    TOF_TRY(alloc_t(c, a, &c->d_leaf_tri, (size_t)std::max(T, 1)));
    c->bvh_info = tof_bvh_info{};
    c->bvh_info.builder = c->bvh_builder;
    c->bvh_info.num_triangles = T;
    const auto tb0 = std::chrono::steady_clock::now();
    int slot = 0;
    if (c->bvh_builder == TOF_BVH_DEVICE && T > 0) {
        // mesh object m: leaf slots [m_slot[m], m_slot[m + 1]), triangles from m_tri[m]
        std::vector<int> m_slot{0}, m_tri;
        for (int o = 0; o < d->num_objects; ++o) {
            const Obj& ob = objs[o];
            if (ob.type != TOF_OBJ_GRID) continue;
            m_tri.push_back(ob.tri_base);
            m_slot.push_back(m_slot.back() + 2 * ob.nu * ob.nv);
            c->mesh_objs.push_back(o);
        }
        const size_t wb = tofh::blas_build_bytes(T, m_tri.size());
        void* ws = nullptr;
        TOF_TRY(dev_alloc(c, c->build_mem, &ws, wb));
        tofh::BlasResult br;
        const tof_status bs =
            tofh::build_blas_device(ws, wb, c->d_tv, c->d_lv, m_slot, m_tri, c->n_tlas_cap, c->d_leaf_tri, br);
        free_all(c, c->build_mem);
        TOF_TRY(bs);
        blas = std::move(br.nodes);
        heights = std::move(br.heights);
        c->blas_root = br.roots;
        c->obj_lbox = br.lbox;
        c->bvh_info.rounds = br.rounds;
    }
    for (int o = 0; o < d->num_objects && !(c->bvh_builder == TOF_BVH_DEVICE && T > 0); ++o) {
        const Obj& ob = objs[o];
        if (ob.type != TOF_OBJ_GRID) continue;
        const int nt = 2 * ob.nu * ob.nv;
        std::vector<tofh::BvhPrim> prims(nt);
        float lb[6] = {3e38f, 3e38f, 3e38f, -3e38f, -3e38f, -3e38f};
        for (int i = 0; i < nt; ++i) {
            const int4 v = tv[ob.tri_base + i];
            const int vi[3] = {v.x, v.y, v.z};
            tofh::BvhPrim& p = prims[i];
            for (int k = 0; k < 3; ++k) {
                p.lo[k] = 3e38f;
                p.hi[k] = -3e38f;
            }
            for (int q = 0; q < 3; ++q)
                for (int k = 0; k < 3; ++k) {
                    const float x = d->vertices[3 * vi[q] + k];
                    p.lo[k] = std::min(p.lo[k], x);
                    p.hi[k] = std::max(p.hi[k], x);
                    lb[k] = std::min(lb[k], x);
                    lb[3 + k] = std::max(lb[3 + k], x);
                }
        }
        const int32_t root = tofh::build_bvh4(prims, 4, c->n_tlas_cap + (int)blas.size(), slot, blas, heights, order);
        for (int i = 0; i < nt; ++i) leaf_tri[slot + i] = ob.tri_base + order[i];
        slot += nt;
        c->mesh_objs.push_back(o);
        c->blas_root.push_back(root);
        c->obj_lbox.insert(c->obj_lbox.end(), lb, lb + 6);
    }
    c->n_blas = (int)blas.size();
    c->n_nodes = c->n_tlas_cap + c->n_blas;
    // refit order of the objects' trees: by height, children first
    std::vector<uint32_t> border;
    c->level_off.assign(1, 0);
    const int hmax = heights.empty() ? -1 : *std::max_element(heights.begin(), heights.end());
    for (int h = 0; h <= hmax; ++h) {
        for (int i = 0; i < c->n_blas; ++i)
            if (heights[i] == h) border.push_back((uint32_t)(c->n_tlas_cap + i));
        c->level_off.push_back((int)border.size());
    }
    if (T && c->bvh_builder != TOF_BVH_DEVICE)
        HIP_TRY(hipMemcpy(c->d_leaf_tri, leaf_tri.data(), sizeof(int) * T, hipMemcpyHostToDevice));
    c->bvh_info.num_nodes = c->n_blas;
    c->bvh_info.num_levels = hmax + 1;
    c->bvh_info.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb0).count();
    for (auto& g : c->geom) {
        TOF_TRY(alloc_t(c, a, &g.xf, 12 * (size_t)objs.size()));
        TOF_TRY(alloc_t(c, a, &g.vel, 6 * (size_t)objs.size()));
        HIP_TRY(hipMemset(g.vel, 0, sizeof(float) * 6 * objs.size()));
        g.vel_host.assign(6 * objs.size(), 0.f);
        TOF_TRY(alloc_t(c, a, &g.wv, std::max(d->num_vertices, 1)));
        TOF_TRY(alloc_t(c, a, &g.wr, std::max(d->num_vertices, 1)));
        TOF_TRY(alloc_t(c, a, &g.nodes, (size_t)c->n_nodes));
        TOF_TRY(alloc_t(c, a, &g.nodesq, (size_t)c->n_nodes));
        TOF_TRY(alloc_t(c, a, &g.order, (size_t)c->n_nodes));
        TOF_TRY(alloc_t(c, a, &g.leaves, 3 * (size_t)std::max(T, 1)));
        HIP_TRY(hipMemset(g.nodes, 0, sizeof(Node4) * (size_t)c->n_nodes));
        HIP_TRY(hipMemset(g.nodesq, 0, sizeof(NodeQ) * (size_t)c->n_nodes));
        if (c->n_blas) {
            HIP_TRY(hipMemcpy(g.nodes + c->n_tlas_cap, blas.data(), sizeof(Node4) * blas.size(), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(g.order, border.data(), sizeof(uint32_t) * border.size(), hipMemcpyHostToDevice));
        }
    }
    c->h_objs = objs;
    c->n_obj = d->num_objects;
    c->n_mat = d->num_materials;
    c->n_vert = d->num_vertices;
    c->n_tri = T;
    c->n_sph = (int)sph.size();
    c->scale = d->scene_scale;
    // per frame: transforms, the tree over the objects and its refit order
    c->pinned_bytes = pinned_slot_bytes(objs.size(), (size_t)c->n_tlas_cap);
    if (c->hbase && 2 * c->pinned_bytes > c->hsize) return TOF_ERR_OUT_OF_MEMORY;
    for (int i = 0; i < 2; ++i) {
        if (c->xf_pinned[i] && !c->hbase) (void)hipHostFree(c->xf_pinned[i]);
        c->xf_pinned[i] = nullptr;
        if (c->hbase)
            c->xf_pinned[i] = (float*)(c->hbase + i * c->pinned_bytes);
        else
            HIP_TRY(hipHostMalloc((void**)&c->xf_pinned[i], c->pinned_bytes));
        if (!c->xf_ev[i]) HIP_TRY(hipEventCreateWithFlags(&c->xf_ev[i], hipEventDisableTiming));
    }
    // the null-stream copies and fills must have landed before a frame on
    // any other stream reads them
    HIP_TRY(hipStreamSynchronize(nullptr));
    c->has_scene = true;
    return TOF_OK;
}

tof_status tof_sensor_set(tof_ctx* c, const tof_sensor_desc* d) {
    if (!c || !d) return TOF_ERR_INVALID_ARG;
    const int B = d->n_bins + (d->gate_enabled ? 1 : 0);
    bool ok = d->width >= 1 && d->height >= 1 && d->full_width >= d->width && d->full_height >= d->height &&
              d->crop_x0 >= 0 && d->crop_y0 >= 0 && d->crop_x0 + d->width <= d->full_width &&
              d->crop_y0 + d->height <= d->full_height && (long long)d->full_width * d->full_height < (1LL << 31) &&
              (d->camera_model == TOF_CAMERA_PINHOLE || d->camera_model == TOF_CAMERA_ORTHO) &&
              (d->light_model == TOF_LIGHT_POINT || d->light_model == TOF_LIGHT_CONFOCAL) && B >= 1 &&
              d->n_bins >= 0 && d->n_bins <= 8192 && (d->n_bins == 0 || d->bin_width > 0.f) &&
              (!d->gate_enabled || d->gate_width > 0.f) && d->n_min >= 1 && d->n_min <= d->n_max && d->n_max <= kMaxVerts &&
              d->m_init >= 1 && d->m_init <= 255 && d->spatial_rounds >= 0 && d->spatial_rounds <= 8 &&
              d->spatial_k >= 0 && d->spatial_k <= kMaxK && (d->spatial_rounds == 0 || d->spatial_k == 0 || d->spatial_radius >= 1) &&
              d->spatial_radius <= 1024 && d->m_cap > 0.f && d->newton_tol_rel > 0.f && d->newton_max_iter >= 0 &&
              d->newton_max_iter <= 64 && d->j_max >= 1.f &&
              (d->shift_mode == TOF_SHIFT_NAIVE || d->shift_mode == TOF_SHIFT_PATHLEN) &&
              d->debug_stage >= TOF_STAGE_CANONICAL && d->debug_stage <= TOF_STAGE_FINAL &&
              d->bin_radius >= 0 && d->bin_radius <= 4 && std::isfinite(d->shrink_k) && d->shrink_k >= 1.f &&
              d->shrink_k <= 1000.f && std::isfinite(d->shrink_r) && d->shrink_r >= 0.f && d->shrink_r <= 1.f &&
              (d->domain == TOF_DOMAIN_TIME || d->domain == TOF_DOMAIN_VELOCITY) &&
              (d->round_trip == 0 || d->round_trip == 1) && (d->mis_mode == 0 || d->mis_mode == 1) &&
              (d->domain == TOF_DOMAIN_TIME || (d->bin_radius == 0 && d->shrink_k == 1.f)) &&
              std::isfinite(d->light_intensity) && std::isfinite(d->gate_center) && std::isfinite(d->bin_t0);
    // items (one per non-empty pixel-plane of a pass) are 32-bit indices;
    // task numbers are counted modulo 2^32, as only their differences within
    // a chunk (at most its task capacity) are ever used
    ok = ok && (unsigned long long)d->width * d->height * B < (1ULL << 31);
    if (ok) {
        // owners of queued visibility segments (indices of the floats a blocked
        // ray zeroes: 4 per task, one per MIS term, 20 per pixel) stay below 2^31
        const size_t P = (size_t)d->width * d->height;
        const tofh::ChunkPlan pc = tofh::plan_chunks(P, (size_t)B, d->spatial_k, d->bin_radius);
        ok = 4 * pc.task_cap < ((size_t)1 << 31) && pc.term_cap < ((size_t)1 << 31) &&
             P * kRecWords < ((size_t)1 << 31);
    }
    if (!ok) return TOF_ERR_INVALID_ARG;
    if (c->has_sensor) {
        // a move of the gate alone keeps the history: the next temporal reuse
        // shifts previous-frame paths by the move (Sec. 4.1)
        tof_sensor_desc moved = c->sd;
        moved.gate_center = d->gate_center;
        if (std::memcmp(&moved, d, sizeof(moved)) == 0) {
            c->sd.gate_center = d->gate_center;
            c->s.gate_c = d->gate_center;
            return TOF_OK;
        }
    }
    if (c->budget && c->scene_mem.bytes + sensor_footprint(*d) > c->budget) return TOF_ERR_OUT_OF_MEMORY;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    free_all(c, c->sensor_mem);
    c->has_sensor = false;
    c->prev_valid = false;
    c->slot[0].valid = c->slot[1].valid = false;
    const size_t P = (size_t)d->width * d->height;
    const size_t words = ((size_t)B + 31) / 32;
    for (int i = 0; i < 3; ++i) TOF_TRY(alloc_set(c, c->sets[i], P, B, words));
    Alloc& a = c->sensor_mem;
    for (int i = 0; i < 2; ++i) {
        SlotHost& h = c->slot[i];
        TOF_TRY(alloc_t(c, a, &h.gb_obj, P));
        TOF_TRY(alloc_t(c, a, &h.gb_xi0, P));
        TOF_TRY(alloc_t(c, a, &h.gb_xi1, P));
        TOF_TRY(alloc_t(c, a, &h.gb_p, P));
        TOF_TRY(alloc_t(c, a, &h.gb_n, P));
    }
    TOF_TRY(alloc_t(c, a, &c->pt, P * B));
    c->pt_zero = c->pt_zero_pending = false;
    TOF_TRY(alloc_t(c, a, &c->direct, P));
    TOF_TRY(alloc_t(c, a, &c->prev_pix, P));
    TOF_TRY(alloc_t(c, a, &c->wsum, 2 * P));
    TOF_TRY(alloc_t(c, a, &c->nb, P * (size_t)std::max(d->spatial_k, 1)));
    const tofh::ChunkPlan& pl = c->alloc_plan = tofh::plan_chunks(P, (size_t)B, d->spatial_k, d->bin_radius);
    TOF_TRY(alloc_t(c, a, &c->items, P * B));
    TOF_TRY(alloc_t(c, a, &c->task0, P * B));
    TOF_TRY(alloc_t(c, a, &c->tasks, pl.task_cap));
    TOF_TRY(alloc_t(c, a, &c->fwd, pl.task_cap));
    c->wide = nullptr;
    if (shrink_mix(*d)) TOF_TRY(alloc_t(c, a, &c->wide, kRecF4 * P));
    TOF_TRY(alloc_t(c, a, &c->shv, 2 * pl.task_cap));
    TOF_TRY(alloc_t(c, a, &c->term, pl.term_cap));
    TOF_TRY(alloc_t(c, a, &c->rays, 2 * pl.ray_cap));
    TOF_TRY(alloc_t(c, a, &c->ray_count, (size_t)tofd::kRaySubQueues * tofd::kCounterStride));
    TOF_TRY(alloc_t(c, a, &c->mis_list, pl.term_cap));
    TOF_TRY(alloc_t(c, a, &c->mis_count, (size_t)tofd::kRaySubQueues * tofd::kCounterStride));
    TOF_TRY(alloc_t(c, a, &c->count, 64));
    c->item_slots = 4 * 4096;
    c->item_used = 0;
    TOF_TRY(alloc_t(c, a, &c->item_hist, c->item_slots));
    c->max_items = P * B;
    c->sd = *d;
    Sens& s = c->s;
    s.W = d->width;
    s.H = d->height;
    s.FW = d->full_width;
    s.FH = d->full_height;
    s.cx0 = d->crop_x0;
    s.cy0 = d->crop_y0;
    s.cam_model = d->camera_model;
    s.light_model = d->light_model;
    s.count_leg = d->count_camera_leg;
    s.jitter = d->jitter;
    s.light_I = d->light_intensity;
    s.gate_en = d->gate_enabled ? 1 : 0;
    s.gate_c = d->gate_center;
    s.gate_w = d->gate_width;
    s.n_bins = d->n_bins;
    s.t0 = d->bin_t0;
    s.bw = d->bin_width;
    s.n_min = d->n_min;
    s.n_max = d->n_max;
    s.m_init = d->m_init;
    s.temporal = d->temporal;
    s.rounds = d->spatial_rounds;
    s.k = d->spatial_k;
    s.radius = d->spatial_radius;
    s.m_cap = d->m_cap;
    s.tol_rel = d->newton_tol_rel;
    s.max_it = d->newton_max_iter;
    s.j_max = d->j_max;
    s.shift_mode = d->shift_mode;
    s.round_trip = d->round_trip;
    s.mis_mode = d->mis_mode;
    s.include_direct = d->include_direct;
    s.debug_stage = d->debug_stage;
    s.br = d->bin_radius;
    s.mw = wide_trees(*d);
    s.shrink_k = s.mw > 0 ? d->shrink_k : 1.f;   // R = 0: no tree samples the wide gate
    s.domain = d->domain;
    s.P = (int)P;
    s.B = B;
    s.mask_words = (int)words;
    s.seed = c->seed;
    c->ray_budget = 0;
    c->plan = plan_of(c, 0);
    c->fin_prev = 2;
    c->has_sensor = true;
    return TOF_OK;
}

tof_status tof_debug_set_ray_budget(tof_ctx* c, size_t rays, size_t* spatial_items_per_chunk) {
    if (!c) return TOF_ERR_INVALID_ARG;
    if (!c->has_sensor) return TOF_ERR_NOT_READY;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    const tofh::ChunkPlan& full = c->alloc_plan;   // what the work space holds
    const tofh::ChunkPlan pl = plan_of(c, rays);
    if (pl.task_cap > full.task_cap || pl.term_cap > full.term_cap || pl.ray_cap > full.ray_cap)
        return TOF_ERR_INVALID_ARG;
    c->plan = pl;
    c->ray_budget = rays;
    if (spatial_items_per_chunk) *spatial_items_per_chunk = pl.ci[1];
    return TOF_OK;
}

tof_status tof_set_launch_config(tof_ctx* c, const tof_launch_config* cfg) {
    if (!c || !cfg) return TOF_ERR_INVALID_ARG;
    const unsigned sb = cfg->shift_blocks ? cfg->shift_blocks : tofh::kShiftGrid;
    const unsigned vb = cfg->vis_blocks ? cfg->vis_blocks : tofh::kVisGrid;
    const int vw = cfg->vis_waves ? (int)cfg->vis_waves : 6;
    const int mt = cfg->merge_tasks ? (int)cfg->merge_tasks : 2;
    if (sb % 64 != 0 || sb > tofh::kShiftGrid || vb % 64 != 0 || vb > kMaxVisBlocks) return TOF_ERR_INVALID_ARG;
    if ((vw != 5 && vw != 6) || (mt != 1 && mt != 2 && mt != 4)) return TOF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    c->shift_blocks = sb;
    c->vis_blocks = vb;
    c->vis_waves = vw;
    c->merge_tasks = mt;
    if (c->has_sensor) c->plan = plan_of(c, c->ray_budget);
    return TOF_OK;
}

tof_status tof_set_bvh_builder(tof_ctx* c, int32_t builder) {
    if (!c || (builder != TOF_BVH_HOST && builder != TOF_BVH_DEVICE)) return TOF_ERR_INVALID_ARG;
    c->bvh_builder = builder;
    return TOF_OK;
}

tof_status tof_get_bvh_info(tof_ctx* c, tof_bvh_info* out, int32_t* leaf_triangles) {
    if (!c || !out) return TOF_ERR_INVALID_ARG;
    if (!c->has_scene) return TOF_ERR_NOT_READY;
    *out = c->bvh_info;
    if (leaf_triangles && c->n_tri > 0) {
        HIP_TRY(hipSetDevice(c->device));
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(leaf_triangles, c->d_leaf_tri, sizeof(int32_t) * (size_t)c->n_tri, hipMemcpyDeviceToHost));
    }
    return TOF_OK;
}

tof_status tof_get_launch_config(tof_ctx* c, tof_launch_config* out) {
    if (!c || !out) return TOF_ERR_INVALID_ARG;
    out->shift_blocks = c->shift_blocks;
    out->vis_blocks = c->vis_blocks;
    out->vis_waves = (uint32_t)c->vis_waves;
    out->merge_tasks = (uint32_t)c->merge_tasks;
    return TOF_OK;
}

tof_status tof_autotune(tof_ctx* c, const tof_frame_desc* frames, int n_frames, void* stream,
                        tof_launch_config* chosen) {
    if (!c || !frames || n_frames < 2 || n_frames > 64) return TOF_ERR_INVALID_ARG;
    if (!c->has_scene || !c->has_sensor) return TOF_ERR_NOT_READY;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    // the tuning frames leave no trace but the chosen shape: the counters and
    // the frame count are restored and the temporal history is dropped
    std::vector<unsigned long long> saved(kCounterBytes / sizeof(unsigned long long));
    HIP_TRY(hipMemcpy(saved.data(), c->counters, kCounterBytes, hipMemcpyDeviceToHost));
    const uint64_t frames0 = c->frames;
    const bool timing = c->timing;
    const unsigned sb0 = c->shift_blocks, vb0 = c->vis_blocks;
    const int vw0 = c->vis_waves, mt0 = c->merge_tasks;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    tof_status res = TOF_OK;
    unsigned best_sb = sb0, best_vb = vb0;
    int best_vw = vw0, best_mt = mt0;
    float best_ms = 3e38f;
    // one candidate: the frames from the first, without history; the later
    // half timed (the earlier half fills the reservoirs)
    auto trial = [&](unsigned sb, unsigned vb, int vw, int mt) -> tof_status {
        c->shift_blocks = sb;
        c->vis_blocks = vb;
        c->vis_waves = vw;
        c->merge_tasks = mt;
        c->plan = plan_of(c, c->ray_budget);
        c->prev_valid = false;
        for (int i = 0; i < n_frames; ++i) {
            if (i == n_frames / 2 && hipEventRecord(ev[0], st) != hipSuccess) return TOF_ERR_DEVICE;
            TOF_TRY(tof_render_frame(c, frames + i, nullptr, nullptr, nullptr, nullptr, stream));
        }
        float ms = 0.f;
        if (hipEventRecord(ev[1], st) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
            hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
            return TOF_ERR_DEVICE;
        if (ms < best_ms) {
            best_ms = ms;
            best_sb = sb;
            best_vb = vb;
            best_vw = vw;
            best_mt = mt;
        }
        return TOF_OK;
    };
    c->timing = false;
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) res = TOF_ERR_DEVICE;
    // coordinate search: the shift kernels' blocks at the default visibility
    // grid, then the visibility blocks, the visibility kernel's occupancy and
    // the merge tile, each at the best of the steps before
    for (unsigned sb : {tofh::kShiftGrid, tofh::kShiftGrid / 2, tofh::kShiftGrid / 4})
        if (res == TOF_OK) res = trial(sb, tofh::kVisGrid, 6, 2);
    const unsigned sb_best = best_sb;
    for (unsigned vb : {tofh::kVisGrid / 4, tofh::kVisGrid / 2, tofh::kVisGrid * 2})
        if (res == TOF_OK) res = trial(sb_best, vb, 6, 2);
    const unsigned vb_best = best_vb;
    if (res == TOF_OK) res = trial(sb_best, vb_best, 5, 2);
    const int vw_best = best_vw;
    for (int mt : {1, 4})
        if (res == TOF_OK) res = trial(sb_best, vb_best, vw_best, mt);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (res == TOF_OK) {
        c->shift_blocks = best_sb;
        c->vis_blocks = best_vb;
        c->vis_waves = best_vw;
        c->merge_tasks = best_mt;
    } else {
        c->shift_blocks = sb0;
        c->vis_blocks = vb0;
        c->vis_waves = vw0;
        c->merge_tasks = mt0;
    }
    c->plan = plan_of(c, c->ray_budget);
    c->timing = timing;
    c->prev_valid = false;
    if (quiesce(c) == hipSuccess &&
        hipMemcpy(c->counters, saved.data(), kCounterBytes, hipMemcpyHostToDevice) == hipSuccess) {
        c->frames = frames0;
    } else if (res == TOF_OK) {
        res = TOF_ERR_DEVICE;
    }
    if (chosen) {
        chosen->shift_blocks = c->shift_blocks;
        chosen->vis_blocks = c->vis_blocks;
        chosen->vis_waves = (uint32_t)c->vis_waves;
        chosen->merge_tasks = (uint32_t)c->merge_tasks;
    }
    return res;
}

tof_status tof_debug_set_history(tof_ctx* c, const tof_history_desc* h) {
    if (!c || !h) return TOF_ERR_INVALID_ARG;
    if (!c->has_scene || !c->has_sensor || !c->slot[0].valid) return TOF_ERR_NOT_READY;
    if (!h->W || !h->phat || !h->len || !h->pre_pdf || !h->origin_pixel || !h->origin_frame || !h->meta ||
        !h->vertex_obj || !h->vertex_xi || !h->M || !h->mask)
        return TOF_ERR_INVALID_ARG;
    const size_t P = (size_t)c->s.P, B = (size_t)c->s.B, PB = P * B, words = (size_t)c->s.mask_words;
    for (size_t i = 0; i < 4 * PB; ++i)
        if (h->vertex_obj[i] < -1 || h->vertex_obj[i] >= c->n_obj) return TOF_ERR_INVALID_ARG;
    for (size_t i = 0; i < PB; ++i) {
        uint32_t m = h->meta[i];
        if (((m >> 8) & 15u) > (uint32_t)kMaxVerts || ((m >> 12) & 15u) > (uint32_t)kMaxVerts ||
            ((m >> 16) & 15u) > 1u || (m >> 17) != 0u)
            return TOF_ERR_INVALID_ARG;
    }
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    ResSet& r = c->sets[c->fin_prev];
    std::vector<float> packed(PB * kRecWords, 0.f);
    auto u2f = [](uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; };
    for (size_t i = 0; i < PB; ++i) {
        float* q = packed.data() + i * kRecWords;
        q[0] = h->W[i];
        q[1] = h->phat[i];
        q[2] = h->len[i];
        q[3] = h->pre_pdf[i];
        q[4] = u2f(h->origin_pixel[i]);
        q[5] = u2f(h->origin_frame[i]);
        const uint32_t m = h->meta[i];
        uint32_t w6, w7;
        rec_pack_meta((int)(m & 255u), (int)((m >> 8) & 15u), (int)((m >> 12) & 15u), (int)((m >> 16) & 15u),
                      h->vertex_obj[i], h->vertex_obj[PB + i], h->vertex_obj[2 * PB + i], h->vertex_obj[3 * PB + i],
                      w6, w7);
        q[6] = u2f(w6);
        q[7] = u2f(w7);
        for (int v = 0; v < 4; ++v) {
            q[8 + 2 * v] = h->vertex_xi[(2 * v) * PB + i];
            q[9 + 2 * v] = h->vertex_xi[(2 * v + 1) * PB + i];
        }
    }
    HIP_TRY(hipMemcpy(r.rec, packed.data(), sizeof(float) * packed.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(r.M, h->M, 4 * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(r.mask, h->mask, 4 * P * words, hipMemcpyHostToDevice));
    HIP_TRY(hipStreamSynchronize(nullptr));
    c->prev_valid = true;
    return TOF_OK;
}

tof_status tof_set_kernel_timing(tof_ctx* c, int enabled) {
    if (!c) return TOF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    c->timing = enabled != 0;
    c->ev_used = 0;
    for (int k = 0; k < TOF_K_COUNT; ++k) {
        c->acc_ms[k] = 0.0;
        c->acc_n[k] = 0;
    }
    for (int q = 0; q < 4; ++q) c->acc_items[q] = 0;
    c->item_used = 0;
    HIP_TRY(hipMemcpy(c->work0, c->counters, kCounterBytes, hipMemcpyDeviceToHost));
    return TOF_OK;
}

tof_status tof_get_kernel_times(tof_ctx* c, tof_kernel_times* out) {
    if (!c || !out) return TOF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    timer_reduce(c);
    if (c->item_used) {
        std::vector<uint32_t> h(c->item_used);
        HIP_TRY(hipMemcpy(h.data(), c->item_hist, 4 * c->item_used, hipMemcpyDeviceToHost));
        for (size_t i = 0; i + 3 < c->item_used; i += 4)
            for (int q = 0; q < 4; ++q) c->acc_items[q] += h[i + q];
        c->item_used = 0;
    }
    for (int k = 0; k < TOF_K_COUNT; ++k) {
        out->ms[k] = c->acc_ms[k];
        out->launches[k] = c->acc_n[k];
    }
    for (int q = 0; q < 4; ++q) out->work_items[q] = c->acc_items[q];
    unsigned long long h[TOF_K_COUNT * kBank];
    HIP_TRY(hipMemcpy(h, c->counters, kCounterBytes, hipMemcpyDeviceToHost));
    for (int k = 0; k < TOF_K_COUNT; ++k) {
        auto d = [&](int i) { return (uint64_t)(h[k * kBank + i] - c->work0[k * kBank + i]); };
        out->work[k].rays = d(ST_RAYS);
        out->work[k].node_visits = d(ST_NODES);
        out->work[k].tri_tests = d(ST_TRIS);
        out->work[k].shifts = d(ST_SHIFTS);
        out->work[k].newton_attempts = d(ST_NEWTON_ATT);
        out->work[k].newton_iters = d(ST_NEWTON_ITERS);
    }
    return TOF_OK;
}

tof_status tof_reservoirs_reset(tof_ctx* c) {
    if (!c) return TOF_ERR_INVALID_ARG;
    c->prev_valid = false;
    return TOF_OK;
}

tof_status tof_get_stats(tof_ctx* c, tof_stats* out) {
    if (!c || !out) return TOF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(quiesce(c));
    unsigned long long hb[TOF_K_COUNT * kBank];
    HIP_TRY(hipMemcpy(hb, c->counters, kCounterBytes, hipMemcpyDeviceToHost));
    unsigned long long h[kBank] = {};
    for (int k = 0; k < TOF_K_COUNT; ++k)
        for (int i = 0; i < kBank; ++i) h[i] += hb[k * kBank + i];
    out->shifts = h[ST_SHIFTS];
    out->shifts_ok = h[ST_SHIFTS_OK] - h[ST_VISFAIL];   // provisional successes minus blocked ones
    out->newton_attempts = h[ST_NEWTON_ATT];
    out->newton_converged = h[ST_NEWTON_CONV];
    out->newton_iters = h[ST_NEWTON_ITERS];
    out->newton_paths_ok = h[ST_NEWTON_OK] - h[ST_VISFAIL_NEWTON];
    out->rays = h[ST_RAYS];
    out->frames = c->frames;
    out->bvh_overflow = h[ST_OVERFLOW];
    out->node_visits = h[ST_NODES];
    out->tri_tests = h[ST_TRIS];
    out->bad_records = h[ST_BADREC];
    return TOF_OK;
}

// A reuse pass (mode 0 temporal, 1 spatial) after its work list is built:
// for every chunk of plan.ci[mode] items, the chunk's tasks, their forward
// shifts and the visibility of those, the MIS shifts and their visibility,
// then the merge of the chunk's items into `out`.  Chunks past the last item
// find an empty window and do nothing.
tof_status run_pass(tof_ctx* c, tofh::FrameArgs& a, int mode, const ResSet& A, const ResSet& Bp, const int* links,
                    int round, const ResSet& out, hipStream_t st) {
    const int kf = mode == 0 ? TOF_K_TEMPORAL_FWD : TOF_K_SPATIAL_FWD;
    const int km = mode == 0 ? TOF_K_TEMPORAL_MIS : TOF_K_SPATIAL_MIS;
    const int kv = mode == 0 ? TOF_K_TEMPORAL_VIS : TOF_K_SPATIAL_VIS;
    const int kg = mode == 0 ? TOF_K_TEMPORAL_MERGE : TOF_K_SPATIAL_MERGE;
    const tofh::ChunkPlan& pl = c->plan;
    const size_t K = mode == 0 ? 1 : (mode == 1 ? (size_t)c->s.k : 2 * (size_t)c->s.br);
    // at most 4 segments per shift across frames (temporal), 2 within one frame
    const size_t seg = mode == 0 ? 4 : 2;
    const size_t ct = pl.ct[mode], ci = pl.ci[mode];
    const size_t ncounters = (size_t)tofd::kRaySubQueues * tofd::kCounterStride;
    const size_t NQ = tofd::kRaySubQueues;
    uint32_t* win = c->count + 2;
    // a chunk has at most ct tasks, ct / NQ per sub-queue (fixed grid)
    const tofd::RayQueue qf{c->rays, c->ray_count, (uint32_t)(seg * ct / NQ)};
    const tofd::RayQueue qm{c->rays, c->ray_count, (uint32_t)(seg * K * ct / NQ)};
    const tofd::IdxQueue lq{c->mis_list, c->mis_count, (uint32_t)(K * ct / NQ)};
    auto vis = [&](int slot, const tofd::RayQueue& q, float* kill) -> hipError_t {
        hipError_t e = timer_mark(c, kv, st);
        if (e != hipSuccess) return e;
        a.counters = c->counters + (size_t)kv * kBank;
        tofh::launch_vis(a, slot, q, kill, pl.vis_grid[mode], c->vis_waves, st);
        return timer_mark(c, kv, st);
    };
    // the chunks that hold items: all the plan allows, or (when more than one
    // is possible, and the frame is not being recorded into a graph) those
    // below the count k_items wrote, read back here
    size_t n_items = c->max_items;
    if (c->sync_counts && !c->capturing && n_items > ci) {
        HIP_TRY(hipMemcpyAsync(c->count_host, c->count, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        n_items = std::min<size_t>(n_items, c->count_host[0]);
    }
    for (size_t i0 = 0; i0 < n_items; i0 += ci) {
        HIP_TRY(timer_mark(c, kf, st));
        tofh::launch_tasks(c->items, c->task0, c->count, i0, ci, c->tasks, win, st);
        tofh::launch_fill_u32(c->ray_count, 0u, ncounters, st);
        a.counters = c->counters + (size_t)kf * kBank;
        tofh::launch_fwd(a, mode, A, Bp, links, c->items, c->tasks, win, c->fwd, c->shv, qf, pl.grid[mode], st);
        HIP_TRY(timer_mark(c, kf, st));
        HIP_TRY(vis(0, qf, (float*)c->fwd));
        HIP_TRY(timer_mark(c, km, st));
        tofh::launch_fill_u32(c->ray_count, 0u, ncounters, st);
        tofh::launch_fill_u32(c->mis_count, 0u, ncounters, st);
        a.counters = c->counters + (size_t)km * kBank;
        tofh::launch_mis(a, mode, A, Bp, links, c->items, c->tasks, win, c->fwd, c->shv, c->term, lq, qm,
                         pl.grid[mode], st);
        HIP_TRY(timer_mark(c, km, st));
        HIP_TRY(vis(mode == 0 ? 1 : 0, qm, c->term));
        HIP_TRY(timer_mark(c, kg, st));
        a.counters = c->counters + (size_t)kg * kBank;
        tofh::launch_merge(a, mode, A, Bp, links, c->items, c->tasks, c->task0, c->count, i0, ci, win, c->fwd, c->term,
                           c->shv, round, out, c->merge_tasks, st);
        HIP_TRY(timer_mark(c, kg, st));
    }
    return TOF_OK;
}

tof_status tof_render_frame(tof_ctx* c, const tof_frame_desc* fr, float* out_image, float* out_hist,
                            float* out_pt_image, float* out_pt_hist, void* stream) {
    if (!c || !fr) return TOF_ERR_INVALID_ARG;
    if (!c->has_scene || !c->has_sensor) return TOF_ERR_NOT_READY;
    if (!fr->object_xforms) return TOF_ERR_INVALID_ARG;
    if ((out_image || out_pt_image) && !c->sd.gate_enabled) return TOF_ERR_INVALID_ARG;
    if ((out_hist || out_pt_hist) && c->sd.n_bins == 0) return TOF_ERR_INVALID_ARG;
    for (int k = 0; k < 12 * c->n_obj; ++k)
        if (!std::isfinite(fr->object_xforms[k])) return TOF_ERR_INVALID_ARG;
    if (!finite3(fr->cam_pos) || !finite3(fr->cam_fwd) || !finite3(fr->cam_up) || !finite3(fr->light_pos))
        return TOF_ERR_INVALID_ARG;
    const bool vel = c->s.domain == TOF_DOMAIN_VELOCITY;
    if (vel) {
        if (!finite3(fr->cam_vel) || !finite3(fr->light_vel)) return TOF_ERR_INVALID_ARG;
        if (fr->object_velocities)
            for (int k = 0; k < 6 * c->n_obj; ++k)
                if (!std::isfinite(fr->object_velocities[k])) return TOF_ERR_INVALID_ARG;
    }
    V3 fwd = hv(fr->cam_fwd[0], fr->cam_fwd[1], fr->cam_fwd[2]);
    V3 up = hv(fr->cam_up[0], fr->cam_up[1], fr->cam_up[2]);
    V3 rc = hcross(fwd, up);
    if (!(rc.x * rc.x + rc.y * rc.y + rc.z * rc.z > 0.f)) return TOF_ERR_INVALID_ARG;
    if (c->sd.camera_model == TOF_CAMERA_PINHOLE && !(fr->fov_y_deg > 0.f && fr->fov_y_deg < 180.f))
        return TOF_ERR_INVALID_ARG;
    if (c->sd.camera_model == TOF_CAMERA_ORTHO && !(fr->ortho_half[0] > 0.f && fr->ortho_half[1] > 0.f))
        return TOF_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // a caller recording the frame into a graph (stream capture): the events
    // the host waits on (the pinned upload ring, the frame's end) are left to
    // it, to record on the stream after it has launched the graph
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap == hipStreamCaptureStatusActive;
    c->capturing = capturing;
    if (!capturing) {   // an earlier recording that never launched leaves nothing to record
        c->xf_pending = -1;
        c->done_pending = false;
    }
    const size_t O = (size_t)c->n_obj;
    // rotate: the previous call's frame becomes slot 1
    if (c->slot[0].valid) std::swap(c->slot[0], c->slot[1]);
    SlotHost& cur = c->slot[0];
    const SlotHost& prev = c->slot[1];
    // this frame's velocities (velocity domain; none = at rest)
    std::vector<float> vel_now;
    if (vel) {
        vel_now.assign(6 * O, 0.f);
        if (fr->object_velocities) std::memcpy(vel_now.data(), fr->object_velocities, sizeof(float) * 6 * O);
    }
    bool same = prev.valid && c->geom[prev.geom].built &&
                std::memcmp(c->geom[prev.geom].xf_host.data(), fr->object_xforms, sizeof(float) * 12 * O) == 0 &&
                (!vel || c->geom[prev.geom].vel_host == vel_now);
    if (same) {
        cur.geom = prev.geom;
    } else {
        cur.geom = prev.valid ? 1 - prev.geom : 0;
        GeomBuf& g = c->geom[cur.geom];
        g.xf_host.assign(fr->object_xforms, fr->object_xforms + 12 * O);
        int ring = c->xf_ring;
        c->xf_ring ^= 1;
        // the pinned slot's last upload is done (under capture the caller has
        // waited for it before the capture began: prepare_frame_capture)
        if (!capturing) HIP_TRY(hipEventSynchronize(c->xf_ev[ring]));
        char* pin = (char*)c->xf_pinned[ring];
        std::memcpy(pin, fr->object_xforms, sizeof(float) * 12 * O);
        HIP_TRY(hipMemcpyAsync(g.xf, pin, sizeof(float) * 12 * O, hipMemcpyHostToDevice, st));
        std::vector<int> levels = c->level_off;
        if (!c->mesh_objs.empty()) {
            // the tree over the objects' world boxes (corners of the object-space
            // boxes moved by this frame's transforms; grouping only, the device
            // refit computes the exact boxes)
            const size_t M = c->mesh_objs.size();
            std::vector<tofh::BvhPrim> prims(M);
            for (size_t m = 0; m < M; ++m) {
                const float* x = fr->object_xforms + 12 * c->mesh_objs[m];
                const float* lb = &c->obj_lbox[6 * m];
                tofh::BvhPrim& p = prims[m];
                for (int k = 0; k < 3; ++k) {
                    p.lo[k] = 3e38f;
                    p.hi[k] = -3e38f;
                }
                for (int corner = 0; corner < 8; ++corner) {
                    const float q[3] = {lb[(corner & 1) ? 3 : 0], lb[(corner & 2) ? 4 : 1], lb[(corner & 4) ? 5 : 2]};
                    for (int k = 0; k < 3; ++k) {
                        const float w = x[4 * k] * q[0] + x[4 * k + 1] * q[1] + x[4 * k + 2] * q[2] + x[4 * k + 3];
                        p.lo[k] = std::min(p.lo[k], w);
                        p.hi[k] = std::max(p.hi[k], w);
                    }
                }
            }
            std::vector<Node4> tl;
            std::vector<int> th, torder;
            const int32_t root = tofh::build_bvh4(prims, 1, 0, 0, tl, th, torder);
            if (root < 0) {   // a single object: a root with one child
                tl.assign(1, Node4{});
                th.assign(1, 0);
                tl[0].child = make_int4(c->blas_root[0], -1, -1, -1);
                tl[0].meta = make_int4(1, 0, 0, 0);
            } else {
                for (Node4& n : tl) {
                    int* ch = &n.child.x;
                    for (int j = 0; j < n.meta.x; ++j)
                        if (ch[j] < 0) ch[j] = c->blas_root[torder[ch[j] & 0x0FFFFFFF]];
                }
            }
            const int nt = (int)tl.size();   // <= n_tlas_cap: fewer 4-wide nodes than objects
            std::vector<uint32_t> tord;
            const int thmax = *std::max_element(th.begin(), th.end());
            for (int h = 0; h <= thmax; ++h) {
                for (int i = 0; i < nt; ++i)
                    if (th[i] == h) tord.push_back((uint32_t)i);
                levels.push_back(c->n_blas + (int)tord.size());
            }
            char* pn = pin + sizeof(float) * 12 * O;
            char* po = pn + sizeof(Node4) * c->n_tlas_cap;
            std::memcpy(pn, tl.data(), sizeof(Node4) * nt);
            std::memcpy(po, tord.data(), sizeof(uint32_t) * nt);
            HIP_TRY(hipMemcpyAsync(g.nodes, pn, sizeof(Node4) * nt, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(g.order + c->n_blas, po, sizeof(uint32_t) * nt, hipMemcpyHostToDevice, st));
        }
        if (vel) {
            char* pv = pin + sizeof(float) * 12 * O + (sizeof(Node4) + sizeof(uint32_t)) * c->n_tlas_cap;
            std::memcpy(pv, vel_now.data(), sizeof(float) * 6 * O);
            HIP_TRY(hipMemcpyAsync(g.vel, pv, sizeof(float) * 6 * O, hipMemcpyHostToDevice, st));
            g.vel_host = vel_now;
        }
        if (capturing)
            c->xf_pending = ring;   // recorded by the caller once the graph is launched
        else
            HIP_TRY(hipEventRecord(c->xf_ev[ring], st));
        HIP_TRY(timer_mark(c, TOF_K_BVH, st));
        tofh::launch_world_verts(c->d_lv, c->d_vobj, g.xf, g.wv, g.wr, c->n_vert, st);
        tofh::launch_leaf_gather(c->d_leaf_tri, c->d_tv, g.wv, c->n_tri, g.leaves, st);
        tofh::launch_refit(g.nodes, g.nodesq, g.order, levels, g.leaves, c->n_tri, st);
        HIP_TRY(timer_mark(c, TOF_K_BVH, st));
        g.built = true;
    }
    cur.valid = true;
    cur.cam_pos = hv(fr->cam_pos[0], fr->cam_pos[1], fr->cam_pos[2]);
    cur.cam_fwd = hnorm(fwd);
    cur.cam_right = hnorm(hcross(cur.cam_fwd, up));
    cur.cam_up = hcross(cur.cam_right, cur.cam_fwd);
    cur.tan_half = std::tan(0.5 * (double)fr->fov_y_deg * 3.14159265358979323846 / 180.0);
    cur.aspect = (float)((double)c->sd.full_width / (double)c->sd.full_height);
    cur.ohx = fr->ortho_half[0];
    cur.ohy = fr->ortho_half[1];
    cur.gate_c = c->s.gate_c;
    cur.light_pos = hv(fr->light_pos[0], fr->light_pos[1], fr->light_pos[2]);
    cur.cam_vel = vel ? hv(fr->cam_vel[0], fr->cam_vel[1], fr->cam_vel[2]) : hv(0.f, 0.f, 0.f);
    cur.light_vel = vel ? hv(fr->light_vel[0], fr->light_vel[1], fr->light_vel[2]) : hv(0.f, 0.f, 0.f);

    tofh::FrameArgs a;
    a.s = c->s;
    a.S.objs = c->d_objs;
    a.S.mats = c->d_mats;
    a.S.tri_info = c->d_tri;
    a.S.sphere_ids = c->d_sph;
    a.S.n_obj = c->n_obj;
    a.S.n_sph = c->n_sph;
    a.S.n_tri = c->n_tri;
    a.S.eps = 1e-4f * c->scale;
    a.S.dmin = 0.01f * c->scale;
    a.F.g[0] = slot_dev(c, 0);
    a.F.g[1] = prev.valid ? slot_dev(c, 1) : slot_dev(c, 0);
    a.frame = (uint32_t)fr->frame_index;
    const size_t P = (size_t)c->s.P, B = (size_t)c->s.B;

    tofh::GBufOut gout{cur.gb_obj, cur.gb_xi0, cur.gb_xi1, cur.gb_p, cur.gb_n};
    HIP_TRY(timer_mark(c, TOF_K_GBUFFER, st));
    a.counters = c->counters + (size_t)TOF_K_GBUFFER * kBank;
    tofh::launch_gbuffer(a, gout, st);
    HIP_TRY(timer_mark(c, TOF_K_GBUFFER, st));
    // the plain-PT deposits start from zero: cleared by the last frame's
    // splat, else filled here
    if (!c->pt_zero) tofh::launch_fill_u32((uint32_t*)c->pt, 0u, P * B, st);
    c->pt_zero = false;   // until this frame's splat has been issued
    c->pt_zero_pending = false;
    ResSet& can = c->sets[0];
    const int spare = c->fin_prev == 1 ? 2 : 1;   // the set not holding the previous frame's final
    ResSet& tmp = c->sets[spare];
    HIP_TRY(timer_mark(c, TOF_K_INITIAL, st));
    a.counters = c->counters + (size_t)TOF_K_INITIAL * kBank;
    ResSet wide{};
    wide.rec = c->wide;
    tofh::launch_initial(a, can, wide, c->pt, c->direct, st);
    if (c->s.gate_en && c->s.shrink_k > 1.f) {
        // shrink mapping of the gate reservoirs, in chunks of the spatial
        // pass's task count (at most 2 visibility segments per pixel)
        const tofh::ChunkPlan& pl = c->plan;
        const size_t ct = pl.ct[1], NQ = tofd::kRaySubQueues;
        const tofd::RayQueue qs{c->rays, c->ray_count, (uint32_t)(2 * ct / NQ)};
        float* kill = (float*)(can.rec + (size_t)c->s.n_bins * P * kRecF4);
        if (c->wide) {   // R < 1: merge of the gate and the shrunk wide-gate samples
            const tofd::RayQueue q4{c->rays, c->ray_count, (uint32_t)(4 * ct / NQ)};
            for (size_t p0 = 0; p0 < P; p0 += ct) {
                const size_t np = std::min(ct, P - p0);
                tofh::launch_fill_u32(c->ray_count, 0u, (size_t)tofd::kRaySubQueues * tofd::kCounterStride, st);
                tofh::launch_shrink_mix(a, can, wide, p0, np, q4, c->fwd, pl.grid[1], st);
                tofh::launch_vis(a, 0, q4, (float*)c->fwd, pl.vis_grid[1], c->vis_waves, st);
                tofh::launch_shrink_mix_fin(a, can, wide, p0, np, c->fwd, st);
            }
        } else {
            for (size_t p0 = 0; p0 < P; p0 += ct) {
                tofh::launch_fill_u32(c->ray_count, 0u, (size_t)tofd::kRaySubQueues * tofd::kCounterStride, st);
                tofh::launch_shrink(a, can, p0, std::min(ct, P - p0), qs, pl.grid[1], st);
                tofh::launch_vis(a, 0, qs, kill, pl.vis_grid[1], c->vis_waves, st);
            }
            tofh::launch_shrink_fin(a, can, st);
        }
    }
    HIP_TRY(timer_mark(c, TOF_K_INITIAL, st));
    const bool record_items = c->timing && c->item_used + 4 <= c->item_slots;
    uint32_t* item_slot = record_items ? c->item_hist + c->item_used : nullptr;
    if (record_items) {
        tofh::launch_fill_u32(item_slot, 0u, 4, st);
        c->item_used += 4;
    }
    const ResSet* shown = nullptr;
    if (c->s.debug_stage == TOF_STAGE_CANONICAL) shown = &can;
    const ResSet* cur_set = &can;
    bool temporal_done = false;
    if (c->s.temporal && c->prev_valid && prev.valid) {
        const ResSet& pf = c->sets[c->fin_prev];
        HIP_TRY(timer_mark(c, TOF_K_TEMPORAL_PREP, st));
        a.counters = c->counters + (size_t)TOF_K_TEMPORAL_PREP * kBank;
        tofh::launch_reproject(a, can, pf, c->prev_pix, tmp.M, st);
        tofh::launch_fill_u32(c->count, 0u, 2, st);
        tofh::launch_items(a, 0, can, pf, c->prev_pix, 2, c->items, c->task0, c->count, tmp.mask, c->wsum, st);
        HIP_TRY(timer_mark(c, TOF_K_TEMPORAL_PREP, st));
        TOF_TRY(run_pass(c, a, 0, can, pf, c->prev_pix, 0, tmp, st));
        if (item_slot) HIP_TRY(hipMemcpyAsync(item_slot, c->count, 8, hipMemcpyDeviceToDevice, st));
        cur_set = &tmp;
        temporal_done = true;
    }
    a.counters = c->counters + (size_t)TOF_K_SPLAT * kBank;
    if (c->s.debug_stage == TOF_STAGE_TEMPORAL) {
        tofh::launch_splat(a, *cur_set, c->pt, true, c->direct, out_image, out_hist, out_pt_image, out_pt_hist, st);
    } else if (shown) {
        tofh::launch_splat(a, *shown, c->pt, true, c->direct, out_image, out_hist, out_pt_image, out_pt_hist, st);
    }
    // the bin-axis pass and the spatial rounds alternate between sets 1 and
    // 2 (the previous frame's final has been read, or is not read this frame)
    int cur_idx = temporal_done ? spare : 0;
    auto next_out = [&]() { return cur_idx == 0 ? spare : 3 - cur_idx; };
    if (c->s.br > 0 && c->s.n_bins > 1) {
        const int out_idx = next_out();
        ResSet& in = c->sets[cur_idx];
        ResSet& out = c->sets[out_idx];
        HIP_TRY(timer_mark(c, TOF_K_SPATIAL_PREP, st));
        a.counters = c->counters + (size_t)TOF_K_SPATIAL_PREP * kBank;
        HIP_TRY(hipMemcpyAsync(out.M, in.M, sizeof(float) * P, hipMemcpyDeviceToDevice, st));
        tofh::launch_fill_u32(c->count, 0u, 2, st);
        tofh::launch_items(a, 2, in, in, nullptr, 2 * c->s.br + 1, c->items, c->task0, c->count, out.mask, c->wsum,
                           st);
        if (c->s.gate_en) tofh::launch_copy_plane(a, in, out, c->s.n_bins, st);
        HIP_TRY(timer_mark(c, TOF_K_SPATIAL_PREP, st));
        TOF_TRY(run_pass(c, a, 2, in, in, nullptr, 0, out, st));
        cur_idx = out_idx;
    }
    for (int r = 0; r < c->s.rounds && c->s.k > 0; ++r) {
        const int out_idx = next_out();
        ResSet& in = c->sets[cur_idx];
        ResSet& out = c->sets[out_idx];
        HIP_TRY(timer_mark(c, TOF_K_SPATIAL_PREP, st));
        a.counters = c->counters + (size_t)TOF_K_SPATIAL_PREP * kBank;
        tofh::launch_neighbours(a, r, in, c->nb, out.M, st);
        tofh::launch_fill_u32(c->count, 0u, 2, st);
        tofh::launch_items(a, 1, in, in, c->nb, c->s.k + 1, c->items, c->task0, c->count, out.mask, c->wsum, st);
        HIP_TRY(timer_mark(c, TOF_K_SPATIAL_PREP, st));
        TOF_TRY(run_pass(c, a, 1, in, in, c->nb, r, out, st));
        if (item_slot && r == 0) HIP_TRY(hipMemcpyAsync(item_slot + 2, c->count, 8, hipMemcpyDeviceToDevice, st));
        cur_idx = out_idx;
    }
    // a final still in the canonical set (no pass ran) trades places with the
    // spare set, so that the next frame's initial samples do not overwrite it
    if (cur_idx == 0) {
        std::swap(c->sets[0], c->sets[spare]);
        cur_idx = spare;
    }
    const int fin_new = cur_idx;
    a.counters = c->counters + (size_t)TOF_K_SPLAT * kBank;
    if (c->s.debug_stage == TOF_STAGE_FINAL) {
        HIP_TRY(timer_mark(c, TOF_K_SPLAT, st));
        tofh::launch_splat(a, c->sets[fin_new], c->pt, true, c->direct, out_image, out_hist, out_pt_image,
                           out_pt_hist, st);
        HIP_TRY(timer_mark(c, TOF_K_SPLAT, st));
    }
    if (c->timing && c->ev_used > 4096) {   // bound the pool: fold finished pairs
        HIP_TRY(hipStreamSynchronize(st));
        timer_reduce(c);
    }
    if (hipGetLastError() != hipSuccess) return TOF_ERR_DEVICE;
    // exactly one splat per frame reads (and clears) every deposit; a
    // recorded frame's only once its graph has been launched
    if (capturing) c->pt_zero_pending = true;
    else c->pt_zero = true;
    if (capturing)
        c->done_pending = true;
    else
        HIP_TRY(hipEventRecord(c->done, st));
    c->has_work = true;
    c->fin_prev = fin_new;
    c->prev_valid = true;
    c->frames++;
    return TOF_OK;
}

// The per-frame work space of a context: work lists, chunk workspace (tasks,
// shift terms, MIS list, ray queue and their counters), plain-PT staging,
// reprojection and neighbour tables.  Only frame state lives elsewhere
// (reservoirs, G-buffers, geometry, event counters).
struct FrameWork {
    float* pt;
    float2* direct;
    int* prev_pix;
    uint32_t* wsum;
    int* nb;
    uint2* items;
    uint32_t* task0;
    uint2* tasks;
    float4* fwd;
    float4* wide;
    float4* shv;
    float* term;
    float4* rays;
    uint32_t* ray_count;
    uint32_t* mis_list;
    uint32_t* mis_count;
    uint32_t* count;
};

static FrameWork work_of(const tof_ctx* c) {
    return FrameWork{c->pt,   c->direct, c->prev_pix, c->wsum,      c->nb,       c->items,     c->task0,
                     c->tasks, c->fwd,   c->wide,     c->shv,       c->term,     c->rays,      c->ray_count,
                     c->mis_list, c->mis_count, c->count};
}

static void set_work(tof_ctx* c, const FrameWork& w) {
    c->pt = w.pt;
    c->direct = w.direct;
    c->prev_pix = w.prev_pix;
    c->wsum = w.wsum;
    c->nb = w.nb;
    c->items = w.items;
    c->task0 = w.task0;
    c->tasks = w.tasks;
    c->fwd = w.fwd;
    c->wide = w.wide;
    c->shv = w.shv;
    c->term = w.term;
    c->rays = w.rays;
    c->ray_count = w.ray_count;
    c->mis_list = w.mis_list;
    c->mis_count = w.mis_count;
    c->count = w.count;
}

// Lay the context's frame work space for chunk plan `pl` out from `base`
// (256-byte aligned parts, the sizes tof_sensor_set allocates for its plan);
// returns the bytes it spans.  base == nullptr only measures.
static size_t carve_work(const tof_ctx* c, const tofh::ChunkPlan& pl, char* base, FrameWork& w) {
    size_t off = 0;
    auto take = [&](auto*& ptr, size_t count) {
        using T = typename std::remove_reference<decltype(*ptr)>::type;
        off = (off + 255) & ~(size_t)255;
        ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
    };
    const size_t P = (size_t)c->s.P, B = (size_t)c->s.B;
    const size_t nq = (size_t)tofd::kRaySubQueues * tofd::kCounterStride;
    take(w.pt, P * B);
    take(w.direct, P);
    take(w.prev_pix, P);
    take(w.wsum, 2 * P);
    take(w.nb, P * (size_t)std::max(c->s.k, 1));
    take(w.items, P * B);
    take(w.task0, P * B);
    take(w.tasks, pl.task_cap);
    take(w.fwd, pl.task_cap);
    w.wide = nullptr;
    if (shrink_mix(c->sd)) take(w.wide, kRecF4 * P);
    take(w.shv, 2 * pl.task_cap);
    take(w.term, pl.term_cap);
    take(w.rays, 2 * pl.ray_cap);
    take(w.ray_count, nq);
    take(w.mis_list, pl.term_cap);
    take(w.mis_count, nq);
    take(w.count, 64);
    return off;
}

tof_status tof_render_frame_noalloc(tof_ctx* c, const tof_frame_desc* fr, float* out_image, float* out_hist,
                                    float* out_pt_image, float* out_pt_hist, void* stream) {
    if (!c || !fr) return TOF_ERR_INVALID_ARG;
    if (!c->has_scene || !c->has_sensor) return TOF_ERR_NOT_READY;
    // the context's chunk plan, or one with a lower ray budget (more, smaller
    // chunks of the reuse passes; results do not depend on the chunking) so
    // that the work space fits the array
    FrameWork w{};
    tofh::ChunkPlan pl = c->plan;
    size_t rays = pl.rays;
    while (carve_work(c, pl, nullptr, w) > kScratchBytes) {
        if (rays <= 1) return TOF_ERR_OUT_OF_MEMORY;   // the per-(pixel, plane) parts alone do not fit
        rays /= 2;
        pl = plan_of(c, rays);
    }
    HIP_TRY(hipSetDevice(c->device));
    void* base = nullptr;
    HIP_TRY(scratch_ptr(c->device, &base));
    carve_work(c, pl, static_cast<char*>(base), w);
    // every buffer of the work space is written by the frame's own kernels
    // before it is read (counters and chunk windows by k_fill_u32 launches),
    // so the previous call's contents do not matter
    const FrameWork own = work_of(c);
    const tofh::ChunkPlan own_plan = c->plan;
    const bool timing = c->timing, sync_counts = c->sync_counts;
    c->timing = false;   // event timing creates events on demand: not recorded here
    c->sync_counts = false;   // no wait for the device inside the call: every chunk is launched
    // the array's deposits are whatever its last user left: filled here;
    // the context's own buffer keeps its state
    const bool pt_zero = c->pt_zero;
    c->pt_zero = false;
    set_work(c, w);
    c->plan = pl;
    const tof_status st = tof_render_frame(c, fr, out_image, out_hist, out_pt_image, out_pt_hist, stream);
    set_work(c, own);
    c->plan = own_plan;
    c->timing = timing;
    c->sync_counts = sync_counts;
    c->pt_zero = pt_zero;
    return st;
}

}  // extern "C"
