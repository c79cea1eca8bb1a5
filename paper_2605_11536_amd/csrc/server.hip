// Request loop over render streams on one device (host code).
//
// Every stream is a full ToF ReSTIR context (scene, sensor, resident
// reservoirs, G-buffers and geometry of the last two frames) with its own HIP
// stream.  A stream is admitted when its footprint fits in what the server's
// HBM budget has left; otherwise it waits, first come first served, until a
// close frees memory.  A submitted frame of an admitted stream is enqueued on
// the stream's HIP stream at once, so frames of different streams run
// concurrently on the device while frames of one stream stay in order (their
// temporal reuse depends on it); frames of a waiting stream are held and
// enqueued when it is admitted.  Completion is tracked with one HIP event per
// frame.  All calls may come from any host thread (one mutex).
//
// Memory: the server allocates its whole HBM budget once, as one arena, plus
// a small pinned host arena for the streams' upload rings.  An admitted
// stream gets one contiguous region of its footprint (best fit) that its
// context fills front to back, so admission calls no hipMalloc (whose page
// clearing costs ~10 ms per GB) and closing calls no hipFree (which waits
// for the whole device).  A closed stream's region returns to the arena once
// its HIP stream is idle; waiting streams are then admitted in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "tof.h"
#include "arena.h"
#include "tof_internal.h"

namespace {

// deep copy of a scene description (the caller's arrays may go away before
// the stream is admitted)
struct SceneCopy {
    std::vector<int32_t> type, material, grid, mtype;
    std::vector<float> sphere, mparams, vertices;
    tof_scene_desc desc{};

    explicit SceneCopy(const tof_scene_desc& d) {
        const size_t O = (size_t)d.num_objects, M = (size_t)d.num_materials, V = (size_t)std::max(d.num_vertices, 0);
        type.assign(d.object_type, d.object_type + O);
        material.assign(d.object_material, d.object_material + O);
        grid.assign(d.object_grid, d.object_grid + 5 * O);
        sphere.assign(d.object_sphere, d.object_sphere + 4 * O);
        mtype.assign(d.material_type, d.material_type + M);
        mparams.assign(d.material_params, d.material_params + 3 * M);
        if (V) vertices.assign(d.vertices, d.vertices + 3 * V);
        desc = d;
        desc.object_type = type.data();
        desc.object_material = material.data();
        desc.object_grid = grid.data();
        desc.object_sphere = sphere.data();
        desc.material_type = mtype.data();
        desc.material_params = mparams.data();
        desc.vertices = V ? vertices.data() : nullptr;
    }
};

struct Request {
    uint64_t ticket = 0;
    int stream = -1;
    tof_frame_desc frame{};
    std::vector<float> xforms;
    std::vector<float> velocities;   // copy of the caller's array (empty = NULL): a held frame outlives it
    float* out[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t start = nullptr;      // recorded on the stream right before the frame's work
    hipEvent_t done = nullptr;
    bool dispatched = false;
    int waiters = 0;                 // tof_server_wait calls blocked on `done`: only they retire the ticket
    tof_status status = TOF_OK;
};

struct Region {
    size_t dev_off = 0, dev_bytes = 0, host_off = 0, host_bytes = 0;
};

struct Stream {
    int id = -1;
    std::unique_ptr<SceneCopy> scene;
    tof_sensor_desc sensor{};
    uint64_t seed = 0;
    size_t footprint = 0, pinned = 0;
    Region region;
    tof_ctx* ctx = nullptr;
    hipStream_t hs = nullptr;
    hipGraphExec_t exec = nullptr;   // the last frame's graph (graph mode), updated frame to frame
    bool admitted = false, failed = false;
    std::deque<uint64_t> held;   // frames submitted before admission
};

}  // namespace

struct Closed {
    tof_ctx* ctx = nullptr;
    hipStream_t hs = nullptr;
    size_t footprint = 0;
    Region region;
    hipGraphExec_t exec = nullptr;
};

struct tof_server {
    int device = 0;
    size_t budget = 0, used = 0;
    char* dev_base = nullptr;     // the HBM arena
    char* host_base = nullptr;    // the pinned host arena
    size_t host_size = 0;
    tofh::Arena dev_arena, host_arena;
    std::vector<hipStream_t> idle_streams;
    std::vector<Closed> closed;   // closed streams whose region is not returned yet
    std::mutex mu;
    bool graphs = false;          // frames recorded into a graph per stream and launched as one
    int next_stream = 0;
    uint64_t next_ticket = 1;
    std::map<int, Stream> streams;
    std::deque<int> waiting;     // streams in admission order
    std::map<uint64_t, std::unique_ptr<Request>> requests;
};

namespace {

constexpr size_t kPinnedArena = (size_t)64 << 20;

tof_status hip_status(hipError_t e) { return e == hipSuccess ? TOF_OK : TOF_ERR_DEVICE; }

// Graph mode: the frame's work is recorded by stream capture into a graph
// and launched as one; the stream's executable graph is updated from it when
// the frame has the same shape as the last (kernels, copies and their order),
// else built anew.  A recording that fails is ended before returning.
tof_status render_graph(Stream& st, Request& r) {
    const tof_status ep = tofh::prepare_frame_capture(st.ctx);
    if (ep != TOF_OK) return ep;
    if (hipStreamBeginCapture(st.hs, hipStreamCaptureModeRelaxed) != hipSuccess) return TOF_ERR_DEVICE;
    tof_status e = tof_render_frame(st.ctx, &r.frame, r.out[0], r.out[1], r.out[2], r.out[3], (void*)st.hs);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(st.hs, &g) != hipSuccess && e == TOF_OK) e = TOF_ERR_DEVICE;
    if (e == TOF_OK) {
        bool updated = false;
        if (st.exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            updated = hipGraphExecUpdate(st.exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
            if (!updated) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(st.exec);
                st.exec = nullptr;
            }
        }
        if (!updated && hipGraphInstantiate(&st.exec, g, nullptr, nullptr, 0) != hipSuccess) {
            st.exec = nullptr;
            e = TOF_ERR_DEVICE;
        }
        if (e == TOF_OK && hipGraphLaunch(st.exec, st.hs) != hipSuccess) e = TOF_ERR_DEVICE;
        if (e == TOF_OK) e = tofh::record_frame_events(st.ctx, st.hs);
    }
    if (g) (void)hipGraphDestroy(g);
    return e;
}

tof_status dispatch(tof_server* s, Stream& st, Request& r) {
    tof_status e = hip_status(hipEventRecord(r.start, st.hs));
    if (e == TOF_OK)
        e = s->graphs ? render_graph(st, r)
                      : tof_render_frame(st.ctx, &r.frame, r.out[0], r.out[1], r.out[2], r.out[3], (void*)st.hs);
    if (e == TOF_OK) e = hip_status(hipEventRecord(r.done, st.hs));
    r.status = e;
    r.dispatched = true;
    return e;
}

void release(tof_server* s, tof_ctx* ctx, hipStream_t hs, const Region& r, hipGraphExec_t exec) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ctx) tof_destroy(ctx);   // region context: waits for its own frames only
    if (hs) s->idle_streams.push_back(hs);
    s->dev_arena.free(r.dev_off, r.dev_bytes);
    s->host_arena.free(r.host_off, r.host_bytes);
}

// return the regions of closed streams whose HIP stream is idle
void reap(tof_server* s) {
    for (size_t i = 0; i < s->closed.size();) {
        Closed& z = s->closed[i];
        if (hipStreamQuery(z.hs) != hipSuccess) {
            ++i;
            continue;
        }
        release(s, z.ctx, z.hs, z.region, z.exec);
        s->used -= z.footprint;
        s->closed[i] = s->closed.back();
        s->closed.pop_back();
    }
}

// Create the context of a stream in a region of the arenas and enqueue its
// held frames.  *no_room when no hole fits it (nothing changed).
tof_status admit(tof_server* s, Stream& st, bool* no_room) {
    *no_room = false;
    Region r;
    r.dev_bytes = st.footprint;
    r.host_bytes = st.pinned;
    if (!s->dev_arena.alloc(r.dev_bytes, r.dev_off)) {
        *no_room = true;
        return TOF_OK;
    }
    if (!s->host_arena.alloc(r.host_bytes, r.host_off)) {
        s->dev_arena.free(r.dev_off, r.dev_bytes);
        *no_room = true;
        return TOF_OK;
    }
    tof_status e = tofh::create_in_region(&st.ctx, s->device, s->dev_base + r.dev_off, r.dev_bytes,
                                          s->host_base + r.host_off, r.host_bytes, st.seed);
    if (e == TOF_OK) e = tof_scene_upload(st.ctx, &st.scene->desc);
    if (e == TOF_OK) e = tof_sensor_set(st.ctx, &st.sensor);
    if (e == TOF_OK) {
        if (!s->idle_streams.empty()) {
            st.hs = s->idle_streams.back();
            s->idle_streams.pop_back();
        } else {
            e = hip_status(hipStreamCreateWithFlags(&st.hs, hipStreamNonBlocking));
        }
    }
    if (e != TOF_OK) {
        release(s, st.ctx, st.hs, r, nullptr);
        st.ctx = nullptr;
        st.hs = nullptr;
        return e;
    }
    st.region = r;
    st.admitted = true;
    s->used += st.footprint;
    while (!st.held.empty()) {
        Request& q = *s->requests[st.held.front()];
        st.held.pop_front();
        dispatch(s, st, q);
    }
    return TOF_OK;
}

// admit waiting streams, first come first served, while the first one fits
void admit_waiting(tof_server* s) {
    reap(s);
    while (!s->waiting.empty()) {
        Stream& st = s->streams[s->waiting.front()];
        bool no_room = false;
        const tof_status e = admit(s, st, &no_room);
        if (no_room) break;
        s->waiting.pop_front();
        if (e != TOF_OK) {   // its frames fail; the stream stays closed to new work
            for (uint64_t t : st.held) {
                s->requests[t]->status = e;
                s->requests[t]->dispatched = true;
            }
            st.held.clear();
            st.failed = true;
        }
    }
}

}  // namespace

extern "C" {

tof_status tof_server_create(tof_server** out, int device, size_t hbm_budget_bytes) {
    if (!out || hbm_budget_bytes == 0) return TOF_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TOF_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return TOF_ERR_DEVICE;
    tof_server* s = new (std::nothrow) tof_server();
    if (!s) return TOF_ERR_OUT_OF_MEMORY;
    s->device = device;
    s->budget = (hbm_budget_bytes + 255) & ~(size_t)255;
    s->host_size = kPinnedArena;
    if (hipMalloc((void**)&s->dev_base, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return TOF_ERR_OUT_OF_MEMORY;
    }
    if (hipHostMalloc((void**)&s->host_base, s->host_size) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(s->dev_base);
        delete s;
        return TOF_ERR_OUT_OF_MEMORY;
    }
    s->dev_arena.reset(s->budget);
    s->host_arena.reset(s->host_size);
    *out = s;
    return TOF_OK;
}

void tof_server_destroy(tof_server* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : s->requests) {
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
        if (kv.second->start) (void)hipEventDestroy(kv.second->start);
    }
    for (auto& kv : s->streams)
        if (kv.second.admitted) release(s, kv.second.ctx, kv.second.hs, kv.second.region, kv.second.exec);
    for (Closed& z : s->closed) release(s, z.ctx, z.hs, z.region, z.exec);
    for (hipStream_t h : s->idle_streams) (void)hipStreamDestroy(h);
    (void)hipFree(s->dev_base);
    (void)hipHostFree(s->host_base);
    delete s;
}

tof_status tof_server_open(tof_server* s, const tof_scene_desc* scene, const tof_sensor_desc* sensor, uint64_t seed,
                           int* stream_id, int* admitted) {
    if (!s || !scene || !sensor || !stream_id) return TOF_ERR_INVALID_ARG;
    size_t fp = 0;
    tof_status e = tof_footprint(scene, sensor, &fp);
    if (e != TOF_OK) return e;
    const size_t pinned = tofh::scene_pinned_bytes(*scene);
    std::lock_guard<std::mutex> lock(s->mu);
    if (fp > s->budget || pinned > s->host_size) return TOF_ERR_OUT_OF_MEMORY;   // could never be admitted
    if (hipSetDevice(s->device) != hipSuccess) return TOF_ERR_DEVICE;
    const int id = s->next_stream++;
    Stream& st = s->streams[id];
    st.id = id;
    st.scene.reset(new SceneCopy(*scene));
    st.sensor = *sensor;
    st.seed = seed;
    st.footprint = fp;
    st.pinned = pinned;
    s->waiting.push_back(id);
    admit_waiting(s);
    if (st.failed) {   // admission itself failed (invalid settings, device error)
        s->streams.erase(id);
        return TOF_ERR_DEVICE;
    }
    *stream_id = id;
    if (admitted) *admitted = st.admitted ? 1 : 0;
    return TOF_OK;
}

tof_status tof_server_submit(tof_server* s, int stream_id, const tof_frame_desc* frame, float* out_image,
                             float* out_hist, float* out_pt_image, float* out_pt_hist, uint64_t* ticket) {
    if (!s || !frame || !frame->object_xforms || !ticket) return TOF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end() || it->second.failed) return TOF_ERR_INVALID_ARG;
    Stream& st = it->second;
    if (hipSetDevice(s->device) != hipSuccess) return TOF_ERR_DEVICE;
    std::unique_ptr<Request> r(new Request());
    r->ticket = s->next_ticket++;
    r->stream = stream_id;
    r->frame = *frame;
    r->xforms.assign(frame->object_xforms, frame->object_xforms + 12 * (size_t)st.scene->desc.num_objects);
    r->frame.object_xforms = r->xforms.data();
    if (frame->object_velocities) {
        r->velocities.assign(frame->object_velocities,
                             frame->object_velocities + 6 * (size_t)st.scene->desc.num_objects);
        r->frame.object_velocities = r->velocities.data();
    }
    r->out[0] = out_image;
    r->out[1] = out_hist;
    r->out[2] = out_pt_image;
    r->out[3] = out_pt_hist;
    if (hipEventCreate(&r->done) != hipSuccess) return TOF_ERR_DEVICE;
    if (hipEventCreate(&r->start) != hipSuccess) {
        (void)hipEventDestroy(r->done);
        return TOF_ERR_DEVICE;
    }
    Request& rr = *r;
    s->requests[r->ticket] = std::move(r);
    *ticket = rr.ticket;
    if (st.admitted) return dispatch(s, st, rr);
    st.held.push_back(rr.ticket);
    return TOF_OK;
}

// Poll a dispatched request under the server lock.  A finished request is
// retired (event destroyed, ticket erased) unless a tof_server_wait is blocked
// on its event, or `retire` is false: the waiter retires it.
static tof_status poll_locked(tof_server* s, std::map<uint64_t, std::unique_ptr<Request>>::iterator it, int* done,
                              bool retire, float* gpu_ms) {
    Request& r = *it->second;
    *done = 0;
    if (!r.dispatched) return TOF_OK;
    tof_status st = r.status;
    if (st == TOF_OK) {
        const hipError_t q = hipEventQuery(r.done);
        if (q == hipErrorNotReady) return TOF_OK;
        if (q != hipSuccess) st = TOF_ERR_DEVICE;
    }
    *done = 1;
    if (gpu_ms) {
        *gpu_ms = -1.f;
        float ms = 0.f;
        if (st == TOF_OK && hipEventElapsedTime(&ms, r.start, r.done) == hipSuccess) *gpu_ms = ms;
    }
    if (!retire || r.waiters > 0) return st;
    (void)hipEventDestroy(r.done);
    (void)hipEventDestroy(r.start);
    s->requests.erase(it);
    if (!s->closed.empty()) admit_waiting(s);
    return st;
}

tof_status tof_server_query(tof_server* s, uint64_t ticket, int* done) {
    return tof_server_query_timed(s, ticket, done, nullptr);
}

tof_status tof_server_query_timed(tof_server* s, uint64_t ticket, int* done, float* gpu_ms) {
    if (!s || !done) return TOF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return TOF_ERR_INVALID_ARG;
    return poll_locked(s, it, done, true, gpu_ms);
}

tof_status tof_server_wait(tof_server* s, uint64_t ticket) {
    if (!s) return TOF_ERR_INVALID_ARG;
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->requests.find(ticket);
        if (it == s->requests.end()) return TOF_ERR_INVALID_ARG;
        if (!it->second->dispatched) return TOF_ERR_NOT_READY;   // its stream is not admitted yet
        it->second->waiters++;    // keeps the event alive while this thread blocks on it
        ev = it->second->done;
    }
    const hipError_t e = hipEventSynchronize(ev);
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return TOF_ERR_INVALID_ARG;   // cannot happen: only waiters retire it now
    it->second->waiters--;
    int done = 0;
    const tof_status st = poll_locked(s, it, &done, it->second->waiters == 0, nullptr);
    if (e != hipSuccess) return TOF_ERR_DEVICE;
    return st;
}

tof_status tof_server_close(tof_server* s, int stream_id) {
    if (!s) return TOF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end()) return TOF_ERR_INVALID_ARG;
    Stream& st = it->second;
    if (hipSetDevice(s->device) != hipSuccess) return TOF_ERR_DEVICE;
    if (st.admitted) {
        // its region returns once its queued frames are done (see reap)
        s->closed.push_back(Closed{st.ctx, st.hs, st.footprint, st.region, st.exec});
    } else {
        for (auto w = s->waiting.begin(); w != s->waiting.end(); ++w)
            if (*w == stream_id) {
                s->waiting.erase(w);
                break;
            }
        for (uint64_t t : st.held) {   // frames that never ran
            s->requests[t]->status = TOF_ERR_NOT_READY;
            s->requests[t]->dispatched = true;
        }
    }
    s->streams.erase(it);
    admit_waiting(s);
    return TOF_OK;
}

tof_status tof_server_set_graphs(tof_server* s, int enabled) {
    if (!s || (enabled != 0 && enabled != 1)) return TOF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    s->graphs = enabled != 0;
    return TOF_OK;
}

tof_status tof_server_info(tof_server* s, size_t* used_bytes, int* admitted, int* waiting) {
    if (!s) return TOF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    reap(s);
    int a = 0;
    for (auto& kv : s->streams) a += kv.second.admitted ? 1 : 0;
    if (used_bytes) *used_bytes = s->used;
    if (admitted) *admitted = a;
    if (waiting) *waiting = (int)s->waiting.size();
    return TOF_OK;
}

}  // extern "C"
