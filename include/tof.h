/*
 * tof.h -- C ABI of the ToF ReSTIR hot path on AMD Instinct MI355X (gfx950).
 *
 * The library renders time-of-flight measurements -- a time-gated image and/or
 * a transient histogram per frame -- with spatio-temporal reservoir
 * resampling and the path-length-aware shift of Kim, Jarosz and Pediredla,
 * "ToF ReSTIR" (ACM TOG 45(4), 2026):
 *   - the measurement is the ToF path integral (Sec. 3.1,
 *     eq. tof_path_integral) with box time gates;
 *   - per pixel and per time bin a reservoir is filled by RIS over path-tree
 *     sub-paths (Sec. 3.2.1, 3.2.4; Sec. 4.5 per-bin deposit);
 *   - temporal and spatial reuse use generalized RIS with the generalized
 *     balance heuristic (Sec. 3.2.3, eq. GRIS_resampling_weight and
 *     eq. GRIS_MIS_weight);
 *   - reused paths are shifted by random replay + reconnection and then the
 *     reconnection vertex is moved by a Newton solve so that the shifted path
 *     keeps its optical length (Sec. 4.1 eq. path_length_constraint, Sec. 4.2,
 *     Sec. 4.3 average-gradient gauge and implicit-function Jacobian).
 *
 * Conventions shared by every entry point:
 *   - Status codes only; no exception crosses the ABI.  On any error nothing
 *     observable changes (no partial state).
 *   - Host pointers passed in descriptors are read during the call only; the
 *     caller keeps ownership.  Device pointers (outputs) are owned by the
 *     caller and must stay valid until the work enqueued on `stream` finishes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - One context per host thread, or external locking.
 *   - Units: c = 1, so time and optical path length are the same quantity.
 */
#ifndef TOF_H
#define TOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tof_ctx tof_ctx;

typedef enum {
    TOF_OK = 0,
    TOF_ERR_INVALID_ARG = -1,      /* a NULL/out-of-range argument or inconsistent descriptor */
    TOF_ERR_OUT_OF_MEMORY = -2,    /* footprint above the context's HBM budget, or hipMalloc failed */
    TOF_ERR_INVALID_SCENE = -3,    /* NaN/Inf vertices, bad object ranges, degenerate objects */
    TOF_ERR_NOT_READY = -4,        /* render before a scene upload and a sensor set */
    TOF_ERR_DEVICE = -5,           /* a HIP runtime error (launch, copy, fault) */
    TOF_ERR_UNIMPLEMENTED = -6
} tof_status;

enum { TOF_OBJ_GRID = 0, TOF_OBJ_SPHERE = 1 };
enum { TOF_MAT_LAMBERT = 0, TOF_MAT_GGX = 1 };
enum { TOF_CAMERA_PINHOLE = 0, TOF_CAMERA_ORTHO = 1 };
enum { TOF_LIGHT_POINT = 0, TOF_LIGHT_CONFOCAL = 1 };
enum { TOF_SHIFT_NAIVE = 0, TOF_SHIFT_PATHLEN = 1 };
/* What the planes measure: the optical path length l (Sec. 3.1), or the path
 * velocity u = -dl/dt (Sec. 4.6, eq. optical_path_velocity; the Doppler
 * frequency shift is f0 u / c) in scene units per second. */
enum { TOF_DOMAIN_TIME = 0, TOF_DOMAIN_VELOCITY = 1 };
enum { TOF_STAGE_CANONICAL = 0, TOF_STAGE_TEMPORAL = 1, TOF_STAGE_FINAL = 2 };

/* Scene: rigid objects made of a regular vertex lattice ("grid": cell (i,j)
 * split into triangles (V[i,j],V[i+1,j],V[i,j+1]) and (V[i+1,j+1],V[i,j+1],
 * V[i+1,j]); the surface chart is xi = (u,v) in cell units) or analytic
 * spheres (chart xi = (theta, phi) about the object's local z axis).  These
 * charts carry the 2-D parameterisation of the reconnection vertex
 * (Sec. 4.2).  All arrays are host memory, copied during the call. */
typedef struct {
    int32_t num_objects;
    const int32_t* object_type;      /* [num_objects] TOF_OBJ_* */
    const int32_t* object_material;  /* [num_objects] index into the material arrays */
    const int32_t* object_grid;      /* [num_objects*5] nu, nv, wrap_u, wrap_v, vertex_offset
                                        (grid: (nu+1)*(nv+1) object-local vertices, row-major in v) */
    const float* object_sphere;      /* [num_objects*4] local centre xyz, radius (spheres) */
    int32_t num_materials;
    const int32_t* material_type;    /* [num_materials] TOF_MAT_* */
    const float* material_params;    /* [num_materials*3] albedo (Lambert), alpha, F0 (GGX) */
    int32_t num_vertices;
    const float* vertices;           /* [num_vertices*3] object-local positions */
    float scene_scale;               /* s_c: ray offsets are 1e-4*s_c, reconnection distance 0.01*s_c */
} tof_scene_desc;

/* Sensor, time domain and reuse settings.  The time domain is a gate
 * [gate_center - gate_width/2, gate_center + gate_width/2) and/or n_bins
 * histogram bins [bin_t0 + b*bin_width, bin_t0 + (b+1)*bin_width); each has its
 * own reservoir plane per pixel (Sec. 4.5).  In the velocity domain the same
 * gate and bins lie on the path-velocity axis, and the reconnection shift keeps
 * the path velocity instead of the length (Sec. 4.6).  Rendering may be restricted to a
 * crop [crop_x0, crop_x0+width) x [crop_y0, crop_y0+height) of a full_width x
 * full_height image (random streams are keyed by full-image pixel index). */
typedef struct {
    int32_t width, height, full_width, full_height, crop_x0, crop_y0;
    int32_t camera_model;            /* TOF_CAMERA_*; ORTHO scans a plane (NLOS relay wall) */
    int32_t light_model;             /* TOF_LIGHT_*; CONFOCAL = laser spot at each pixel's primary hit */
    int32_t count_camera_leg;        /* include |camera - first hit| in the path length */
    int32_t jitter;                  /* box-filter pixel jitter */
    float light_intensity;           /* point intensity, or laser power for CONFOCAL */
    int32_t gate_enabled;
    float gate_center, gate_width;
    int32_t n_bins;
    float bin_t0, bin_width;
    int32_t n_min, n_max;            /* scattering vertices per path, 1 <= n_min <= n_max <= 4 */
    int32_t m_init;                  /* path trees per pixel, 1..32 */
    int32_t temporal;                /* temporal reuse on/off */
    int32_t spatial_rounds, spatial_k, spatial_radius;   /* rounds 0..4, k 0..8, radius px */
    float m_cap;                     /* confidence cap of the temporal candidate */
    float newton_tol_rel;            /* Newton tolerance as a fraction of the gate/bin width */
    int32_t newton_max_iter;
    float j_max;                     /* shifts with |J| outside [1/j_max, j_max] are rejected */
    int32_t shift_mode;              /* TOF_SHIFT_NAIVE (replay+reconnect) or TOF_SHIFT_PATHLEN */
    int32_t include_direct;          /* add the deterministic 1-vertex term */
    int32_t debug_stage;             /* TOF_STAGE_*: which reservoirs the splat shows */
    int32_t bin_radius;              /* bin-axis reuse (Sec. 4.5) between the temporal and the spatial
                                        pass: bin b resamples bins b +- 1..bin_radius of the same pixel,
                                        shifted by Delta l = (b - b') * bin_width; 0 = off, at most 4 */
    float shrink_k;                  /* shrink mapping of initial gate samples (Sec. 4.4.2): candidates come
                                        from a gate shrink_k times wider (same centre) and the RIS winner
                                        is moved into the gate by the path-length-aware shift with
                                        Delta l = (l - l0) / K + l0 - l, its weight scaled by the shift's
                                        Jacobian / K; all samples in the wide gate (the paper's R = 1,
                                        biased low where shrinks fail).  1 = off, at most 1000 */
    int32_t domain;                  /* TOF_DOMAIN_*; the velocity domain requires bin_radius 0 and
                                        shrink_k 1 (both shifts are defined on path lengths) */
    float shrink_r;                  /* with shrink_k > 1: the fraction R in [0, 1] of the m_init path trees
                                        whose gate candidates come from the wide gate (the first
                                        round(R m_init) trees).  R = 1: all, as described at shrink_k.
                                        0 < round(R m_init) < m_init: the others sample the gate itself
                                        and the two reservoirs are merged into the gate by GRIS with the
                                        generalized balance heuristic (Sec. 4.4.2), unbiased; the wide
                                        technique's density at a gate path comes through the inverse
                                        map, Delta l = K (l - l0) + l0 - l.  round(R m_init) = 0: no
                                        shrink mapping */
    int32_t round_trip;              /* 1: a path-length-aware shift is kept only if the inverse shift of its
                                        result (the same Newton iteration from the shifted vertex, Delta l
                                        negated) converges back to within the reconnection distance
                                        0.01 s_c of the source's reconnection vertex.  GRIS is unbiased only
                                        if each shift is a bijection (Sec. 3.2.3); the gauge of Sec. 4.3
                                        makes the exact root reversible, but the iteration can land on
                                        another root or fail one way only near paths whose length is
                                        stationary on the chart (the first return of a confocal scan), which
                                        biases the reuse upward there.  0: no check; 0 or 1 */
    int32_t mis_mode;                /* MIS weights of the spatial reuse passes: 0 the generalized balance
                                        heuristic (Sec. 3.2.3, eq. GRIS_MIS_weight); 1 pairwise MIS, the
                                        canonical technique split into as many parts as there are
                                        neighbours, each part paired with one neighbour under the balance
                                        heuristic and the pair weighted by its share of the confidence
                                        (also unbiased; K MIS shifts per pixel-plane instead of K (K + 1)).
                                        Temporal and bin-axis reuse use the former in both */
} tof_sensor_desc;

/* Per-frame poses.  object_xforms: host [num_objects*12], rigid 3x4 row-major
 * [R | t] mapping object-local to world coordinates for this frame.  The
 * velocities are read in the velocity domain only (all finite, else
 * TOF_ERR_INVALID_ARG): object_velocities is host [num_objects*6] or NULL (all
 * at rest), linear v then angular w per object, so that a point x of the
 * object moves at v + w x (x - t); cam_vel and light_vel move the camera and
 * the point light (the confocal spot moves with the surface it lies on). */
typedef struct {
    int32_t frame_index;             /* keys the random streams of this frame */
    float cam_pos[3], cam_fwd[3], cam_up[3];
    float fov_y_deg;                 /* pinhole vertical field of view */
    float ortho_half[2];             /* orthographic half extents */
    float light_pos[3];              /* point light position */
    const float* object_xforms;
    const float* object_velocities;
    float cam_vel[3], light_vel[3];
} tof_frame_desc;

typedef struct {
    uint64_t shifts;                 /* shift attempts (temporal + spatial, incl. MIS shifts) */
    uint64_t shifts_ok;              /* shifts with a non-zero target in the destination */
    uint64_t newton_attempts;        /* path-length shifts that reached the Newton solve */
    uint64_t newton_converged;       /* "Newton SR" numerator (Sec. 6, Table 1) */
    uint64_t newton_iters;           /* iterations summed over converged solves */
    uint64_t newton_paths_ok;        /* "actual SR" numerator: converged and fully valid */
    uint64_t rays;                   /* closest-hit + shadow rays traced */
    uint64_t frames;                 /* frames rendered */
    uint64_t bvh_overflow;           /* traversal stack overflows (must be 0) */
    uint64_t node_visits;            /* BVH internal nodes visited (four child-box tests each) */
    uint64_t tri_tests;              /* ray/triangle tests */
    uint64_t bad_records;            /* reservoir records rejected as malformed (must be 0) */
} tof_stats;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps what the
 * context may allocate (0 = no cap).  seed keys every random stream
 * (Philox4x64-10 with key (seed, 0)).  *out receives the context. */
tof_status tof_create(tof_ctx** out, int device, size_t hbm_budget_bytes, uint64_t seed);

/* Release every device allocation of the context (synchronizes the device). */
void tof_destroy(tof_ctx* ctx);

/* Copy the scene to the device and validate it (TOF_ERR_INVALID_ARG for fewer
 * than 1 or more than 4095 objects, since a reservoir record names a path's
 * vertex objects in 12 bits; TOF_ERR_INVALID_SCENE for malformed objects or
 * 2^28 triangles or more).  Drops reservoir history. */
tof_status tof_scene_upload(tof_ctx* ctx, const tof_scene_desc* scene);

/* Which builder makes the mesh objects' trees at the next tof_scene_upload
 * (the traversal the paper's GPU ray tracing needs, Sec. 6; any tree gives
 * the same hits: closest hit is the least (distance, triangle id) and the
 * boxes are conservative, so images do not depend on the builder).
 * TOF_BVH_HOST: binned SAH on the host, collapsed to 4-wide nodes (the
 * default).  TOF_BVH_DEVICE: built on the GPU from a Morton-ordered radix
 * sort by agglomerative clustering (PLOC), with SAH leaf sizes and the same
 * collapse; it needs about 260 bytes of device work space per triangle
 * during the upload (counted by tof_footprint).  Both cap leaves at 4
 * triangles.  TOF_ERR_INVALID_ARG for another value. */
enum { TOF_BVH_HOST = 0, TOF_BVH_DEVICE = 1 };
tof_status tof_set_bvh_builder(tof_ctx* ctx, int32_t builder);

/* The mesh objects' trees of the last tof_scene_upload: the builder, the
 * 4-wide node count, the refit levels, the clustering rounds (device
 * builder), the build's wall time in ms (host-side, readbacks included),
 * and, when leaf_triangles is not NULL, the triangle of every leaf slot
 * ([num_triangles] host array, filled after a device synchronization).
 * TOF_ERR_NOT_READY before a scene upload. */
typedef struct {
    int32_t builder;
    int32_t num_nodes;
    int32_t num_levels;
    int32_t rounds;
    int32_t num_triangles;
    int32_t pad;
    double build_ms;
} tof_bvh_info;
tof_status tof_get_bvh_info(tof_ctx* ctx, tof_bvh_info* info, int32_t* leaf_triangles);

/* Set sensor and time-domain settings and (re)allocate per-pixel state after
 * checking the footprint against the budget.  Any change drops the temporal
 * history (reservoirs are reset), except a move of gate_center alone: that
 * keeps the history, and the next frame's temporal reuse shifts the previous
 * frame's paths by the move, Delta l = new centre - old centre (Sec. 4.1,
 * time-gate shifting).  Bins never move.  TOF_ERR_INVALID_ARG for settings
 * out of range, including width * height * planes >= 2^31 (work items use
 * 32-bit indices).  Per-(pixel, plane) reservoirs are
 * allocated densely; the reuse passes run over chunks of work items whose
 * work space is sized to a ray budget, so the footprint grows with the
 * planes mainly through the reservoirs. */
tof_status tof_sensor_set(tof_ctx* ctx, const tof_sensor_desc* sensor);

/* Render one frame asynchronously on `stream`, in the order of the ReSTIR
 * pipeline (Sec. 3.2.4: initial candidates, temporal reuse, spatial reuse,
 * final shading; Sec. 6 real-time temporal reuse): BVH refit for the frame's
 * transforms, G-buffer, path trees + initial RIS, temporal reuse (when a
 * previous frame exists), spatial rounds, splat.  Outputs are device float32
 * arrays owned by the caller, plane-major, each value divided by its gate or
 * bin width; any may be NULL:
 *   out_image    [height*width]           ReSTIR gate image
 *   out_hist     [n_bins*height*width]    ReSTIR transient histogram
 *   out_pt_image / out_pt_hist            plain ToF path tracing of the same frame
 * The frames of one context depend on each other (temporal reuse, scratch
 * work lists): issue them on one stream, or order the streams.  Calls that
 * read or replace the context's state (stats, timing, history, scene, sensor)
 * wait for the last frame issued, not for the whole device.  When a reuse
 * pass may need more than one chunk of work items (large sensors: planes x
 * pixels beyond one chunk's capacity), the call reads back the pass's item
 * count after counting them on `stream` (a wait for the device that far) and
 * launches only the chunks that hold items; contexts of the server,
 * tof_render_frame_noalloc and a frame issued under stream capture never
 * wait, and launch every chunk the plan allows.  Under stream capture the
 * call also leaves out the events the context's host waits use (the pinned
 * upload ring, the frame's end): recording a frame into a graph is done by
 * the server's graph mode, which records them after launching the graph.
 * The bin-axis
 * pass and the shrink mapping count into the spatial and initial kernel
 * groups of tof_kernel_times.
 * Errors: TOF_ERR_NOT_READY without scene+sensor; TOF_ERR_INVALID_ARG for a
 * NULL frame/xforms or an image requested without a gate; TOF_ERR_DEVICE on a
 * HIP error. */
tof_status tof_render_frame(tof_ctx* ctx, const tof_frame_desc* frame, float* out_image, float* out_hist,
                            float* out_pt_image, float* out_pt_hist, void* stream);

/* For callers that cannot allocate device memory while they render: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The same frame as tof_render_frame (same arguments, errors and
 * results) with its per-frame work space -- work lists, shift terms, MIS list,
 * ray queue and their counters, plain-PT staging, reprojection and neighbour
 * tables -- taken from one static device array of the library instead of the
 * context's buffers: 64 MiB per GPU, held from the first tof_create on that
 * GPU until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree, pinned or event allocation); the context's reservoirs, G-buffers
 * and geometry are used as always.  The reuse passes run over as many chunks
 * as it takes for their work space to fit the array (results do not depend on
 * the chunking).  TOF_ERR_OUT_OF_MEMORY when even the smallest chunks do not
 * fit: the parts sized per (pixel, plane), 16 bytes each, plus 4 (spatial_k +
 * 3) bytes per pixel and about 4 MiB for the smallest chunk must stay under
 * 64 MiB (about 3.5 M pixel-planes with 5 neighbours, e.g. 128x128 pixels
 * with 200 planes).  Every call on a GPU uses that GPU's one array: frames of
 * this entry point that may overlap on one GPU (unordered streams, or several
 * host threads) race on it and must be ordered by the caller.  Kernel timing
 * is not recorded for these frames. */
tof_status tof_render_frame_noalloc(tof_ctx* ctx, const tof_frame_desc* frame, float* out_image, float* out_hist,
                                    float* out_pt_image, float* out_pt_hist, void* stream);

/* Launch shape of the reuse passes: the most blocks (of 128 lanes) that a
 * shift kernel (forward and MIS shifts, the shrink mapping) and the
 * visibility kernel launch per chunk; the occupancy the visibility kernel is
 * compiled for (waves per SIMD: its register budget); the tile of the
 * resampling merge (tasks whose loads a lane issues at once).
 * shift_blocks: a multiple of 64 up to 8192, vis_blocks: a multiple of 64 up
 * to 65536, vis_waves: 5 or 6, merge_tasks: 1, 2 or 4; 0 = the default
 * (8192, 16384, 6, 2).  A smaller shift grid also makes the chunks smaller
 * (each chunk is a whole number of grid sweeps).  Results do not depend on
 * any of them, only speed: which lane shifts or traces what changes, not
 * what is computed.  For callers that tune per workload (frame size, planes,
 * scene); not in the paper.  Kept across sensor changes.  Waits for the
 * context's last frame.  TOF_ERR_INVALID_ARG for a value out of range. */
typedef struct {
    uint32_t shift_blocks;
    uint32_t vis_blocks;
    uint32_t vis_waves;
    uint32_t merge_tasks;
} tof_launch_config;
tof_status tof_set_launch_config(tof_ctx* ctx, const tof_launch_config* config);
tof_status tof_get_launch_config(tof_ctx* ctx, tof_launch_config* config);

/* Pick the launch shape for this context's scene and sensor by timing:
 * frames[0 .. n_frames-1] (host descriptors, 2 <= n_frames <= 64) are
 * rendered from an empty history, once per candidate, on `stream`, and the
 * later half of each run is timed with HIP events; the candidates are the
 * shift grids 8192, 4096, 2048 at the default visibility grid, then the
 * visibility grids 4096, 8192, 32768 at the best of those, then the
 * visibility kernel at 5 waves per SIMD, then merge tiles of 1 and 4
 * tasks, each step at the best so far (a coordinate search).  The fastest is
 * set and returned in *chosen (may be NULL).  The tuning frames leave no other
 * trace: the counters of tof_get_stats are restored, the temporal history is
 * dropped (the next frame renders without temporal reuse), nothing is
 * written to any output.  Errors as tof_render_frame; on an error the
 * previous shape stays. */
tof_status tof_autotune(tof_ctx* ctx, const tof_frame_desc* frames, int n_frames, void* stream,
                        tof_launch_config* chosen);

/* Drop the temporal history (the previous frame's final reservoirs that
 * temporal reuse resamples, Sec. 3.2.4 and Sec. 6): the next frame renders
 * without temporal reuse.  Waits for the context's last frame. */
tof_status tof_reservoirs_reset(tof_ctx* ctx);

/* Accumulated counters (waits for the context's last frame). */
tof_status tof_get_stats(tof_ctx* ctx, tof_stats* out);

/* Reservoir planes of one reservoir set in host memory.  P = width*height,
 * B = n_bins + gate_enabled; element [plane*P + pixel].  meta packs
 * tree | n<<8 | k<<12 | nsfx<<16 (n = path vertices, k = reconnection index,
 * 0 = pure replay); vertex_obj is [4][P*B] (x_{k-1}, p, next vertex or -1 for
 * the light, suffix vertex); vertex_xi is [4][2][P*B] chart coordinates;
 * M is the per-pixel confidence; mask bit (plane) of word [plane/32][pixel]
 * marks non-empty reservoirs. */
typedef struct {
    const float* W;
    const float* phat;
    const float* len;
    const float* pre_pdf;
    const uint32_t* origin_pixel;
    const uint32_t* origin_frame;
    const uint32_t* meta;
    const int32_t* vertex_obj;
    const float* vertex_xi;
    const float* M;
    const uint32_t* mask;
} tof_history_desc;

/* Test support (per-frame parity from an identical history): replace the
 * temporal history -- the final reservoirs of the previously rendered frame --
 * with host-provided reservoirs.  Needs one rendered frame (its G-buffer and
 * geometry stay those of that frame).  Synchronous.  TOF_ERR_NOT_READY before
 * the first frame; TOF_ERR_INVALID_ARG on NULL pointers or out-of-range
 * object ids. */
tof_status tof_debug_set_history(tof_ctx* ctx, const tof_history_desc* history);

/* Test support (the chunked reuse passes at small sizes): lower the ray budget
 * that sizes the chunks of the reuse passes to `rays` (0 = the default), so
 * that a small frame runs its passes over several chunks; a chunk still holds
 * at least one sweep of the smallest grid (8192 tasks).  Results do not
 * depend on the chunking.  *spatial_items_per_chunk (may be NULL) receives the
 * items of a spatial chunk.  Waits for the context's last frame; the next
 * tof_sensor_set restores the default.  TOF_ERR_NOT_READY before a sensor is
 * set. */
tof_status tof_debug_set_ray_budget(tof_ctx* ctx, size_t rays, size_t* spatial_items_per_chunk);

/* Per-kernel GPU timing with HIP events recorded on the render stream around
 * each launch (off by default).  Kernel ids index tof_kernel_times. */
enum {
    TOF_K_BVH = 0,        /* world vertices + refit of the two-level BVH of a moved frame */
    TOF_K_GBUFFER,
    TOF_K_INITIAL,        /* path trees + per-plane RIS + plain PT deposit */
    TOF_K_TEMPORAL_PREP,  /* reprojection + work list */
    TOF_K_TEMPORAL_FWD,   /* temporal forward shifts into the pixel */
    TOF_K_TEMPORAL_MIS,   /* temporal MIS shifts into the other domain */
    TOF_K_TEMPORAL_VIS,   /* visibility rays queued by the temporal shifts */
    TOF_K_TEMPORAL_MERGE, /* temporal weights + reservoir merge */
    TOF_K_SPATIAL_PREP,   /* neighbour choice + work list */
    TOF_K_SPATIAL_FWD,    /* spatial forward shifts into the pixel */
    TOF_K_SPATIAL_MIS,    /* spatial MIS shifts into the neighbours */
    TOF_K_SPATIAL_VIS,    /* visibility rays queued by the spatial shifts */
    TOF_K_SPATIAL_MERGE,  /* spatial weights + reservoir merge */
    TOF_K_SPLAT,
    TOF_K_COUNT
};
typedef struct {
    uint64_t rays;                   /* closest-hit + shadow rays */
    uint64_t node_visits;            /* BVH internal nodes visited */
    uint64_t tri_tests;              /* ray/triangle tests */
    uint64_t shifts;                 /* shift attempts counted by the group */
    uint64_t newton_attempts;        /* Newton solves started */
    uint64_t newton_iters;           /* Newton iterations of converged solves */
} tof_kernel_work;
typedef struct {
    double ms[TOF_K_COUNT];          /* summed event time per kernel group */
    uint64_t launches[TOF_K_COUNT];  /* timed launches per group */
    uint64_t work_items[4];          /* in timed frames: temporal items, temporal candidate tasks,
                                        spatial items, spatial candidate tasks (first round) */
    tof_kernel_work work[TOF_K_COUNT]; /* events per group since timing was enabled; the merge
                                          groups re-derive selected shifts without counting them */
} tof_kernel_times;

/* Enable or disable event timing; enabling clears the accumulated times. */
tof_status tof_set_kernel_timing(tof_ctx* ctx, int enabled);

/* Accumulated per-kernel times and work since timing was enabled
 * (synchronizes). */
tof_status tof_get_kernel_times(tof_ctx* ctx, tof_kernel_times* out);

/* Static string for a status code. */
const char* tof_status_string(tof_status status);

/* ------------------------------------------------------------------------
 * Serving: a request loop over render streams on one device.
 *
 * Each stream is a full context (scene, sensor, resident reservoirs and the
 * last two frames' G-buffers and geometry) with its own HIP stream.  A stream
 * is admitted when its footprint (tof_footprint) fits in what the server's
 * HBM budget has left, else it waits, first come first served, until a close
 * frees memory.  Frames of admitted streams are enqueued on submission, so
 * frames of different streams run concurrently on the device while the
 * frames of one stream run in order (their temporal reuse depends on it);
 * frames of a waiting stream are held and enqueued on admission.  Results are
 * the same as rendering the stream alone with tof_render_frame.  The calls
 * may come from several host threads; one thread should wait for a ticket.
 * ------------------------------------------------------------------------ */
typedef struct tof_server tof_server;

/* Upper bound of the device memory a context with this scene and sensor
 * allocates (scene upload + sensor set). */
tof_status tof_footprint(const tof_scene_desc* scene, const tof_sensor_desc* sensor, size_t* bytes);

/* A server on HIP device `device` whose streams together use at most
 * hbm_budget_bytes (> 0) of device memory. */
tof_status tof_server_create(tof_server** out, int device, size_t hbm_budget_bytes);

/* Waits for all work, releases every stream. */
void tof_server_destroy(tof_server* server);

/* Open a stream (scene and sensor are copied; seed keys its random streams).
 * *stream_id receives its id and *admitted (may be NULL) whether it was
 * admitted at once.  TOF_ERR_OUT_OF_MEMORY if its footprint exceeds the whole
 * budget. */
tof_status tof_server_open(tof_server* server, const tof_scene_desc* scene, const tof_sensor_desc* sensor,
                           uint64_t seed, int* stream_id, int* admitted);

/* Queue a frame of a stream (the frame description and transforms are
 * copied); outputs as for tof_render_frame, device buffers that must stay
 * valid until the frame is done.  *ticket identifies the frame. */
tof_status tof_server_submit(tof_server* server, int stream_id, const tof_frame_desc* frame, float* out_image,
                             float* out_hist, float* out_pt_image, float* out_pt_hist, uint64_t* ticket);

/* Non-blocking: *done = 1 once the frame finished (its status is returned and
 * the ticket is retired), else 0. */
tof_status tof_server_query(tof_server* server, uint64_t ticket, int* done);

/* tof_server_query that also gives, once the frame is done, the time in
 * milliseconds between the start and the end of its work on its HIP stream
 * (*gpu_ms, -1 if unknown): the frame's service time under the load of the
 * other streams; its queueing delay is what the caller saw beyond that. */
tof_status tof_server_query_timed(tof_server* server, uint64_t ticket, int* done, float* gpu_ms);

/* Block until the frame finished; returns its status and retires the ticket.
 * TOF_ERR_NOT_READY while its stream waits for admission.  While a wait is
 * blocked on a ticket, tof_server_query on it reports the state but leaves the
 * ticket to the wait, which retires it. */
tof_status tof_server_wait(tof_server* server, uint64_t ticket);

/* Close a stream; its queued frames still run.  Its memory is freed once no
 * frame of any stream is in flight, or at once (waiting for the device) when
 * a waiting stream needs it, and then admits waiting streams.  Frames held by
 * a stream that was never admitted end with TOF_ERR_NOT_READY. */
tof_status tof_server_close(tof_server* server, int stream_id);

/* Device memory held by admitted streams and by closed streams not yet
 * freed, the number of admitted streams, streams waiting. */
tof_status tof_server_info(tof_server* server, size_t* used_bytes, int* admitted, int* waiting);

/* Graph mode (enabled = 1; 0, the default, turns it off) for the frames
 * dispatched after the call: each frame's work is recorded by stream capture
 * into a HIP graph and launched as one graph on the stream's HIP stream; a
 * stream keeps its executable graph and updates it from the next frame when
 * the frame has the same shape (kernels, copies, their order), else builds it
 * anew.  Results are the same as without graphs.  For callers that want
 * fewer launches per frame (a launch-bound mix of small frames); not in the
 * paper.  TOF_ERR_INVALID_ARG for other values. */
tof_status tof_server_set_graphs(tof_server* server, int enabled);

#ifdef __cplusplus
}
#endif
#endif /* TOF_H */
