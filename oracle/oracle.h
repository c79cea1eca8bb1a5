/*
 * ToF ReSTIR CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 reference implementation of the ToF ReSTIR frame
 * (path trees with NEE, per-bin RIS reservoirs, temporal and spatial GRIS
 * reuse with the path-length-aware Newton shift, splat).  It exists so that
 * tests, the smoke check and the benchmark's CPU baseline can compare the
 * HIP path against it; no product code may link or call it.
 *
 * It shares no code with the HIP library: every routine here (Philox, BVH,
 * intersection, BSDFs, shift, reuse) is written separately.
 *
 * Parity status of each part is listed at the top of oracle.cpp.
 */
#ifndef TOF_ORACLE_H
#define TOF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t num_objects;
    const int32_t* obj_type;      /* 0 = grid, 1 = sphere */
    const int32_t* obj_material;
    const int32_t* obj_grid;      /* [num_objects*5]: nu, nv, wrap_u, wrap_v, vertex_offset */
    const float* obj_sphere;      /* [num_objects*4]: local centre xyz, radius */
    int32_t num_materials;
    const int32_t* mat_type;      /* 0 = Lambert, 1 = GGX */
    const float* mat_params;      /* [num_materials*3]: albedo, alpha, f0 */
    int32_t num_vertices;
    const float* vertices;        /* [num_vertices*3] object-local */
    float scene_scale;
} orc_scene;

typedef struct {
    int32_t width, height, full_width, full_height, crop_x0, crop_y0;
    int32_t camera_model, light_model, count_camera_leg, jitter;
    double light_intensity;
    int32_t gate_enabled;
    double gate_center, gate_width;
    int32_t n_bins;
    double bin_t0, bin_width;
    int32_t n_min, n_max, m_init, temporal, spatial_rounds, spatial_k, spatial_radius;
    double m_cap, newton_tol_rel;
    int32_t newton_max_iter;
    double j_max;
    int32_t shift_mode, include_direct, debug_stage;
    int32_t bin_radius;           /* bin-axis reuse: bins b +- 1..bin_radius of the same pixel (0 = off) */
    double shrink_k;              /* shrink mapping: initial gate samples from a gate shrink_k times wider (1 = off) */
    double shrink_r;              /* fraction R of the path trees sampled from the wide gate (1 = all) */
    int32_t domain;               /* 0: planes over path length; 1: over path velocity u = -dl/dt (Doppler) */
    int32_t round_trip;           /* keep a Newton shift only if the inverse shift returns to the source vertex */
    int32_t mis_mode;             /* spatial reuse: 0 generalized balance heuristic, 1 pairwise MIS */
    uint64_t seed;
} orc_sensor;

typedef struct {
    int32_t index;
    float cam_pos[3], cam_fwd[3], cam_up[3];
    float fov_y_deg;
    float ortho_half[2];
    float light_pos[3];
    const float* xforms;          /* [num_objects*12], rigid 3x4 row-major */
    const float* velocities;      /* [num_objects*6] or NULL: linear v, angular w (point x moves at v + w x (x - t)) */
    float cam_vel[3], light_vel[3];
} orc_frame;

/* lifecycle */
void* orc_create(const orc_scene* scene, const orc_sensor* sensor, int num_threads);
void orc_destroy(void* ctx);
void orc_reset(void* ctx);
/* Move the time gate's centre, keeping the reservoir history: the next
 * temporal reuse shifts previous-frame paths by the move (Sec. 4.1). */
void orc_set_gate_center(void* ctx, double center);

/* One full frame.  Outputs are FP64, plane-major [B][H][W]; any may be NULL.
 * gate image = gate plane / gate width; histogram bins / bin width.
 * pt_* are the plain (no reuse) ToF path-tracing estimates of the same frame.
 * Returns 0 on success. */
int orc_render_frame(void* ctx, const orc_frame* frame, double* out_image, double* out_hist,
                     double* out_pt_image, double* out_pt_hist);

/* Counters: shifts, shifts_ok, newton_attempts, newton_converged,
 * newton_iters_sum, newton_paths_ok, rays, reserved. */
void orc_get_stats(void* ctx, uint64_t out[8]);

/* Diagnostics of the resampling weights, summed over every merge so far with
 * a positive weight sum, for the temporal pass (out[0..4]) and the spatial
 * rounds (out[5..9]): merges, effective sample count (sum w)^2 / sum w^2,
 * candidates with w > 0, candidates present (non-empty reservoirs, before
 * their shift), share of the canonical candidate in the weight sum.  A
 * diagnostic, not part of what the hot path computes. */
void orc_get_merge_diag(void* ctx, double out[10]);

/* Export the final reservoirs of the last rendered frame (the temporal
 * history of the next frame) in a flat plane-major layout, element
 * [plane*P + pixel]: W, phat, len, pre_pdf, origin pixel, origin frame,
 * meta = tree | n<<8 | k<<12 | nsfx<<16, vertex objects [4][P*B] (-1 = none
 * or light), vertex chart coordinates [4][2][P*B], M [P], non-empty mask
 * [ceil(B/32)][P].  Values are rounded to float32.  Returns 0 if a history
 * exists. */
int orc_export_history(void* ctx, float* W, float* phat, float* len, float* pre_pdf, uint32_t* opix, uint32_t* ofr,
                       uint32_t* meta, int32_t* vobj, float* vxi, float* M, uint32_t* mask);

/* ---- unit-level entry points used by the pin tests ---- */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Make `frame` the current frame geometry (slot 0) without rendering. */
int orc_load_frame(void* ctx, const orc_frame* frame);

/* Closest hit in the current frame.  Returns the primitive id (triangles
 * first, then spheres) or -1; out = {t, object, xi0, xi1}. */
int orc_trace(void* ctx, const double o[3], const double d[3], int brute_force, double out[4]);

/* Any-hit query in the current frame, the one shadow rays use: 1 if a
 * primitive is hit at t in (0, tmax) along the normalized direction d. */
int orc_occluded(void* ctx, const double o[3], const double d[3], double tmax);

/* BSDF values f_s(wi, wo[i]) of object obj's material at a point with normal
 * n, for count directions wo [count*3] (directions normalized inside; wi
 * points away from the surface). */
void orc_bsdf(void* ctx, int obj, const double n[3], const double wi[3], const double* wo, int count, double* out);

/* The BSDF sampler of the path trees and the random replay, applied to count
 * uniform pairs u [count*2]: wo [count*3] and its solid-angle density pdf
 * [count] (0 where the sample is rejected).  Returns the accepted count. */
int orc_bsdf_sample(void* ctx, int obj, const double n[3], const double wi[3], const double* u, int count, double* wo,
                    double* pdf);

/* Position, chart Jacobian and normal of chart point (obj, xi) in the current
 * frame.  out = {p(3), J_u(3), J_v(3), n(3)}.  Returns 1 if xi is on the chart. */
int orc_chart(void* ctx, int obj, const double xi[2], double out[12]);

/* Path-length Newton solve on object `obj` in the current frame.
 * Source length L_src(xi) = c_src + |a_src - p(xi)| + |b_src - p(xi)|, same for
 * the destination.  out = {xi'0, xi'1, iterations, |det dxi'/dxi|,
 * |det dp'/dp|, F1, F2, status}.  Returns 1 on convergence. */
int orc_newton(void* ctx, int obj, const double xi[2], const double a_src[3], const double b_src[3],
               double c_src, const double a_dst[3], const double b_dst[3], double c_dst,
               double dl0, double tol, int max_iter, double out[8]);

/* The path-velocity function of the reconnection vertex on object obj's chart
 * in the loaded frame (velocity domain): U(xi) = c + (va - v(p)).w_a +
 * (v(p) - vb).w_b, w_a the unit vector a -> p, w_b p -> b.  out = {U, dU/du,
 * dU/dv, d2U/du2, d2U/dudv, d2U/dv2}.  Returns 1 if the chart point exists. */
int orc_vel_eval(void* ctx, int obj, const double xi[2], const double a[3], const double va[3], const double b[3],
                 const double vb[3], double c, double out[6]);

/* MIS weights of the spatial reuse at one path y of the pixel's domain
 * (mode 0 generalized balance heuristic, 1 pairwise): out[0] the canonical
 * technique's, out[1 + j] neighbour j's; M[j] < 0 marks a neighbour without
 * a pixel (weight 0), d[j] domain j's density term at y, dc the canonical
 * target at y, mq the canonical confidence. */
void orc_mis_weights(int mode, int K, const double* M, double mq, const double* d, double dc, double* out);

/* Weighted reservoir streaming of n candidate weights with uniforms u. */
int orc_wrs(const double* w, const double* u, int n, double* w_sum);

#ifdef __cplusplus
}
#endif
#endif
