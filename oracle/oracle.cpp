/*
 * ToF ReSTIR CPU oracle (FP64) -- TEST INFRASTRUCTURE ONLY; no product code
 * links or calls it.  See oracle.h.
 *
 * What it computes, following the paper (Kim, Jarosz, Pediredla, "ToF ReSTIR",
 * ACM TOG 45(4) 2026):
 *   - the time-of-flight path integral I(tau) = int W_tau(l(x)) f(x) dmu(x)
 *     (Sec. 3.1, eq. tof_path_integral), estimated with path trees and NEE to a
 *     delta light (Sec. 5, "Light Source");
 *   - RIS / weighted reservoir sampling (Sec. 3.2.1 and 3.2.4), one reservoir
 *     per pixel and time bin (Sec. 4.5) seeded by per-bin path deposit
 *     (Sec. 4.5, comparison with Jarabo's path reuse);
 *   - GRIS with the generalized balance heuristic (Sec. 3.2.3,
 *     eq. GRIS_resampling_weight and eq. GRIS_MIS_weight);
 *   - the hybrid replay/reconnection shift followed by the path-length-aware
 *     perturbation of the reconnection vertex (Sec. 4.1, eq.
 *     path_length_constraint) with the average-gradient gauge, Newton with
 *     backtracking, and the implicit-function Jacobian (Sec. 4.3);
 *   - gradient and Hessian of the length function (Sec. 4.3, "Gradient and
 *     Hessian Evaluation"), including the curvature term Q on sphere charts;
 *   - the four-stage frame: initial, temporal, spatial, final shading
 *     (Sec. 3.2.4), with an optional reuse along the bin axis between the
 *     temporal and the spatial stage (Sec. 4.5: a histogram bin takes the
 *     samples of the bins around it in the same pixel, shifted by the bins'
 *     distance, Delta l = (b - b') * bin width);
 *   - optionally, initial gate samples drawn in a gate K times wider and the
 *     RIS winner shrunk into the gate (Sec. 4.4.2, shrink mapping, with all
 *     samples in the wide gate, R = 1, or a fraction R < 1 of the path trees
 *     there and the rest in the gate, the two reservoirs merged by GRIS with
 *     the generalized balance heuristic, which is unbiased);
 *   - the Doppler domain (Sec. 4.6): planes over the path velocity
 *     u = -dl/dt (eq. optical_path_velocity, refractive index 1) with the
 *     vertices moving rigidly with their objects, and the same shift under a
 *     path-velocity constraint; its gradient and Hessian are derived here
 *     (the supplement that holds them is not available).
 * Where a passage is ambiguous or garbled, the code states the reading it
 * takes.
 *
 * Pins (tests/test_oracle_*.py): Philox against numpy's Philox4x64-10; BVH
 * closest hit against brute force; the closed-form transient of a Lambertian
 * plane; the confocal radial closed form of the Newton shift; finite-difference
 * Jacobians; the gate constraint; the identity shift; bijectivity; WRS
 * selection frequencies; unbiasedness of the full ReSTIR estimator against
 * plain path tracing; the path velocity against a time difference of the
 * path length of the moved scene, its chart gradient and Hessian against
 * finite differences, and the closed-form Doppler spectrum of a receding
 * Lambertian plane.  Parity of the complete multi-pass image beyond these
 * properties is "parity unpinned" (no per-pixel values exist in the paper).
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// small vector algebra
// ---------------------------------------------------------------------------
struct V3 {
    double x = 0, y = 0, z = 0;
    V3() = default;
    V3(double a, double b, double c) : x(a), y(b), z(c) {}
    double operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline V3 operator-(V3 a) { return {-a.x, -a.y, -a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double length(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return (1.0 / length(a)) * a; }

const double PI = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor bijection with the key bumped by the Weyl constants.
// ---------------------------------------------------------------------------
void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

enum { PASS_JITTER = 0, PASS_BSDF = 1, PASS_RIS = 2, PASS_TEMPORAL = 3, PASS_SPATIAL = 4, PASS_BIN = 16,
       PASS_SHRINK_MIX = 17 };

struct Draw {
    uint64_t x[4];
    // uniform in [0,1) from the top 24 bits: exact in FP32 and FP64
    double u(int i) const { return (double)(x[i] >> 40) * (1.0 / 16777216.0); }
};

Draw draw(uint64_t seed, uint64_t pixel, uint64_t frame, uint64_t pass, uint64_t a, uint64_t b) {
    uint64_t ctr[4] = {pixel, frame, (pass << 56) | (a << 32) | b, 0};
    uint64_t key[2] = {seed, 0};
    Draw d;
    philox4x64_10(ctr, key, d.x);
    return d;
}

// ---------------------------------------------------------------------------
// scene description
// ---------------------------------------------------------------------------
struct Material { int type; double albedo, alpha, f0; };
struct Object {
    int type, material;
    int nu, nv, wrap_u, wrap_v, voff;
    V3 centre; double radius;
    int tri_base;
};
struct TriRef { int obj, i, j, h; };

struct Vertex {           // a surface point in one frame
    int obj = -1;
    double xi[2] = {0, 0};
    V3 p, n;
};

struct ChartEval {
    bool on = false, ok = false;
    V3 p, ju, jv, puu, puv, pvv, n;
};

struct BNode { double lo[3], hi[3]; int left, right, first, count; };

// ---------------------------------------------------------------------------
// MIS weight of technique t at a path y of the pixel's domain (Sec. 3.2.3,
// eq. GRIS_MIS_weight): t = -1 the canonical technique, t = j a neighbour's.
// M[l] < 0 marks a neighbour without a pixel; d[l] is domain l's density term
// at y (phat_l of y shifted into l, times |J|; for t = j the stored
// phat_j(x_j) / |J_{j->q}|), dc = phat_q(y), mq the canonical confidence.
// Generalized balance heuristic: M_t d_t / (mq dc + sum_l M_l d_l).  Pairwise
// (opt-in): the canonical technique is split into Kv parts of confidence
// mq / Kv, part l paired with neighbour l under the balance heuristic, pair l
// weighted by (M_l + mq / Kv) / (mq + sum_l M_l); a neighbour's weight needs
// only its own term and dc.
// ---------------------------------------------------------------------------
double mis_weight(int mode, int t, int K, const double* M, double mq, const double* d, double dc) {
    int kv = 0;
    double mtot = mq;
    for (int l = 0; l < K; ++l)
        if (M[l] >= 0.0) {
            ++kv;
            mtot += M[l];
        }
    if (mode == 1 && kv > 0) {
        const double mqk = mq / kv;
        if (t >= 0) return (M[t] + mqk) / mtot * (M[t] * d[t] / (M[t] * d[t] + mqk * dc));
        double m = 0.0;
        for (int l = 0; l < K; ++l)
            if (M[l] >= 0.0) m += (M[l] + mqk) / mtot * (mqk * dc / (mqk * dc + M[l] * d[l]));
        return m;
    }
    double den = mq * dc;
    for (int l = 0; l < K; ++l)
        if (M[l] >= 0.0) den += M[l] * d[l];
    return (t >= 0 ? M[t] * d[t] : mq * dc) / den;
}

struct FrameGeom {
    bool valid = false;
    int index = 0;
    double gate_center = 0.0;    // the time gate's centre when the frame was rendered
    std::vector<double> xf;      // per object: 3x4 row-major
    std::vector<V3> wv;          // world vertices
    std::vector<BNode> nodes;
    std::vector<int> order;      // triangle ids in BVH leaf order
    V3 cam_pos, cam_fwd, cam_right, cam_up;
    double tan_half = 0, aspect = 1, ortho_hx = 0, ortho_hy = 0;
    V3 light_pos;
    std::vector<double> ov;      // per object: linear velocity v, angular velocity w
    V3 cam_vel, light_vel;
};

struct GBuf { bool hit = false; Vertex v; };

struct VRef { int obj = -1; double xi[2] = {0, 0}; };

struct PathRec {
    uint32_t opix = 0, ofr = 0;
    int tree = 0, n = 0, k = 0, nsfx = 0;
    VRef xkm1, p, p2, sfx[2];
    double len = 0, pre_pdf = 1, phat = 0;
};

struct Res { PathRec y; double W = 0; };

// Diagnostics of the resampling weights of one merge (a pixel-plane whose
// weights sum to more than zero), summed per pass kind (0 temporal, 1
// spatial): items, effective sample count (sum w)^2 / sum w^2, candidates
// with w > 0, candidates present (non-empty, before their shift), share of
// the canonical candidate's weight.
struct MergeDiag {
    double d[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    void item(int kind, double ws, double w2, int npos, int npresent, double w0) {
        d[kind][0] += 1.0;
        d[kind][1] += ws * ws / w2;
        d[kind][2] += npos;
        d[kind][3] += npresent;
        d[kind][4] += w0 / ws;
    }
};

struct Stats {
    uint64_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    MergeDiag md;
    void add(const Stats& o) {
        for (int i = 0; i < 8; ++i) c[i] += o.c[i];
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i < 5; ++i) md.d[k][i] += o.md.d[k][i];
    }
};
enum { ST_SHIFTS = 0, ST_SHIFTS_OK, ST_NEWTON_ATT, ST_NEWTON_CONV, ST_NEWTON_ITERS, ST_NEWTON_OK, ST_RAYS };

typedef std::map<int, Res> PixelRes;   // non-empty planes only

struct Oracle {
    // scene
    std::vector<Object> objs;
    std::vector<Material> mats;
    std::vector<V3> lverts;
    std::vector<TriRef> tris;
    double sc = 1, eps = 1e-4, dmin = 0.01;
    // sensor
    orc_sensor s;
    int P = 0, B = 0;            // pixels in the crop, planes
    int nthreads = 1;
    // state: slot 0 = current frame, slot 1 = previous frame
    FrameGeom fg[2];
    std::vector<GBuf> gb[2];
    std::vector<PixelRes> fin_prev;
    std::vector<double> M_prev;
    bool prev_valid = false;
    Stats stats;

    // -------------------------------------------------------------------
    const Material& mat_of(int obj) const { return mats[objs[obj].material]; }
    bool rough(int obj) const {
        const Material& m = mat_of(obj);
        return m.type == 0 || m.alpha >= 0.2;
    }

    // -------------------------------------------------------------------
    // frame geometry
    // -------------------------------------------------------------------
    V3 xf_point(const FrameGeom& F, int o, V3 q) const {
        const double* m = &F.xf[12 * o];
        return {m[0] * q.x + m[1] * q.y + m[2] * q.z + m[3],
                m[4] * q.x + m[5] * q.y + m[6] * q.z + m[7],
                m[8] * q.x + m[9] * q.y + m[10] * q.z + m[11]};
    }
    V3 xf_dir(const FrameGeom& F, int o, V3 q) const {
        const double* m = &F.xf[12 * o];
        return {m[0] * q.x + m[1] * q.y + m[2] * q.z, m[4] * q.x + m[5] * q.y + m[6] * q.z,
                m[8] * q.x + m[9] * q.y + m[10] * q.z};
    }
    V3 xf_inv_point(const FrameGeom& F, int o, V3 p) const {
        const double* m = &F.xf[12 * o];
        V3 d = {p.x - m[3], p.y - m[7], p.z - m[11]};
        return {m[0] * d.x + m[4] * d.y + m[8] * d.z, m[1] * d.x + m[5] * d.y + m[9] * d.z,
                m[2] * d.x + m[6] * d.y + m[10] * d.z};
    }
    V3 gvert(const FrameGeom& F, int o, int i, int j) const {
        const Object& ob = objs[o];
        return F.wv[ob.voff + j * (ob.nu + 1) + i];
    }
    void tri_verts(const FrameGeom& F, int t, V3& a, V3& b, V3& c) const {
        const TriRef& r = tris[t];
        if (r.h == 0) {
            a = gvert(F, r.obj, r.i, r.j); b = gvert(F, r.obj, r.i + 1, r.j); c = gvert(F, r.obj, r.i, r.j + 1);
        } else {
            a = gvert(F, r.obj, r.i + 1, r.j + 1); b = gvert(F, r.obj, r.i, r.j + 1); c = gvert(F, r.obj, r.i + 1, r.j);
        }
    }

    void build_bvh(FrameGeom& F) {
        int T = (int)tris.size();
        F.order.resize(T);
        std::vector<V3> cen(T);
        for (int t = 0; t < T; ++t) {
            F.order[t] = t;
            V3 a, b, c;
            tri_verts(F, t, a, b, c);
            cen[t] = (1.0 / 3.0) * (a + b + c);
        }
        F.nodes.clear();
        if (T == 0) return;
        build_node(F, cen, 0, T);
    }
    int build_node(FrameGeom& F, const std::vector<V3>& cen, int first, int count) {
        int id = (int)F.nodes.size();
        F.nodes.push_back(BNode());
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
        for (int q = first; q < first + count; ++q) {
            V3 a, b, c;
            tri_verts(F, F.order[q], a, b, c);
            for (int ax = 0; ax < 3; ++ax) {
                lo[ax] = std::min(lo[ax], std::min(a[ax], std::min(b[ax], c[ax])));
                hi[ax] = std::max(hi[ax], std::max(a[ax], std::max(b[ax], c[ax])));
                clo[ax] = std::min(clo[ax], cen[F.order[q]][ax]);
                chi[ax] = std::max(chi[ax], cen[F.order[q]][ax]);
            }
        }
        BNode nd;
        for (int ax = 0; ax < 3; ++ax) {   // pad so the slab test is conservative
            double pad = 1e-9 * (std::fabs(lo[ax]) + std::fabs(hi[ax]) + 1.0);
            nd.lo[ax] = lo[ax] - pad;
            nd.hi[ax] = hi[ax] + pad;
        }
        if (count <= 4) {
            nd.left = nd.right = -1; nd.first = first; nd.count = count;
            F.nodes[id] = nd;
            return id;
        }
        int axis = 0;
        for (int ax = 1; ax < 3; ++ax)
            if (chi[ax] - clo[ax] > chi[axis] - clo[axis]) axis = ax;
        int mid = first + count / 2;
        std::nth_element(F.order.begin() + first, F.order.begin() + mid, F.order.begin() + first + count,
                         [&](int x, int y) {
                             double cx = cen[x][axis], cy = cen[y][axis];
                             return cx < cy || (cx == cy && x < y);
                         });
        nd.first = 0; nd.count = 0;
        nd.left = build_node(F, cen, first, mid - first);
        nd.right = build_node(F, cen, mid, first + count - mid);
        F.nodes[id] = nd;
        return id;
    }

    void load_frame(FrameGeom& F, const orc_frame* fr) {
        F.valid = true;
        F.index = fr->index;
        F.gate_center = s.gate_center;
        int O = (int)objs.size();
        F.xf.assign(12 * O, 0.0);
        for (int k = 0; k < 12 * O; ++k) F.xf[k] = (double)fr->xforms[k];
        F.wv.resize(lverts.size());
        for (int o = 0; o < O; ++o) {
            const Object& ob = objs[o];
            if (ob.type != 0) continue;
            int nvtx = (ob.nu + 1) * (ob.nv + 1);
            for (int q = 0; q < nvtx; ++q) F.wv[ob.voff + q] = xf_point(F, o, lverts[ob.voff + q]);
        }
        build_bvh(F);
        F.cam_pos = {fr->cam_pos[0], fr->cam_pos[1], fr->cam_pos[2]};
        V3 fwd = normalize(V3(fr->cam_fwd[0], fr->cam_fwd[1], fr->cam_fwd[2]));
        V3 up = {fr->cam_up[0], fr->cam_up[1], fr->cam_up[2]};
        F.cam_fwd = fwd;
        F.cam_right = normalize(cross(fwd, up));
        F.cam_up = cross(F.cam_right, fwd);
        F.tan_half = std::tan(0.5 * (double)fr->fov_y_deg * PI / 180.0);
        F.aspect = (double)s.full_width / (double)s.full_height;
        F.ortho_hx = fr->ortho_half[0];
        F.ortho_hy = fr->ortho_half[1];
        F.light_pos = {fr->light_pos[0], fr->light_pos[1], fr->light_pos[2]};
        F.ov.assign(6 * O, 0.0);
        if (fr->velocities)
            for (int k = 0; k < 6 * O; ++k) F.ov[k] = (double)fr->velocities[k];
        F.cam_vel = {fr->cam_vel[0], fr->cam_vel[1], fr->cam_vel[2]};
        F.light_vel = {fr->light_vel[0], fr->light_vel[1], fr->light_vel[2]};
    }

    // -------------------------------------------------------------------
    // surface charts (Sec. 4.2): xi -> p on a grid object (piecewise-affine
    // in cell units) or on a sphere ((theta, phi) about the local z axis).
    // -------------------------------------------------------------------
    ChartEval chart(const FrameGeom& F, int obj, double u, double v) const {
        ChartEval c;
        const Object& ob = objs[obj];
        if (ob.type == 0) {
            c.on = true;
            double uu = u, vv = v;
            if (ob.wrap_u) uu = u - ob.nu * std::floor(u / ob.nu);
            else if (u < 0.0 || u > (double)ob.nu) c.on = false;
            if (ob.wrap_v) vv = v - ob.nv * std::floor(v / ob.nv);
            else if (v < 0.0 || v > (double)ob.nv) c.on = false;
            int i = (int)std::floor(uu), j = (int)std::floor(vv);
            i = std::min(std::max(i, 0), ob.nu - 1);
            j = std::min(std::max(j, 0), ob.nv - 1);
            double a = uu - i, b = vv - j;
            V3 v00 = gvert(F, obj, i, j), v10 = gvert(F, obj, i + 1, j);
            V3 v01 = gvert(F, obj, i, j + 1), v11 = gvert(F, obj, i + 1, j + 1);
            if (a + b <= 1.0) {
                c.p = v00 + a * (v10 - v00) + b * (v01 - v00);
                c.ju = v10 - v00;
                c.jv = v01 - v00;
            } else {
                c.p = v11 + (1.0 - a) * (v01 - v11) + (1.0 - b) * (v10 - v11);
                c.ju = v11 - v01;
                c.jv = v11 - v10;
            }
            V3 cr = cross(c.ju, c.jv);
            double l = length(cr);
            c.ok = l > 0.0;
            if (c.ok) c.n = (1.0 / l) * cr;
        } else {
            double th = u, ph = v, r = ob.radius;
            double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
            V3 radial = {st * cp, st * sp, ct};
            c.p = xf_point(F, obj, ob.centre + r * radial);
            c.ju = xf_dir(F, obj, V3(r * ct * cp, r * ct * sp, -r * st));
            c.jv = xf_dir(F, obj, V3(-r * st * sp, r * st * cp, 0.0));
            c.puu = xf_dir(F, obj, -r * radial);
            c.puv = xf_dir(F, obj, V3(-r * ct * sp, r * ct * cp, 0.0));
            c.pvv = xf_dir(F, obj, V3(-r * st * cp, -r * st * sp, 0.0));
            c.n = xf_dir(F, obj, radial);
            c.on = th >= 1e-3 && th <= PI - 1e-3;
            c.ok = true;
        }
        return c;
    }
    double wrap_coord(int obj, int dim, double x) const {
        const Object& ob = objs[obj];
        if (ob.type == 0) {
            if (dim == 0 && ob.wrap_u) return x - ob.nu * std::floor(x / ob.nu);
            if (dim == 1 && ob.wrap_v) return x - ob.nv * std::floor(x / ob.nv);
            return x;
        }
        if (dim == 1) return x - 2.0 * PI * std::floor(x / (2.0 * PI));
        return x;
    }
    Vertex vertex_at(const FrameGeom& F, int obj, const double xi[2]) const {
        Vertex vx;
        vx.obj = obj;
        vx.xi[0] = xi[0];
        vx.xi[1] = xi[1];
        ChartEval c = chart(F, obj, xi[0], xi[1]);
        vx.p = c.p;
        vx.n = c.n;
        return vx;
    }
    Vertex vertex_at(const FrameGeom& F, const VRef& r) const { return vertex_at(F, r.obj, r.xi); }

    // -------------------------------------------------------------------
    // ray casting: watertight ray/triangle test (Woop, Benthin, Wald,
    // JCGT 2013), analytic spheres, a median-split BVH.
    // -------------------------------------------------------------------
    static bool isect_tri(V3 o, V3 d, V3 v0, V3 v1, V3 v2, double tmax, double& t, double& b1, double& b2) {
        int kz = 0;
        if (std::fabs(d.y) > std::fabs(d[kz])) kz = 1;
        if (std::fabs(d.z) > std::fabs(d[kz])) kz = 2;
        int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
        if (d[kz] < 0.0) std::swap(kx, ky);
        double sx = d[kx] / d[kz], sy = d[ky] / d[kz], sz = 1.0 / d[kz];
        V3 A = v0 - o, B = v1 - o, C = v2 - o;
        double ax = A[kx] - sx * A[kz], ay = A[ky] - sy * A[kz];
        double bx = B[kx] - sx * B[kz], by = B[ky] - sy * B[kz];
        double cx = C[kx] - sx * C[kz], cy = C[ky] - sy * C[kz];
        double U = cx * by - cy * bx, Vv = ax * cy - ay * cx, W = bx * ay - by * ax;
        if ((U < 0 || Vv < 0 || W < 0) && (U > 0 || Vv > 0 || W > 0)) return false;
        double det = U + Vv + W;
        if (det == 0.0) return false;
        double T = U * (sz * A[kz]) + Vv * (sz * B[kz]) + W * (sz * C[kz]);
        double tt = T / det;
        if (!(tt > 0.0 && tt < tmax)) return false;
        t = tt;
        b1 = Vv / det;
        b2 = W / det;
        return true;
    }
    static bool isect_sphere(V3 o, V3 d, V3 c, double r, double tmax, double& t) {
        V3 oc = o - c;
        double b = dot(oc, d), cc = dot(oc, oc) - r * r;
        double disc = b * b - cc;
        if (disc < 0.0) return false;
        double sq = std::sqrt(disc);
        double t0 = -b - sq, t1 = -b + sq;
        if (t0 > 0.0 && t0 < tmax) { t = t0; return true; }
        if (t1 > 0.0 && t1 < tmax) { t = t1; return true; }
        return false;
    }
    static bool slab(const BNode& nd, V3 o, V3 d, double tmax) {
        double tn = 0.0, tf = tmax;
        for (int ax = 0; ax < 3; ++ax) {
            if (d[ax] == 0.0) {
                if (o[ax] < nd.lo[ax] || o[ax] > nd.hi[ax]) return false;
                continue;
            }
            double t1 = (nd.lo[ax] - o[ax]) / d[ax], t2 = (nd.hi[ax] - o[ax]) / d[ax];
            if (t1 > t2) std::swap(t1, t2);
            tn = std::max(tn, t1);
            tf = std::min(tf, t2);
            if (tn > tf) return false;
        }
        return true;
    }

    struct Hit { bool hit = false; int prim = -1; int obj = -1; double t = 0, b1 = 0, b2 = 0; };

    // closest hit; ties in t go to the smaller primitive id
    Hit closest(const FrameGeom& F, V3 o, V3 d, bool brute = false) const {
        Hit best;
        double tb = 1e300;
        auto consider_tri = [&](int t) {
            V3 a, b, c;
            tri_verts(F, t, a, b, c);
            double tt, b1, b2;
            if (isect_tri(o, d, a, b, c, tb * (1.0 + 1e-12) + 1e-300, tt, b1, b2)) {
                if (tt < tb || (tt == tb && t < best.prim)) {
                    tb = tt; best.hit = true; best.prim = t; best.obj = tris[t].obj; best.t = tt; best.b1 = b1; best.b2 = b2;
                }
            }
        };
        if (brute) {
            for (int t = 0; t < (int)tris.size(); ++t) consider_tri(t);
        } else if (!F.nodes.empty()) {
            std::vector<int> stack;
            stack.push_back(0);
            while (!stack.empty()) {
                int ni = stack.back();
                stack.pop_back();
                const BNode& nd = F.nodes[ni];
                if (!slab(nd, o, d, tb)) continue;
                if (nd.left < 0) {
                    for (int q = nd.first; q < nd.first + nd.count; ++q) consider_tri(F.order[q]);
                } else {
                    stack.push_back(nd.left);
                    stack.push_back(nd.right);
                }
            }
        }
        int T = (int)tris.size();
        for (int ob = 0; ob < (int)objs.size(); ++ob) {
            if (objs[ob].type != 1) continue;
            double tt;
            V3 cw = xf_point(F, ob, objs[ob].centre);
            int prim = T + ob;
            if (isect_sphere(o, d, cw, objs[ob].radius, tb * (1.0 + 1e-12) + 1e-300, tt)) {
                if (tt < tb || (tt == tb && prim < best.prim)) {
                    tb = tt; best.hit = true; best.prim = prim; best.obj = ob; best.t = tt;
                }
            }
        }
        return best;
    }

    bool occluded(const FrameGeom& F, V3 o, V3 d, double tmax) const {
        if (!F.nodes.empty()) {
            std::vector<int> stack;
            stack.push_back(0);
            while (!stack.empty()) {
                int ni = stack.back();
                stack.pop_back();
                const BNode& nd = F.nodes[ni];
                if (!slab(nd, o, d, tmax)) continue;
                if (nd.left < 0) {
                    for (int q = nd.first; q < nd.first + nd.count; ++q) {
                        V3 a, b, c;
                        tri_verts(F, F.order[q], a, b, c);
                        double tt, b1, b2;
                        if (isect_tri(o, d, a, b, c, tmax, tt, b1, b2)) return true;
                    }
                } else {
                    stack.push_back(nd.left);
                    stack.push_back(nd.right);
                }
            }
        }
        for (int ob = 0; ob < (int)objs.size(); ++ob) {
            if (objs[ob].type != 1) continue;
            double tt;
            if (isect_sphere(o, d, xf_point(F, ob, objs[ob].centre), objs[ob].radius, tmax, tt)) return true;
        }
        return false;
    }

    // chart coordinates of a hit, then the vertex re-evaluated from its chart
    Vertex hit_vertex(const FrameGeom& F, const Hit& h, V3 o, V3 d) const {
        double xi[2];
        if (h.prim < (int)tris.size()) {
            const TriRef& r = tris[h.prim];
            if (r.h == 0) { xi[0] = r.i + h.b1; xi[1] = r.j + h.b2; }
            else { xi[0] = r.i + 1 - h.b1; xi[1] = r.j + 1 - h.b2; }
        } else {
            const Object& ob = objs[h.obj];
            V3 q = xf_inv_point(F, h.obj, o + h.t * d) - ob.centre;
            double ct = std::min(1.0, std::max(-1.0, q.z / ob.radius));
            xi[0] = std::acos(ct);
            double ph = std::atan2(q.y, q.x);
            if (ph < 0.0) ph += 2.0 * PI;
            xi[1] = ph;
        }
        return vertex_at(F, h.obj, xi);
    }

    V3 offset(V3 p, V3 n, V3 dir) const { return dot(n, dir) > 0.0 ? p + eps * n : p - eps * n; }

    bool trace(const FrameGeom& F, const Vertex& from, V3 dir, Vertex& out) const {
        V3 o = offset(from.p, from.n, dir);
        Hit h = closest(F, o, dir);
        if (!h.hit) return false;
        out = hit_vertex(F, h, o, dir);
        return true;
    }
    bool visible_pts(const FrameGeom& F, const Vertex& a, const Vertex& b) const {
        V3 o = offset(a.p, a.n, b.p - a.p);
        V3 t = offset(b.p, b.n, a.p - b.p);
        V3 dv = t - o;
        double dist = length(dv);
        return !occluded(F, o, (1.0 / dist) * dv, dist);
    }

    // -------------------------------------------------------------------
    // domains: pixel of the current (slot 0) or previous (slot 1) frame
    // -------------------------------------------------------------------
    uint64_t full_pixel(int pix) const {
        int x = pix % s.width, y = pix / s.width;
        return (uint64_t)(s.crop_y0 + y) * (uint64_t)s.full_width + (uint64_t)(s.crop_x0 + x);
    }
    V3 toward_camera(int slot, const Vertex& y1) const {
        const FrameGeom& F = fg[slot];
        if (s.camera_model == 0) return normalize(F.cam_pos - y1.p);
        return -F.cam_fwd;
    }
    // -------------------------------------------------------------------
    // The quantity the planes measure (Sec. 3.1 for time, Sec. 4.6 for
    // Doppler): the optical path length l, or the path velocity
    // u = -dl/dt = sum over segments of (v_from - v_to) . w, w the unit vector
    // of the segment (eq. optical_path_velocity), with the vertices moving
    // with their objects' instantaneous rigid motion.
    // -------------------------------------------------------------------
    struct EP { V3 p, v; };   // a path vertex: position and velocity
    V3 vel_at(const FrameGeom& F, int obj, V3 x) const {
        if (obj < 0 || F.ov.empty()) return V3();
        const double* q = &F.ov[6 * obj];
        V3 t = {F.xf[12 * obj + 3], F.xf[12 * obj + 7], F.xf[12 * obj + 11]};
        return V3(q[0], q[1], q[2]) + cross(V3(q[3], q[4], q[5]), x - t);
    }
    EP ep(const FrameGeom& F, const Vertex& y) const { return EP{y.p, vel_at(F, y.obj, y.p)}; }
    // contribution of the segment from -> to
    double seg_q(const EP& from, const EP& to) const {
        V3 d = to.p - from.p;
        double l = length(d);
        if (s.domain == 0) return l;
        return dot(from.v - to.v, (1.0 / l) * d);
    }
    double camera_leg(int slot, const Vertex& y1) const {
        if (!s.count_camera_leg) return 0.0;
        const FrameGeom& F = fg[slot];
        if (s.domain == 1) {
            V3 dir = s.camera_model == 0 ? normalize(y1.p - F.cam_pos) : F.cam_fwd;
            return dot(F.cam_vel - vel_at(F, y1.obj, y1.p), dir);
        }
        if (s.camera_model == 0) return length(y1.p - F.cam_pos);
        return dot(y1.p - F.cam_pos, F.cam_fwd);
    }
    // Delta lights (Sec. 5, "Light Source"): an isotropic point light, or the
    // confocal laser spot at the domain's primary hit re-emitting with the
    // wall's Lambertian BRDF.
    V3 light_pos(int slot, int pix) const {
        if (s.light_model == 0) return fg[slot].light_pos;
        return gb[slot][pix].v.p;
    }
    EP light_ep(int slot, int pix) const {
        if (s.light_model == 0) return EP{fg[slot].light_pos, fg[slot].light_vel};
        return ep(fg[slot], gb[slot][pix].v);
    }
    double light_emit(int slot, int pix, V3 x) const {
        if (s.light_model == 0) return s.light_intensity;
        const Vertex& g = gb[slot][pix].v;
        V3 w = normalize(x - g.p);
        double cw = dot(g.n, w), cs = dot(g.n, -fg[slot].cam_fwd);
        if (cw * cs <= 0.0) return 0.0;
        const Material& m = mat_of(g.obj);
        return s.light_intensity * m.albedo / PI * std::fabs(cw);
    }
    bool light_visible(int slot, int pix, const Vertex& x) const {
        const FrameGeom& F = fg[slot];
        if (s.light_model == 0) {
            V3 o = offset(x.p, x.n, F.light_pos - x.p);
            V3 dv = F.light_pos - o;
            double dist = length(dv);
            return !occluded(F, o, (1.0 / dist) * dv, dist);
        }
        return visible_pts(F, x, gb[slot][pix].v);
    }

    // -------------------------------------------------------------------
    // BSDFs: Lambert and GGX (Walter et al. 2007, separable Smith G,
    // Schlick Fresnel), sampled cosine-weighted / proportional to D cos.
    // -------------------------------------------------------------------
    static void onb(V3 n, V3& t, V3& b) {   // Duff et al., JCGT 2017
        double sg = std::copysign(1.0, n.z);
        double a = -1.0 / (sg + n.z);
        double bb = n.x * n.y * a;
        t = {1.0 + sg * n.x * n.x * a, sg * bb, -sg * n.x};
        b = {bb, sg + n.y * n.y * a, -n.y};
    }
    static double ggx_d(double alpha, double ch) {
        double a2 = alpha * alpha;
        double den = ch * ch * (a2 - 1.0) + 1.0;
        return a2 / (PI * den * den);
    }
    static double ggx_g1(double alpha, double c) {
        double a2 = alpha * alpha;
        return 2.0 * c / (c + std::sqrt(a2 + (1.0 - a2) * c * c));
    }
    double bsdf(int obj, V3 n, V3 wi, V3 wo) const {
        double ci = dot(n, wi), co = dot(n, wo);
        if (ci * co <= 0.0) return 0.0;
        const Material& m = mat_of(obj);
        if (m.type == 0) return m.albedo / PI;
        ci = std::fabs(ci); co = std::fabs(co);
        V3 ns = dot(n, wi) > 0.0 ? n : -n;
        V3 h = normalize(wi + wo);
        double ch = dot(ns, h);
        double D = ggx_d(m.alpha, ch);
        double G = ggx_g1(m.alpha, ci) * ggx_g1(m.alpha, co);
        double F = m.f0 + (1.0 - m.f0) * std::pow(1.0 - dot(wi, h), 5.0);
        return D * G * F / (4.0 * ci * co);
    }
    bool bsdf_sample(int obj, V3 n, V3 wi, double u1, double u2, V3& wo, double& pdf) const {
        double ci = dot(n, wi);
        if (ci == 0.0) return false;
        V3 ns = ci > 0.0 ? n : -n;
        V3 t, b;
        onb(ns, t, b);
        const Material& m = mat_of(obj);
        if (m.type == 0) {
            double r = std::sqrt(u1), ph = 2.0 * PI * u2;
            double z = std::sqrt(std::max(0.0, 1.0 - u1));
            wo = normalize(r * std::cos(ph) * t + r * std::sin(ph) * b + z * ns);
            pdf = dot(ns, wo) / PI;
            return pdf > 0.0;
        }
        double a2 = m.alpha * m.alpha;
        double t2 = a2 * u1 / (1.0 - u1);
        double ch = 1.0 / std::sqrt(1.0 + t2);
        double sh = std::sqrt(std::max(0.0, 1.0 - ch * ch));
        double ph = 2.0 * PI * u2;
        V3 h = sh * std::cos(ph) * t + sh * std::sin(ph) * b + ch * ns;
        double wh = dot(wi, h);
        wo = normalize(2.0 * wh * h - wi);
        if (dot(ns, wo) <= 0.0) return false;
        pdf = ggx_d(m.alpha, ch) * ch / (4.0 * std::fabs(wh));
        return pdf > 0.0;
    }

    // -------------------------------------------------------------------
    // time gate / bins (Sec. 3.1 W_tau; half-open boxes)
    // -------------------------------------------------------------------
    // the gate plane of a frame slot uses the gate centre of that frame;
    // index n_bins + 1 stands for the wide gate of the shrink mapping (K
    // times the gate, same centre), the domain of its wide-gate samples
    double gate_half(int pl) const { return 0.5 * s.gate_width * (pl == s.n_bins + 1 ? s.shrink_k : 1.0); }
    double plane_lo(int pl, int slot = 0) const {
        return pl < s.n_bins ? s.bin_t0 + pl * s.bin_width : fg[slot].gate_center - gate_half(pl);
    }
    double plane_hi(int pl, int slot = 0) const {
        return pl < s.n_bins ? s.bin_t0 + (pl + 1) * s.bin_width : fg[slot].gate_center + gate_half(pl);
    }
    double plane_width(int pl) const { return pl < s.n_bins ? s.bin_width : 2.0 * gate_half(pl); }
    bool in_plane(int pl, double len, int slot = 0) const {
        return len >= plane_lo(pl, slot) && len < plane_hi(pl, slot);
    }
    // path trees whose gate candidates come from the wide gate: R x M_init
    int wide_trees() const {
        const double r = std::min(1.0, std::max(0.0, s.shrink_r));
        return (int)std::lround(r * (double)s.m_init);
    }
    bool shrink_on() const { return s.gate_enabled && s.shrink_k > 1.0 && wide_trees() > 0; }
    // R < 1: wide-gate and gate samples, combined with MIS
    bool shrink_mix() const { return shrink_on() && wide_trees() < s.m_init; }
    // the wide ("rough") gate of the shrink mapping: K times the gate, same centre
    bool in_rough_gate(double len) const {
        const double c = fg[0].gate_center, h = 0.5 * s.shrink_k * s.gate_width;
        return len >= c - h && len < c + h;
    }
    // Delta l of a temporal shift from the previous frame into the current one
    // (Sec. 4.1, time-gate shifting): the gate's move; bins do not move
    double gate_shift(int pl) const { return pl < s.n_bins ? 0.0 : fg[0].gate_center - fg[1].gate_center; }
    int bin_of(double len) const {
        if (s.n_bins <= 0) return -1;
        double f = std::floor((len - s.bin_t0) / s.bin_width);
        if (!(f > -2.0 && f < (double)s.n_bins + 1.0)) return -1;
        int b = (int)f;
        if (b >= 0 && b < s.n_bins && len < plane_lo(b)) b -= 1;
        if (b >= -1 && b + 1 < s.n_bins && b + 1 >= 0 && len >= plane_lo(b + 1)) b += 1;
        if (b < 0 || b >= s.n_bins || !in_plane(b, len)) return -1;
        return b;
    }

    // reconnection criterion (Sec. 4.1, first consecutive rough vertices)
    bool recon_ok(const Vertex& a, const Vertex& b) const {
        return rough(a.obj) && rough(b.obj) && length(b.p - a.p) >= dmin;
    }

    // -------------------------------------------------------------------
    // path contribution f(y) in the product solid-angle measure of the
    // sampled directions, with NEE to the delta light (no visibility).
    // -------------------------------------------------------------------
    // throughput of the path ys -> light in a frame slot; len receives the
    // plane quantity (path length or path velocity)
    double path_eval(int slot, int pix, const std::vector<Vertex>& ys, double& len) const {
        const FrameGeom& F = fg[slot];
        V3 wi = toward_camera(slot, ys[0]);
        double f = 1.0;
        len = camera_leg(slot, ys[0]);
        for (size_t j = 0; j + 1 < ys.size(); ++j) {
            V3 dv = ys[j + 1].p - ys[j].p;
            double dl = length(dv);
            V3 wo = (1.0 / dl) * dv;
            f *= bsdf(ys[j].obj, ys[j].n, wi, wo) * std::fabs(dot(ys[j].n, wo));
            len += seg_q(ep(F, ys[j]), ep(F, ys[j + 1]));
            wi = -wo;
        }
        const Vertex& y = ys.back();
        V3 L = light_pos(slot, pix);
        V3 dv = L - y.p;
        double dl = length(dv);
        V3 wo = (1.0 / dl) * dv;
        f *= bsdf(y.obj, y.n, wi, wo) * std::fabs(dot(y.n, wo)) * light_emit(slot, pix, y.p) / (dl * dl);
        len += seg_q(ep(F, y), light_ep(slot, pix));
        return f;
    }

    // -------------------------------------------------------------------
    // Newton solve of the path constraint with the average-gradient gauge
    // (Sec. 4.3; Sec. 4.6 swaps the path length for the path velocity).
    // Reading: the constraint functions use the source endpoints at xi and
    // the destination endpoints at xi', and dF2/dxi' is derived by
    // differentiating F2 (the printed sign of its Hessian term is not used).
    //
    // The constraint function of the reconnection vertex p = p(xi) with fixed
    // neighbours a and b is c + phi_a(p) + phi_b(p), where
    //   time:     phi_a(p) = |p - a|
    //   velocity: phi_a(p) = (v_a - v(p)) . d,  d = (p - a) / |p - a|,
    // the second being the two segments' terms of the path velocity written
    // from a's side (a segment's term does not depend on its direction).  With
    // the rigid motion v(p) = V + W x (p - t), l = |p - a|, w = v_a - v(p) and
    // P = I - d d^T (the supplement with these derivations is not available;
    // they are derived here and pinned by finite differences):
    //   grad phi_a = W x d + P w / l
    //   Hess phi_a x = (d (d.(W x x)) - (d.x) (W x d)) / l
    //                  - ((d.w) P x + d (P w . x) + P w (d.x)) / l^2
    // and in chart coordinates g = J^T grad, H = J^T Hess J + grad . p_ij.
    // -------------------------------------------------------------------
    struct LenEval { bool ok = false; double L = 0, g[2] = {0, 0}, H[2][2] = {{0, 0}, {0, 0}}; double area = 0; };
    LenEval len_eval(const FrameGeom& F, int obj, double u, double v, const EP& a, const EP& b, double c) const {
        return constraint_eval(F, obj, u, v, a, b, c, s.domain);
    }
    LenEval constraint_eval(const FrameGeom& F, int obj, double u, double v, const EP& a, const EP& b, double c,
                            int domain) const {
        LenEval e;
        ChartEval ch = chart(F, obj, u, v);
        if (!ch.ok) return e;
        const V3 vp = vel_at(F, obj, ch.p);
        const V3 W = F.ov.empty() ? V3() : V3(F.ov[6 * obj + 3], F.ov[6 * obj + 4], F.ov[6 * obj + 5]);
        double val = c;
        V3 grad;
        V3 Hju, Hjv;   // Hess_p applied to the chart tangents
        for (const EP* e2 : {&a, &b}) {
            V3 r = ch.p - e2->p;
            double l = length(r);
            if (!(l > 0.0)) return e;
            V3 d = (1.0 / l) * r;
            if (domain == 0) {
                val += l;
                grad = grad + d;
                auto Hx = [&](V3 x) { return (1.0 / l) * (x - dot(d, x) * d); };
                Hju = Hju + Hx(ch.ju);
                Hjv = Hjv + Hx(ch.jv);
            } else {
                V3 w = e2->v - vp;
                V3 Pw = w - dot(d, w) * d;
                val += dot(w, d);
                grad = grad + cross(W, d) + (1.0 / l) * Pw;
                auto Hx = [&](V3 x) {
                    V3 t1 = (1.0 / l) * (dot(d, cross(W, x)) * d - dot(d, x) * cross(W, d));
                    V3 t2 = dot(d, w) * (x - dot(d, x) * d) + dot(Pw, x) * d + dot(d, x) * Pw;
                    return t1 - (1.0 / (l * l)) * t2;
                };
                Hju = Hju + Hx(ch.ju);
                Hjv = Hjv + Hx(ch.jv);
            }
        }
        e.L = val;
        e.g[0] = dot(grad, ch.ju);
        e.g[1] = dot(grad, ch.jv);
        e.H[0][0] = dot(ch.ju, Hju) + dot(grad, ch.puu);
        e.H[0][1] = dot(ch.ju, Hjv) + dot(grad, ch.puv);
        e.H[1][0] = e.H[0][1];
        e.H[1][1] = dot(ch.jv, Hjv) + dot(grad, ch.pvv);
        e.area = length(cross(ch.ju, ch.jv));
        e.ok = true;
        return e;
    }

    struct NewtonOut { bool conv = false; double xi[2] = {0, 0}; int iters = 0; double det_dxi = 0, det_area = 0, F[2] = {0, 0}; int status = 0; };

    NewtonOut newton(const FrameGeom& FS, const FrameGeom& FD, int obj, const double xi[2], const EP& as,
                     const EP& bs, double cs, const EP& ad, const EP& bd, double cd, double dl0, double tol,
                     int maxit) const {
        NewtonOut out;
        LenEval S = len_eval(FS, obj, xi[0], xi[1], as, bs, cs);
        if (!S.ok) { out.status = 1; return out; }
        auto Fval = [&](const double xp[2], LenEval& D, double Fv[2]) {
            D = len_eval(FD, obj, xp[0], xp[1], ad, bd, cd);
            if (!D.ok) return false;
            double m0 = 0.5 * (S.g[0] + D.g[0]), m1 = 0.5 * (S.g[1] + D.g[1]);
            double d0 = xp[0] - xi[0], d1 = xp[1] - xi[1];
            Fv[0] = D.L - S.L - dl0;
            Fv[1] = -m1 * d0 + m0 * d1;         // (R m)^T (xi' - xi), R = 90 deg rotation
            return true;
        };
        // dF/dxi' = [grad L_dst ; (R m - 0.5 H_dst R d)^T]
        auto jac_dst = [&](const double xp[2], const LenEval& D, double J[2][2]) {
            double m0 = 0.5 * (S.g[0] + D.g[0]), m1 = 0.5 * (S.g[1] + D.g[1]);
            double d0 = xp[0] - xi[0], d1 = xp[1] - xi[1];
            double rd0 = -d1, rd1 = d0;
            J[0][0] = D.g[0];
            J[0][1] = D.g[1];
            J[1][0] = -m1 - 0.5 * (D.H[0][0] * rd0 + D.H[0][1] * rd1);
            J[1][1] = m0 - 0.5 * (D.H[1][0] * rd0 + D.H[1][1] * rd1);
        };
        double xp[2] = {xi[0], xi[1]};
        LenEval D;
        double Fv[2];
        if (!Fval(xp, D, Fv)) { out.status = 1; return out; }
        int it = 0;
        while (true) {
            if (std::fabs(Fv[0]) <= tol && std::fabs(Fv[1]) <= tol) break;
            if (it >= maxit) { out.status = 2; out.F[0] = Fv[0]; out.F[1] = Fv[1]; return out; }
            double J[2][2];
            jac_dst(xp, D, J);
            double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            if (std::fabs(det) < 1e-12) { out.status = 3; return out; }
            double step0 = -(J[1][1] * Fv[0] - J[0][1] * Fv[1]) / det;
            double step1 = -(-J[1][0] * Fv[0] + J[0][0] * Fv[1]) / det;
            double norm0 = std::hypot(Fv[0], Fv[1]);
            bool accepted = false;
            double alpha = 1.0;
            for (int ls = 0; ls < 4; ++ls, alpha *= 0.5) {   // backtracking line search
                double xt[2] = {xp[0] + alpha * step0, xp[1] + alpha * step1};
                LenEval Dt;
                double Ft[2];
                if (Fval(xt, Dt, Ft) && std::hypot(Ft[0], Ft[1]) < norm0) {
                    xp[0] = xt[0]; xp[1] = xt[1]; D = Dt; Fv[0] = Ft[0]; Fv[1] = Ft[1];
                    accepted = true;
                    break;
                }
            }
            if (!accepted) { out.status = 4; return out; }
            ++it;
        }
        // implicit-function Jacobian: |det dxi'/dxi| = |det dF/dxi| / |det dF/dxi'|
        double Jd[2][2];
        jac_dst(xp, D, Jd);
        double m0 = 0.5 * (S.g[0] + D.g[0]), m1 = 0.5 * (S.g[1] + D.g[1]);
        double d0 = xp[0] - xi[0], d1 = xp[1] - xi[1];
        double rd0 = -d1, rd1 = d0;
        double Js[2][2];   // dF/dxi = [-grad L_src ; -(R m + 0.5 H_src R d)^T]
        Js[0][0] = -S.g[0];
        Js[0][1] = -S.g[1];
        Js[1][0] = -(-m1 + 0.5 * (S.H[0][0] * rd0 + S.H[0][1] * rd1));
        Js[1][1] = -(m0 + 0.5 * (S.H[1][0] * rd0 + S.H[1][1] * rd1));
        double detd = Jd[0][0] * Jd[1][1] - Jd[0][1] * Jd[1][0];
        double dets = Js[0][0] * Js[1][1] - Js[0][1] * Js[1][0];
        if (std::fabs(detd) < 1e-12) { out.status = 3; return out; }
        out.conv = true;
        out.xi[0] = xp[0];
        out.xi[1] = xp[1];
        out.iters = it;
        out.det_dxi = std::fabs(dets) / std::fabs(detd);
        // chart -> surface area factor sqrt(det J'^T J') / sqrt(det J^T J)
        out.det_area = D.area / S.area * out.det_dxi;
        out.F[0] = Fv[0];
        out.F[1] = Fv[1];
        return out;
    }

    // -------------------------------------------------------------------
    // shift T_{src -> dst} of a stored path (Sec. 4.1): random replay up to
    // the vertex before the reconnection vertex, reconnection, then the
    // path-length-aware perturbation of the reconnection vertex.
    // -------------------------------------------------------------------
    struct ShiftOut { bool ok = false; PathRec y; double J = 0, phat = 0; };

    ShiftOut shift(const PathRec& x, int src_slot, int src_pix, int dst_slot, int dst_pix, int plane, double dl0,
                   Stats& st) const {
        ShiftOut R;
        st.c[ST_SHIFTS]++;
        const GBuf& g = gb[dst_slot][dst_pix];
        if (!g.hit) return R;
        const FrameGeom& FS = fg[src_slot];
        const FrameGeom& FD = fg[dst_slot];
        std::vector<Vertex> ys;
        ys.push_back(g.v);
        double pdf_y = 1.0;
        V3 wi = toward_camera(dst_slot, ys[0]);
        int nrep = (x.k == 0) ? x.n - 1 : x.k - 2;
        for (int i = 1; i <= nrep; ++i) {
            const Vertex cur = ys.back();
            Draw u = draw(s.seed, x.opix, x.ofr, PASS_BSDF, (uint64_t)x.tree, (uint64_t)i);
            V3 wo;
            double pdf;
            if (!bsdf_sample(cur.obj, cur.n, wi, u.u(0), u.u(1), wo, pdf)) return R;
            Vertex nx;
            st.c[ST_RAYS]++;
            if (!trace(FD, cur, wo, nx)) return R;
            // the offset path must not reconnect earlier than the base path
            if (recon_ok(cur, nx)) return R;
            pdf_y *= pdf;
            ys.push_back(nx);
            wi = -wo;
        }
        // Every rejection below is a plain conjunction, so the order of the
        // tests does not change the result; rays are traced last so that only
        // shifts that would contribute pay for them (the ray count depends on
        // this order).
        if (x.k == 0) {   // pure random replay
            double len;
            double C = path_eval(dst_slot, dst_pix, ys, len);
            if (!(C > 0.0)) return R;
            double J = x.pre_pdf / pdf_y;
            if (!(J >= 1.0 / s.j_max && J <= s.j_max)) return R;
            double ph = in_plane(plane, len, dst_slot) ? C : 0.0;
            if (!(ph > 0.0)) return R;
            st.c[ST_RAYS]++;
            if (!light_visible(dst_slot, dst_pix, ys.back())) return R;   // the only visibility ray
            R.y = x;
            R.y.len = len;
            R.y.pre_pdf = pdf_y;
            R.y.phat = ph;
            R.J = J;
            R.phat = ph;
            R.ok = true;
            st.c[ST_SHIFTS_OK]++;
            return R;
        }

        const Vertex ykm1 = ys.back();
        if (!rough(ykm1.obj)) return R;
        const int obj = x.p.obj;
        Vertex xkm1_s = vertex_at(FS, x.xkm1);
        Vertex p_s = vertex_at(FS, x.p);
        const bool p2light = x.p2.obj < 0;
        Vertex p2_s, p2_d;
        EP p2s_ep, p2d_ep;
        if (p2light) {
            p2s_ep = light_ep(src_slot, src_pix);
            p2d_ep = light_ep(dst_slot, dst_pix);
        } else {
            p2_s = vertex_at(FS, x.p2);
            p2_d = vertex_at(FD, x.p2);
            p2s_ep = ep(FS, p2_s);
            p2d_ep = ep(FD, p2_d);
        }
        std::vector<Vertex> sfx_d;
        for (int q = 0; q < x.nsfx; ++q) sfx_d.push_back(vertex_at(FD, x.sfx[q]));
        // the rest of the path's quantity, fixed while p moves
        const EP xkm1_ep = ep(FS, xkm1_s), p_ep = ep(FS, p_s), ykm1_ep = ep(FD, ykm1);
        double c_src = x.len - seg_q(xkm1_ep, p_ep) - seg_q(p_ep, p2s_ep);
        double c_dst = camera_leg(dst_slot, ys[0]);
        for (size_t j = 0; j + 1 < ys.size(); ++j) c_dst += seg_q(ep(FD, ys[j]), ep(FD, ys[j + 1]));
        if (!p2light) {
            EP prev = p2d_ep;
            for (const Vertex& v : sfx_d) { c_dst += seg_q(prev, ep(FD, v)); prev = ep(FD, v); }
            c_dst += seg_q(prev, light_ep(dst_slot, dst_pix));
        }
        double xi2[2] = {x.p.xi[0], x.p.xi[1]};
        double det_area;
        if (s.shift_mode == 1) {
            st.c[ST_NEWTON_ATT]++;
            double tol = s.newton_tol_rel * plane_width(plane);
            NewtonOut no = newton(FS, FD, obj, x.p.xi, xkm1_ep, p2s_ep, c_src, ykm1_ep, p2d_ep, c_dst, dl0, tol,
                                  s.newton_max_iter);
            if (!no.conv) return R;
            if (s.round_trip) {
                // GRIS needs every shift to be a bijection (Sec. 3.2.3); the
                // gauge makes the exact root reversible (Sec. 4.3), but near a
                // stationary length the iteration can reach another root or
                // fail in one direction only.  Keep the shift only if the
                // inverse shift (destination and source swapped, Delta l
                // negated) brings the vertex back to the source vertex.
                NewtonOut bk = newton(FD, FS, obj, no.xi, ykm1_ep, p2d_ep, c_dst, xkm1_ep, p2s_ep, c_src, -dl0, tol,
                                      s.newton_max_iter);
                if (!bk.conv) return R;
                ChartEval cb = chart(FS, obj, bk.xi[0], bk.xi[1]);
                if (!cb.ok || length(cb.p - p_s.p) > dmin) return R;
            }
            st.c[ST_NEWTON_CONV]++;
            st.c[ST_NEWTON_ITERS] += (uint64_t)no.iters;
            xi2[0] = no.xi[0];
            xi2[1] = no.xi[1];
            det_area = no.det_area;
        } else {
            ChartEval cs = chart(FS, obj, xi2[0], xi2[1]), cd = chart(FD, obj, xi2[0], xi2[1]);
            if (!cs.ok || !cd.ok) return R;
            det_area = length(cross(cd.ju, cd.jv)) / length(cross(cs.ju, cs.jv));
        }
        ChartEval cp = chart(FD, obj, xi2[0], xi2[1]);
        if (!cp.on || !cp.ok) return R;
        Vertex pd;
        pd.obj = obj;
        pd.xi[0] = wrap_coord(obj, 0, xi2[0]);
        pd.xi[1] = wrap_coord(obj, 1, xi2[1]);
        pd.p = cp.p;
        pd.n = cp.n;
        if (length(pd.p - ykm1.p) < dmin) return R;
        std::vector<Vertex> yfull = ys;
        yfull.push_back(pd);
        if (!p2light) {
            yfull.push_back(p2_d);
            for (const Vertex& v : sfx_d) yfull.push_back(v);
        }
        double len;
        double C = path_eval(dst_slot, dst_pix, yfull, len);
        // Jacobian of the whole shift in the product solid-angle measure
        double J = x.pre_pdf / pdf_y;
        V3 ey = ykm1.p - pd.p, ex = xkm1_s.p - p_s.p;
        double ly = length(ey), lx = length(ex);
        double gy = std::fabs(dot(pd.n, (1.0 / ly) * ey)) / (ly * ly);
        double gx = std::fabs(dot(p_s.n, (1.0 / lx) * ex)) / (lx * lx);
        J *= gy / gx * det_area;
        if (!p2light) {
            V3 e2d = pd.p - p2_d.p, e2s = p_s.p - p2_s.p;
            double l2d = length(e2d), l2s = length(e2s);
            double g2d = std::fabs(dot(p2_d.n, (1.0 / l2d) * e2d)) / (l2d * l2d);
            double g2s = std::fabs(dot(p2_s.n, (1.0 / l2s) * e2s)) / (l2s * l2s);
            J *= g2d / g2s;
        }
        if (!(J >= 1.0 / s.j_max && J <= s.j_max)) return R;
        double ph = in_plane(plane, len, dst_slot) ? C : 0.0;
        if (!(ph > 0.0)) return R;
        // visibility of the moved edges; the suffix is re-tested when the two
        // domains belong to different frames (the scene may have moved).  All
        // of the shift's visibility rays are traced (and counted), then the
        // shift fails if any is blocked.
        bool vis = true;
        st.c[ST_RAYS]++;
        vis = visible_pts(FD, ykm1, pd) && vis;
        if (p2light) {
            st.c[ST_RAYS]++;
            vis = light_visible(dst_slot, dst_pix, pd) && vis;
        } else {
            st.c[ST_RAYS]++;
            vis = visible_pts(FD, pd, p2_d) && vis;
            if (src_slot != dst_slot) {
                Vertex prev = p2_d;
                for (const Vertex& v : sfx_d) {
                    st.c[ST_RAYS]++;
                    vis = visible_pts(FD, prev, v) && vis;
                    prev = v;
                }
                st.c[ST_RAYS]++;
                vis = light_visible(dst_slot, dst_pix, prev) && vis;
            }
        }
        if (!vis) return R;
        R.y = x;
        R.y.xkm1.obj = ykm1.obj;
        R.y.xkm1.xi[0] = ykm1.xi[0];
        R.y.xkm1.xi[1] = ykm1.xi[1];
        R.y.p.obj = obj;
        R.y.p.xi[0] = pd.xi[0];
        R.y.p.xi[1] = pd.xi[1];
        R.y.len = len;
        R.y.pre_pdf = pdf_y;
        R.y.phat = ph;
        R.J = J;
        R.phat = ph;
        R.ok = true;
        st.c[ST_SHIFTS_OK]++;
        if (s.shift_mode == 1) st.c[ST_NEWTON_OK]++;
        return R;
    }

    // -------------------------------------------------------------------
    // passes
    // -------------------------------------------------------------------
    void gbuffer_pass(int slot, uint64_t frame) {
        const FrameGeom& F = fg[slot];
        gb[slot].assign(P, GBuf());
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
        for (int pix = 0; pix < P; ++pix) {
            int x = pix % s.width, y = pix / s.width;
            double fx = s.crop_x0 + x, fy = s.crop_y0 + y;
            double u0 = 0.5, u1 = 0.5;
            if (s.jitter) {
                Draw d = draw(s.seed, full_pixel(pix), frame, PASS_JITTER, 0, 0);
                u0 = d.u(0);
                u1 = d.u(1);
            }
            double sx = 2.0 * (fx + u0) / s.full_width - 1.0;
            double sy = 1.0 - 2.0 * (fy + u1) / s.full_height;
            V3 o, dir;
            if (s.camera_model == 0) {
                o = F.cam_pos;
                dir = normalize(F.cam_fwd + (sx * F.tan_half * F.aspect) * F.cam_right + (sy * F.tan_half) * F.cam_up);
            } else {
                o = F.cam_pos + (sx * F.ortho_hx) * F.cam_right + (sy * F.ortho_hy) * F.cam_up;
                dir = F.cam_fwd;
            }
            Hit h = closest(F, o, dir);
            if (h.hit) {
                gb[slot][pix].hit = true;
                gb[slot][pix].v = hit_vertex(F, h, o, dir);
            }
        }
    }

    // Shrink mapping (Sec. 4.4.2): the gate reservoir's winner x, drawn with
    // the target f * 1[l in the rough gate], is moved by the path-length-aware
    // shift of its own pixel with Delta l = (l - l0) / K + l0 - l (l0 the gate
    // centre), so that its length lands in the gate at the same relative
    // position; the Jacobian of this map is the shift's times 1/K, and the
    // sample's contribution weight is multiplied by it.  A path without a
    // reconnection vertex (or under the naive shift) cannot be shrunk: it is
    // kept unchanged if it already lies in the gate.  A failed shrink empties
    // the reservoir (with all samples in the wide gate, R = 1, the estimate is
    // biased low where shrinks fail, as the paper notes).
    void shrink_gate_sample(int pix, PixelRes& pr, Stats& st) {
        auto it = pr.find(s.n_bins);
        if (it == pr.end()) return;
        Res& r = it->second;
        if (s.shift_mode != 1 || r.y.k < 2) {
            if (!in_plane(s.n_bins, r.y.len)) pr.erase(it);
            return;
        }
        const double l0 = fg[0].gate_center, K = s.shrink_k, l = r.y.len;
        ShiftOut sh = shift(r.y, 0, pix, 0, pix, s.n_bins, (l - l0) / K + l0 - l, st);
        if (!sh.ok) {
            pr.erase(it);
            return;
        }
        r.W *= sh.J / K;
        r.y = sh.y;
    }

    // R < 1 (Sec. 4.4.2): the gate's canonical reservoir (gate samples of the
    // last (1 - R) M_init trees, confidence M_n) and the wide-gate reservoir
    // (the first R M_init trees, confidence M_w) are merged by GRIS with the
    // generalized balance heuristic (eq. GRIS_MIS_weight, eq.
    // GRIS_resampling_weight) into the gate: the wide sample y_w enters
    // shrunk, y' = T(y_w) with |J| = |J_shift| / K, and the density of the
    // wide technique at a gate path y is p_w(T^-1(y)) |J_{T^-1}(y)|, with
    // T^-1 the expansion Delta l = K (l - l0) + l0 - l into the wide gate and
    // |J_{T^-1}| = K |J_shift|; a failed expansion means the wide technique
    // cannot produce y.  Paths that cannot be moved (no reconnection vertex,
    // or the naive shift) map by the identity where they lie in the gate.
    // One uniform (pass 17) selects between the two candidates.
    void shrink_mix_sample(int pix, uint64_t frame, PixelRes& pr, Stats& st) {
        const int gp = s.n_bins, wp = s.n_bins + 1;
        const double Mw = (double)wide_trees(), Mn = (double)(s.m_init - wide_trees());
        const double l0 = fg[0].gate_center, K = s.shrink_k;
        auto movable = [&](const PathRec& y) { return s.shift_mode == 1 && y.k >= 2; };
        double wa = 0.0, wb = 0.0, pa = 0.0, pb = 0.0;
        PathRec ya, yb;
        auto itn = pr.find(gp);
        if (itn != pr.end()) {   // the canonical gate sample
            const Res& r = itn->second;
            ya = r.y;
            pa = r.y.phat;
            double p_wide = 0.0;
            if (!movable(r.y)) {
                p_wide = pa;
            } else {
                const double l = r.y.len;
                ShiftOut e = shift(r.y, 0, pix, 0, pix, wp, K * (l - l0) + l0 - l, st);
                if (e.ok) p_wide = e.phat * e.J * K;
            }
            wa = Mn * pa / (Mn * pa + Mw * p_wide) * pa * r.W;
        }
        auto itw = pr.find(wp);
        if (itw != pr.end()) {   // the wide-gate sample, shrunk
            const Res& r = itw->second;
            double J = 0.0;
            if (!movable(r.y)) {
                if (in_plane(gp, r.y.len)) {
                    yb = r.y;
                    pb = r.y.phat;
                    J = 1.0;
                }
            } else {
                const double l = r.y.len;
                ShiftOut sh = shift(r.y, 0, pix, 0, pix, gp, (l - l0) / K + l0 - l, st);
                if (sh.ok) {
                    yb = sh.y;
                    pb = sh.phat;
                    J = sh.J / K;
                }
            }
            if (J > 0.0) {
                const double p_wide = r.y.phat / J;   // p_w(y_w) |J_{T^-1}(y')|
                wb = Mw * p_wide / (Mn * pb + Mw * p_wide) * pb * r.W * J;
            }
            pr.erase(itw);
        }
        const double ws = wa + wb;
        if (!(ws > 0.0)) {
            pr.erase(gp);
            return;
        }
        const Draw u = draw(s.seed, full_pixel(pix), frame, PASS_SHRINK_MIX, 0, 0);
        const bool pick_b = u.u(0) * ws < wb;
        Res& out = pr[gp];
        out.y = pick_b ? yb : ya;
        out.W = ws / (pick_b ? pb : pa);
    }

    // initial candidates: path trees with NEE at every vertex, each sub-path
    // deposited into the reservoir of its bin (and the gate) (Sec. 4.5).
    void initial_pass(uint64_t frame, std::vector<PixelRes>& can, std::vector<double>& Mc,
                      std::vector<double>& pt, std::vector<double>& direct_c, std::vector<double>& direct_l) {
        can.assign(P, PixelRes());
        Mc.assign(P, 0.0);
        pt.assign((size_t)B * P, 0.0);
        direct_c.assign(P, 0.0);
        direct_l.assign(P, 0.0);
        std::vector<Stats> ts(nthreads);
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
        for (int pix = 0; pix < P; ++pix) {
#ifdef _OPENMP
            Stats& st = ts[omp_get_thread_num()];
#else
            Stats& st = ts[0];
#endif
            const GBuf& g = gb[0][pix];
            if (!g.hit) continue;
            Mc[pix] = (double)s.m_init;
            const FrameGeom& F = fg[0];
            uint64_t fp = full_pixel(pix);
            std::map<int, double> wsum;
            for (int tree = 0; tree < s.m_init; ++tree) {
                std::vector<Vertex> vs;
                std::vector<double> pdfs;   // pdfs[j-1] = p(omega_j)
                vs.push_back(g.v);
                double beta = 1.0, pdf = 1.0, len = camera_leg(0, g.v);
                V3 wi = toward_camera(0, g.v);
                int kfound = 0;
                for (int i = 1; i <= s.n_max; ++i) {
                    const Vertex xi = vs.back();
                    if (i >= 2 && kfound == 0 && recon_ok(vs[i - 2], vs[i - 1])) kfound = i;
                    bool want = (i >= 2 && i >= s.n_min) || (i == 1 && s.include_direct && s.n_min <= 1);
                    if (want) {
                        V3 L = light_pos(0, pix);
                        V3 dv = L - xi.p;
                        double dl = length(dv);
                        V3 wl = (1.0 / dl) * dv;
                        double fs = bsdf(xi.obj, xi.n, wi, wl);
                        double C = beta * fs * std::fabs(dot(xi.n, wl)) * light_emit(0, pix, xi.p) / (dl * dl);
                        if (C > 0.0) {
                            st.c[ST_RAYS]++;
                            if (!light_visible(0, pix, xi)) C = 0.0;
                        }
                        double l_i = len + seg_q(ep(F, xi), light_ep(0, pix));
                        if (C > 0.0 && i == 1) {
                            if (tree == 0) { direct_c[pix] = C; direct_l[pix] = l_i; }
                        } else if (C > 0.0) {
                            PathRec rec;
                            rec.opix = (uint32_t)fp;
                            rec.ofr = (uint32_t)frame;
                            rec.tree = tree;
                            rec.n = i;
                            rec.k = kfound;
                            rec.len = l_i;
                            rec.phat = C;
                            if (kfound >= 2) {
                                int k = kfound;
                                rec.pre_pdf = 1.0;
                                for (int j = 1; j <= k - 2; ++j) rec.pre_pdf *= pdfs[j - 1];
                                auto ref = [&](const Vertex& v) { VRef r; r.obj = v.obj; r.xi[0] = v.xi[0]; r.xi[1] = v.xi[1]; return r; };
                                rec.xkm1 = ref(vs[k - 2]);
                                rec.p = ref(vs[k - 1]);
                                if (k < i) rec.p2 = ref(vs[k]);
                                rec.nsfx = 0;
                                for (int q = k + 1; q < i; ++q) rec.sfx[rec.nsfx++] = ref(vs[q]);
                            } else {
                                rec.pre_pdf = pdf;
                            }
                            Draw u = draw(s.seed, fp, frame, PASS_RIS, (uint64_t)tree, (uint64_t)i);
                            // plain PT deposits into the planes; the reservoirs
                            // take the gate's candidates from the wide gate
                            // when the shrink mapping is on (all trees, R = 1;
                            // the first R x M_init trees with R < 1, whose
                            // wide-gate reservoir is kept apart, and the
                            // others from the gate).  Each sampling technique
                            // normalizes by its own number of trees.
                            const bool gate_pt = s.gate_enabled && in_plane(s.n_bins, l_i);
                            const bool wide_tree = shrink_on() && tree < wide_trees();
                            const bool gate_res = wide_tree ? in_rough_gate(l_i) : gate_pt;
                            const int gate_key = wide_tree && shrink_mix() ? s.n_bins + 1 : s.n_bins;
                            const double m_gate = !shrink_mix() ? (double)s.m_init
                                                  : (wide_tree ? (double)wide_trees()
                                                               : (double)(s.m_init - wide_trees()));
                            int planes[2] = {bin_of(l_i), gate_res ? gate_key : -1};
                            if (planes[0] >= 0) pt[(size_t)planes[0] * P + pix] += C / pdf / (double)s.m_init;
                            if (gate_pt) pt[(size_t)s.n_bins * P + pix] += C / pdf / (double)s.m_init;
                            for (int q = 0; q < 2; ++q) {
                                int pl = planes[q];
                                if (pl < 0) continue;
                                const double w = C / ((q == 0 ? (double)s.m_init : m_gate) * pdf);
                                double& ws = wsum[pl];
                                ws += w;
                                if (u.u(q) * ws < w) can[pix][pl].y = rec;
                            }
                        }
                    }
                    if (i == s.n_max) break;
                    Draw u = draw(s.seed, fp, frame, PASS_BSDF, (uint64_t)tree, (uint64_t)i);
                    V3 wo;
                    double pw;
                    if (!bsdf_sample(xi.obj, xi.n, wi, u.u(0), u.u(1), wo, pw)) break;
                    double fcos = bsdf(xi.obj, xi.n, wi, wo) * std::fabs(dot(xi.n, wo));
                    Vertex nx;
                    st.c[ST_RAYS]++;
                    if (!trace(F, xi, wo, nx)) break;
                    beta *= fcos;
                    pdf *= pw;
                    pdfs.push_back(pw);
                    len += seg_q(ep(F, xi), ep(F, nx));
                    vs.push_back(nx);
                    wi = -wo;
                }
            }
            for (auto& kv : can[pix]) kv.second.W = wsum[kv.first] / kv.second.y.phat;
            if (shrink_mix()) shrink_mix_sample(pix, frame, can[pix], st);
            else if (shrink_on()) shrink_gate_sample(pix, can[pix], st);
        }
        for (auto& t : ts) stats.add(t);
    }

    int reproject(int pix) const {
        const GBuf& g = gb[0][pix];
        const FrameGeom& F = fg[1];
        V3 p = chart(F, g.v.obj, g.v.xi[0], g.v.xi[1]).p;
        V3 v = p - F.cam_pos;
        double px, py;
        if (s.camera_model == 0) {
            double z = dot(v, F.cam_fwd);
            if (!(z > 0.0)) return -1;
            double sx = dot(v, F.cam_right) / z / (F.tan_half * F.aspect);
            double sy = dot(v, F.cam_up) / z / F.tan_half;
            px = 0.5 * (sx + 1.0) * s.full_width;
            py = 0.5 * (1.0 - sy) * s.full_height;
        } else {
            px = 0.5 * (dot(v, F.cam_right) / F.ortho_hx + 1.0) * s.full_width;
            py = 0.5 * (1.0 - dot(v, F.cam_up) / F.ortho_hy) * s.full_height;
        }
        double fx = std::floor(px) - s.crop_x0, fy = std::floor(py) - s.crop_y0;
        if (!(fx >= 0.0 && fx < s.width && fy >= 0.0 && fy < s.height)) return -1;
        int q = (int)fy * s.width + (int)fx;
        if (!gb[1][q].hit || gb[1][q].v.obj != g.v.obj) return -1;
        return q;
    }

    // temporal reuse: GRIS of the canonical and the previous frame's final
    // reservoir with the generalized balance heuristic (Sec. 3.2.3, 3.2.4)
    void temporal_pass(uint64_t frame, const std::vector<PixelRes>& can, const std::vector<double>& Mc,
                       std::vector<PixelRes>& out, std::vector<double>& Mo) {
        out.assign(P, PixelRes());
        Mo.assign(P, 0.0);
        std::vector<Stats> ts(nthreads);
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
        for (int pix = 0; pix < P; ++pix) {
#ifdef _OPENMP
            Stats& st = ts[omp_get_thread_num()];
#else
            Stats& st = ts[0];
#endif
            if (!gb[0][pix].hit) continue;
            int qp = reproject(pix);
            double mc = Mc[pix];
            double mp = qp >= 0 ? std::min(M_prev[qp], s.m_cap) : 0.0;
            Mo[pix] = mc + mp;
            std::vector<int> planes;
            for (auto& kv : can[pix]) planes.push_back(kv.first);
            if (qp >= 0)
                for (auto& kv : fin_prev[qp]) planes.push_back(kv.first);
            std::sort(planes.begin(), planes.end());
            planes.erase(std::unique(planes.begin(), planes.end()), planes.end());
            uint64_t fp = full_pixel(pix);
            for (int pl : planes) {
                Draw u = draw(s.seed, fp, frame, PASS_TEMPORAL, 0, (uint64_t)pl);
                double ws = 0.0, w2 = 0.0, w0 = 0.0;
                int npos = 0, npresent = 0;
                bool have = false;
                PathRec sel;
                auto itc = can[pix].find(pl);
                if (itc != can[pix].end()) {
                    const Res& xr = itc->second;
                    double ph = xr.y.phat;
                    double den = mc * ph;
                    if (qp >= 0) {
                        ShiftOut sh = shift(xr.y, 0, pix, 1, qp, pl, -gate_shift(pl), st);
                        if (sh.ok) den += mp * sh.phat * sh.J;
                    }
                    double w = (mc * ph / den) * ph * xr.W;
                    ws += w;
                    w2 += w * w;
                    w0 = w;
                    ++npresent;
                    npos += w > 0.0;
                    if (u.u(0) * ws < w) { sel = xr.y; have = true; }
                }
                if (qp >= 0) {
                    auto itp = fin_prev[qp].find(pl);
                    if (itp != fin_prev[qp].end()) {
                        const Res& xr = itp->second;
                        ++npresent;
                        ShiftOut sh = shift(xr.y, 1, qp, 0, pix, pl, gate_shift(pl), st);
                        if (sh.ok) {
                            double a = mp * xr.y.phat / sh.J;
                            double m = a / (a + mc * sh.phat);
                            double w = m * sh.phat * xr.W * sh.J;
                            ws += w;
                            w2 += w * w;
                            npos += w > 0.0;
                            if (u.u(1) * ws < w) { sel = sh.y; have = true; }
                        }
                    }
                }
                if (ws > 0.0) st.md.item(0, ws, w2, npos, npresent, w0);
                if (have && ws > 0.0) {
                    Res r;
                    r.y = sel;
                    r.W = ws / sel.phat;
                    out[pix][pl] = r;
                }
            }
        }
        for (auto& t : ts) stats.add(t);
    }

    // Bin-axis reuse (Sec. 4.5, transient histograms): the reservoir of bin b
    // of a pixel resamples its own sample and those of bins b + o, o in
    // {-1, +1, -2, +2, ...} up to bin_radius, of the same pixel and frame.  A
    // sample of bin b' enters bin b through the path-length-aware shift with
    // Delta l = (b - b') * bin width (Sec. 4.1, eq. path_length_constraint);
    // weights are the generalized balance heuristic over the bin domains
    // (Sec. 3.2.3), every domain with the pixel's confidence M, which the
    // pass leaves unchanged.  The gate plane passes through.
    static int bin_offset(int l) { return (l / 2 + 1) * ((l & 1) ? 1 : -1); }

    void bin_pass(uint64_t frame, const std::vector<PixelRes>& in, const std::vector<double>& Mi,
                  std::vector<PixelRes>& out, std::vector<double>& Mo) {
        out.assign(P, PixelRes());
        Mo = Mi;
        const int K = 2 * s.bin_radius;
        const double bw = s.bin_width;
        std::vector<Stats> ts(nthreads);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
        for (int pix = 0; pix < P; ++pix) {
#ifdef _OPENMP
            Stats& st = ts[omp_get_thread_num()];
#else
            Stats& st = ts[0];
#endif
            if (!gb[0][pix].hit) continue;
            const double m = Mi[pix];
            auto itg = in[pix].find(s.n_bins);
            if (s.gate_enabled && itg != in[pix].end()) out[pix][s.n_bins] = itg->second;
            std::vector<int> planes;
            for (auto& kv : in[pix]) {
                if (kv.first >= s.n_bins) continue;
                planes.push_back(kv.first);
                for (int l = 0; l < K; ++l) {
                    const int b = kv.first - bin_offset(l);   // bins whose domain l is this one
                    if (b >= 0 && b < s.n_bins) planes.push_back(b);
                }
            }
            std::sort(planes.begin(), planes.end());
            planes.erase(std::unique(planes.begin(), planes.end()), planes.end());
            uint64_t fp = full_pixel(pix);
            for (int b : planes) {
                auto dom = [&](int l) { const int c = b + bin_offset(l); return c >= 0 && c < s.n_bins ? c : -1; };
                double ws = 0.0;
                bool have = false;
                PathRec sel;
                auto uni = [&](int cand) {
                    Draw d = draw(s.seed, fp, frame, PASS_BIN, 0, (uint64_t)(b * 4 + cand / 4));
                    return d.u(cand % 4);
                };
                auto itq = in[pix].find(b);
                if (itq != in[pix].end()) {
                    const Res& xr = itq->second;
                    double ph = xr.y.phat;
                    double den = m * ph;
                    for (int l = 0; l < K; ++l) {
                        const int bl = dom(l);
                        if (bl < 0) continue;
                        ShiftOut sh = shift(xr.y, 0, pix, 0, pix, bl, (bl - b) * bw, st);
                        if (sh.ok) den += m * sh.phat * sh.J;
                    }
                    double w = (m * ph / den) * ph * xr.W;
                    ws += w;
                    if (uni(0) * ws < w) { sel = xr.y; have = true; }
                }
                for (int j = 0; j < K; ++j) {
                    const int bj = dom(j);
                    if (bj < 0) continue;
                    auto itj = in[pix].find(bj);
                    if (itj == in[pix].end()) continue;
                    const Res& xr = itj->second;
                    ShiftOut sh = shift(xr.y, 0, pix, 0, pix, b, (b - bj) * bw, st);
                    if (!sh.ok) continue;
                    double a = m * xr.y.phat / sh.J;
                    double den = a + m * sh.phat;
                    for (int l = 0; l < K; ++l) {
                        const int bl = dom(l);
                        if (l == j || bl < 0) continue;
                        ShiftOut t2 = shift(sh.y, 0, pix, 0, pix, bl, (bl - b) * bw, st);
                        if (t2.ok) den += m * t2.phat * t2.J;
                    }
                    double w = (a / den) * sh.phat * xr.W * sh.J;
                    ws += w;
                    if (uni(j + 1) * ws < w) { sel = sh.y; have = true; }
                }
                if (have && ws > 0.0) {
                    Res r;
                    r.y = sel;
                    r.W = ws / sel.phat;
                    out[pix][b] = r;
                }
            }
        }
        for (auto& t : ts) stats.add(t);
    }

    // neighbour choice: integer rejection sampling in the disk of radius r
    void neighbours(int pix, uint64_t frame, int round, std::vector<int>& nb) const {
        nb.assign(s.spatial_k, -1);
        int x = pix % s.width, y = pix / s.width;
        uint64_t fp = full_pixel(pix);
        int64_t R = s.spatial_radius;
        uint64_t span = (uint64_t)(2 * R + 1);
        for (int sl = 0; sl < s.spatial_k; ++sl) {
            for (int t = 0; t < 8; ++t) {
                Draw d = draw(s.seed, fp, frame, PASS_SPATIAL + (uint64_t)round, 1, (uint64_t)(sl * 16 + t / 2));
                uint64_t a = d.x[(t & 1) ? 2 : 0] >> 32, b = d.x[(t & 1) ? 3 : 1] >> 32;
                int64_t dx = (int64_t)((a * span) >> 32) - R;
                int64_t dy = (int64_t)((b * span) >> 32) - R;
                if (dx * dx + dy * dy > R * R || (dx == 0 && dy == 0)) continue;
                int64_t nx = x + dx, ny = y + dy;
                if (nx >= 0 && nx < s.width && ny >= 0 && ny < s.height) {
                    int q = (int)(ny * s.width + nx);
                    if (gb[0][q].hit) nb[sl] = q;
                }
                break;
            }
        }
    }

    // spatial reuse round: canonical + k neighbours, GBH MIS (Sec. 3.2.3)
    void spatial_pass(uint64_t frame, int round, const std::vector<PixelRes>& in, const std::vector<double>& Mi,
                      std::vector<PixelRes>& out, std::vector<double>& Mo) {
        out.assign(P, PixelRes());
        Mo.assign(P, 0.0);
        std::vector<Stats> ts(nthreads);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
        for (int pix = 0; pix < P; ++pix) {
#ifdef _OPENMP
            Stats& st = ts[omp_get_thread_num()];
#else
            Stats& st = ts[0];
#endif
            if (!gb[0][pix].hit) continue;
            std::vector<int> nb;
            neighbours(pix, frame, round, nb);
            const int K = s.spatial_k;
            double mq = Mi[pix];
            std::vector<double> ms(K, 0.0);
            double mtot = mq;
            std::vector<int> planes;
            for (auto& kv : in[pix]) planes.push_back(kv.first);
            for (int sl = 0; sl < K; ++sl) {
                if (nb[sl] < 0) continue;
                ms[sl] = Mi[nb[sl]];
                mtot += ms[sl];
                for (auto& kv : in[nb[sl]]) planes.push_back(kv.first);
            }
            Mo[pix] = mtot;
            std::sort(planes.begin(), planes.end());
            planes.erase(std::unique(planes.begin(), planes.end()), planes.end());
            uint64_t fp = full_pixel(pix);
            // confidences of the domains (-1: no neighbour pixel); pairwise
            // MIS shifts only the canonical sample into the neighbours
            std::vector<double> Ml(K, -1.0), dl(K, 0.0);
            for (int l = 0; l < K; ++l)
                if (nb[l] >= 0) Ml[l] = ms[l];
            const bool pairwise = s.mis_mode == 1;
            for (int pl : planes) {
                double ws = 0.0;
                bool have = false;
                PathRec sel;
                auto uni = [&](int cand) {
                    Draw d = draw(s.seed, fp, frame, PASS_SPATIAL + (uint64_t)round, 2, (uint64_t)(pl * 2 + cand / 4));
                    return d.u(cand % 4);
                };
                double w2 = 0.0, w0 = 0.0;
                int npos = 0, npresent = 0;
                auto itq = in[pix].find(pl);
                if (itq != in[pix].end()) {
                    const Res& xr = itq->second;
                    double ph = xr.y.phat;
                    for (int l = 0; l < K; ++l) {
                        dl[l] = 0.0;
                        if (nb[l] < 0) continue;
                        ShiftOut sh = shift(xr.y, 0, pix, 0, nb[l], pl, 0.0, st);
                        if (sh.ok) dl[l] = sh.phat * sh.J;
                    }
                    double w = mis_weight(s.mis_mode, -1, K, Ml.data(), mq, dl.data(), ph) * ph * xr.W;
                    ws += w;
                    w2 += w * w;
                    w0 = w;
                    ++npresent;
                    npos += w > 0.0;
                    if (uni(0) * ws < w) { sel = xr.y; have = true; }
                }
                for (int j = 0; j < K; ++j) {
                    if (nb[j] < 0) continue;
                    auto itj = in[nb[j]].find(pl);
                    if (itj == in[nb[j]].end()) continue;
                    const Res& xr = itj->second;
                    ++npresent;
                    ShiftOut sh = shift(xr.y, 0, nb[j], 0, pix, pl, 0.0, st);
                    if (!sh.ok) continue;
                    for (int l = 0; l < K; ++l) {
                        dl[l] = 0.0;
                        if (l == j || nb[l] < 0 || pairwise) continue;
                        ShiftOut t2 = shift(sh.y, 0, pix, 0, nb[l], pl, 0.0, st);
                        if (t2.ok) dl[l] = t2.phat * t2.J;
                    }
                    dl[j] = xr.y.phat / sh.J;
                    double w = mis_weight(s.mis_mode, j, K, Ml.data(), mq, dl.data(), sh.phat) * sh.phat * xr.W * sh.J;
                    ws += w;
                    w2 += w * w;
                    npos += w > 0.0;
                    if (uni(j + 1) * ws < w) { sel = sh.y; have = true; }
                }
                if (ws > 0.0) st.md.item(1, ws, w2, npos, npresent, w0);
                if (have && ws > 0.0) {
                    Res r;
                    r.y = sel;
                    r.W = ws / sel.phat;
                    out[pix][pl] = r;
                }
            }
        }
        for (auto& t : ts) stats.add(t);
    }

    int render(const orc_frame* fr, double* img, double* hist, double* pt_img, double* pt_hist) {
        // rotate: the previous call's frame becomes slot 1
        if (fg[0].valid) {
            fg[1] = fg[0];
            gb[1] = gb[0];
        }
        load_frame(fg[0], fr);
        uint64_t frame = (uint64_t)(uint32_t)fr->index;
        gbuffer_pass(0, frame);
        std::vector<PixelRes> can, tmp, fin;
        std::vector<double> Mc, Mt, Mf, pt, dc, dl;
        initial_pass(frame, can, Mc, pt, dc, dl);
        const std::vector<PixelRes>* cur = &can;
        const std::vector<double>* curM = &Mc;
        if (s.temporal && prev_valid) {
            temporal_pass(frame, can, Mc, tmp, Mt);
            cur = &tmp;
            curM = &Mt;
        }
        const std::vector<PixelRes>* stage_t = cur;
        std::vector<PixelRes> rin, bins;
        std::vector<double> rM, bM;
        if (s.bin_radius > 0 && s.n_bins > 1) {
            bin_pass(frame, *cur, *curM, bins, bM);
            cur = &bins;
            curM = &bM;
        }
        for (int r = 0; r < s.spatial_rounds; ++r) {
            std::vector<PixelRes> o;
            std::vector<double> oM;
            spatial_pass(frame, r, *cur, *curM, o, oM);
            rin.swap(o);
            rM.swap(oM);
            cur = &rin;
            curM = &rM;
        }
        fin = *cur;
        Mf = *curM;
        const std::vector<PixelRes>* shown = s.debug_stage == 0 ? &can : (s.debug_stage == 1 ? stage_t : &fin);
        auto splat = [&](int pl, int pix, bool restir) {
            double v = 0.0;
            if (restir) {
                auto it = (*shown)[pix].find(pl);
                if (it != (*shown)[pix].end()) v = it->second.W * it->second.y.phat;
            } else {
                v = pt[(size_t)pl * P + pix];
            }
            if (s.include_direct && dc[pix] > 0.0 && in_plane(pl, dl[pix])) v += dc[pix];
            return v / plane_width(pl);
        };
        for (int pix = 0; pix < P; ++pix) {
            if (s.gate_enabled) {
                if (img) img[pix] = splat(s.n_bins, pix, true);
                if (pt_img) pt_img[pix] = splat(s.n_bins, pix, false);
            }
            for (int b = 0; b < s.n_bins; ++b) {
                if (hist) hist[(size_t)b * P + pix] = splat(b, pix, true);
                if (pt_hist) pt_hist[(size_t)b * P + pix] = splat(b, pix, false);
            }
        }
        fin_prev.swap(fin);
        M_prev.swap(Mf);
        prev_valid = true;
        return 0;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// C entry points
// ---------------------------------------------------------------------------
extern "C" {

void* orc_create(const orc_scene* sc, const orc_sensor* sn, int num_threads) {
    // the bin-axis and shrink shifts are defined here for path lengths only
    if (sn->domain < 0 || sn->domain > 1) return nullptr;
    if (sn->domain == 1 && (sn->bin_radius > 0 || sn->shrink_k > 1.0)) return nullptr;
    Oracle* o = new Oracle();
    o->s = *sn;
    o->nthreads = num_threads > 0 ? num_threads : 1;
    for (int m = 0; m < sc->num_materials; ++m)
        o->mats.push_back({sc->mat_type[m], (double)sc->mat_params[3 * m], (double)sc->mat_params[3 * m + 1],
                           (double)sc->mat_params[3 * m + 2]});
    for (int v = 0; v < sc->num_vertices; ++v)
        o->lverts.push_back(V3(sc->vertices[3 * v], sc->vertices[3 * v + 1], sc->vertices[3 * v + 2]));
    for (int ob = 0; ob < sc->num_objects; ++ob) {
        Object obj;
        obj.type = sc->obj_type[ob];
        obj.material = sc->obj_material[ob];
        const int32_t* g = sc->obj_grid + 5 * ob;
        obj.nu = g[0]; obj.nv = g[1]; obj.wrap_u = g[2]; obj.wrap_v = g[3]; obj.voff = g[4];
        const float* sp = sc->obj_sphere + 4 * ob;
        obj.centre = V3(sp[0], sp[1], sp[2]);
        obj.radius = sp[3];
        obj.tri_base = (int)o->tris.size();
        if (obj.type == 0)
            for (int j = 0; j < obj.nv; ++j)
                for (int i = 0; i < obj.nu; ++i)
                    for (int h = 0; h < 2; ++h) o->tris.push_back({ob, i, j, h});
        o->objs.push_back(obj);
    }
    o->sc = sc->scene_scale;
    o->eps = 1e-4 * o->sc;
    o->dmin = 0.01 * o->sc;
    o->P = sn->width * sn->height;
    o->B = sn->n_bins + (sn->gate_enabled ? 1 : 0);
    return o;
}

void orc_destroy(void* ctx) { delete (Oracle*)ctx; }

void orc_reset(void* ctx) {
    Oracle* o = (Oracle*)ctx;
    o->prev_valid = false;
    o->fin_prev.clear();
    o->M_prev.clear();
}

void orc_set_gate_center(void* ctx, double center) {
    // the history is kept: the next temporal pass shifts it by the gate's move
    ((Oracle*)ctx)->s.gate_center = center;
}

int orc_render_frame(void* ctx, const orc_frame* frame, double* out_image, double* out_hist, double* out_pt_image,
                     double* out_pt_hist) {
    return ((Oracle*)ctx)->render(frame, out_image, out_hist, out_pt_image, out_pt_hist);
}

void orc_get_stats(void* ctx, uint64_t out[8]) {
    Oracle* o = (Oracle*)ctx;
    for (int i = 0; i < 8; ++i) out[i] = o->stats.c[i];
}

void orc_get_merge_diag(void* ctx, double out[10]) {
    Oracle* o = (Oracle*)ctx;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 5; ++i) out[5 * k + i] = o->stats.md.d[k][i];
}

int orc_export_history(void* ctx, float* W, float* phat, float* len, float* pre_pdf, uint32_t* opix, uint32_t* ofr,
                       uint32_t* meta, int32_t* vobj, float* vxi, float* M, uint32_t* mask) {
    Oracle* o = (Oracle*)ctx;
    if (!o->prev_valid) return 1;
    const size_t P = (size_t)o->P, B = (size_t)o->B, PB = P * B;
    const size_t words = (B + 31) / 32;
    for (size_t i = 0; i < words * P; ++i) mask[i] = 0u;
    for (size_t pix = 0; pix < P; ++pix) {
        M[pix] = (float)o->M_prev[pix];
        for (const auto& kv : o->fin_prev[pix]) {
            const size_t pl = (size_t)kv.first, idx = pl * P + pix;
            const PathRec& y = kv.second.y;
            W[idx] = (float)kv.second.W;
            phat[idx] = (float)y.phat;
            len[idx] = (float)y.len;
            pre_pdf[idx] = (float)y.pre_pdf;
            opix[idx] = y.opix;
            ofr[idx] = y.ofr;
            meta[idx] = (uint32_t)y.tree | ((uint32_t)y.n << 8) | ((uint32_t)y.k << 12) | ((uint32_t)y.nsfx << 16);
            const VRef* vr[4] = {&y.xkm1, &y.p, &y.p2, &y.sfx[0]};
            for (int q = 0; q < 4; ++q) {
                vobj[q * PB + idx] = vr[q]->obj;
                vxi[(2 * q) * PB + idx] = (float)vr[q]->xi[0];
                vxi[(2 * q + 1) * PB + idx] = (float)vr[q]->xi[1];
            }
            mask[(pl >> 5) * P + pix] |= 1u << (pl & 31);
        }
    }
    return 0;
}

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) { philox4x64_10(ctr, key, out); }

int orc_load_frame(void* ctx, const orc_frame* frame) {
    Oracle* o = (Oracle*)ctx;
    o->load_frame(o->fg[0], frame);
    return 0;
}

int orc_trace(void* ctx, const double o3[3], const double d3[3], int brute_force, double out[4]) {
    Oracle* o = (Oracle*)ctx;
    V3 org(o3[0], o3[1], o3[2]), dir = normalize(V3(d3[0], d3[1], d3[2]));
    Oracle::Hit h = o->closest(o->fg[0], org, dir, brute_force != 0);
    if (!h.hit) return -1;
    Vertex v = o->hit_vertex(o->fg[0], h, org, dir);
    out[0] = h.t;
    out[1] = h.obj;
    out[2] = v.xi[0];
    out[3] = v.xi[1];
    return h.prim;
}

void orc_mis_weights(int mode, int K, const double* M, double mq, const double* d, double dc, double* out) {
    out[0] = mis_weight(mode, -1, K, M, mq, d, dc);
    for (int j = 0; j < K; ++j) out[1 + j] = M[j] >= 0.0 ? mis_weight(mode, j, K, M, mq, d, dc) : 0.0;
}

int orc_occluded(void* ctx, const double o3[3], const double d3[3], double tmax) {
    Oracle* o = (Oracle*)ctx;
    V3 org(o3[0], o3[1], o3[2]), dir = normalize(V3(d3[0], d3[1], d3[2]));
    return o->occluded(o->fg[0], org, dir, tmax) ? 1 : 0;
}

void orc_bsdf(void* ctx, int obj, const double n[3], const double wi[3], const double* wo, int count, double* out) {
    Oracle* o = (Oracle*)ctx;
    const V3 nn = normalize(V3(n[0], n[1], n[2])), wn = normalize(V3(wi[0], wi[1], wi[2]));
    for (int i = 0; i < count; ++i)
        out[i] = o->bsdf(obj, nn, wn, normalize(V3(wo[3 * i], wo[3 * i + 1], wo[3 * i + 2])));
}

int orc_bsdf_sample(void* ctx, int obj, const double n[3], const double wi[3], const double* u, int count, double* wo,
                    double* pdf) {
    Oracle* o = (Oracle*)ctx;
    const V3 nn = normalize(V3(n[0], n[1], n[2])), wn = normalize(V3(wi[0], wi[1], wi[2]));
    int accepted = 0;
    for (int i = 0; i < count; ++i) {
        V3 w;
        double p = 0.0;
        const bool ok = o->bsdf_sample(obj, nn, wn, u[2 * i], u[2 * i + 1], w, p);
        wo[3 * i] = w.x; wo[3 * i + 1] = w.y; wo[3 * i + 2] = w.z;
        pdf[i] = ok ? p : 0.0;
        accepted += ok ? 1 : 0;
    }
    return accepted;
}

int orc_chart(void* ctx, int obj, const double xi[2], double out[12]) {
    Oracle* o = (Oracle*)ctx;
    ChartEval c = o->chart(o->fg[0], obj, xi[0], xi[1]);
    V3 vs[4] = {c.p, c.ju, c.jv, c.n};
    for (int k = 0; k < 4; ++k) {
        out[3 * k] = vs[k].x;
        out[3 * k + 1] = vs[k].y;
        out[3 * k + 2] = vs[k].z;
    }
    return (c.on && c.ok) ? 1 : 0;
}

int orc_newton(void* ctx, int obj, const double xi[2], const double as[3], const double bs[3], double cs,
               const double ad[3], const double bd[3], double cd, double dl0, double tol, int max_iter,
               double out[8]) {
    Oracle* o = (Oracle*)ctx;
    auto at_rest = [](const double* q) { return Oracle::EP{V3(q[0], q[1], q[2]), V3()}; };
    Oracle::NewtonOut no = o->newton(o->fg[0], o->fg[0], obj, xi, at_rest(as), at_rest(bs), cs, at_rest(ad),
                                     at_rest(bd), cd, dl0, tol, max_iter);
    out[0] = no.xi[0];
    out[1] = no.xi[1];
    out[2] = no.iters;
    out[3] = no.det_dxi;
    out[4] = no.det_area;
    out[5] = no.F[0];
    out[6] = no.F[1];
    out[7] = no.status;
    return no.conv ? 1 : 0;
}

int orc_vel_eval(void* ctx, int obj, const double xi[2], const double a[3], const double va[3], const double b[3],
                 const double vb[3], double c, double out[6]) {
    Oracle* o = (Oracle*)ctx;
    Oracle::EP ea{V3(a[0], a[1], a[2]), V3(va[0], va[1], va[2])}, eb{V3(b[0], b[1], b[2]), V3(vb[0], vb[1], vb[2])};
    Oracle::LenEval e = o->constraint_eval(o->fg[0], obj, xi[0], xi[1], ea, eb, c, 1);
    out[0] = e.L;
    out[1] = e.g[0];
    out[2] = e.g[1];
    out[3] = e.H[0][0];
    out[4] = e.H[0][1];
    out[5] = e.H[1][1];
    return e.ok ? 1 : 0;
}

int orc_wrs(const double* w, const double* u, int n, double* w_sum) {
    double ws = 0.0;
    int sel = -1;
    for (int i = 0; i < n; ++i) {
        ws += w[i];
        if (u[i] * ws < w[i]) sel = i;
    }
    *w_sum = ws;
    return sel;
}

}  // extern "C"
