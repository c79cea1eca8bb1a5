// Device-side building blocks of the ToF ReSTIR hot path (gfx950).
//
// Everything here is __device__ code shared by the kernels of this library:
// Philox4x64-10 streams, surface charts (Sec. 4.2), BSDFs, LDS-stack BVH
// traversal, path evaluation with NEE to delta lights (Sec. 5), and the
// path-length-aware shift (Sec. 4.1-4.3).  Evaluation is FP32; the 2x2 Newton
// solve and the Jacobian determinants are FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tofd {

constexpr float kPi = 3.14159265358979323846f;
#ifndef TOF_STACK_DEPTH
#define TOF_STACK_DEPTH 48
#endif
#ifndef TOF_VIS_STACK_DEPTH
#define TOF_VIS_STACK_DEPTH 24
#endif
constexpr int kStackDepth = TOF_STACK_DEPTH;           // per-lane traversal stack entries (LDS)
constexpr int kVisStackDepth = TOF_VIS_STACK_DEPTH;    // the same for the visibility pass
constexpr int kMaxVerts = 4;         // scattering vertices per path
constexpr int kMaxK = 8;             // spatial neighbours

// ---------------------------------------------------------------------------
// vectors
// ---------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 mk(float a, float b, float c) { return V3{a, b, c}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator-(V3 a) { return V3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float len(V3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ V3 nrm(V3 a) { return (1.0f / len(a)) * a; }
__device__ __forceinline__ float comp(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// ---------------------------------------------------------------------------
// data model (mirrors the C ABI's scene description)
// ---------------------------------------------------------------------------
struct Obj {
    int type, material, nu, nv, wrap_u, wrap_v, voff, tri_base;
    float cx, cy, cz, r;
};
struct Mat {
    int type;
    float albedo, alpha, f0;
};
struct TriInfo {
    int obj, i, j, h;
};
// Binary BVH node of the builder, holding both child boxes; child index has
// bit 31 set for a leaf (sorted primitive position).
struct Node {
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int c0, c1, parent, pad;
};
// Traversal node: four child boxes, one 128-byte line.  Component j of each
// float4 belongs to child j; child[j] >= 0 is a Node4 index, bit 31 set marks
// a leaf: (count - 1) << 28 | first triangle slot, count <= 8; meta.x =
// number of children (1..4).  Node 0 is the root of the tree over the
// objects, whose leaves are the roots of the objects' trees.
struct Node4 {
    float4 lox, loy, loz, hix, hiy, hiz;
    int4 child;
    int4 meta;
};

// The node as traversal reads it: 64 bytes, four 16-byte loads instead of
// eight.  Child boxes are quantized to 8 bits per plane relative to the
// node's box: plane = org + q * 2^e per axis, with lower planes rounded down
// and upper planes up, so every child box contains its exact (padded) box.
// q0 = (lo_x, hi_x, lo_y, hi_y), q1 = (lo_z, hi_z, exponents, child count),
// one byte per child in each word, exponents biased by 127 in bytes 0..2.
struct NodeQ {
    float4 org;
    uint4 q0, q1;
    int4 child;
};
static_assert(sizeof(NodeQ) == 64, "NodeQ is one 64-byte line");

struct SceneDev {
    const Obj* objs;
    const Mat* mats;
    const TriInfo* tri_info;
    const int* sphere_ids;
    int n_obj, n_sph, n_tri;
    float eps, dmin;
};

// One frame's geometry, camera, light and G-buffer.
struct SlotDev {
    // vertices turned into world orientation about their object's origin
    // (world position = origin + wr): differences of nearby vertices stay exact
    // to FP32 rounding of the edge, where absolute world positions would carry
    // their rounding at the object's distance from the world origin
    const float4* wr;
    const float* xf;        // object transforms, 12 floats each
    const NodeQ* nodes;     // 4-wide traversal nodes (quantized), root at 0
    int n_nodes;
    const float4* leaves;   // 3 float4 per sorted triangle: v0 (w = tri id bits), v1, v2
    int n_tri;
    V3 cam_pos, cam_fwd, cam_right, cam_up;
    float tan_half, aspect, ohx, ohy;
    V3 light_pos;
    // instantaneous velocities (velocity domain only): per object linear v and
    // angular w, 6 floats each; camera and point light
    const float* vel;
    V3 cam_vel, light_vel;
    float gate_c;           // the time gate's centre when the frame was rendered
    // G-buffer (obj = -1: no primary hit)
    const int* gb_obj;
    const float* gb_xi0;
    const float* gb_xi1;
    const float4* gb_p;     // xyz = position
    const float4* gb_n;     // xyz = normal
};

struct Sens {
    int W, H, FW, FH, cx0, cy0, cam_model, light_model, count_leg, jitter;
    float light_I;
    int gate_en;
    float gate_c, gate_w;
    int n_bins;
    float t0, bw;
    int n_min, n_max, m_init, temporal, rounds, k, radius;
    float m_cap, tol_rel;
    int max_it;
    float j_max;
    int shift_mode, include_direct, debug_stage;
    int br;                  // bin-axis reuse radius (0 = off)
    float shrink_k;          // shrink mapping of initial gate samples (1 = off)
    int mw;                  // path trees sampling the wide gate (R x M_init; all = R 1, shrink only)
    int domain;              // planes over 0: path length, 1: path velocity
    int round_trip;          // keep a Newton shift only if its inverse returns to the source vertex
    int mis_mode;            // spatial reuse: 0 generalized balance heuristic, 1 pairwise MIS
    int P, B, mask_words;
    uint64_t seed;
};

// Reuse passes: 0 temporal, 1 spatial, 2 bin axis (Sec. 4.5).  K = the
// number of other domains per item; bin-axis domain l of bin b is bin
// b + bin_offset(l), offsets -1, +1, -2, +2, ...
__host__ __device__ __forceinline__ int pass_K(const Sens& s, int mode) { return mode == 0 ? 1 : (mode == 1 ? s.k : 2 * s.br); }
__host__ __device__ __forceinline__ int bin_offset(int l) { return (l / 2 + 1) * ((l & 1) ? 1 : -1); }

struct VRef {
    int obj;
    float xi0, xi1;
};
struct Rec {
    uint32_t opix, ofr;
    int tree, n, k, nsfx;
    VRef v[4];              // x_{k-1}, p, p2 (obj -1 = light), suffix
    float len, pre_pdf, phat;
};

// Reservoirs: one 64-byte record (4 x float4, half a 128-byte line) per
// (plane, pixel), index [plane * P + pixel].  Reuse work lists visit a
// pixel's planes together, so neighbouring lanes touch different planes; a
// contiguous, line-aligned record keeps each lane's access inside one line.
// Words: 0 W, 1 phat, 2 len, 3 pre_pdf, 4 origin pixel, 5 origin frame,
// 6 tree (8 bits) | n << 8 (3) | k << 11 (3) | nsfx << 14 (1) | the high 4
// bits of object 2 << 15 | object 3 << 19 (12), 7 object 0 (12) | object 1
// << 12 (12) | the low 8 bits of object 2 << 24, 8..15 (xi0, xi1) of the four
// vertex refs.  Objects are 12-bit, 0xFFF standing for -1 (none, or the
// light), so a scene holds at most 4095 objects.  M (confidence) and the
// non-empty bitmask are per pixel.
constexpr int kRecWords = 16;
constexpr int kRecF4 = kRecWords / 4;
constexpr int kMaxObjects = 4095;

struct ResSet {
    float4* rec;             // [P * B * kRecF4]
    float* M;                // [P]
    uint32_t* mask;          // [mask_words * P]: bit set <=> reservoir non-empty
};

__device__ __forceinline__ float& rec_W(const ResSet& R, size_t idx) { return ((float*)R.rec)[idx * kRecWords]; }
__device__ __forceinline__ float rec_phat(const ResSet& R, size_t idx) { return ((const float*)R.rec)[idx * kRecWords + 1]; }

// words 6 and 7 from the path's counts and its four vertex objects (-1 allowed)
__host__ __device__ __forceinline__ void rec_pack_meta(int tree, int n, int k, int nsfx, int o0, int o1, int o2,
                                                       int o3, uint32_t& w6, uint32_t& w7) {
    const uint32_t b0 = (uint32_t)o0 & 0xFFFu, b1 = (uint32_t)o1 & 0xFFFu, b2 = (uint32_t)o2 & 0xFFFu,
                   b3 = (uint32_t)o3 & 0xFFFu;
    w6 = ((uint32_t)tree & 255u) | (((uint32_t)n & 7u) << 8) | (((uint32_t)k & 7u) << 11) |
         (((uint32_t)nsfx & 1u) << 14) | ((b2 >> 8) << 15) | (b3 << 19);
    w7 = b0 | (b1 << 12) | ((b2 & 255u) << 24);
}
__host__ __device__ __forceinline__ int rec_obj(uint32_t b) { return b == 0xFFFu ? -1 : (int)b; }

__device__ __forceinline__ void store_rec(const ResSet& R, size_t idx, const Rec& r, float W) {
    float4* q = R.rec + idx * kRecF4;
    uint32_t w6, w7;
    rec_pack_meta(r.tree, r.n, r.k, r.nsfx, r.v[0].obj, r.v[1].obj, r.v[2].obj, r.v[3].obj, w6, w7);
    q[0] = make_float4(W, r.phat, r.len, r.pre_pdf);
    q[1] = make_float4(__uint_as_float(r.opix), __uint_as_float(r.ofr), __uint_as_float(w6), __uint_as_float(w7));
    q[2] = make_float4(r.v[0].xi0, r.v[0].xi1, r.v[1].xi0, r.v[1].xi1);
    q[3] = make_float4(r.v[2].xi0, r.v[2].xi1, r.v[3].xi0, r.v[3].xi1);
}
__device__ __forceinline__ Rec load_rec(const ResSet& R, size_t idx, float& W) {
    const float4* q = R.rec + idx * kRecF4;
    float4 a = q[0], b = q[1], c = q[2], d = q[3];
    Rec r;
    W = a.x;
    r.phat = a.y;
    r.len = a.z;
    r.pre_pdf = a.w;
    r.opix = __float_as_uint(b.x);
    r.ofr = __float_as_uint(b.y);
    const uint32_t m = __float_as_uint(b.z), o = __float_as_uint(b.w);
    r.tree = (int)(m & 255u);
    r.n = (int)((m >> 8) & 7u);
    r.k = (int)((m >> 11) & 7u);
    r.nsfx = (int)((m >> 14) & 1u);
    r.v[0] = VRef{rec_obj(o & 0xFFFu), c.x, c.y};
    r.v[1] = VRef{rec_obj((o >> 12) & 0xFFFu), c.z, c.w};
    r.v[2] = VRef{rec_obj(((m >> 15) & 15u) << 8 | (o >> 24)), d.x, d.y};
    r.v[3] = VRef{rec_obj(m >> 19), d.z, d.w};
    return r;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the stream layout
// counter = (pixel, frame, pass << 56 | a << 32 | b, 0), key = (seed, 0)
// ---------------------------------------------------------------------------
enum { PASS_JITTER = 0, PASS_BSDF = 1, PASS_RIS = 2, PASS_TEMPORAL = 3, PASS_SPATIAL = 4, PASS_BIN = 16,
       PASS_SHRINK_MIX = 17 };

struct Draw {
    uint64_t x[4];
    __device__ __forceinline__ float u(int i) const { return (float)(x[i] >> 40) * (1.0f / 16777216.0f); }
    // the same for an index known only at run time, by selects (an indexed
    // read of x would put the draw in scratch memory)
    __device__ __forceinline__ float u_sel(int i) const {
        const uint64_t v = i == 0 ? x[0] : (i == 1 ? x[1] : (i == 2 ? x[2] : x[3]));
        return (float)(v >> 40) * (1.0f / 16777216.0f);
    }
};

__device__ __forceinline__ Draw philox(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t pass, uint64_t a,
                                       uint64_t b) {
    uint64_t x0 = c0, x1 = c1, x2 = (pass << 56) | (a << 32) | b, x3 = 0;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
        uint64_t hi0 = __umul64hi(m0, x0), lo0 = m0 * x0;
        uint64_t hi1 = __umul64hi(m1, x2), lo1 = m1 * x2;
        uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    Draw d;
    d.x[0] = x0;
    d.x[1] = x1;
    d.x[2] = x2;
    d.x[3] = x3;
    return d;
}

// ---------------------------------------------------------------------------
// transforms and charts
// ---------------------------------------------------------------------------
__device__ __forceinline__ V3 xf_point(const float* m, V3 q) {
    return mk(m[0] * q.x + m[1] * q.y + m[2] * q.z + m[3], m[4] * q.x + m[5] * q.y + m[6] * q.z + m[7],
              m[8] * q.x + m[9] * q.y + m[10] * q.z + m[11]);
}
__device__ __forceinline__ V3 xf_dir(const float* m, V3 q) {
    return mk(m[0] * q.x + m[1] * q.y + m[2] * q.z, m[4] * q.x + m[5] * q.y + m[6] * q.z,
              m[8] * q.x + m[9] * q.y + m[10] * q.z);
}
__device__ __forceinline__ V3 xf_inv_point(const float* m, V3 p) {
    V3 d = mk(p.x - m[3], p.y - m[7], p.z - m[11]);
    return mk(m[0] * d.x + m[4] * d.y + m[8] * d.z, m[1] * d.x + m[5] * d.y + m[9] * d.z,
              m[2] * d.x + m[6] * d.y + m[10] * d.z);
}
__device__ __forceinline__ V3 ld3(const float4* a, int i) {
    float4 v = a[i];
    return mk(v.x, v.y, v.z);
}

struct Chart {
    bool on, ok;
    V3 p, ju, jv, puu, puv, pvv, n;
};

// xi -> p on a grid object (piecewise affine, cell units) or a sphere
// ((theta, phi) about the local z axis), with first and second derivatives.
__device__ inline Chart chart_eval(const SceneDev& S, const SlotDev& G, int obj, float u, float v) {
    Chart c;
    const Obj ob = S.objs[obj];
    V3 z = mk(0.f, 0.f, 0.f);
    c.puu = z;
    c.puv = z;
    c.pvv = z;
    if (ob.type == 0) {
        c.on = true;
        float uu = u, vv = v;
        if (ob.wrap_u) uu = u - (float)ob.nu * floorf(u / (float)ob.nu);
        else if (u < 0.f || u > (float)ob.nu) c.on = false;
        if (ob.wrap_v) vv = v - (float)ob.nv * floorf(v / (float)ob.nv);
        else if (v < 0.f || v > (float)ob.nv) c.on = false;
        int i = (int)floorf(uu), j = (int)floorf(vv);
        i = min(max(i, 0), ob.nu - 1);
        j = min(max(j, 0), ob.nv - 1);
        float a = uu - (float)i, b = vv - (float)j;
        int row = ob.nu + 1;
        int base = ob.voff + j * row + i;
        // the cell's lower triangle (v00, v10, v01) or its upper one (v11, v01, v10)
        const float* m = G.xf + 12 * obj;
        const V3 org = mk(m[3], m[7], m[11]);
        if (a + b <= 1.0f) {
            const V3 r0 = ld3(G.wr, base), ru = ld3(G.wr, base + 1), rv = ld3(G.wr, base + row);
            c.ju = ru - r0;
            c.jv = rv - r0;
            c.p = org + (r0 + a * c.ju + b * c.jv);
        } else {
            const V3 r0 = ld3(G.wr, base + row + 1), ru = ld3(G.wr, base + row), rv = ld3(G.wr, base + 1);
            c.ju = r0 - ru;
            c.jv = r0 - rv;
            c.p = org + (r0 - (1.0f - a) * c.ju - (1.0f - b) * c.jv);
        }
        V3 cr = cross(c.ju, c.jv);
        float l = len(cr);
        c.ok = l > 0.f;
        c.n = c.ok ? (1.0f / l) * cr : z;
    } else {
        const float* m = G.xf + 12 * obj;
        float th = u, ph = v, r = ob.r;
        float st = sinf(th), ct = cosf(th), sp = sinf(ph), cp = cosf(ph);
        V3 radial = mk(st * cp, st * sp, ct);
        c.p = xf_point(m, mk(ob.cx, ob.cy, ob.cz) + r * radial);
        c.ju = xf_dir(m, mk(r * ct * cp, r * ct * sp, -r * st));
        c.jv = xf_dir(m, mk(-r * st * sp, r * st * cp, 0.f));
        c.puu = xf_dir(m, -r * radial);
        c.puv = xf_dir(m, mk(-r * ct * sp, r * ct * cp, 0.f));
        c.pvv = xf_dir(m, mk(-r * st * cp, -r * st * sp, 0.f));
        c.n = xf_dir(m, radial);
        c.on = th >= 1e-3f && th <= kPi - 1e-3f;
        c.ok = true;
    }
    return c;
}

__device__ __forceinline__ float wrap_coord(const SceneDev& S, int obj, int dim, float x) {
    const Obj& ob = S.objs[obj];
    if (ob.type == 0) {
        if (dim == 0 && ob.wrap_u) return x - (float)ob.nu * floorf(x / (float)ob.nu);
        if (dim == 1 && ob.wrap_v) return x - (float)ob.nv * floorf(x / (float)ob.nv);
        return x;
    }
    if (dim == 1) return x - 2.0f * kPi * floorf(x / (2.0f * kPi));
    return x;
}

struct Vtx {
    int obj;
    float xi0, xi1;
    V3 p, n;
};

__device__ __forceinline__ Vtx vertex_at(const SceneDev& S, const SlotDev& G, int obj, float xi0, float xi1) {
    Chart c = chart_eval(S, G, obj, xi0, xi1);
    Vtx v;
    v.obj = obj;
    v.xi0 = xi0;
    v.xi1 = xi1;
    v.p = c.p;
    v.n = c.n;
    return v;
}
__device__ __forceinline__ Vtx gbuf_vertex(const SlotDev& G, int pix) {
    Vtx v;
    v.obj = G.gb_obj[pix];
    v.xi0 = G.gb_xi0[pix];
    v.xi1 = G.gb_xi1[pix];
    float4 p = G.gb_p[pix], n = G.gb_n[pix];
    v.p = mk(p.x, p.y, p.z);
    v.n = mk(n.x, n.y, n.z);
    return v;
}

// ---------------------------------------------------------------------------
// ray casting: watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013),
// analytic spheres, BVH with a per-lane stack in LDS ([depth][lane] layout)
// ---------------------------------------------------------------------------
// Contraction into FMAs is disabled here: the edge functions of two triangles
// sharing an edge must be exact negations of each other, which is what makes
// the test watertight; a fused multiply-add rounds the two orders differently
// and opens cracks along shared edges.
__device__ __forceinline__ bool isect_tri(V3 o, V3 d, int kx, int ky, int kz, float sx, float sy, float sz, V3 v0,
                                          V3 v1, V3 v2, float tmax, float& t, float& b1, float& b2) {
#pragma clang fp contract(off)
    V3 A = v0 - o, B = v1 - o, C = v2 - o;
    float Akz = comp(A, kz), Bkz = comp(B, kz), Ckz = comp(C, kz);
    float ax = comp(A, kx) - sx * Akz, ay = comp(A, ky) - sy * Akz;
    float bx = comp(B, kx) - sx * Bkz, by = comp(B, ky) - sy * Bkz;
    float cx = comp(C, kx) - sx * Ckz, cy = comp(C, ky) - sy * Ckz;
    float U = cx * by - cy * bx, Vv = ax * cy - ay * cx, W = bx * ay - by * ax;
    if ((U < 0.f || Vv < 0.f || W < 0.f) && (U > 0.f || Vv > 0.f || W > 0.f)) return false;
    float det = U + Vv + W;
    if (det == 0.f) return false;
    float T = U * (sz * Akz) + Vv * (sz * Bkz) + W * (sz * Ckz);
    float tt = T / det;
    if (!(tt > 0.f && tt < tmax)) return false;
    t = tt;
    b1 = Vv / det;
    b2 = W / det;
    return true;
}

// Ray/sphere intersection for a unit direction d, in the form of Haines,
// Guenther and Akenine-Moeller ("Precision Improvements for Ray/Sphere
// Intersection", Ray Tracing Gems, 2019): the discriminant r^2 - |l|^2 comes
// from the centre's distance |l| to the ray instead of b^2 - (|f|^2 - r^2),
// which cancels in FP32 when the sphere is small against its distance (an
// error of 1e-6 in the hit point of a ray that meets the sphere obliquely
// becomes 1e-4 of a contribution whose light direction grazes the sphere);
// the roots are q and (|f|^2 - r^2) / q, without cancellation.
__device__ __forceinline__ bool isect_sphere(V3 o, V3 d, V3 c, float r, float tmax, float& t) {
    const V3 f = o - c;
    const float b = -dot(f, d);             // ray parameter of the point nearest the centre
    const float ll = len(f + b * d);        // distance from the centre to the ray
    const float disc = (r - ll) * (r + ll);
    if (disc < 0.f) return false;
    const float q = b + copysignf(sqrtf(disc), b);
    if (q == 0.f) return false;
    const float cc = dot(f, f) - r * r;
    const float ta = cc / q, tb = q;
    const float t0 = fminf(ta, tb), t1 = fmaxf(ta, tb);
    if (t0 > 0.f && t0 < tmax) {
        t = t0;
        return true;
    }
    if (t1 > 0.f && t1 < tmax) {
        t = t1;
        return true;
    }
    return false;
}

struct RayPre {
    V3 o, d, inv;
    int kx, ky, kz;
    float sx, sy, sz;
};
__device__ __forceinline__ RayPre ray_pre(V3 o, V3 d) {
    RayPre r;
    r.o = o;
    r.d = d;
    auto safe_inv = [](float x) { return fabsf(x) > 1e-20f ? 1.0f / x : copysignf(1e20f, x); };
    r.inv = mk(safe_inv(d.x), safe_inv(d.y), safe_inv(d.z));
    int kz = 0;
    if (fabsf(d.y) > fabsf(comp(d, kz))) kz = 1;
    if (fabsf(d.z) > fabsf(comp(d, kz))) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (comp(d, kz) < 0.f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    float dz = comp(d, kz);
    r.sx = comp(d, kx) / dz;
    r.sy = comp(d, ky) / dz;
    r.sz = 1.0f / dz;
    return r;
}

// ray/box slab test; tn = entry distance (clamped at 0)
__device__ __forceinline__ bool slab(float lox, float loy, float loz, float hix, float hiy, float hiz, const RayPre& r,
                                     float tmax, float& tn) {
    const float x1 = (lox - r.o.x) * r.inv.x, x2 = (hix - r.o.x) * r.inv.x;
    const float y1 = (loy - r.o.y) * r.inv.y, y2 = (hiy - r.o.y) * r.inv.y;
    const float z1 = (loz - r.o.z) * r.inv.z, z2 = (hiz - r.o.z) * r.inv.z;
    const float a = fmaxf(fmaxf(fminf(x1, x2), fminf(y1, y2)), fmaxf(fminf(z1, z2), 0.f));
    const float b = fminf(fminf(fmaxf(x1, x2), fmaxf(y1, y2)), fminf(fmaxf(z1, z2), tmax));
    tn = a;
    return a <= b;
}

struct Hit {
    int prim, obj;
    float t, b1, b2;
};

// per-lane event counters; one lane's share of a launch fits 32 bits
constexpr int kNumCounters = 14;
struct Counters {
    uint32_t c[kNumCounters];
};
enum { ST_SHIFTS = 0, ST_SHIFTS_OK, ST_NEWTON_ATT, ST_NEWTON_CONV, ST_NEWTON_ITERS, ST_NEWTON_OK, ST_RAYS, ST_FRAMES,
       ST_OVERFLOW, ST_NODES, ST_TRIS, ST_BADREC, ST_VISFAIL, ST_VISFAIL_NEWTON };
// A queued segment's owner (the index of the float its blocking zeroes) carries
// this flag when the shift moved its reconnection vertex by Newton: blocked
// Newton shifts are counted apart ("actual SR" of the Newton statistics).
// Owners stay below 2^31 (tof_sensor_set checks the sizes that bound them).
constexpr uint32_t kOwnerNewton = 0x80000000u;

// Closest hit (any_hit = false; ties in t go to the smaller primitive id) or
// any hit in (0, tmax) (any_hit = true).  `stack` points at this lane's LDS
// column; consecutive entries are `stride` apart.
__device__ inline bool traverse(const SceneDev& S, const SlotDev& G, V3 o, V3 d, float tmax, bool any_hit, int depth, Hit& h,
                                uint32_t* stack, int stride, Counters& st) {
    RayPre r = ray_pre(o, d);
    float tb = tmax;
    h.prim = -1;
    h.obj = -1;
    const int T = G.n_tri;
    auto test_leaf = [&](int k) -> bool {
        if ((unsigned)k >= (unsigned)T) {   // never for a well-formed tree
            st.c[ST_OVERFLOW]++;
            return false;
        }
        st.c[ST_TRIS]++;
        float4 a = G.leaves[3 * k], b = G.leaves[3 * k + 1], c = G.leaves[3 * k + 2];
        float t, b1, b2;
        float lim = any_hit ? tmax : __fmul_rn(tb, 1.0000001f) + 1e-30f;
        if (isect_tri(r.o, r.d, r.kx, r.ky, r.kz, r.sx, r.sy, r.sz, mk(a.x, a.y, a.z), mk(b.x, b.y, b.z),
                      mk(c.x, c.y, c.z), lim, t, b1, b2)) {
            int id = __float_as_int(a.w);
            if (any_hit) return true;
            if (t < tb || (t == tb && id < h.prim)) {
                tb = t;
                h.prim = id;
                h.t = t;
                h.b1 = b1;
                h.b2 = b2;
            }
        }
        return false;
    };
    if (T > 0) {
        // Leaves are postponed (Aila and Laine 2009): a lane that meets leaf
        // children keeps them as pending and, while other lanes of the wave
        // still look for theirs, goes on through inner nodes, pushing leaves
        // it meets meanwhile onto its stack; the wave then tests the pending
        // leaves together, instead of one leaf phase per node visit with few
        // lanes active.  Visit order does not change a result: closest hit
        // is the minimum of (t, primitive id) over the triangles whose boxes
        // the ray enters before the current best t, any hit is any of them.
        constexpr uint32_t kDone = 0xFFFFFFFFu;   // not a leaf reference: leaves start below 2^28
        constexpr float kInfT = 3.0e38f;
        int sp = 0;
        uint32_t node = 0;           // inner node, leaf reference (bit 31), or kDone
        uint32_t pmask = 0;          // pending leaves: bits of pcc
        int4 pcc = make_int4(0, 0, 0, 0);
        auto push = [&](uint32_t n) {
            if (sp < depth) {
                stack[sp * stride] = n;
                ++sp;
            } else {
                st.c[ST_OVERFLOW]++;
            }
        };
        auto pop = [&]() -> uint32_t {
            if (sp == 0) return kDone;
            --sp;
            return stack[sp * stride];
        };
        // any valid walk visits each node at most once, so this bound only
        // stops a malformed tree
        int budget = 2 * G.n_nodes + 64;
        while (node != kDone || pmask) {
            // inner nodes until every lane of the wave has a pending leaf or
            // is done; no speculation once the stack could not take a node's
            // leaves
            while (node < 0x80000000u && (pmask == 0 || sp + 4 <= depth)) {
                if (--budget <= 0 || node >= (uint32_t)G.n_nodes) {   // never for a well-formed tree
                    st.c[ST_OVERFLOW]++;
                    node = kDone;
                    sp = 0;
                    break;
                }
                // the whole 64-byte node, loaded unconditionally, boxes decoded
                const NodeQ* nq = G.nodes + node;
                const float4 org = nq->org;
                const uint4 q0 = nq->q0, q1 = nq->q1;
                const int4 cc = nq->child;
                const int nc = (int)q1.w;
                const float sx = __int_as_float((int)((q1.z & 0xFFu) << 23));
                const float sy = __int_as_float((int)(((q1.z >> 8) & 0xFFu) << 23));
                const float sz = __int_as_float((int)(((q1.z >> 16) & 0xFFu) << 23));
                auto deq = [](uint32_t w, float o, float sc) {
                    return make_float4(fmaf((float)(w & 0xFFu), sc, o), fmaf((float)((w >> 8) & 0xFFu), sc, o),
                                       fmaf((float)((w >> 16) & 0xFFu), sc, o), fmaf((float)(w >> 24), sc, o));
                };
                const float4 lx = deq(q0.x, org.x, sx), hx = deq(q0.y, org.x, sx);
                const float4 ly = deq(q0.z, org.y, sy), hy = deq(q0.w, org.y, sy);
                const float4 lz = deq(q1.x, org.z, sz), hz = deq(q1.y, org.z, sz);
                st.c[ST_NODES]++;
                // all four boxes, without branches; children j >= nc are padding
                float t0, t1, t2, t3;
                const bool h0 = slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, r, tb, t0);
                const bool h1 = slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, r, tb, t1) && nc > 1;
                const bool h2 = slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, r, tb, t2) && nc > 2;
                const bool h3 = slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, r, tb, t3) && nc > 3;
                const bool f0 = cc.x < 0, f1 = cc.y < 0, f2 = cc.z < 0, f3 = cc.w < 0;   // leaves
                const uint32_t leaves = (h0 && f0 ? 1u : 0u) | (h1 && f1 ? 2u : 0u) | (h2 && f2 ? 4u : 0u) |
                                        (h3 && f3 ? 8u : 0u);
                if (leaves) {
                    if (pmask == 0) {
                        pmask = leaves;
                        pcc = cc;
                    } else {   // speculative: keep them for later
                        if (leaves & 1u) push((uint32_t)cc.x);
                        if (leaves & 2u) push((uint32_t)cc.y);
                        if (leaves & 4u) push((uint32_t)cc.z);
                        if (leaves & 8u) push((uint32_t)cc.w);
                    }
                }
                // key = entry distance of an internal child that is hit, +inf otherwise
                float k0 = (h0 && !f0) ? t0 : kInfT, k1 = (h1 && !f1) ? t1 : kInfT;
                float k2 = (h2 && !f2) ? t2 : kInfT, k3 = (h3 && !f3) ? t3 : kInfT;
                int n0 = cc.x, n1 = cc.y, n2 = cc.z, n3 = cc.w;
                // sorting network on (key, node): nearest first
                auto cswap = [](float& ka, int& na, float& kb, int& nb) {
                    if (kb < ka) {
                        const float kt = ka;
                        ka = kb;
                        kb = kt;
                        const int nt = na;
                        na = nb;
                        nb = nt;
                    }
                };
                if (any_hit) {
                    // any hit: order does not matter for a ray that is not
                    // blocked; only bring the nearest to the front
                    cswap(k0, n0, k1, n1);
                    cswap(k2, n2, k3, n3);
                    cswap(k0, n0, k2, n2);
                } else {
                    cswap(k0, n0, k1, n1);
                    cswap(k2, n2, k3, n3);
                    cswap(k0, n0, k2, n2);
                    cswap(k1, n1, k3, n3);
                    cswap(k1, n1, k2, n2);
                }
                if (k0 < kInfT) {
                    // the others onto the stack, farthest deepest
                    if (k3 < kInfT) push((uint32_t)n3);
                    if (k2 < kInfT) push((uint32_t)n2);
                    if (k1 < kInfT) push((uint32_t)n1);
                    node = (uint32_t)n0;
                } else {
                    node = pop();
                }
                // a leaf taken from the stack becomes the pending one if there is none
                if (node != kDone && node >= 0x80000000u && pmask == 0) {
                    pmask = 1u;
                    pcc.x = (int)node;
                    node = pop();
                }
                if (__all(pmask != 0)) break;
            }
            // leaf phase: the pending leaves, then leaves met on the stack
            // while no inner node is next
            while (pmask) {
                const int j = __ffs(pmask) - 1;
                pmask &= pmask - 1;
                const uint32_t c = (uint32_t)(j == 0 ? pcc.x : (j == 1 ? pcc.y : (j == 2 ? pcc.z : pcc.w)));
                const int first = (int)(c & 0x0FFFFFFFu), cnt = (int)((c >> 28) & 7u) + 1;
                for (int k = first; k < first + cnt; ++k)
                    if (test_leaf(k)) return true;
                if (pmask == 0 && node != kDone && node >= 0x80000000u) {
                    pmask = 1u;
                    pcc.x = (int)node;
                    node = pop();
                }
            }
        }
    }
    for (int q = 0; q < S.n_sph; ++q) {
        int ob = S.sphere_ids[q];
        const Obj& O = S.objs[ob];
        V3 cw = xf_point(G.xf + 12 * ob, mk(O.cx, O.cy, O.cz));
        float t;
        float lim = any_hit ? tmax : __fmul_rn(tb, 1.0000001f) + 1e-30f;
        if (isect_sphere(r.o, r.d, cw, O.r, lim, t)) {
            if (any_hit) return true;
            int prim = T + ob;
            if (t < tb || (t == tb && prim < h.prim)) {
                tb = t;
                h.prim = prim;
                h.obj = ob;
                h.t = t;
            }
        }
    }
    if (any_hit) return false;
    if (h.prim >= 0 && h.prim < T) h.obj = S.tri_info[h.prim].obj;
    return h.prim >= 0;
}

__device__ __forceinline__ Vtx hit_vertex(const SceneDev& S, const SlotDev& G, const Hit& h, V3 o, V3 d) {
    float xi0, xi1;
    if (h.prim < S.n_tri) {
        TriInfo ti = S.tri_info[h.prim];
        if (ti.h == 0) {
            xi0 = (float)ti.i + h.b1;
            xi1 = (float)ti.j + h.b2;
        } else {
            xi0 = (float)(ti.i + 1) - h.b1;
            xi1 = (float)(ti.j + 1) - h.b2;
        }
    } else {
        const Obj& ob = S.objs[h.obj];
        V3 q = xf_inv_point(G.xf + 12 * h.obj, o + h.t * d) - mk(ob.cx, ob.cy, ob.cz);
        float ct = fminf(1.0f, fmaxf(-1.0f, q.z / ob.r));
        xi0 = acosf(ct);
        float ph = atan2f(q.y, q.x);
        if (ph < 0.f) ph += 2.0f * kPi;
        xi1 = ph;
    }
    return vertex_at(S, G, h.obj, xi0, xi1);
}

__device__ __forceinline__ V3 offset_pt(const SceneDev& S, V3 p, V3 n, V3 dir) {
    return dot(n, dir) > 0.f ? p + S.eps * n : p - S.eps * n;
}

// A visibility query as a segment (offset origin, unit direction, length).
struct Seg {
    V3 o, d;
    float t;
};
__device__ __forceinline__ Seg seg_pts(const SceneDev& S, const Vtx& a, const Vtx& b) {
    V3 o = offset_pt(S, a.p, a.n, b.p - a.p);
    V3 t = offset_pt(S, b.p, b.n, a.p - b.p);
    V3 dv = t - o;
    float dist = len(dv);
    return Seg{o, (1.0f / dist) * dv, dist};
}
__device__ __forceinline__ Seg seg_point(const SceneDev& S, const Vtx& a, V3 L) {
    V3 o = offset_pt(S, a.p, a.n, L - a.p);
    V3 dv = L - o;
    float dist = len(dv);
    return Seg{o, (1.0f / dist) * dv, dist};
}

struct Tracer {
    const SceneDev& S;
    uint32_t* stack;
    int stride;
    int depth;          // stack entries per lane
    Counters& st;

    __device__ bool trace(const SlotDev& G, const Vtx& from, V3 dir, Vtx& out) {
        V3 o = offset_pt(S, from.p, from.n, dir);
        Hit h;
        st.c[ST_RAYS]++;
        if (!traverse(S, G, o, dir, 3.0e38f, false, depth, h, stack, stride, st)) return false;
        out = hit_vertex(S, G, h, o, dir);
        return true;
    }
    __device__ bool visible(const SlotDev& G, const Seg& sg) {
        Hit h;
        st.c[ST_RAYS]++;
        return !traverse(S, G, sg.o, sg.d, sg.t, true, depth, h, stack, stride, st);
    }
};

// ---------------------------------------------------------------------------
// Deferred visibility.  A shift appends its visibility segments to a queue
// (two float4 per ray: origin and length, direction and owner); a separate
// pass traces them (persistent lanes, or one ray per lane in small scenes)
// and zeroes kill[owner] when one is blocked.  The queue is split into kRaySubQueues parts, each with its own
// counter on its own cache line, chosen by block index: appends take one
// atomic per wave on one of 64 addresses (atomics on a single address
// serialize in L2).  Within a wave's allocation, segment e of every lane is
// stored contiguously, so a wave of the visibility pass traces rays of one
// kind from neighbouring shifts.
// ---------------------------------------------------------------------------
constexpr int kRaySubQueues = 64;
constexpr int kCounterStride = 32;   // u32 words between counters (128 B)

struct RayQueue {
    float4* buf;        // [kRaySubQueues][sub_cap] rays, 2 float4 each
    uint32_t* count;    // count[s * kCounterStride]: rays in sub-queue s
    uint32_t sub_cap;

    // slots for this lane's n segments: slot of segment e = out + e-major offset
    __device__ bool alloc(uint32_t n, uint32_t slot[4]) const {
        const int lane = (int)__lane_id();
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        uint32_t off = 0, rank[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint64_t m = __ballot(n > (uint32_t)e);
            rank[e] = off + (uint32_t)__popcll(m & lt);
            off += (uint32_t)__popcll(m);
        }
        const uint64_t act = __ballot(1);
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t sub = blockIdx.x % kRaySubQueues;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(count + sub * kCounterStride, off);
        base = __shfl(base, leader, 64);
        bool fits = base + off <= sub_cap;
#pragma unroll
        for (int e = 0; e < 4; ++e) slot[e] = sub * sub_cap + base + rank[e];
        return fits;
    }
    __device__ void put(uint32_t i, const Seg& sg, uint32_t owner) const {
        buf[2 * (size_t)i] = make_float4(sg.o.x, sg.o.y, sg.o.z, sg.t);
        buf[2 * (size_t)i + 1] = make_float4(sg.d.x, sg.d.y, sg.d.z, __uint_as_float(owner));
    }
};

// Any-hit tracing of queued segments by one wave with persistent lanes (Aila
// and Laine 2009, "dynamic fetch"): the wave owns the chunks c0, c0 + cstep,
// c0 + 2 cstep, ... of `chunk` rays each of a sub-queue of n rays, and a lane
// whose ray is finished takes the next ray of those chunks before the next
// traversal phase, so that the wave does not idle behind its longest ray.
// Chunks dealt round robin spread costly regions of the queue over many
// waves.  Rays go to lanes in queue order; a blocked segment zeroes
// kill[owner].
// The traversal is the any-hit case of traverse(): the same 64-byte nodes,
// postponed leaves and stack discipline, and the same triangle and sphere
// tests, so each segment's result does not depend on which lane traces it or
// in which order.  Every phase moves each active lane by at least one node
// or leaf, a ray's node visits are bounded by its budget, and the wave
// leaves once its range is taken and every lane is idle.
__device__ inline void trace_vis_chunks(const SceneDev& S, const SlotDev& G, const float4* __restrict__ buf,
                                        uint32_t n, uint32_t c0, uint32_t cstep, uint32_t chunk,
                                        float* __restrict__ kill, uint32_t* stack, int stride, int depth,
                                        Counters& st) {
    constexpr uint32_t kDone = 0xFFFFFFFFu;
    const int T = G.n_tri;
    const int lane = (int)__lane_id();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // wave-uniform: next ray and end of the current chunk
    uint64_t c = c0;
    uint32_t cursor = (uint32_t)min((uint64_t)n, c * chunk);
    uint32_t end = (uint32_t)min((uint64_t)n, c * chunk + chunk);
    bool have = false;         // this lane traces a ray
    RayPre r;
    r.o = r.d = r.inv = mk(0.f, 0.f, 0.f);
    r.kx = r.ky = r.kz = 0;
    r.sx = r.sy = r.sz = 0.f;
    float tmax = 0.f;
    uint32_t owner = 0;
    int sp = 0, budget = 0;
    uint32_t node = kDone, pmask = 0;
    int4 pcc = make_int4(0, 0, 0, 0);
    auto blocked = [&]() {
        const float old = atomicExch(kill + (owner & ~kOwnerNewton), 0.f);
        if (old != 0.f) {
            st.c[ST_VISFAIL]++;
            if (owner & kOwnerNewton) st.c[ST_VISFAIL_NEWTON]++;
        }
    };
    auto push = [&](uint32_t n) {
        if (sp < depth) {
            stack[sp * stride] = n;
            ++sp;
        } else {
            st.c[ST_OVERFLOW]++;
        }
    };
    auto pop = [&]() -> uint32_t {
        if (sp == 0) return kDone;
        --sp;
        return stack[sp * stride];
    };
    while (true) {
        // refill: idle lanes take the next rays of the wave's chunks in lane
        // order, across the end of a chunk into the next one
        const uint64_t idle = __ballot(!have);
        if (idle && cursor < end) {
            const uint32_t rank = (uint32_t)__popcll(idle & lt), tot = (uint32_t)__popcll(idle);
            const uint32_t rem = end - cursor;
            const uint64_t cn = c + cstep;   // the next chunk
            const uint32_t nb = (uint32_t)min((uint64_t)n, cn * chunk), ne = (uint32_t)min((uint64_t)n, cn * chunk + chunk);
            const uint32_t i = rank < rem ? cursor + rank : nb + (rank - rem);
            const bool take = rank < rem || i < ne;
            if (tot < rem) {
                cursor += tot;
            } else {   // this chunk is taken: go on in the next (empty when past the queue)
                c = cn;
                cursor = min(ne, nb + (tot - rem));
                end = ne;
            }
            if (!have && take) {
                const float4 r0 = buf[2 * (size_t)i], r1 = buf[2 * (size_t)i + 1];
                st.c[ST_RAYS]++;
                r = ray_pre(mk(r0.x, r0.y, r0.z), mk(r1.x, r1.y, r1.z));
                tmax = r0.w;
                owner = __float_as_uint(r1.w);
                // analytic spheres first (any hit: the order of tests is free)
                bool hit = false;
                for (int q = 0; q < S.n_sph && !hit; ++q) {
                    const int ob = S.sphere_ids[q];
                    const Obj& O = S.objs[ob];
                    float t;
                    hit = isect_sphere(r.o, r.d, xf_point(G.xf + 12 * ob, mk(O.cx, O.cy, O.cz)), O.r, tmax, t);
                }
                if (hit) {
                    blocked();
                } else if (T > 0) {
                    have = true;
                    sp = 0;
                    node = 0;
                    pmask = 0;
                    budget = 2 * G.n_nodes + 64;
                }
            }
        }
        if (cursor >= end && c * chunk < n) {   // an exhausted chunk: on to the next one
            c += cstep;
            cursor = (uint32_t)min((uint64_t)n, c * chunk);
            end = (uint32_t)min((uint64_t)n, c * chunk + chunk);
        }
        if (!__any(have)) {
            if (cursor >= end) break;
            continue;
        }
        if (!have) continue;
        // inner nodes until every active lane has a pending leaf or is done
        while (node < 0x80000000u && (pmask == 0 || sp + 4 <= depth)) {
            if (--budget <= 0 || node >= (uint32_t)G.n_nodes) {   // never for a well-formed tree
                st.c[ST_OVERFLOW]++;
                node = kDone;
                sp = 0;
                break;
            }
            const NodeQ* nq = G.nodes + node;
            const float4 org = nq->org;
            const uint4 q0 = nq->q0, q1 = nq->q1;
            const int4 cc = nq->child;
            const int nc = (int)q1.w;
            const float sx = __int_as_float((int)((q1.z & 0xFFu) << 23));
            const float sy = __int_as_float((int)(((q1.z >> 8) & 0xFFu) << 23));
            const float sz = __int_as_float((int)(((q1.z >> 16) & 0xFFu) << 23));
            auto deq = [](uint32_t w, float o, float sc) {
                return make_float4(fmaf((float)(w & 0xFFu), sc, o), fmaf((float)((w >> 8) & 0xFFu), sc, o),
                                   fmaf((float)((w >> 16) & 0xFFu), sc, o), fmaf((float)(w >> 24), sc, o));
            };
            const float4 lx = deq(q0.x, org.x, sx), hx = deq(q0.y, org.x, sx);
            const float4 ly = deq(q0.z, org.y, sy), hy = deq(q0.w, org.y, sy);
            const float4 lz = deq(q1.x, org.z, sz), hz = deq(q1.y, org.z, sz);
            st.c[ST_NODES]++;
            float t0, t1, t2, t3;
            const bool h0 = slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, r, tmax, t0);
            const bool h1 = slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, r, tmax, t1) && nc > 1;
            const bool h2 = slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, r, tmax, t2) && nc > 2;
            const bool h3 = slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, r, tmax, t3) && nc > 3;
            const bool f0 = cc.x < 0, f1 = cc.y < 0, f2 = cc.z < 0, f3 = cc.w < 0;
            const uint32_t leaves = (h0 && f0 ? 1u : 0u) | (h1 && f1 ? 2u : 0u) | (h2 && f2 ? 4u : 0u) |
                                    (h3 && f3 ? 8u : 0u);
            if (leaves) {
                if (pmask == 0) {
                    pmask = leaves;
                    pcc = cc;
                } else {
                    if (leaves & 1u) push((uint32_t)cc.x);
                    if (leaves & 2u) push((uint32_t)cc.y);
                    if (leaves & 4u) push((uint32_t)cc.z);
                    if (leaves & 8u) push((uint32_t)cc.w);
                }
            }
            constexpr float kInfT = 3.0e38f;
            float k0 = (h0 && !f0) ? t0 : kInfT, k1 = (h1 && !f1) ? t1 : kInfT;
            float k2 = (h2 && !f2) ? t2 : kInfT, k3 = (h3 && !f3) ? t3 : kInfT;
            int n0 = cc.x, n1 = cc.y, n2 = cc.z, n3 = cc.w;
            auto cswap = [](float& ka, int& na, float& kb, int& nb) {
                if (kb < ka) {
                    const float kt = ka;
                    ka = kb;
                    kb = kt;
                    const int nt = na;
                    na = nb;
                    nb = nt;
                }
            };
            // only the nearest child to the front
            cswap(k0, n0, k1, n1);
            cswap(k2, n2, k3, n3);
            cswap(k0, n0, k2, n2);
            if (k0 < kInfT) {
                if (k3 < kInfT) push((uint32_t)n3);
                if (k2 < kInfT) push((uint32_t)n2);
                if (k1 < kInfT) push((uint32_t)n1);
                node = (uint32_t)n0;
            } else {
                node = pop();
            }
            if (node != kDone && node >= 0x80000000u && pmask == 0) {
                pmask = 1u;
                pcc.x = (int)node;
                node = pop();
            }
            if (__all(pmask != 0)) break;
        }
        // leaf phase: the pending leaves, then leaves met on the stack while
        // no inner node is next
        bool hit = false;
        while (pmask && !hit) {
            const int j = __ffs(pmask) - 1;
            pmask &= pmask - 1;
            const uint32_t c = (uint32_t)(j == 0 ? pcc.x : (j == 1 ? pcc.y : (j == 2 ? pcc.z : pcc.w)));
            const int first = (int)(c & 0x0FFFFFFFu), cnt = (int)((c >> 28) & 7u) + 1;
            for (int k = first; k < first + cnt; ++k) {
                if ((unsigned)k >= (unsigned)T) {   // never for a well-formed tree
                    st.c[ST_OVERFLOW]++;
                    break;
                }
                st.c[ST_TRIS]++;
                const float4 a = G.leaves[3 * k], b = G.leaves[3 * k + 1], cv = G.leaves[3 * k + 2];
                float t, b1, b2;
                if (isect_tri(r.o, r.d, r.kx, r.ky, r.kz, r.sx, r.sy, r.sz, mk(a.x, a.y, a.z), mk(b.x, b.y, b.z),
                              mk(cv.x, cv.y, cv.z), tmax, t, b1, b2)) {
                    hit = true;
                    break;
                }
            }
            if (!hit && pmask == 0 && node != kDone && node >= 0x80000000u) {
                pmask = 1u;
                pcc.x = (int)node;
                node = pop();
            }
        }
        if (hit) {
            blocked();
            have = false;
            pmask = 0;
            node = kDone;
        } else if (node == kDone && pmask == 0) {
            have = false;
        }
    }
}

// A list of u32 work indices in kRaySubQueues sub-lists (same scheme as the
// ray queue): alloc(n) gives this lane n consecutive slots.
struct IdxQueue {
    uint32_t* buf;      // [kRaySubQueues][sub_cap]
    uint32_t* count;    // count[s * kCounterStride]
    uint32_t sub_cap;

    __device__ bool alloc(uint32_t n, uint32_t& first) const {
        const int lane = (int)__lane_id();
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {   // n < 16
            const uint64_t m = __ballot((n >> b) & 1u);
            pre += (uint32_t)__popcll(m & lt) << b;
            tot += (uint32_t)__popcll(m) << b;
        }
        const uint64_t act = __ballot(1);
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t sub = blockIdx.x % kRaySubQueues;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(count + sub * kCounterStride, tot);
        base = __shfl(base, leader, 64);
        first = sub * sub_cap + base + pre;
        return base + tot <= sub_cap;
    }
};

// ---------------------------------------------------------------------------
// BSDFs: Lambert, GGX (Walter et al. 2007; separable Smith G; Schlick F)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_rough(const SceneDev& S, int obj) {
    const Mat& m = S.mats[S.objs[obj].material];
    return m.type == 0 || m.alpha >= 0.2f;
}
__device__ __forceinline__ void onb(V3 n, V3& t, V3& b) {   // Duff et al., JCGT 2017
    float sg = copysignf(1.0f, n.z);
    float a = -1.0f / (sg + n.z);
    float bb = n.x * n.y * a;
    t = mk(1.0f + sg * n.x * n.x * a, sg * bb, -sg * n.x);
    b = mk(bb, sg + n.y * n.y * a, -n.y);
}
// GGX normal distribution written with sin^2 of the half-vector angle:
// D = a^2 / (pi (sin^2 + a^2 cos^2)^2), the same function as
// a^2 / (pi (cos^2 (a^2 - 1) + 1)^2) without the cancellation of
// 1 - cos^2 near the lobe peak at small roughness.
__device__ __forceinline__ float ggx_d_sc(float alpha, float sh2, float ch2) {
    float a2 = alpha * alpha;
    float den = sh2 + a2 * ch2;
    return a2 / (kPi * den * den);
}
__device__ __forceinline__ float ggx_g1(float alpha, float c) {
    float a2 = alpha * alpha;
    return 2.0f * c / (c + sqrtf(a2 + (1.0f - a2) * c * c));
}
__device__ inline float bsdf_eval(const SceneDev& S, int obj, V3 n, V3 wi, V3 wo) {
    float ci = dot(n, wi), co = dot(n, wo);
    if (ci * co <= 0.f) return 0.f;
    const Mat m = S.mats[S.objs[obj].material];
    if (m.type == 0) return m.albedo / kPi;
    V3 ns = ci > 0.f ? n : -n;
    ci = fabsf(ci);
    co = fabsf(co);
    V3 h = nrm(wi + wo);
    float ch = dot(ns, h);
    V3 xh = cross(ns, h);
    float D = ggx_d_sc(m.alpha, dot(xh, xh), ch * ch);
    float G = ggx_g1(m.alpha, ci) * ggx_g1(m.alpha, co);
    float x = 1.0f - dot(wi, h);
    float x2 = x * x;
    float F = m.f0 + (1.0f - m.f0) * (x2 * x2 * x);
    return D * G * F / (4.0f * ci * co);
}
__device__ inline bool bsdf_sample(const SceneDev& S, int obj, V3 n, V3 wi, float u1, float u2, V3& wo, float& pdf) {
    float ci = dot(n, wi);
    if (ci == 0.f) return false;
    V3 ns = ci > 0.f ? n : -n;
    V3 t, b;
    onb(ns, t, b);
    const Mat m = S.mats[S.objs[obj].material];
    if (m.type == 0) {
        float r = sqrtf(u1), ph = 2.0f * kPi * u2;
        float z = sqrtf(fmaxf(0.f, 1.0f - u1));
        float sp, cp;
        sincosf(ph, &sp, &cp);
        wo = nrm(r * cp * t + r * sp * b + z * ns);
        pdf = dot(ns, wo) / kPi;
        return pdf > 0.f;
    }
    float a2 = m.alpha * m.alpha;
    float t2 = a2 * u1 / (1.0f - u1);
    float ch = 1.0f / sqrtf(1.0f + t2);
    float sh = sqrtf(t2) * ch;   // sin = tan cos, without the cancellation of 1 - cos^2
    float ph = 2.0f * kPi * u2;
    float sp, cp;
    sincosf(ph, &sp, &cp);
    V3 h = sh * cp * t + sh * sp * b + ch * ns;
    float wh = dot(wi, h);
    wo = nrm(2.0f * wh * h - wi);
    if (dot(ns, wo) <= 0.f) return false;
    // sin^2 = t2 cos^2 for the sampled half vector (tan^2 = t2)
    pdf = ggx_d_sc(m.alpha, t2 * ch * ch, ch * ch) * ch / (4.0f * fabsf(wh));
    return pdf > 0.f;
}

// ---------------------------------------------------------------------------
// time planes: bins [t0 + b w, t0 + (b+1) w) and the gate (plane n_bins)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float plane_lo(const Sens& s, int pl) {
    return pl < s.n_bins ? s.t0 + (float)pl * s.bw : s.gate_c - 0.5f * s.gate_w;
}
__device__ __forceinline__ float plane_hi(const Sens& s, int pl) {
    return pl < s.n_bins ? s.t0 + (float)(pl + 1) * s.bw : s.gate_c + 0.5f * s.gate_w;
}
// plane n_bins + 1 stands for the wide gate of the shrink mapping (shrink_k
// times the gate, same centre), the domain of the wide-gate samples
__device__ __forceinline__ float plane_width(const Sens& s, int pl) {
    return pl < s.n_bins ? s.bw : (pl == s.n_bins + 1 ? s.shrink_k * s.gate_w : s.gate_w);
}
// the wide gate of the shrink mapping: shrink_k times the gate, same centre
__device__ __forceinline__ bool in_rough_gate(const Sens& s, float l) {
    const float h = 0.5f * s.shrink_k * s.gate_w;
    return l >= s.gate_c - h && l < s.gate_c + h;
}
__device__ __forceinline__ bool in_plane(const Sens& s, int pl, float l) {
    return l >= plane_lo(s, pl) && l < plane_hi(s, pl);
}
// the same, with the gate plane of the frame held in slot G
__device__ __forceinline__ bool in_plane_at(const Sens& s, const SlotDev& G, int pl, float l) {
    if (pl < s.n_bins) return in_plane(s, pl, l);
    const float h = pl == s.n_bins + 1 ? 0.5f * s.shrink_k * s.gate_w : 0.5f * s.gate_w;
    return l >= G.gate_c - h && l < G.gate_c + h;
}
// Delta l of a temporal shift from the previous frame into the current one
// (Sec. 4.1, time-gate shifting): the gate's move; bins do not move
__device__ __forceinline__ float gate_shift(const Sens& s, const SlotDev& cur, const SlotDev& prev, int pl) {
    return pl < s.n_bins ? 0.f : cur.gate_c - prev.gate_c;
}
__device__ __forceinline__ int bin_of(const Sens& s, float l) {
    if (s.n_bins <= 0) return -1;
    float f = floorf((l - s.t0) / s.bw);
    if (!(f > -2.0f && f < (float)s.n_bins + 1.0f)) return -1;
    int b = (int)f;
    if (b >= 0 && b < s.n_bins && l < plane_lo(s, b)) b -= 1;
    if (b >= -1 && b + 1 < s.n_bins && b + 1 >= 0 && l >= plane_lo(s, b + 1)) b += 1;
    if (b < 0 || b >= s.n_bins || !in_plane(s, b, l)) return -1;
    return b;
}

// ---------------------------------------------------------------------------
// domains: a pixel of the current (slot 0) or previous (slot 1) frame
// ---------------------------------------------------------------------------
struct Frames {
    SlotDev g[2];
};

__device__ __forceinline__ uint64_t full_pixel(const Sens& s, int pix) {
    int x = pix % s.W, y = pix / s.W;
    return (uint64_t)(s.cy0 + y) * (uint64_t)s.FW + (uint64_t)(s.cx0 + x);
}
__device__ __forceinline__ V3 toward_camera(const Sens& s, const SlotDev& G, const Vtx& y1) {
    if (s.cam_model == 0) return nrm(G.cam_pos - y1.p);
    return -G.cam_fwd;
}
// ---------------------------------------------------------------------------
// Path velocity (Sec. 4.6, eq. optical_path_velocity, refractive index 1):
// u = -dl/dt = sum over segments of (v_from - v_to) . w, w the segment's unit
// vector.  A point p of object o moves rigidly at v_o + w_o x (p - t_o), t_o
// the translation of the object's transform.
// ---------------------------------------------------------------------------
__device__ __forceinline__ V3 vel_at(const SlotDev& G, int obj, V3 p) {
    if (obj < 0) return mk(0.f, 0.f, 0.f);
    const float* q = G.vel + 6 * obj;
    const float* m = G.xf + 12 * obj;
    return mk(q[0], q[1], q[2]) + cross(mk(q[3], q[4], q[5]), p - mk(m[3], m[7], m[11]));
}
// the term of the segment from (pa, va) to (pb, vb)
__device__ __forceinline__ float seg_u(V3 pa, V3 va, V3 pb, V3 vb) {
    const V3 d = pb - pa;
    return dot(va - vb, (1.0f / len(d)) * d);
}
// the plane quantity of the camera leg: its length (to the image plane for
// the orthographic camera), or its term of u
template <bool VEL>
__device__ __forceinline__ float camera_leg(const Sens& s, const SlotDev& G, const Vtx& y1) {
    if (!s.count_leg) return 0.f;
    if (VEL) {
        const V3 dir = s.cam_model == 0 ? nrm(y1.p - G.cam_pos) : G.cam_fwd;
        return dot(G.cam_vel - vel_at(G, y1.obj, y1.p), dir);
    }
    if (s.cam_model == 0) return len(y1.p - G.cam_pos);
    return dot(y1.p - G.cam_pos, G.cam_fwd);
}
// delta lights (Sec. 5): isotropic point, or the confocal laser spot at the
// domain's primary hit re-emitting with the wall's Lambertian BRDF
__device__ __forceinline__ V3 light_pos(const Sens& s, const SlotDev& G, int pix) {
    if (s.light_model == 0) return G.light_pos;
    float4 p = G.gb_p[pix];
    return mk(p.x, p.y, p.z);
}
__device__ __forceinline__ V3 light_vel(const Sens& s, const SlotDev& G, int pix) {
    if (s.light_model == 0) return G.light_vel;
    float4 p = G.gb_p[pix];
    return vel_at(G, G.gb_obj[pix], mk(p.x, p.y, p.z));
}
__device__ __forceinline__ float light_emit(const Sens& s, const SceneDev& S, const SlotDev& G, int pix, V3 x) {
    if (s.light_model == 0) return s.light_I;
    Vtx g = gbuf_vertex(G, pix);
    V3 w = nrm(x - g.p);
    float cw = dot(g.n, w), cs = dot(g.n, -G.cam_fwd);
    if (cw * cs <= 0.f) return 0.f;
    const Mat& m = S.mats[S.objs[g.obj].material];
    return s.light_I * m.albedo / kPi * fabsf(cw);
}
__device__ __forceinline__ Seg seg_light(const Sens& s, const SceneDev& S, const SlotDev& G, int pix, const Vtx& x) {
    if (s.light_model == 0) return seg_point(S, x, G.light_pos);
    return seg_pts(S, x, gbuf_vertex(G, pix));
}

__device__ __forceinline__ bool recon_ok(const SceneDev& S, const Vtx& a, const Vtx& b) {
    return is_rough(S, a.obj) && is_rough(S, b.obj) && len(b.p - a.p) >= S.dmin;
}

// ---------------------------------------------------------------------------
// Newton solve of the path-length constraint (Sec. 4.3), average-gradient
// gauge.  Length functions use the source endpoints at xi and the
// destination endpoints at xi'; dF2/dxi' is the derivative of F2 itself.
// The length function and its derivatives are evaluated in NReal (FP32 by
// default); the 2x2 Newton step and both determinants are solved in FP64.
// ---------------------------------------------------------------------------
#ifndef TOF_NEWTON_FP64
#define TOF_NEWTON_FP64 0
#endif
#if TOF_NEWTON_FP64
typedef double NReal;
#else
typedef float NReal;
#endif

template <typename T>
struct T3 {
    T x, y, z;
};
template <typename T>
__device__ __forceinline__ T3<T> operator+(T3<T> a, T3<T> b) { return T3<T>{a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ __forceinline__ T3<T> operator-(T3<T> a, T3<T> b) { return T3<T>{a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __forceinline__ T3<T> operator*(T s, T3<T> a) { return T3<T>{s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ __forceinline__ T tdot(T3<T> a, T3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ T3<T> tcross(T3<T> a, T3<T> b) {
    return T3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ T tlen(T3<T> a) { return sqrt(tdot(a, a)); }
template <typename T>
__device__ __forceinline__ T3<T> tof3(V3 a) { return T3<T>{(T)a.x, (T)a.y, (T)a.z}; }
template <typename T>
__device__ __forceinline__ T3<T> tld(const float4* a, int i) {
    float4 v = a[i];
    return T3<T>{(T)v.x, (T)v.y, (T)v.z};
}
template <typename T>
__device__ __forceinline__ T3<T> txf(const float* m, T3<T> q, T w) {
    return T3<T>{(T)m[0] * q.x + (T)m[1] * q.y + (T)m[2] * q.z + w * (T)m[3],
                 (T)m[4] * q.x + (T)m[5] * q.y + (T)m[6] * q.z + w * (T)m[7],
                 (T)m[8] * q.x + (T)m[9] * q.y + (T)m[10] * q.z + w * (T)m[11]};
}

template <typename T>
struct ChartT {
    bool ok;
    T3<T> p, ju, jv, puu, puv, pvv;
};

template <typename T>
__device__ inline ChartT<T> chart_eval_t(const SceneDev& S, const SlotDev& G, int obj, T u, T v) {
    ChartT<T> c;
    const Obj ob = S.objs[obj];
    T3<T> z = T3<T>{0, 0, 0};
    c.puu = z;
    c.puv = z;
    c.pvv = z;
    if (ob.type == 0) {
        T uu = u, vv = v;
        if (ob.wrap_u) uu = u - (T)ob.nu * floor(u / (T)ob.nu);
        if (ob.wrap_v) vv = v - (T)ob.nv * floor(v / (T)ob.nv);
        T fi = floor(uu), fj = floor(vv);
        int i = (int)fmin(fmax(fi, (T)0), (T)(ob.nu - 1));
        int j = (int)fmin(fmax(fj, (T)0), (T)(ob.nv - 1));
        T a = uu - (T)i, b = vv - (T)j;
        int row = ob.nu + 1;
        int base = ob.voff + j * row + i;
        const float* m = G.xf + 12 * obj;
        const T3<T> org = T3<T>{(T)m[3], (T)m[7], (T)m[11]};
        if (a + b <= (T)1) {
            const T3<T> r0 = tld<T>(G.wr, base), ru = tld<T>(G.wr, base + 1), rv = tld<T>(G.wr, base + row);
            c.ju = ru - r0;
            c.jv = rv - r0;
            c.p = org + (r0 + a * c.ju + b * c.jv);
        } else {
            const T3<T> r0 = tld<T>(G.wr, base + row + 1), ru = tld<T>(G.wr, base + row), rv = tld<T>(G.wr, base + 1);
            c.ju = r0 - ru;
            c.jv = r0 - rv;
            c.p = org + (r0 - ((T)1 - a) * c.ju - ((T)1 - b) * c.jv);
        }
        c.ok = tlen(tcross(c.ju, c.jv)) > (T)0;
    } else {
        const float* m = G.xf + 12 * obj;
        T th = u, ph = v, r = (T)ob.r;
        T st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
        T3<T> radial = T3<T>{st * cp, st * sp, ct};
        c.p = txf(m, T3<T>{(T)ob.cx, (T)ob.cy, (T)ob.cz} + r * radial, (T)1);
        c.ju = txf(m, T3<T>{r * ct * cp, r * ct * sp, -r * st}, (T)0);
        c.jv = txf(m, T3<T>{-r * st * sp, r * st * cp, (T)0}, (T)0);
        c.puu = txf(m, (-r) * radial, (T)0);
        c.puv = txf(m, T3<T>{-r * ct * sp, r * ct * cp, (T)0}, (T)0);
        c.pvv = txf(m, T3<T>{-r * st * cp, -r * st * sp, (T)0}, (T)0);
        c.ok = true;
    }
    return c;
}

template <typename T>
struct LenEvalT {
    bool ok;
    T L, g0, g1, h00, h01, h11;
};

// l(xi) = c + |a - p(xi)| + |b - p(xi)|, its chart gradient J^T(-s) and
// Hessian J^T A J + Q with A = sum (I - d d^T)/|p_i - p|, Q_ij = (-s).p_ij
template <typename T>
__device__ __forceinline__ LenEvalT<T> len_eval_t(const SceneDev& S, const SlotDev& G, int obj, T u, T v, T3<T> a, T3<T> b,
                                         T c) {
    LenEvalT<T> e;
    e.ok = false;
    ChartT<T> ch = chart_eval_t<T>(S, G, obj, u, v);
    if (!ch.ok) return e;
    T3<T> r1 = a - ch.p, r2 = b - ch.p;
    T l1 = tlen(r1), l2 = tlen(r2);
    if (!(l1 > (T)0 && l2 > (T)0)) return e;
    T i1 = (T)1 / l1, i2 = (T)1 / l2;
    T3<T> d1 = i1 * r1, d2 = i2 * r2;
    T3<T> sv = d1 + d2;
    e.L = c + l1 + l2;
    e.g0 = -tdot(sv, ch.ju);
    e.g1 = -tdot(sv, ch.jv);
    T3<T> Aju = i1 * (ch.ju - tdot(d1, ch.ju) * d1) + i2 * (ch.ju - tdot(d2, ch.ju) * d2);
    T3<T> Ajv = i1 * (ch.jv - tdot(d1, ch.jv) * d1) + i2 * (ch.jv - tdot(d2, ch.jv) * d2);
    e.h00 = tdot(ch.ju, Aju) - tdot(sv, ch.puu);
    e.h01 = tdot(ch.ju, Ajv) - tdot(sv, ch.puv);
    e.h11 = tdot(ch.jv, Ajv) - tdot(sv, ch.pvv);
    e.ok = true;
    return e;
}

template <typename T>
__device__ __forceinline__ T seg_u_t(T3<T> pa, T3<T> va, T3<T> pb, T3<T> vb) {
    const T3<T> d = pb - pa;
    return tdot(va - vb, ((T)1 / tlen(d)) * d);
}

// The path-velocity counterpart of len_eval_t (Sec. 4.6): U(xi) = c +
// phi_a(p) + phi_b(p) with phi_a(p) = (v_a - v(p)) . d, d = (p - a) / |p - a|
// (a segment's term does not depend on its direction) and v(p) = V + W x
// (p - t) the object's rigid motion.  With l = |p - a|, w = v_a - v(p) and
// P = I - d d^T:
//   grad phi_a = W x d + P w / l
//   Hess phi_a x = (d (d.(W x x)) - (d.x)(W x d)) / l
//                  - ((d.w) P x + d (P w . x) + P w (d.x)) / l^2
// (derived from the definition; the supplement that holds the paper's own
// derivation is not available), and in the chart g = J^T grad,
// H = J^T Hess J + grad . p_ij.
template <typename T>
__device__ __forceinline__ LenEvalT<T> vel_eval_t(const SceneDev& S, const SlotDev& G, int obj, T u, T v, T3<T> a,
                                                  T3<T> va, T3<T> b, T3<T> vb, T c) {
    LenEvalT<T> e;
    e.ok = false;
    ChartT<T> ch = chart_eval_t<T>(S, G, obj, u, v);
    if (!ch.ok) return e;
    const float* q = G.vel + 6 * obj;
    const float* m = G.xf + 12 * obj;
    const T3<T> W = T3<T>{(T)q[3], (T)q[4], (T)q[5]};
    const T3<T> vp = T3<T>{(T)q[0], (T)q[1], (T)q[2]} + tcross(W, ch.p - T3<T>{(T)m[3], (T)m[7], (T)m[11]});
    const T3<T> z = T3<T>{0, 0, 0};
    T val = c;
    T3<T> grad = z, Hju = z, Hjv = z;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const T3<T> ep = side ? b : a, ev = side ? vb : va;
        const T3<T> r = ch.p - ep;
        const T l = tlen(r);
        if (!(l > (T)0)) return e;
        const T il = (T)1 / l;
        const T3<T> d = il * r;
        const T3<T> w = ev - vp;
        const T dw = tdot(d, w);
        const T3<T> Pw = w - dw * d;
        const T3<T> Wd = tcross(W, d);
        val = val + dw;
        grad = grad + Wd + il * Pw;
        const T3<T> xs[2] = {ch.ju, ch.jv};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const T3<T> x = xs[k];
            const T dx = tdot(d, x);
            const T3<T> t1 = il * (tdot(d, tcross(W, x)) * d - dx * Wd);
            const T3<T> t2 = dw * (x - dx * d) + tdot(Pw, x) * d + dx * Pw;
            const T3<T> hx = t1 - (il * il) * t2;
            if (k == 0) Hju = Hju + hx;
            else Hjv = Hjv + hx;
        }
    }
    e.L = val;
    e.g0 = tdot(grad, ch.ju);
    e.g1 = tdot(grad, ch.jv);
    e.h00 = tdot(ch.ju, Hju) + tdot(grad, ch.puu);
    e.h01 = tdot(ch.ju, Hjv) + tdot(grad, ch.puv);
    e.h11 = tdot(ch.jv, Hjv) + tdot(grad, ch.pvv);
    e.ok = true;
    return e;
}

// the constraint function of the plane quantity (length or velocity)
template <typename T, bool VEL>
__device__ __forceinline__ LenEvalT<T> con_eval_t(const SceneDev& S, const SlotDev& G, int obj, T u, T v, T3<T> a,
                                                  T3<T> va, T3<T> b, T3<T> vb, T c) {
    if (VEL) return vel_eval_t<T>(S, G, obj, u, v, a, va, b, vb, c);
    return len_eval_t<T>(S, G, obj, u, v, a, b, c);
}

struct NewtonOut {
    bool conv;
    float xi0, xi1;
    int iters;
    double det_area;
};

// Endpoints a, b carry velocities va, vb (read in the velocity domain only).
// JAC = false: the caller needs only the solution (the round trip of a
// shift); the implicit-function Jacobian's area factor is not formed (the
// determinant of dF/dxi' is still tested, as part of convergence).
template <typename T, bool VEL, bool JAC = true>
__device__ inline NewtonOut newton_solve(const SceneDev& S, const SlotDev& GS, const SlotDev& GD, int obj, T xs0,
                                         T xs1, T3<T> as, T3<T> vas, T3<T> bs, T3<T> vbs, T cs, T3<T> ad, T3<T> vad,
                                         T3<T> bd, T3<T> vbd, T cd, T dl0, T tol, int maxit) {
    NewtonOut out;
    out.conv = false;
    out.iters = 0;
    const LenEvalT<T> Sv = con_eval_t<T, VEL>(S, GS, obj, xs0, xs1, as, vas, bs, vbs, cs);
    if (!Sv.ok) return out;
    T xp0 = xs0, xp1 = xs1;
    LenEvalT<T> D = con_eval_t<T, VEL>(S, GD, obj, xp0, xp1, ad, vad, bd, vbd, cd);
    if (!D.ok) return out;
    // F = [L_dst(xi') - L_src(xi) - dl ; (R m)^T (xi' - xi)], R = 90 degree rotation
    T F0 = D.L - Sv.L - dl0;
    T F1 = (T)0;
    int it = 0;
    while (true) {
        if (fabs(F0) <= tol && fabs(F1) <= tol) break;
        if (it >= maxit) return out;
        const T m0 = (T)0.5 * (Sv.g0 + D.g0), m1 = (T)0.5 * (Sv.g1 + D.g1);
        const T rd0 = -(xp1 - xs1), rd1 = xp0 - xs0;
        // dF/dxi' = [grad L_dst ; (R m - 0.5 H_dst R d)^T], solved in FP64
        const double J00 = D.g0, J01 = D.g1;
        const double J10 = (double)(-m1 - (T)0.5 * (D.h00 * rd0 + D.h01 * rd1));
        const double J11 = (double)(m0 - (T)0.5 * (D.h01 * rd0 + D.h11 * rd1));
        const double det = J00 * J11 - J01 * J10;
        if (fabs(det) < 1e-12) return out;
        const double s0 = -(J11 * (double)F0 - J01 * (double)F1) / det;
        const double s1 = -(-J10 * (double)F0 + J00 * (double)F1) / det;
        const T norm0 = sqrt(F0 * F0 + F1 * F1);
        bool accepted = false;
        T alpha = (T)1;
        for (int ls = 0; ls < 4; ++ls, alpha *= (T)0.5) {   // backtracking line search
            const T x0 = xp0 + alpha * (T)s0, x1 = xp1 + alpha * (T)s1;
            const LenEvalT<T> Dt = con_eval_t<T, VEL>(S, GD, obj, x0, x1, ad, vad, bd, vbd, cd);
            if (!Dt.ok) continue;
            const T n0 = (T)0.5 * (Sv.g0 + Dt.g0), n1 = (T)0.5 * (Sv.g1 + Dt.g1);
            const T G0 = Dt.L - Sv.L - dl0;
            const T G1 = -n1 * (x0 - xs0) + n0 * (x1 - xs1);
            if (sqrt(G0 * G0 + G1 * G1) < norm0) {
                xp0 = x0;
                xp1 = x1;
                D = Dt;
                F0 = G0;
                F1 = G1;
                accepted = true;
                break;
            }
        }
        if (!accepted) return out;
        ++it;
    }
    // implicit-function Jacobian |det dxi'/dxi| = |det dF/dxi| / |det dF/dxi'|
    const T m0 = (T)0.5 * (Sv.g0 + D.g0), m1 = (T)0.5 * (Sv.g1 + D.g1);
    const T rd0 = -(xp1 - xs1), rd1 = xp0 - xs0;
    const double Jd00 = D.g0, Jd01 = D.g1;
    const double Jd10 = (double)(-m1 - (T)0.5 * (D.h00 * rd0 + D.h01 * rd1));
    const double Jd11 = (double)(m0 - (T)0.5 * (D.h01 * rd0 + D.h11 * rd1));
    const double Js00 = -(double)Sv.g0, Js01 = -(double)Sv.g1;
    const double Js10 = -(double)(-m1 + (T)0.5 * (Sv.h00 * rd0 + Sv.h01 * rd1));
    const double Js11 = -(double)(m0 + (T)0.5 * (Sv.h01 * rd0 + Sv.h11 * rd1));
    const double detd = Jd00 * Jd11 - Jd01 * Jd10;
    const double dets = Js00 * Js11 - Js01 * Js10;
    if (fabs(detd) < 1e-12) return out;
    out.conv = true;
    out.xi0 = (float)xp0;
    out.xi1 = (float)xp1;
    out.iters = it;
    out.det_area = 0.0;
    if (!JAC) return out;
    // chart -> surface: sqrt(det J'^T J') / sqrt(det J^T J)
    const ChartT<T> cd_ = chart_eval_t<T>(S, GD, obj, xp0, xp1);
    const ChartT<T> cs_ = chart_eval_t<T>(S, GS, obj, xs0, xs1);
    const double area = (double)tlen(tcross(cd_.ju, cd_.jv)) / (double)tlen(tcross(cs_.ju, cs_.jv));
    out.conv = true;
    out.xi0 = (float)xp0;
    out.xi1 = (float)xp1;
    out.iters = it;
    out.det_area = area * (fabs(dets) / fabs(detd));
    return out;
}

// ---------------------------------------------------------------------------
// shift T_{src -> dst} (Sec. 4.1): random replay up to x_{k-1}, reconnection
// at p, Newton perturbation of p, full Jacobian in the product solid-angle
// measure, target in the destination plane, then visibility of the moved
// edges (the suffix too when the domains belong to different frames).
// Returns only what changes in the record.
// ---------------------------------------------------------------------------
struct ShiftOut {
    bool ok;
    float J, phat, len, pre_pdf;
    VRef v0, v1;
};

__device__ __forceinline__ void apply_shift(Rec& y, const ShiftOut& r) {
    y.v[0] = r.v0;
    y.v[1] = r.v1;
    y.len = r.len;
    y.pre_pdf = r.pre_pdf;
    y.phat = r.phat;
}

// a stored record may only be shifted if every object it names exists and its
// vertex counts are in range (the shift dereferences them)
__device__ __forceinline__ bool rec_valid(const SceneDev& S, const Rec& x) {
    const unsigned no = (unsigned)S.n_obj;
    if (x.n < 1 || x.n > kMaxVerts) return false;
    if (x.k == 0) return true;
    if (x.k < 2 || x.k > x.n) return false;
    if ((unsigned)x.v[0].obj >= no || (unsigned)x.v[1].obj >= no) return false;
    if (x.v[2].obj != -1 && (unsigned)x.v[2].obj >= no) return false;
    if (x.nsfx != 0 && (x.nsfx != 1 || (unsigned)x.v[3].obj >= no)) return false;
    return true;
}

// The returned ok is provisional: the shift's visibility segments are queued
// under `owner` and a blocked one zeroes the owner's weight later.  VEL: the
// planes measure the path velocity and the perturbation keeps it (Sec. 4.6).
template <bool VEL>
__device__ __forceinline__ ShiftOut shift_path(const Sens& s, const SceneDev& S, const Frames& F, Tracer& tr, const Rec& x,
                                      int src_slot, int src_pix, int dst_slot, int dst_pix, int plane, float dl0,
                                      const RayQueue& q, uint32_t owner) {
    ShiftOut R;
    R.ok = false;
    Counters& st = tr.st;
    st.c[ST_SHIFTS]++;
    if (!rec_valid(S, x)) {
        st.c[ST_BADREC]++;
        return R;
    }
    const SlotDev& GS = F.g[src_slot];
    const SlotDev& GD = F.g[dst_slot];
    if (GD.gb_obj[dst_pix] < 0) return R;
    // replay in primary sample space, evaluating the prefix as we go
    Vtx cur = gbuf_vertex(GD, dst_pix);
    V3 wi_s = toward_camera(s, GD, cur);   // incoming direction for sampling
    V3 wi_e = wi_s;                        // incoming direction for evaluation (from positions)
    float plen = camera_leg<VEL>(s, GD, cur);
    NReal cpre = (NReal)plen;   // prefix length in the Newton precision
    V3 vc = VEL ? vel_at(GD, cur.obj, cur.p) : mk(0.f, 0.f, 0.f);   // velocity of cur
    float beta = 1.0f, pdf_y = 1.0f;
    const int nrep = (x.k == 0) ? x.n - 1 : x.k - 2;
    for (int i = 1; i <= nrep; ++i) {
        Draw u = philox(s.seed, x.opix, x.ofr, PASS_BSDF, (uint64_t)x.tree, (uint64_t)i);
        V3 wo;
        float pdf;
        if (!bsdf_sample(S, cur.obj, cur.n, wi_s, u.u(0), u.u(1), wo, pdf)) return R;
        Vtx nx;
        if (!tr.trace(GD, cur, wo, nx)) return R;
        // the offset path must not reconnect earlier than the base path
        if (recon_ok(S, cur, nx)) return R;
        V3 dv = nx.p - cur.p;
        float dl = len(dv);
        V3 we = (1.0f / dl) * dv;
        beta *= bsdf_eval(S, cur.obj, cur.n, wi_e, we) * fabsf(dot(cur.n, we));
        if (VEL) {
            const V3 vn = vel_at(GD, nx.obj, nx.p);
            const float du = dot(vc - vn, we);
            plen += du;
            cpre += (NReal)du;
            vc = vn;
        } else {
            plen += dl;
            cpre += tlen(tof3<NReal>(nx.p) - tof3<NReal>(cur.p));
        }
        pdf_y *= pdf;
        wi_s = -wo;
        wi_e = -we;
        cur = nx;
    }
    const bool replay_only = x.k == 0;
    const bool p2light = x.v[2].obj < 0;
    const int obj = x.v[1].obj;
    float C;
    double J = (double)x.pre_pdf / (double)pdf_y;
    Vtx pd, p2_d, sfx_d;
    if (replay_only) {   // pure random replay: NEE at y_n
        V3 L = light_pos(s, GD, dst_pix);
        V3 dv = L - cur.p;
        float dl = len(dv);
        V3 wo = (1.0f / dl) * dv;
        C = beta * (bsdf_eval(S, cur.obj, cur.n, wi_e, wo) * fabsf(dot(cur.n, wo)) *
                    light_emit(s, S, GD, dst_pix, cur.p) / (dl * dl));
        plen += VEL ? dot(vc - light_vel(s, GD, dst_pix), wo) : dl;
        R.v0 = x.v[0];
        R.v1 = x.v[1];
    } else {
        if (!is_rough(S, cur.obj)) return R;
        const Vtx xkm1_s = vertex_at(S, GS, x.v[0].obj, x.v[0].xi0, x.v[0].xi1);
        const Vtx p_s = vertex_at(S, GS, obj, x.v[1].xi0, x.v[1].xi1);
        Vtx p2_s;
        V3 p2s_pos, p2d_pos;
        if (p2light) {
            p2s_pos = light_pos(s, GS, src_pix);
            p2d_pos = light_pos(s, GD, dst_pix);
        } else {
            p2_s = vertex_at(S, GS, x.v[2].obj, x.v[2].xi0, x.v[2].xi1);
            p2_d = vertex_at(S, GD, x.v[2].obj, x.v[2].xi0, x.v[2].xi1);
            p2s_pos = p2_s.p;
            p2d_pos = p2_d.p;
        }
        if (x.nsfx > 0) sfx_d = vertex_at(S, GD, x.v[3].obj, x.v[3].xi0, x.v[3].xi1);
        // destination velocities of the fixed vertices after p (velocity domain)
        const V3 vp2d = !VEL ? mk(0.f, 0.f, 0.f) : (p2light ? light_vel(s, GD, dst_pix) : vel_at(GD, p2_d.obj, p2_d.p));
        const V3 vsfx = (VEL && x.nsfx > 0) ? vel_at(GD, sfx_d.obj, sfx_d.p) : mk(0.f, 0.f, 0.f);
        const V3 vlight = VEL ? light_vel(s, GD, dst_pix) : mk(0.f, 0.f, 0.f);
        float xi0 = x.v[1].xi0, xi1 = x.v[1].xi1;
        double det_area;
        if (s.shift_mode == 1) {
            st.c[ST_NEWTON_ATT]++;
            // fixed parts of the two length functions: prefix up to x_{k-1},
            // suffix after p2 (so that L_src(xi) reproduces the stored length)
            NReal c_dst = cpre;
            if (!p2light) {
                V3 prev = p2d_pos, vprev = vp2d;
                if (x.nsfx > 0) {
                    c_dst += VEL ? (NReal)seg_u(prev, vprev, sfx_d.p, vsfx) : (NReal)len(sfx_d.p - prev);
                    prev = sfx_d.p;
                    vprev = vsfx;
                }
                const V3 L = light_pos(s, GD, dst_pix);
                c_dst += VEL ? (NReal)seg_u(prev, vprev, L, vlight) : (NReal)len(L - prev);
            }
            const T3<NReal> xk = chart_eval_t<NReal>(S, GS, x.v[0].obj, x.v[0].xi0, x.v[0].xi1).p;
            const T3<NReal> pp = chart_eval_t<NReal>(S, GS, obj, xi0, xi1).p;
            const T3<NReal> p2s = p2light ? tof3<NReal>(p2s_pos)
                                          : chart_eval_t<NReal>(S, GS, x.v[2].obj, x.v[2].xi0, x.v[2].xi1).p;
            const T3<NReal> p2d = p2light ? tof3<NReal>(p2d_pos)
                                          : chart_eval_t<NReal>(S, GD, x.v[2].obj, x.v[2].xi0, x.v[2].xi1).p;
            const T3<NReal> yk = chart_eval_t<NReal>(S, GD, cur.obj, cur.xi0, cur.xi1).p;
            // endpoint velocities (velocity domain): x_{k-1} and p2 in the
            // source, y_{k-1} and p2 in the destination
            T3<NReal> vxk{0, 0, 0}, vp2s{0, 0, 0}, vyk{0, 0, 0}, vp2dn{0, 0, 0}, vpp{0, 0, 0};
            if (VEL) {
                auto fv = [](T3<NReal> a) { return mk((float)a.x, (float)a.y, (float)a.z); };
                vxk = tof3<NReal>(vel_at(GS, x.v[0].obj, fv(xk)));
                vpp = tof3<NReal>(vel_at(GS, obj, fv(pp)));
                vp2s = tof3<NReal>(p2light ? light_vel(s, GS, src_pix) : vel_at(GS, x.v[2].obj, fv(p2s)));
                vp2dn = tof3<NReal>(p2light ? vlight : vel_at(GD, x.v[2].obj, fv(p2d)));
                vyk = tof3<NReal>(vel_at(GD, cur.obj, fv(yk)));
            }
            const NReal c_src = VEL ? (NReal)x.len - seg_u_t<NReal>(xk, vxk, pp, vpp) - seg_u_t<NReal>(pp, vpp, p2s, vp2s)
                                    : (NReal)x.len - tlen(xk - pp) - tlen(p2s - pp);
            const NReal tol = (NReal)s.tol_rel * (NReal)plane_width(s, plane);
            NewtonOut no = newton_solve<NReal, VEL>(S, GS, GD, obj, (NReal)xi0, (NReal)xi1, xk, vxk, p2s, vp2s, c_src,
                                                    yk, vyk, p2d, vp2dn, c_dst, (NReal)dl0, tol, s.max_it);
            if (!no.conv) return R;
            if (s.round_trip) {
                // GRIS needs the shift to be a bijection (Sec. 3.2.3): keep it
                // only if the inverse shift (source and destination swapped,
                // Delta l negated) brings the vertex back to the source's
                // reconnection vertex, within the reconnection distance
                const NewtonOut bk = newton_solve<NReal, VEL, false>(S, GD, GS, obj, (NReal)no.xi0, (NReal)no.xi1, yk, vyk,
                                                              p2d, vp2dn, c_dst, xk, vxk, p2s, vp2s, c_src,
                                                              -(NReal)dl0, tol, s.max_it);
                if (!bk.conv) return R;
                const ChartT<NReal> cb = chart_eval_t<NReal>(S, GS, obj, (NReal)bk.xi0, (NReal)bk.xi1);
                if (!cb.ok || tlen(cb.p - pp) > (NReal)S.dmin) return R;
            }
            st.c[ST_NEWTON_CONV]++;
            st.c[ST_NEWTON_ITERS] += (uint32_t)no.iters;
            xi0 = no.xi0;
            xi1 = no.xi1;
            det_area = no.det_area;
        } else {
            Chart cs = chart_eval(S, GS, obj, xi0, xi1), cd = chart_eval(S, GD, obj, xi0, xi1);
            if (!cs.ok || !cd.ok) return R;
            det_area = (double)len(cross(cd.ju, cd.jv)) / (double)len(cross(cs.ju, cs.jv));
        }
        const Chart cp = chart_eval(S, GD, obj, xi0, xi1);
        if (!cp.on || !cp.ok) return R;
        pd.obj = obj;
        pd.xi0 = wrap_coord(S, obj, 0, xi0);
        pd.xi1 = wrap_coord(S, obj, 1, xi1);
        pd.p = cp.p;
        pd.n = cp.n;
        V3 e1 = pd.p - cur.p;
        float l1 = len(e1);
        if (l1 < S.dmin) return R;
        // contribution of the offset path beyond y_{k-1}
        V3 w1 = (1.0f / l1) * e1;
        C = beta * (bsdf_eval(S, cur.obj, cur.n, wi_e, w1) * fabsf(dot(cur.n, w1)));
        const V3 vpd = VEL ? vel_at(GD, obj, pd.p) : mk(0.f, 0.f, 0.f);
        plen += VEL ? dot(vc - vpd, w1) : l1;
        V3 wi2 = -w1;
        if (p2light) {
            V3 e2 = light_pos(s, GD, dst_pix) - pd.p;
            float l2 = len(e2);
            V3 w2 = (1.0f / l2) * e2;
            C *= bsdf_eval(S, obj, pd.n, wi2, w2) * fabsf(dot(pd.n, w2)) * light_emit(s, S, GD, dst_pix, pd.p) /
                 (l2 * l2);
            plen += VEL ? dot(vpd - vlight, w2) : l2;
        } else {
            V3 e2 = p2_d.p - pd.p;
            float l2 = len(e2);
            V3 w2 = (1.0f / l2) * e2;
            C *= bsdf_eval(S, obj, pd.n, wi2, w2) * fabsf(dot(pd.n, w2));
            plen += VEL ? dot(vpd - vp2d, w2) : l2;
            Vtx last = p2_d;
            V3 vlast = vp2d;
            V3 wil = -w2;
            if (x.nsfx > 0) {
                V3 e3 = sfx_d.p - p2_d.p;
                float l3 = len(e3);
                V3 w3 = (1.0f / l3) * e3;
                C *= bsdf_eval(S, p2_d.obj, p2_d.n, wil, w3) * fabsf(dot(p2_d.n, w3));
                plen += VEL ? dot(vp2d - vsfx, w3) : l3;
                last = sfx_d;
                vlast = vsfx;
                wil = -w3;
            }
            V3 e4 = light_pos(s, GD, dst_pix) - last.p;
            float l4 = len(e4);
            V3 w4 = (1.0f / l4) * e4;
            C *= bsdf_eval(S, last.obj, last.n, wil, w4) * fabsf(dot(last.n, w4)) *
                 light_emit(s, S, GD, dst_pix, last.p) / (l4 * l4);
            plen += VEL ? dot(vlast - vlight, w4) : l4;
        }
        // Jacobian: replayed directions, reconnection edge, chart area, next edge
        V3 ex = xkm1_s.p - p_s.p;
        float lx = len(ex);
        float gy = fabsf(dot(pd.n, w1)) / (l1 * l1);
        float gx = fabsf(dot(p_s.n, (1.0f / lx) * ex)) / (lx * lx);
        J *= (double)gy / (double)gx * det_area;
        if (!p2light) {
            V3 e2d = pd.p - p2_d.p, e2s = p_s.p - p2_s.p;
            float l2d = len(e2d), l2s = len(e2s);
            float g2d = fabsf(dot(p2_d.n, (1.0f / l2d) * e2d)) / (l2d * l2d);
            float g2s = fabsf(dot(p2_s.n, (1.0f / l2s) * e2s)) / (l2s * l2s);
            J *= (double)g2d / (double)g2s;
        }
        R.v0 = VRef{cur.obj, cur.xi0, cur.xi1};
        R.v1 = VRef{obj, pd.xi0, pd.xi1};
    }
    if (!(C > 0.f)) return R;
    const float Jf = (float)J;
    if (!(Jf >= 1.0f / s.j_max && Jf <= s.j_max)) return R;
    const float ph = in_plane_at(s, GD, plane, plen) ? C : 0.f;
    if (!(ph > 0.f)) return R;
    // visibility last: only shifts that would contribute pay for rays
    const bool newton = s.shift_mode == 1 && !replay_only;
    const uint32_t tag = newton ? kOwnerNewton : 0u;
    const int nseg = replay_only ? 1 : 2 + ((!p2light && src_slot != dst_slot) ? (x.nsfx > 0 ? 2 : 1) : 0);
    uint32_t slot_e[4];
    if (!q.alloc((uint32_t)nseg, slot_e)) {   // the launch sizes its chunk so that this never happens
        st.c[ST_OVERFLOW]++;
        return R;
    }
    for (int e = 0; e < nseg; ++e) {
        Seg sg;
        if (replay_only) sg = seg_light(s, S, GD, dst_pix, cur);
        else if (e == 0) sg = seg_pts(S, cur, pd);
        else if (e == 1) sg = p2light ? seg_light(s, S, GD, dst_pix, pd) : seg_pts(S, pd, p2_d);
        else if (e == 2 && x.nsfx > 0) sg = seg_pts(S, p2_d, sfx_d);
        else sg = seg_light(s, S, GD, dst_pix, x.nsfx > 0 ? sfx_d : p2_d);
        q.put(e == 0 ? slot_e[0] : (e == 1 ? slot_e[1] : (e == 2 ? slot_e[2] : slot_e[3])), sg, owner | tag);
    }
    R.len = plen;
    R.pre_pdf = pdf_y;
    R.phat = ph;
    R.J = Jf;
    R.ok = true;
    st.c[ST_SHIFTS_OK]++;
    if (newton) st.c[ST_NEWTON_OK]++;
    return R;
}

// wave-reduced accumulation of the per-lane counters (one atomic per wave)
__device__ inline void flush_counters(Counters& st, unsigned long long* global) {
#pragma unroll
    for (int i = 0; i < kNumCounters; ++i) {
        unsigned long long v = st.c[i];   // widened before the wave sum
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(global + i, v);
    }
}

}  // namespace tofd
