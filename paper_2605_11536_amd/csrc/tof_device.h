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
constexpr int kStackDepth = 64;      // per-lane traversal stack entries (LDS)
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
// Binary BVH node holding both child boxes; child index has bit 31 set for a
// leaf (sorted primitive position).
struct Node {
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int c0, c1, parent, pad;
};

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
    const float4* wv;       // world vertices
    const float* xf;        // object transforms, 12 floats each
    const Node* nodes;
    const float4* leaves;   // 3 float4 per sorted triangle: v0 (w = tri id bits), v1, v2
    int n_tri;
    V3 cam_pos, cam_fwd, cam_right, cam_up;
    float tan_half, aspect, ohx, ohy;
    V3 light_pos;
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
    int P, B, mask_words;
    uint64_t seed;
};

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

// SoA reservoir planes, element [plane * P + pixel]; M and masks per pixel.
struct ResSet {
    float* W;
    float* phat;
    float* len;
    float* pre_pdf;
    uint32_t* opix;
    uint32_t* ofr;
    uint32_t* meta;          // tree | n << 8 | k << 12 | nsfx << 16
    int* vobj[4];
    float* vxi0[4];
    float* vxi1[4];
    float* M;                // [P]
    uint32_t* mask;          // [mask_words * P]: bit set <=> reservoir non-empty
};

__device__ __forceinline__ void store_rec(const ResSet& R, size_t idx, const Rec& r, float W) {
    R.W[idx] = W;
    R.phat[idx] = r.phat;
    R.len[idx] = r.len;
    R.pre_pdf[idx] = r.pre_pdf;
    R.opix[idx] = r.opix;
    R.ofr[idx] = r.ofr;
    R.meta[idx] = (uint32_t)r.tree | ((uint32_t)r.n << 8) | ((uint32_t)r.k << 12) | ((uint32_t)r.nsfx << 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        R.vobj[q][idx] = r.v[q].obj;
        R.vxi0[q][idx] = r.v[q].xi0;
        R.vxi1[q][idx] = r.v[q].xi1;
    }
}
__device__ __forceinline__ Rec load_rec(const ResSet& R, size_t idx, float& W) {
    Rec r;
    W = R.W[idx];
    r.phat = R.phat[idx];
    r.len = R.len[idx];
    r.pre_pdf = R.pre_pdf[idx];
    r.opix = R.opix[idx];
    r.ofr = R.ofr[idx];
    uint32_t m = R.meta[idx];
    r.tree = (int)(m & 255u);
    r.n = (int)((m >> 8) & 15u);
    r.k = (int)((m >> 12) & 15u);
    r.nsfx = (int)((m >> 16) & 15u);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        r.v[q].obj = R.vobj[q][idx];
        r.v[q].xi0 = R.vxi0[q][idx];
        r.v[q].xi1 = R.vxi1[q][idx];
    }
    return r;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the stream layout
// counter = (pixel, frame, pass << 56 | a << 32 | b, 0), key = (seed, 0)
// ---------------------------------------------------------------------------
enum { PASS_JITTER = 0, PASS_BSDF = 1, PASS_RIS = 2, PASS_TEMPORAL = 3, PASS_SPATIAL = 4 };

struct Draw {
    uint64_t x[4];
    __device__ __forceinline__ float u(int i) const { return (float)(x[i] >> 40) * (1.0f / 16777216.0f); }
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
        V3 v00 = ld3(G.wv, base), v10 = ld3(G.wv, base + 1);
        V3 v01 = ld3(G.wv, base + row), v11 = ld3(G.wv, base + row + 1);
        if (a + b <= 1.0f) {
            c.p = v00 + a * (v10 - v00) + b * (v01 - v00);
            c.ju = v10 - v00;
            c.jv = v01 - v00;
        } else {
            c.p = v11 + (1.0f - a) * (v01 - v11) + (1.0f - b) * (v10 - v11);
            c.ju = v11 - v01;
            c.jv = v11 - v10;
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

__device__ __forceinline__ bool isect_sphere(V3 o, V3 d, V3 c, float r, float tmax, float& t) {
    V3 oc = o - c;
    float b = dot(oc, d), cc = dot(oc, oc) - r * r;
    float disc = b * b - cc;
    if (disc < 0.f) return false;
    float sq = sqrtf(disc);
    float t0 = -b - sq, t1 = -b + sq;
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

__device__ __forceinline__ bool slab(const float* lo, const float* hi, const RayPre& r, float tmax, float& tn) {
    float t1 = (lo[0] - r.o.x) * r.inv.x, t2 = (hi[0] - r.o.x) * r.inv.x;
    float a = fminf(t1, t2), b = fmaxf(t1, t2);
    t1 = (lo[1] - r.o.y) * r.inv.y;
    t2 = (hi[1] - r.o.y) * r.inv.y;
    a = fmaxf(a, fminf(t1, t2));
    b = fminf(b, fmaxf(t1, t2));
    t1 = (lo[2] - r.o.z) * r.inv.z;
    t2 = (hi[2] - r.o.z) * r.inv.z;
    a = fmaxf(a, fminf(t1, t2));
    b = fminf(b, fmaxf(t1, t2));
    a = fmaxf(a, 0.f);
    b = fminf(b, tmax);
    tn = a;
    return a <= b;
}

struct Hit {
    int prim, obj;
    float t, b1, b2;
};

struct Counters {
    uint64_t c[9];
};
enum { ST_SHIFTS = 0, ST_SHIFTS_OK, ST_NEWTON_ATT, ST_NEWTON_CONV, ST_NEWTON_ITERS, ST_NEWTON_OK, ST_RAYS, ST_FRAMES,
       ST_OVERFLOW };

// Closest hit (any_hit = false; ties in t go to the smaller primitive id) or
// any hit in (0, tmax) (any_hit = true).  `stack` points at this lane's LDS
// column; consecutive entries are `stride` apart.
__device__ inline bool traverse(const SceneDev& S, const SlotDev& G, V3 o, V3 d, float tmax, bool any_hit, Hit& h,
                                uint32_t* stack, int stride, Counters& st) {
    RayPre r = ray_pre(o, d);
    float tb = tmax;
    h.prim = -1;
    h.obj = -1;
    const int T = G.n_tri;
    auto test_leaf = [&](int k) -> bool {
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
    if (T == 1) {
        if (test_leaf(0)) return true;
    } else if (T > 1) {
        int sp = 0;
        uint32_t node = 0;
        // a binary tree over T leaves has T-1 internal nodes: any valid walk
        // visits each at most once, so this bound only stops a malformed tree
        int budget = 2 * T + 64;
        while (--budget > 0) {
            const Node& nd = G.nodes[node];
            float t0, t1;
            bool h0 = slab(nd.lo0, nd.hi0, r, tb, t0);
            bool h1 = slab(nd.lo1, nd.hi1, r, tb, t1);
            uint32_t c0 = (uint32_t)nd.c0, c1 = (uint32_t)nd.c1;
            // leaves are tested right away; internal children are visited near-first
            if (h0 && (c0 & 0x80000000u)) {
                if (test_leaf((int)(c0 & 0x7fffffffu))) return true;
                h0 = false;
            }
            if (h1 && (c1 & 0x80000000u)) {
                if (test_leaf((int)(c1 & 0x7fffffffu))) return true;
                h1 = false;
            }
            if (h0 && h1) {
                uint32_t nearc = t0 <= t1 ? c0 : c1, farc = t0 <= t1 ? c1 : c0;
                if (sp < kStackDepth) {
                    stack[sp * stride] = farc;
                    ++sp;
                } else {
                    st.c[ST_OVERFLOW]++;
                }
                node = nearc;
                continue;
            }
            if (h0) {
                node = c0;
                continue;
            }
            if (h1) {
                node = c1;
                continue;
            }
            if (sp == 0) break;
            --sp;
            node = stack[sp * stride];
        }
        if (budget <= 0) st.c[ST_OVERFLOW]++;
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
    Counters& st;

    __device__ bool trace(const SlotDev& G, const Vtx& from, V3 dir, Vtx& out) {
        V3 o = offset_pt(S, from.p, from.n, dir);
        Hit h;
        st.c[ST_RAYS]++;
        if (!traverse(S, G, o, dir, 3.0e38f, false, h, stack, stride, st)) return false;
        out = hit_vertex(S, G, h, o, dir);
        return true;
    }
    // true if every segment is unoccluded (stops at the first blocked one)
    __device__ bool all_visible(const SlotDev& G, const Seg* segs, int n) {
        for (int i = 0; i < n; ++i) {
            Hit h;
            st.c[ST_RAYS]++;
            if (traverse(S, G, segs[i].o, segs[i].d, segs[i].t, true, h, stack, stride, st)) return false;
        }
        return true;
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
    float sh = sqrtf(fmaxf(0.f, 1.0f - ch * ch));
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
__device__ __forceinline__ float plane_width(const Sens& s, int pl) { return pl < s.n_bins ? s.bw : s.gate_w; }
__device__ __forceinline__ bool in_plane(const Sens& s, int pl, float l) {
    return l >= plane_lo(s, pl) && l < plane_hi(s, pl);
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
__device__ __forceinline__ float camera_leg(const Sens& s, const SlotDev& G, const Vtx& y1) {
    if (!s.count_leg) return 0.f;
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

// path contribution in the product solid-angle measure (no visibility)
__device__ inline float path_eval(const Sens& s, const SceneDev& S, const SlotDev& G, int pix, const Vtx* ys, int n,
                                  float& plen) {
    V3 wi = toward_camera(s, G, ys[0]);
    float f = 1.0f;
    plen = camera_leg(s, G, ys[0]);
    for (int j = 0; j + 1 < n; ++j) {
        V3 dv = ys[j + 1].p - ys[j].p;
        float dl = len(dv);
        V3 wo = (1.0f / dl) * dv;
        f *= bsdf_eval(S, ys[j].obj, ys[j].n, wi, wo) * fabsf(dot(ys[j].n, wo));
        plen += dl;
        wi = -wo;
    }
    const Vtx& y = ys[n - 1];
    V3 L = light_pos(s, G, pix);
    V3 dv = L - y.p;
    float dl = len(dv);
    V3 wo = (1.0f / dl) * dv;
    f *= bsdf_eval(S, y.obj, y.n, wi, wo) * fabsf(dot(y.n, wo)) * light_emit(s, S, G, pix, y.p) / (dl * dl);
    plen += dl;
    return f;
}

// ---------------------------------------------------------------------------
// Newton solve of the path-length constraint (Sec. 4.3), average-gradient
// gauge.  Length functions use the source endpoints at xi and the
// destination endpoints at xi'; dF2/dxi' is the derivative of F2 itself.
//
// The solve runs in FP64: near stationary points of the length function the
// system is ill-conditioned and FP32 evaluation of F moves xi' and the
// determinant by up to ~1e-3 relative.  gfx950 issues FP64 vector math at
// half the FP32 rate and the solve is a few hundred flops per shift, small
// next to the traversal of the same shift.
// ---------------------------------------------------------------------------
struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 dk(double a, double b, double c) { return D3{a, b, c}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return D3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 dcross(D3 a, D3 b) {
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dlen(D3 a) { return sqrt(ddot(a, a)); }
__device__ __forceinline__ D3 up3(V3 a) { return D3{a.x, a.y, a.z}; }
__device__ __forceinline__ D3 ldd3(const float4* a, int i) {
    float4 v = a[i];
    return D3{v.x, v.y, v.z};
}
__device__ __forceinline__ D3 dxf_point(const float* m, D3 q) {
    return dk((double)m[0] * q.x + (double)m[1] * q.y + (double)m[2] * q.z + (double)m[3],
              (double)m[4] * q.x + (double)m[5] * q.y + (double)m[6] * q.z + (double)m[7],
              (double)m[8] * q.x + (double)m[9] * q.y + (double)m[10] * q.z + (double)m[11]);
}
__device__ __forceinline__ D3 dxf_dir(const float* m, D3 q) {
    return dk((double)m[0] * q.x + (double)m[1] * q.y + (double)m[2] * q.z,
              (double)m[4] * q.x + (double)m[5] * q.y + (double)m[6] * q.z,
              (double)m[8] * q.x + (double)m[9] * q.y + (double)m[10] * q.z);
}

struct ChartD {
    bool ok;
    D3 p, ju, jv, puu, puv, pvv;
};

// FP64 twin of chart_eval (positions from the frame's FP32 world vertices)
__device__ inline ChartD chart_eval_d(const SceneDev& S, const SlotDev& G, int obj, double u, double v) {
    ChartD c;
    const Obj ob = S.objs[obj];
    D3 z = dk(0.0, 0.0, 0.0);
    c.puu = z;
    c.puv = z;
    c.pvv = z;
    if (ob.type == 0) {
        double uu = u, vv = v;
        if (ob.wrap_u) uu = u - (double)ob.nu * floor(u / (double)ob.nu);
        if (ob.wrap_v) vv = v - (double)ob.nv * floor(v / (double)ob.nv);
        double fi = floor(uu), fj = floor(vv);
        int i = (int)fmin(fmax(fi, 0.0), (double)(ob.nu - 1));
        int j = (int)fmin(fmax(fj, 0.0), (double)(ob.nv - 1));
        double a = uu - (double)i, b = vv - (double)j;
        int row = ob.nu + 1;
        int base = ob.voff + j * row + i;
        D3 v00 = ldd3(G.wv, base), v10 = ldd3(G.wv, base + 1);
        D3 v01 = ldd3(G.wv, base + row), v11 = ldd3(G.wv, base + row + 1);
        if (a + b <= 1.0) {
            c.p = v00 + a * (v10 - v00) + b * (v01 - v00);
            c.ju = v10 - v00;
            c.jv = v01 - v00;
        } else {
            c.p = v11 + (1.0 - a) * (v01 - v11) + (1.0 - b) * (v10 - v11);
            c.ju = v11 - v01;
            c.jv = v11 - v10;
        }
        c.ok = dlen(dcross(c.ju, c.jv)) > 0.0;
    } else {
        const float* m = G.xf + 12 * obj;
        double th = u, ph = v, r = ob.r;
        double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
        D3 radial = dk(st * cp, st * sp, ct);
        c.p = dxf_point(m, dk(ob.cx, ob.cy, ob.cz) + r * radial);
        c.ju = dxf_dir(m, dk(r * ct * cp, r * ct * sp, -r * st));
        c.jv = dxf_dir(m, dk(-r * st * sp, r * st * cp, 0.0));
        c.puu = dxf_dir(m, (-r) * radial);
        c.puv = dxf_dir(m, dk(-r * ct * sp, r * ct * cp, 0.0));
        c.pvv = dxf_dir(m, dk(-r * st * cp, -r * st * sp, 0.0));
        c.ok = true;
    }
    return c;
}

struct LenEval {
    bool ok;
    double L, g0, g1, h00, h01, h11, area;
};

__device__ inline LenEval len_eval(const SceneDev& S, const SlotDev& G, int obj, double u, double v, D3 a, D3 b,
                                   double c) {
    LenEval e;
    e.ok = false;
    ChartD ch = chart_eval_d(S, G, obj, u, v);
    if (!ch.ok) return e;
    D3 r1 = a - ch.p, r2 = b - ch.p;
    double l1 = dlen(r1), l2 = dlen(r2);
    if (!(l1 > 0.0 && l2 > 0.0)) return e;
    D3 d1 = (1.0 / l1) * r1, d2 = (1.0 / l2) * r2;
    D3 sv = d1 + d2;
    e.L = c + l1 + l2;
    e.g0 = -ddot(sv, ch.ju);
    e.g1 = -ddot(sv, ch.jv);
    double i1 = 1.0 / l1, i2 = 1.0 / l2;
    auto A = [&](D3 x) { return i1 * (x - ddot(d1, x) * d1) + i2 * (x - ddot(d2, x) * d2); };
    D3 Aju = A(ch.ju), Ajv = A(ch.jv);
    e.h00 = ddot(ch.ju, Aju) - ddot(sv, ch.puu);
    e.h01 = ddot(ch.ju, Ajv) - ddot(sv, ch.puv);
    e.h11 = ddot(ch.jv, Ajv) - ddot(sv, ch.pvv);
    e.area = dlen(dcross(ch.ju, ch.jv));
    e.ok = true;
    return e;
}

struct NewtonOut {
    bool conv;
    double xi0, xi1;
    int iters;
    double det_area;
};

__device__ inline NewtonOut newton_solve(const SceneDev& S, const SlotDev& GS, const SlotDev& GD, int obj,
                                         double xs0, double xs1, D3 as, D3 bs, double cs, D3 ad, D3 bd, double cd,
                                         double dl0, double tol, int maxit) {
    NewtonOut out;
    out.conv = false;
    out.iters = 0;
    LenEval Sv = len_eval(S, GS, obj, xs0, xs1, as, bs, cs);
    if (!Sv.ok) return out;
    double xp0 = xs0, xp1 = xs1;
    LenEval D = len_eval(S, GD, obj, xp0, xp1, ad, bd, cd);
    if (!D.ok) return out;
    auto Fv = [&](const LenEval& E, double x0, double x1, double& F0, double& F1) {
        double m0 = 0.5 * (Sv.g0 + E.g0), m1 = 0.5 * (Sv.g1 + E.g1);
        double d0 = x0 - xs0, d1 = x1 - xs1;
        F0 = E.L - Sv.L - dl0;
        F1 = -m1 * d0 + m0 * d1;
    };
    auto jac_dst = [&](const LenEval& E, double x0, double x1, double J[4]) {
        double m0 = 0.5 * (Sv.g0 + E.g0), m1 = 0.5 * (Sv.g1 + E.g1);
        double rd0 = -(x1 - xs1), rd1 = x0 - xs0;
        J[0] = E.g0;
        J[1] = E.g1;
        J[2] = -m1 - 0.5 * (E.h00 * rd0 + E.h01 * rd1);
        J[3] = m0 - 0.5 * (E.h01 * rd0 + E.h11 * rd1);
    };
    double F0, F1;
    Fv(D, xp0, xp1, F0, F1);
    int it = 0;
    while (true) {
        if (fabs(F0) <= tol && fabs(F1) <= tol) break;
        if (it >= maxit) return out;
        double J[4];
        jac_dst(D, xp0, xp1, J);
        double det = J[0] * J[3] - J[1] * J[2];
        if (fabs(det) < 1e-12) return out;
        double s0 = -(J[3] * F0 - J[1] * F1) / det;
        double s1 = -(-J[2] * F0 + J[0] * F1) / det;
        double norm0 = sqrt(F0 * F0 + F1 * F1);
        bool accepted = false;
        double alpha = 1.0;
        for (int ls = 0; ls < 4; ++ls, alpha *= 0.5) {   // backtracking line search
            double x0 = xp0 + alpha * s0, x1 = xp1 + alpha * s1;
            LenEval Dt = len_eval(S, GD, obj, x0, x1, ad, bd, cd);
            if (!Dt.ok) continue;
            double G0, G1;
            Fv(Dt, x0, x1, G0, G1);
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
    double Jd[4];
    jac_dst(D, xp0, xp1, Jd);
    double m0 = 0.5 * (Sv.g0 + D.g0), m1 = 0.5 * (Sv.g1 + D.g1);
    double rd0 = -(xp1 - xs1), rd1 = xp0 - xs0;
    double Js00 = -Sv.g0, Js01 = -Sv.g1;
    double Js10 = -(-m1 + 0.5 * (Sv.h00 * rd0 + Sv.h01 * rd1));
    double Js11 = -(m0 + 0.5 * (Sv.h01 * rd0 + Sv.h11 * rd1));
    double detd = Jd[0] * Jd[3] - Jd[1] * Jd[2];
    double dets = Js00 * Js11 - Js01 * Js10;
    if (fabs(detd) < 1e-12) return out;
    out.conv = true;
    out.xi0 = xp0;
    out.xi1 = xp1;
    out.iters = it;
    // chart -> surface: sqrt(det J'^T J') / sqrt(det J^T J)
    out.det_area = D.area / Sv.area * (fabs(dets) / fabs(detd));
    return out;
}

// ---------------------------------------------------------------------------
// shift T_{src -> dst} (Sec. 4.1): random replay up to x_{k-1}, reconnection
// at p, Newton perturbation of p, visibility, full Jacobian in the product
// solid-angle measure, target in the destination plane.
// ---------------------------------------------------------------------------
struct ShiftOut {
    bool ok;
    Rec y;
    float J, phat;
};

__device__ inline ShiftOut shift_path(const Sens& s, const SceneDev& S, const Frames& F, Tracer& tr, const Rec& x,
                                      int src_slot, int src_pix, int dst_slot, int dst_pix, int plane, float dl0) {
    ShiftOut R;
    R.ok = false;
    Counters& st = tr.st;
    st.c[ST_SHIFTS]++;
    const SlotDev& GS = F.g[src_slot];
    const SlotDev& GD = F.g[dst_slot];
    if (GD.gb_obj[dst_pix] < 0) return R;
    Vtx ys[kMaxVerts + 1];
    int ny = 1;
    ys[0] = gbuf_vertex(GD, dst_pix);
    float pdf_y = 1.0f;
    V3 wi = toward_camera(s, GD, ys[0]);
    const int nrep = (x.k == 0) ? x.n - 1 : x.k - 2;
    for (int i = 1; i <= nrep; ++i) {
        const Vtx cur = ys[ny - 1];
        Draw u = philox(s.seed, x.opix, x.ofr, PASS_BSDF, (uint64_t)x.tree, (uint64_t)i);
        V3 wo;
        float pdf;
        if (!bsdf_sample(S, cur.obj, cur.n, wi, u.u(0), u.u(1), wo, pdf)) return R;
        Vtx nx;
        if (!tr.trace(GD, cur, wo, nx)) return R;
        pdf_y *= pdf;
        ys[ny++] = nx;
        wi = -wo;
    }
    for (int kk = 2; kk <= ny; ++kk)
        if (recon_ok(S, ys[kk - 2], ys[kk - 1])) return R;

    if (x.k == 0) {   // pure random replay
        float plen;
        float C = path_eval(s, S, GD, dst_pix, ys, ny, plen);
        if (!(C > 0.f)) return R;
        Seg sg = seg_light(s, S, GD, dst_pix, ys[ny - 1]);
        if (!tr.all_visible(GD, &sg, 1)) return R;
        float J = x.pre_pdf / pdf_y;
        if (!(J >= 1.0f / s.j_max && J <= s.j_max)) return R;
        float ph = in_plane(s, plane, plen) ? C : 0.f;
        if (!(ph > 0.f)) return R;
        R.y = x;
        R.y.len = plen;
        R.y.pre_pdf = pdf_y;
        R.y.phat = ph;
        R.J = J;
        R.phat = ph;
        R.ok = true;
        st.c[ST_SHIFTS_OK]++;
        return R;
    }

    const Vtx ykm1 = ys[ny - 1];
    if (!is_rough(S, ykm1.obj)) return R;
    const int obj = x.v[1].obj;
    const Vtx xkm1_s = vertex_at(S, GS, x.v[0].obj, x.v[0].xi0, x.v[0].xi1);
    const Vtx p_s = vertex_at(S, GS, obj, x.v[1].xi0, x.v[1].xi1);
    const bool p2light = x.v[2].obj < 0;
    Vtx p2_s, p2_d;
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
    Vtx sfx_d;
    if (x.nsfx > 0) sfx_d = vertex_at(S, GD, x.v[3].obj, x.v[3].xi0, x.v[3].xi1);
    // fixed parts of the two length functions (prefix before x_{k-1}, suffix
    // after p2), formed in FP64 so that L_src(xi) reproduces the stored length
    double c_dst = (double)camera_leg(s, GD, ys[0]);
    for (int j = 0; j + 1 < ny; ++j) c_dst += dlen(up3(ys[j + 1].p) - up3(ys[j].p));
    if (!p2light) {
        D3 prev = up3(p2d_pos);
        if (x.nsfx > 0) {
            c_dst += dlen(up3(sfx_d.p) - prev);
            prev = up3(sfx_d.p);
        }
        c_dst += dlen(up3(light_pos(s, GD, dst_pix)) - prev);
    }
    float xi0 = x.v[1].xi0, xi1 = x.v[1].xi1;
    double det_area;
    if (s.shift_mode == 1) {
        st.c[ST_NEWTON_ATT]++;
        double tol = (double)s.tol_rel * (double)plane_width(s, plane);
        // endpoints in FP64 from the FP32 chart points of the two frames
        D3 xkm1_d = chart_eval_d(S, GS, x.v[0].obj, x.v[0].xi0, x.v[0].xi1).p;
        D3 ykm1_d = chart_eval_d(S, GD, ykm1.obj, ykm1.xi0, ykm1.xi1).p;
        D3 p2s_d = p2light ? up3(p2s_pos) : chart_eval_d(S, GS, x.v[2].obj, x.v[2].xi0, x.v[2].xi1).p;
        D3 p2d_d = p2light ? up3(p2d_pos) : chart_eval_d(S, GD, x.v[2].obj, x.v[2].xi0, x.v[2].xi1).p;
        D3 p_d = chart_eval_d(S, GS, obj, xi0, xi1).p;
        double c_src = (double)x.len - dlen(xkm1_d - p_d) - dlen(p2s_d - p_d);
        NewtonOut no = newton_solve(S, GS, GD, obj, xi0, xi1, xkm1_d, p2s_d, c_src, ykm1_d, p2d_d, c_dst,
                                    (double)dl0, tol, s.max_it);
        if (!no.conv) return R;
        st.c[ST_NEWTON_CONV]++;
        st.c[ST_NEWTON_ITERS] += (uint64_t)no.iters;
        xi0 = (float)no.xi0;
        xi1 = (float)no.xi1;
        det_area = no.det_area;
    } else {
        Chart cs = chart_eval(S, GS, obj, xi0, xi1), cd = chart_eval(S, GD, obj, xi0, xi1);
        if (!cs.ok || !cd.ok) return R;
        det_area = (double)len(cross(cd.ju, cd.jv)) / (double)len(cross(cs.ju, cs.jv));
    }
    Chart cp = chart_eval(S, GD, obj, xi0, xi1);
    if (!cp.on || !cp.ok) return R;
    Vtx pd;
    pd.obj = obj;
    pd.xi0 = wrap_coord(S, obj, 0, xi0);
    pd.xi1 = wrap_coord(S, obj, 1, xi1);
    pd.p = cp.p;
    pd.n = cp.n;
    if (len(pd.p - ykm1.p) < S.dmin) return R;
    {
        Seg segs[4];
        int ns = 0;
        segs[ns++] = seg_pts(S, ykm1, pd);
        if (p2light) {
            segs[ns++] = seg_light(s, S, GD, dst_pix, pd);
        } else {
            segs[ns++] = seg_pts(S, pd, p2_d);
            if (src_slot != dst_slot) {   // the scene may have moved: re-test the suffix
                Vtx prev = p2_d;
                if (x.nsfx > 0) {
                    segs[ns++] = seg_pts(S, prev, sfx_d);
                    prev = sfx_d;
                }
                segs[ns++] = seg_light(s, S, GD, dst_pix, prev);
            }
        }
        if (!tr.all_visible(GD, segs, ns)) return R;
    }
    ys[ny++] = pd;
    if (!p2light) {
        ys[ny++] = p2_d;
        if (x.nsfx > 0) ys[ny++] = sfx_d;
    }
    float plen;
    float C = path_eval(s, S, GD, dst_pix, ys, ny, plen);
    double J = (double)x.pre_pdf / (double)pdf_y;
    V3 ey = ykm1.p - pd.p, ex = xkm1_s.p - p_s.p;
    float ly = len(ey), lx = len(ex);
    float gy = fabsf(dot(pd.n, (1.0f / ly) * ey)) / (ly * ly);
    float gx = fabsf(dot(p_s.n, (1.0f / lx) * ex)) / (lx * lx);
    J *= (double)gy / (double)gx * det_area;
    if (!p2light) {
        V3 e2d = pd.p - p2_d.p, e2s = p_s.p - p2_s.p;
        float l2d = len(e2d), l2s = len(e2s);
        float g2d = fabsf(dot(p2_d.n, (1.0f / l2d) * e2d)) / (l2d * l2d);
        float g2s = fabsf(dot(p2_s.n, (1.0f / l2s) * e2s)) / (l2s * l2s);
        J *= (double)g2d / (double)g2s;
    }
    float Jf = (float)J;
    if (!(Jf >= 1.0f / s.j_max && Jf <= s.j_max)) return R;
    float ph = in_plane(s, plane, plen) ? C : 0.f;
    if (!(ph > 0.f)) return R;
    R.y = x;
    R.y.v[0].obj = ykm1.obj;
    R.y.v[0].xi0 = ykm1.xi0;
    R.y.v[0].xi1 = ykm1.xi1;
    R.y.v[1].obj = obj;
    R.y.v[1].xi0 = pd.xi0;
    R.y.v[1].xi1 = pd.xi1;
    R.y.len = plen;
    R.y.pre_pdf = pdf_y;
    R.y.phat = ph;
    R.J = Jf;
    R.phat = ph;
    R.ok = true;
    st.c[ST_SHIFTS_OK]++;
    if (s.shift_mode == 1) st.c[ST_NEWTON_OK]++;
    return R;
}

// wave-reduced accumulation of the per-lane counters (one atomic per wave)
__device__ inline void flush_counters(Counters& st, unsigned long long* global) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        unsigned long long v = st.c[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(global + i, v);
    }
}

}  // namespace tofd
