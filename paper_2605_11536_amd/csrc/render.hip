// Frame kernels of the ToF ReSTIR hot path (gfx950):
//   G-buffer -> path trees + initial per-plane RIS (+ plain PT splat buffer)
//   -> temporal GRIS -> spatial GRIS rounds -> splat.
// Reuse passes work on compacted (pixel, plane) work lists: a pixel's planes
// that are non-empty in any candidate reservoir (block scan + one atomic per
// block), consumed by grid-stride kernels, so empty planes cost no work.
#include "tof_device.h"
#include "tof_internal.h"

using namespace tofd;
using tofh::FrameArgs;
using tofh::GBufOut;

namespace {

// Waves per SIMD the tracing kernels are compiled for: caps their VGPRs at
// 512 / TOF_TRACE_WAVES.  The LDS stacks (TOF_STACK_DEPTH x 4 B per lane)
// must allow as many: 48 entries x 128 lanes = 24 KB per block, 6 blocks per
// CU, 3 waves per SIMD.  Measured on the glossy 512^2 sequence, 3 waves beat
// 2 by 21%; 4 and 5 spill registers and lose 3% and 8%.
#ifndef TOF_TRACE_WAVES
#define TOF_TRACE_WAVES 3
#endif
#define TOF_TRACE_KERNEL __global__ void __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(TOF_TRACE_WAVES)))
constexpr int kTB = 128;   // lanes per block of the tracing kernels

__device__ __forceinline__ bool mask_bit(const uint32_t* mask, int P, int pl, int pix) {
    return (mask[(size_t)(pl >> 5) * P + pix] >> (pl & 31)) & 1u;
}

// ---------------------------------------------------------------------------
// primary visibility (pixel jitter from the JITTER stream)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTB) k_gbuffer(FrameArgs a, GBufOut out) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    const Sens& s = a.s;
    int pix = blockIdx.x * kTB + threadIdx.x;
    if (pix < s.P) {
        const SlotDev& G = a.F.g[0];
        int x = pix % s.W, y = pix / s.W;
        float fx = (float)(s.cx0 + x), fy = (float)(s.cy0 + y);
        float u0 = 0.5f, u1 = 0.5f;
        if (s.jitter) {
            Draw d = philox(s.seed, full_pixel(s, pix), a.frame, PASS_JITTER, 0, 0);
            u0 = d.u(0);
            u1 = d.u(1);
        }
        float sx = 2.0f * (fx + u0) / (float)s.FW - 1.0f;
        float sy = 1.0f - 2.0f * (fy + u1) / (float)s.FH;
        V3 o, dir;
        if (s.cam_model == 0) {
            o = G.cam_pos;
            dir = nrm(G.cam_fwd + (sx * G.tan_half * G.aspect) * G.cam_right + (sy * G.tan_half) * G.cam_up);
        } else {
            o = G.cam_pos + (sx * G.ohx) * G.cam_right + (sy * G.ohy) * G.cam_up;
            dir = G.cam_fwd;
        }
        Hit h;
        if (traverse(a.S, G, o, dir, 3.0e38f, false, kStackDepth, h, stk + threadIdx.x, kTB, st)) {
            Vtx v = hit_vertex(a.S, G, h, o, dir);
            out.obj[pix] = v.obj;
            out.xi0[pix] = v.xi0;
            out.xi1[pix] = v.xi1;
            out.p[pix] = make_float4(v.p.x, v.p.y, v.p.z, 0.f);
            out.n[pix] = make_float4(v.n.x, v.n.y, v.n.z, 0.f);
        } else {
            out.obj[pix] = -1;
            out.xi0[pix] = 0.f;
            out.xi1[pix] = 0.f;
            out.p[pix] = make_float4(0.f, 0.f, 0.f, 0.f);
            out.n[pix] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    flush_counters(st, a.counters);
}

// ---------------------------------------------------------------------------
// path trees with NEE at every vertex; each complete sub-path is a candidate
// of the reservoir of its time bin and of the gate (Sec. 4.5 per-bin deposit),
// and is splatted into the plain path-tracing buffer.  VEL: the planes
// measure the path velocity (Sec. 4.6) instead of the path length.
// ---------------------------------------------------------------------------
template <bool VEL>
TOF_TRACE_KERNEL k_initial(FrameArgs a, ResSet can, ResSet wide, float* __restrict__ pt,
                                                 float2* __restrict__ direct) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, kStackDepth, st};
    const Sens& s = a.s;
    const SceneDev& S = a.S;
    int pix = blockIdx.x * kTB + threadIdx.x;
    if (pix < s.P) {
        const SlotDev& G = a.F.g[0];
        const int P = s.P;
        for (int w = 0; w < s.mask_words; ++w) can.mask[(size_t)w * P + pix] = 0u;
        // the wide-gate reservoir of the shrink mapping with R < 1 (W = 0: empty)
        const bool mix = wide.rec != nullptr;
        if (mix) rec_W(wide, pix) = 0.f;
        float2 dterm = make_float2(0.f, 0.f);
        if (G.gb_obj[pix] < 0) {
            can.M[pix] = 0.f;
        } else {
            can.M[pix] = (float)s.m_init;
            const uint64_t fp = full_pixel(s, pix);
            const Vtx g = gbuf_vertex(G, pix);
            for (int tree = 0; tree < s.m_init; ++tree) {
                Vtx vs[kMaxVerts];
                float pdfs[kMaxVerts];
                vs[0] = g;
                float beta = 1.0f, pdf = 1.0f, plen = camera_leg<VEL>(s, G, g);
                V3 vcur = VEL ? vel_at(G, g.obj, g.p) : mk(0.f, 0.f, 0.f);   // velocity of the last vertex
                V3 wi = toward_camera(s, G, g);
                int kfound = 0;
                for (int i = 1; i <= s.n_max; ++i) {
                    const Vtx xi = vs[i - 1];
                    if (i >= 2 && kfound == 0 && recon_ok(S, vs[i - 2], vs[i - 1])) kfound = i;
                    bool want = (i >= 2 && i >= s.n_min) || (i == 1 && s.include_direct && s.n_min <= 1);
                    if (want) {
                        V3 L = light_pos(s, G, pix);
                        V3 dv = L - xi.p;
                        float dl = len(dv);
                        V3 wl = (1.0f / dl) * dv;
                        float fs = bsdf_eval(S, xi.obj, xi.n, wi, wl);
                        float C = beta * fs * fabsf(dot(xi.n, wl)) * light_emit(s, S, G, pix, xi.p) / (dl * dl);
                        if (C > 0.f) {
                            Seg sg = seg_light(s, S, G, pix, xi);
                            if (!tr.visible(G, sg)) C = 0.f;
                        }
                        const float li = plen + (VEL ? dot(vcur - light_vel(s, G, pix), wl) : dl);
                        if (C > 0.f && i == 1) {
                            if (tree == 0) dterm = make_float2(C, li);
                        } else if (C > 0.f) {
                            Rec rec;
                            rec.opix = (uint32_t)fp;
                            rec.ofr = a.frame;
                            rec.tree = tree;
                            rec.n = i;
                            rec.k = kfound;
                            rec.nsfx = 0;
                            rec.len = li;
                            rec.phat = C;
                            for (int q = 0; q < 4; ++q) rec.v[q] = VRef{-1, 0.f, 0.f};
                            if (kfound >= 2) {
                                const int k = kfound;
                                float pp = 1.0f;
                                for (int j = 1; j <= k - 2; ++j) pp *= pdfs[j - 1];
                                rec.pre_pdf = pp;
                                rec.v[0] = VRef{vs[k - 2].obj, vs[k - 2].xi0, vs[k - 2].xi1};
                                rec.v[1] = VRef{vs[k - 1].obj, vs[k - 1].xi0, vs[k - 1].xi1};
                                if (k < i) rec.v[2] = VRef{vs[k].obj, vs[k].xi0, vs[k].xi1};
                                if (k + 1 < i) {
                                    rec.v[3] = VRef{vs[k + 1].obj, vs[k + 1].xi0, vs[k + 1].xi1};
                                    rec.nsfx = 1;
                                }
                            } else {
                                rec.pre_pdf = pdf;
                            }
                            Draw u = philox(s.seed, fp, a.frame, PASS_RIS, (uint64_t)tree, (uint64_t)i);
                            // plain PT deposits into the planes; the reservoirs take
                            // the gate's candidates from the wide gate when the
                            // shrink mapping is on (every tree with R = 1; with
                            // R < 1 the first R x M_init trees, into a reservoir
                            // of their own, and the others from the gate), each
                            // sampling technique normalized by its own tree count
                            const bool gate_pt = s.gate_en && in_plane(s, s.n_bins, li);
                            const bool wide_tree = s.gate_en && s.shrink_k > 1.f && tree < s.mw;
                            const bool gate_res = wide_tree ? in_rough_gate(s, li) : gate_pt;
                            const float m_gate = !mix ? (float)s.m_init
                                                      : (wide_tree ? (float)s.mw : (float)(s.m_init - s.mw));
                            int planes[2] = {bin_of(s, li), gate_res ? s.n_bins : -1};
                            if (planes[0] >= 0) pt[(size_t)planes[0] * P + pix] += C / pdf / (float)s.m_init;
                            if (gate_pt) pt[(size_t)s.n_bins * P + pix] += C / pdf / (float)s.m_init;
                            for (int q = 0; q < 2; ++q) {
                                int pl = planes[q];
                                if (pl < 0) continue;
                                const float w = C / ((q == 0 ? (float)s.m_init : m_gate) * pdf);
                                if (q == 1 && mix && wide_tree) {
                                    const float ws0 = rec_W(wide, pix);
                                    if (ws0 == 0.f) {
                                        store_rec(wide, pix, rec, w);
                                    } else {
                                        const float ws = ws0 + w;
                                        if (u.u(q) * ws < w) store_rec(wide, pix, rec, ws);
                                        else rec_W(wide, pix) = ws;
                                    }
                                    continue;
                                }
                                size_t idx = (size_t)pl * P + pix;
                                uint32_t* mw = can.mask + (size_t)(pl >> 5) * P + pix;
                                uint32_t bit = 1u << (pl & 31);
                                uint32_t m = *mw;
                                if (!(m & bit)) {   // first candidate of this plane: always selected
                                    *mw = m | bit;
                                    store_rec(can, idx, rec, w);
                                } else {
                                    float ws = rec_W(can, idx) + w;
                                    if (u.u(q) * ws < w) store_rec(can, idx, rec, ws);
                                    else rec_W(can, idx) = ws;
                                }
                            }
                        }
                    }
                    if (i == s.n_max) break;
                    Draw u = philox(s.seed, fp, a.frame, PASS_BSDF, (uint64_t)tree, (uint64_t)i);
                    V3 wo;
                    float pw;
                    if (!bsdf_sample(S, xi.obj, xi.n, wi, u.u(0), u.u(1), wo, pw)) break;
                    float fcos = bsdf_eval(S, xi.obj, xi.n, wi, wo) * fabsf(dot(xi.n, wo));
                    Vtx nx;
                    if (!tr.trace(G, xi, wo, nx)) break;
                    beta *= fcos;
                    pdf *= pw;
                    pdfs[i - 1] = pw;
                    if (VEL) {
                        const V3 vn = vel_at(G, nx.obj, nx.p);
                        plen += seg_u(xi.p, vcur, nx.p, vn);
                        vcur = vn;
                    } else {
                        plen += len(nx.p - xi.p);
                    }
                    vs[i] = nx;
                    wi = -wo;
                }
            }
            // finalize: W = (sum of weights) / phat(selected)
            for (int w = 0; w < s.mask_words; ++w) {
                uint32_t m = can.mask[(size_t)w * P + pix];
                while (m) {
                    int b = __ffs(m) - 1;
                    m &= m - 1;
                    size_t idx = (size_t)(32 * w + b) * P + pix;
                    rec_W(can, idx) = rec_W(can, idx) / rec_phat(can, idx);
                }
            }
            if (mix && rec_W(wide, pix) > 0.f) rec_W(wide, pix) = rec_W(wide, pix) / rec_phat(wide, pix);
        }
        direct[pix] = dterm;
    }
    flush_counters(st, a.counters);
}

// ---------------------------------------------------------------------------
// temporal correspondence: exact rigid motion of the primary hit, projected
// into the previous camera; dropped off-screen or on a different object
// ---------------------------------------------------------------------------
__global__ void k_reproject(FrameArgs a, const float* __restrict__ Mc, const float* __restrict__ Mp,
                            int* __restrict__ prev_pix, float* __restrict__ M_out) {
    const Sens& s = a.s;
    int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= s.P) return;
    const SlotDev& G0 = a.F.g[0];
    const SlotDev& G1 = a.F.g[1];
    int obj = G0.gb_obj[pix];
    int q = -1;
    if (obj >= 0) {
        V3 p = chart_eval(a.S, G1, obj, G0.gb_xi0[pix], G0.gb_xi1[pix]).p;
        V3 v = p - G1.cam_pos;
        float px, py;
        bool ok = true;
        if (s.cam_model == 0) {
            float z = dot(v, G1.cam_fwd);
            ok = z > 0.f;
            float sx = dot(v, G1.cam_right) / z / (G1.tan_half * G1.aspect);
            float sy = dot(v, G1.cam_up) / z / G1.tan_half;
            px = 0.5f * (sx + 1.0f) * (float)s.FW;
            py = 0.5f * (1.0f - sy) * (float)s.FH;
        } else {
            px = 0.5f * (dot(v, G1.cam_right) / G1.ohx + 1.0f) * (float)s.FW;
            py = 0.5f * (1.0f - dot(v, G1.cam_up) / G1.ohy) * (float)s.FH;
        }
        if (ok) {
            float fx = floorf(px) - (float)s.cx0, fy = floorf(py) - (float)s.cy0;
            if (fx >= 0.f && fx < (float)s.W && fy >= 0.f && fy < (float)s.H) {
                int c = (int)fy * s.W + (int)fx;
                if (G1.gb_obj[c] == obj) q = c;
            }
        }
    }
    prev_pix[pix] = q;
    M_out[pix] = obj >= 0 ? Mc[pix] + (q >= 0 ? fminf(Mp[q], s.m_cap) : 0.f) : 0.f;
}

// ---------------------------------------------------------------------------
// spatial neighbours: integer rejection sampling in the disk of radius r
// (off-screen picks and pixels without a primary hit are dropped)
// ---------------------------------------------------------------------------
__global__ void k_neighbours(FrameArgs a, int round, const float* __restrict__ Min, int* __restrict__ nb,
                             float* __restrict__ M_out) {
    const Sens& s = a.s;
    int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= s.P) return;
    const SlotDev& G = a.F.g[0];
    const bool hit = G.gb_obj[pix] >= 0;
    const int x = pix % s.W, y = pix / s.W;
    const uint64_t fp = full_pixel(s, pix);
    const int64_t R = s.radius;
    const uint64_t span = (uint64_t)(2 * R + 1);
    float M = hit ? Min[pix] : 0.f;
    for (int sl = 0; sl < s.k; ++sl) {
        int q = -1;
        if (hit) {
            for (int t = 0; t < 8; ++t) {
                Draw d = philox(s.seed, fp, a.frame, PASS_SPATIAL + (uint64_t)round, 1, (uint64_t)(sl * 16 + t / 2));
                uint64_t ua = d.x[(t & 1) ? 2 : 0] >> 32, ub = d.x[(t & 1) ? 3 : 1] >> 32;
                int64_t dx = (int64_t)((ua * span) >> 32) - R;
                int64_t dy = (int64_t)((ub * span) >> 32) - R;
                if (dx * dx + dy * dy > R * R || (dx == 0 && dy == 0)) continue;
                int64_t nx = x + dx, ny = y + dy;
                if (nx >= 0 && nx < s.W && ny >= 0 && ny < s.H) {
                    int c = (int)(ny * s.W + nx);
                    if (G.gb_obj[c] >= 0) q = c;
                }
                break;
            }
        }
        nb[(size_t)sl * s.P + pix] = q;
        if (q >= 0) M += Min[q];
    }
    M_out[pix] = M;
}

// ---------------------------------------------------------------------------
// work lists.  Mode 0 (temporal): candidates are the canonical reservoir and
// the previous frame's final reservoir at the reprojected pixel.  Mode 1
// (spatial): the pixel's input reservoir and those of its k neighbours.  For
// every plane non-empty in any candidate one item (pixel, plane | cmask << 16)
// is emitted, cmask bit c marking the non-empty candidates, with task0 = the
// index of its first task (item, c), one per non-empty candidate; items and
// tasks are numbered in the same block order, so task0 grows with the item
// index and the tasks of an item range are contiguous.  count[0] and count[1]
// receive the totals.  Task numbers wrap modulo 2^32 on a pass with more
// tasks than that; every later use takes the difference of two of them within
// one chunk, which stays exact.  Also clears the output mask.
// ---------------------------------------------------------------------------
// the bits of mask word w that are planes (not padding)
__device__ __forceinline__ uint32_t planes_in_word(const Sens& s, int w) {
    const int lo = 32 * w;
    return s.B >= lo + 32 ? 0xFFFFFFFFu : (s.B > lo ? (1u << (s.B - lo)) - 1u : 0u);
}
// the bits of mask word w that are histogram bins (not the gate plane, not padding)
__device__ __forceinline__ uint32_t bins_in_word(const Sens& s, int w) {
    const int lo = 32 * w;
    if (w < 0 || s.n_bins <= lo) return 0u;
    return s.n_bins >= lo + 32 ? 0xFFFFFFFFu : (1u << (s.n_bins - lo)) - 1u;
}
__device__ __forceinline__ uint32_t bin_word(const Sens& s, const uint32_t* m, int pix, int w) {
    if (w < 0 || w >= s.mask_words) return 0u;
    return m[(size_t)w * s.P + pix] & bins_in_word(s, w);
}

__device__ __forceinline__ uint32_t cand_word(const FrameArgs& a, int mode, const uint32_t* m1, const uint32_t* m2,
                                              const int* links, int c, int w, int pix) {
    const int P = a.s.P;
    if (mode == 2) {   // bin axis: bit b of candidate c is bin b + o of the pixel; targets are bins too
        if (c == 0) return bin_word(a.s, m1, pix, w);
        const int o = bin_offset(c - 1);
        const uint32_t v = o > 0 ? (bin_word(a.s, m1, pix, w) >> o) | (bin_word(a.s, m1, pix, w + 1) << (32 - o))
                                 : (bin_word(a.s, m1, pix, w) << -o) | (bin_word(a.s, m1, pix, w - 1) >> (32 + o));
        return v & bins_in_word(a.s, w);
    }
    if (c == 0) return m1[(size_t)w * P + pix];
    int q = mode == 0 ? links[pix] : links[(size_t)(c - 1) * P + pix];
    if (q < 0) return 0u;
    return (mode == 0 ? m2 : m1)[(size_t)w * P + q];
}

__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t b, uint32_t& ea, uint32_t& eb, uint32_t* base,
                                            uint32_t* count) {
    __shared__ uint32_t s_a[256], s_b[256];
    __shared__ uint32_t s_base[2];
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t va = (int)threadIdx.x >= off ? s_a[threadIdx.x - off] : 0u;
        uint32_t vb = (int)threadIdx.x >= off ? s_b[threadIdx.x - off] : 0u;
        __syncthreads();
        s_a[threadIdx.x] += va;
        s_b[threadIdx.x] += vb;
        __syncthreads();
    }
    if (threadIdx.x == 255) {
        // one 64-bit add for both totals (count[0] the low word), so that the
        // blocks take their item and task ranges in the same order
        const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long*>(count),
                                                 ((unsigned long long)s_b[255] << 32) | s_a[255]);
        s_base[0] = (uint32_t)old;
        s_base[1] = (uint32_t)(old >> 32);
    }
    __syncthreads();
    ea = s_base[0] + s_a[threadIdx.x] - a;
    eb = s_base[1] + s_b[threadIdx.x] - b;
    (void)base;
}

// per pixel, bit w set when mask word w is non-zero (at most 32 words)
__global__ void __launch_bounds__(256) k_word_sum(const uint32_t* __restrict__ m, int P, int words,
                                                  uint32_t* __restrict__ sum) {
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= P) return;
    uint32_t v = 0;
    for (int w = 0; w < words; ++w)
        if (m[(size_t)w * P + pix]) v |= 1u << w;
    sum[pix] = v;
}

// sum1, sum2: the word summaries of m1 and m2 (k_word_sum), or nullptr: a
// pixel reads only the words some candidate holds samples in
__global__ void __launch_bounds__(256) k_items(FrameArgs a, int mode, const uint32_t* __restrict__ m1,
                                               const uint32_t* __restrict__ m2, const int* __restrict__ links,
                                               int ncand, uint2* __restrict__ items, uint32_t* __restrict__ task0,
                                               uint32_t* __restrict__ count, uint32_t* __restrict__ out_mask,
                                               const uint32_t* __restrict__ sum1, const uint32_t* __restrict__ sum2) {
    const int P = a.s.P;
    int pix = blockIdx.x * 256 + threadIdx.x;
    bool valid = pix < P && a.F.g[0].gb_obj[pix] >= 0;
    uint32_t ni = 0, nt = 0;
    if (pix < P)
        for (int w = 0; w < a.s.mask_words; ++w) out_mask[(size_t)w * P + pix] = 0u;
    // the words any candidate of this pixel holds samples in (all without summaries)
    uint32_t wset = 0xFFFFFFFFu;
    if (valid && sum1) {
        wset = sum1[pix];
        for (int c = 1; c < ncand; ++c) {
            const int q = mode == 0 ? links[pix] : links[(size_t)(c - 1) * P + pix];
            if (q >= 0) wset |= (mode == 0 ? sum2 : sum1)[q];
        }
    }
    if (valid) {
        for (int w = 0; w < a.s.mask_words; ++w) {
            if (!((wset >> (w & 31)) & 1u)) continue;
            uint32_t u = 0;
            const uint32_t live = planes_in_word(a.s, w);
            for (int c = 0; c < ncand; ++c) {
                uint32_t m = cand_word(a, mode, m1, m2, links, c, w, pix) & live;
                u |= m;
                nt += __popc(m);
            }
            ni += __popc(u);
        }
    }
    uint32_t pi, pt_;
    block_scan2(ni, nt, pi, pt_, nullptr, count);
    if (valid && ni) {
        for (int w = 0; w < a.s.mask_words; ++w) {
            if (!((wset >> (w & 31)) & 1u)) continue;
            uint32_t wm[kMaxK + 1];
            uint32_t u = 0;
            const uint32_t live = planes_in_word(a.s, w);
            for (int c = 0; c < ncand; ++c) {
                wm[c] = cand_word(a, mode, m1, m2, links, c, w, pix) & live;
                u |= wm[c];
            }
            while (u) {
                int b = __ffs(u) - 1;
                u &= u - 1;
                uint32_t cm = 0;
                task0[pi] = pt_;
                for (int c = 0; c < ncand; ++c)
                    if ((wm[c] >> b) & 1u) cm |= 1u << c;
                pt_ += (uint32_t)__popc(cm);
                items[pi++] = make_uint2((uint32_t)pix, (uint32_t)(32 * w + b) | (cm << 16));
            }
        }
    }
}

// Tasks of the item chunk [i0, i0 + ci): tasks[t - tb] = (item, c), tb =
// task0[i0]; win = (tb, number of tasks in the chunk) for the later kernels
// of the chunk (both 0 for a chunk past the last item).
__global__ void __launch_bounds__(256) k_tasks(const uint2* __restrict__ items, const uint32_t* __restrict__ task0,
                                               const uint32_t* __restrict__ count, uint32_t i0, uint32_t ci,
                                               uint2* __restrict__ tasks, uint32_t* __restrict__ win) {
    const uint32_t ni = count[0];
    const uint32_t ie = ni - i0 > ci ? i0 + ci : ni;   // used only when i0 < ni
    const uint32_t tb = i0 < ni ? task0[i0] : 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        win[0] = tb;
        win[1] = i0 < ni ? (ie < ni ? task0[ie] : count[1]) - tb : 0u;
    }
    if (i0 >= ni) return;
    for (uint32_t i = i0 + blockIdx.x * 256 + threadIdx.x; i < ie; i += gridDim.x * 256) {
        uint32_t cm = items[i].y >> 16;
        uint32_t t = task0[i] - tb;
        while (cm) {
            const int c = __ffs(cm) - 1;
            cm &= cm - 1;
            tasks[t++] = make_uint2(i, (uint32_t)c);
        }
    }
}

// ---------------------------------------------------------------------------
// candidate weights (Sec. 3.2.3, eq. GRIS_resampling_weight with the
// generalized balance heuristic eq. GRIS_MIS_weight), one shift per lane.
//
// k_fwd, one lane per (item, candidate) task: a neighbour's sample x_c is
// shifted into q (y_c = T_{c->q}(x_c)); fwd[t] = (phat_q(y_c), |J|,
// M_c phat_c(x_c) / |J|, W_c), phat_q = 0 marking a failed shift, and the
// fields the shift rewrote go to shv[2t], shv[2t+1].  The canonical
// candidate (c = 0) records (phat_q(x_q), 1, 0, W_q).
//
// k_mis, one lane per (task, neighbour l): y_c is shifted into l's domain and
// term[t * K + l] = M_l phat_l(T_{q->l}(y_c)) |J| (0 if the shift fails, if
// l has no pixel, or for the candidate's own domain l = c - 1).
//
// The merge forms m_c = (own or M_q phat_q) / (own + M_q phat_q + sum terms).
//
// Pairwise MIS (spatial pass, opt-in): the canonical technique is split into
// Kv parts of confidence M_q / Kv (Kv = neighbours with a pixel), part l
// paired with neighbour l under the balance heuristic and the pair weighted
// by (M_l + M_q / Kv) / M_total.  A neighbour's candidate needs only its own
// forward terms, so only the canonical task has MIS shifts (K per item in
// place of K (K + 1)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cand_src(int mode, const int* links, int P, int pix, int c) {
    return mode == 0 ? links[pix] : (mode == 1 ? links[(size_t)(c - 1) * P + pix] : pix);
}
// plane of candidate c of an item in plane pl
__device__ __forceinline__ int cand_plane(int mode, int pl, int c) { return mode == 2 ? pl + bin_offset(c - 1) : pl; }
// M of a neighbour domain's pixel
__device__ __forceinline__ float dom_M(const Sens& s, int mode, const ResSet& A, const ResSet& Bp, int dpix) {
    return mode == 0 ? fminf(Bp.M[dpix], s.m_cap) : A.M[dpix];
}

template <bool VEL>
TOF_TRACE_KERNEL k_fwd(FrameArgs a, int mode, ResSet A, ResSet Bp, const int* __restrict__ links,
                       const uint2* __restrict__ items, const uint2* __restrict__ tasks,
                       const uint32_t* __restrict__ win, float4* __restrict__ fwd, float4* __restrict__ shv,
                       RayQueue q) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, kStackDepth, st};
    const Sens& s = a.s;
    const int P = s.P;
    const uint32_t n = win[1];
    for (uint32_t t = blockIdx.x * kTB + threadIdx.x; t < n; t += gridDim.x * kTB) {
        const uint2 task = tasks[t];
        const uint2 item = items[task.x];
        const int c = (int)task.y;
        const int pix = (int)item.x, pl = (int)(item.y & 0xFFFFu);
        if (c == 0) {
            const size_t idx = (size_t)pl * P + pix;
            fwd[t] = make_float4(rec_phat(A, idx), 1.0f, 0.f, rec_W(A, idx));
            continue;
        }
        const int src = cand_src(mode, links, P, pix, c);
        const int spl = cand_plane(mode, pl, c);
        float Wx;
        Rec y = load_rec(mode == 0 ? Bp : A, (size_t)spl * P + src, Wx);
        const float xphat = y.phat;
        const float mc = dom_M(s, mode, A, Bp, src);
        // a blocked visibility ray zeroes phat_q (component x of fwd[t])
        const float dl = mode == 0 ? gate_shift(s, a.F.g[0], a.F.g[1], pl)
                                   : (mode == 2 ? (float)(pl - spl) * s.bw : 0.f);
        const ShiftOut sh = shift_path<VEL>(s, a.S, a.F, tr, y, mode == 0 ? 1 : 0, src, 0, pix, pl, dl, q, 4u * t);
        if (!sh.ok) {
            fwd[t] = make_float4(0.f, 1.0f, 0.f, Wx);
            continue;
        }
        apply_shift(y, sh);
        fwd[t] = make_float4(sh.phat, sh.J, mc * xphat / sh.J, Wx);
        shv[2 * (size_t)t] = make_float4(__int_as_float(y.v[0].obj), y.v[0].xi0, y.v[0].xi1, __int_as_float(y.v[1].obj));
        shv[2 * (size_t)t + 1] = make_float4(y.v[1].xi0, y.v[1].xi1, y.len, y.pre_pdf);
    }
    flush_counters(st, a.counters);
}

// MIS work list: for the tasks of the chunk, every (task, neighbour l) pair
// that needs a shift -- all neighbours of a canonical task, the neighbours
// other than the source of a forward-shifted one, none after a failed forward
// shift, never an off-screen neighbour -- as g = t * K + l; term[g] = 0 for all.
__global__ void __launch_bounds__(kTB) k_mis_list(FrameArgs a, int mode, const int* __restrict__ links,
                                                  const uint2* __restrict__ items, const uint2* __restrict__ tasks,
                                                  const uint32_t* __restrict__ win, const float4* __restrict__ fwd,
                                                  float* __restrict__ term, IdxQueue lq) {
    const int P = a.s.P;
    const uint32_t K = (uint32_t)pass_K(a.s, mode);
    const uint32_t n = win[1];
    for (uint32_t t = blockIdx.x * kTB + threadIdx.x; t < n; t += gridDim.x * kTB) {
        uint32_t valid = 0;
        const uint2 task = tasks[t];
        const int c = (int)task.y;
        const uint2 item = items[task.x];
        const int pix = (int)item.x, pl = (int)(item.y & 0xFFFFu);
        // pairwise MIS: only the canonical sample is shifted into the neighbours
        const bool open = c == 0 || (fwd[t].x > 0.f && !(mode == 1 && a.s.mis_mode == 1));
        for (uint32_t l = 0; l < K; ++l) {
            term[(size_t)t * K + l] = 0.f;
            bool dom;
            if (mode == 2) {
                const int dpl = pl + bin_offset((int)l);
                dom = dpl >= 0 && dpl < a.s.n_bins;
            } else {
                dom = (mode == 0 ? links[pix] : links[(size_t)l * P + pix]) >= 0;
            }
            if (open && (int)l != c - 1 && dom) valid |= 1u << l;
        }
        uint32_t first;
        const bool fits = lq.alloc((uint32_t)__popc(valid), first);   // bounded by the chunk size
        if (fits)
            for (uint32_t l = 0; valid; ++l, valid >>= 1)
                if (valid & 1u) lq.buf[first++] = t * K + l;
    }
}

// MIS shifts of the listed pairs; blocks are dealt to the sub-lists round
// robin (and so append their rays to the ray sub-queue of the same index)
template <bool VEL>
TOF_TRACE_KERNEL k_mis(FrameArgs a, int mode, ResSet A, ResSet Bp, const int* __restrict__ links,
                       const uint2* __restrict__ items, const uint2* __restrict__ tasks, IdxQueue lq,
                       const float4* __restrict__ fwd, const float4* __restrict__ shv, float* __restrict__ term,
                       RayQueue q) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, kStackDepth, st};
    const Sens& s = a.s;
    const int P = s.P;
    const uint32_t K = (uint32_t)pass_K(s, mode);
    const uint32_t sub = blockIdx.x % kRaySubQueues;
    const uint32_t n = min(lq.count[sub * kCounterStride], lq.sub_cap);
    const uint32_t* list = lq.buf + (size_t)sub * lq.sub_cap;
    const uint32_t step = (gridDim.x / kRaySubQueues) * kTB;
    for (uint32_t i = (blockIdx.x / kRaySubQueues) * kTB + threadIdx.x; i < n; i += step) {
        const uint32_t g = list[i];
        const uint32_t t = g / K;
        const int l = (int)(g - t * K);
        const uint2 task = tasks[t];
        const int c = (int)task.y;
        const uint2 item = items[task.x];
        const int pix = (int)item.x, pl = (int)(item.y & 0xFFFFu);
        const int dpix = mode == 0 ? links[pix] : (mode == 1 ? links[(size_t)l * P + pix] : pix);
        const int dpl = mode == 2 ? pl + bin_offset(l) : pl;
        float Wx;
        Rec y;
        if (c == 0) {
            y = load_rec(A, (size_t)pl * P + pix, Wx);
        } else {
            const int src = cand_src(mode, links, P, pix, c);
            y = load_rec(mode == 0 ? Bp : A, (size_t)cand_plane(mode, pl, c) * P + src, Wx);
            const float4 s0 = shv[2 * (size_t)t], s1 = shv[2 * (size_t)t + 1];
            y.v[0] = VRef{__float_as_int(s0.x), s0.y, s0.z};
            y.v[1] = VRef{__float_as_int(s0.w), s1.x, s1.y};
            y.len = s1.z;
            y.pre_pdf = s1.w;
            y.phat = fwd[t].x;
        }
        const float dl = mode == 0 ? -gate_shift(s, a.F.g[0], a.F.g[1], pl)
                                   : (mode == 2 ? (float)(dpl - pl) * s.bw : 0.f);
        const ShiftOut sh = shift_path<VEL>(s, a.S, a.F, tr, y, 0, pix, mode == 0 ? 1 : 0, dpix, dpl, dl, q, g);
        if (sh.ok) term[g] = dom_M(s, mode, A, Bp, dpix) * sh.phat * sh.J;
    }
    flush_counters(st, a.counters);
}

// ---------------------------------------------------------------------------
// visibility of queued shift segments in the frame of `slot`; a blocked ray
// zeroes kill[owner] (the first one counts the shift as failed).  Two forms:
// persistent lanes that refill from the wave's share of the queue (k_vis),
// for trees deep enough that rays of one wave take very different numbers of
// steps, and one ray per lane (k_vis_lanes) for small scenes, where a ray is
// a few node visits and the refill bookkeeping costs more than the idle
// lanes it saves.
// ---------------------------------------------------------------------------
constexpr uint32_t kVisChunk = 128;   // rays per chunk of the persistent visibility waves
__global__ void __launch_bounds__(kTB) k_vis_lanes(FrameArgs a, int slot, RayQueue q, float* __restrict__ kill) {
    __shared__ uint32_t stk[kVisStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, kVisStackDepth, st};
    const SlotDev& G = slot ? a.F.g[1] : a.F.g[0];
    // blocks are dealt to the sub-queues round robin
    const uint32_t sub = blockIdx.x % kRaySubQueues;
    const uint32_t nb = gridDim.x / kRaySubQueues;
    const uint32_t n = min(q.count[sub * kCounterStride], q.sub_cap);
    const float4* buf = q.buf + 2 * (size_t)sub * q.sub_cap;
    for (uint32_t i = (blockIdx.x / kRaySubQueues) * kTB + threadIdx.x; i < n; i += nb * kTB) {
        const float4 r0 = buf[2 * (size_t)i], r1 = buf[2 * (size_t)i + 1];
        const Seg sg{mk(r0.x, r0.y, r0.z), mk(r1.x, r1.y, r1.z), r0.w};
        if (!tr.visible(G, sg)) {
            const uint32_t owner = __float_as_uint(r1.w);
            const float old = atomicExch(kill + (owner & ~kOwnerNewton), 0.f);
            if (old != 0.f) {
                st.c[ST_VISFAIL]++;
                if (owner & kOwnerNewton) st.c[ST_VISFAIL_NEWTON]++;
            }
        }
    }
    flush_counters(st, a.counters);
}

// WPE: the waves per SIMD it is compiled for (its register budget; the LDS
// stacks allow at most 6 waves of 128 lanes' stacks per SIMD)
template <int WPE>
__global__ void __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(WPE))) k_vis(FrameArgs a, int slot,
                                                                                    RayQueue q,
                                                                                    float* __restrict__ kill) {
    __shared__ uint32_t stk[kVisStackDepth * kTB];
    Counters st = {};
    const SlotDev& G = slot ? a.F.g[1] : a.F.g[0];
    // blocks are dealt to the sub-queues round robin; the waves of a
    // sub-queue's blocks take its chunks of kVisChunk rays round robin (a
    // short queue leaves the later waves without a chunk)
    constexpr uint32_t kWaves = kTB / 64;
    const uint32_t sub = blockIdx.x % kRaySubQueues;
    const uint32_t n = min(q.count[sub * kCounterStride], q.sub_cap);
    const uint32_t W = (gridDim.x / kRaySubQueues) * kWaves;
    const uint32_t w = (blockIdx.x / kRaySubQueues) * kWaves + threadIdx.x / 64;
    if ((uint64_t)w * kVisChunk < n) {
        const float4* buf = q.buf + 2 * (size_t)sub * q.sub_cap;
        trace_vis_chunks(a.S, G, buf, n, w, W, kVisChunk, kill, stk + threadIdx.x, kTB, kVisStackDepth, st);
    }
    flush_counters(st, a.counters);
}

// ---------------------------------------------------------------------------
// merge: weighted reservoir sampling over the candidates in order, W = sum/phat.
// Weights follow eq. GRIS_resampling_weight with the generalized balance
// heuristic from the terms of k_fwd and k_mis.  A selected neighbour sample is
// its source record with the fields its shift into q rewrote.
//
// A wave takes 64 consecutive items, whose tasks are contiguous.  Its lanes
// first take one item each (pixel, plane, confidences, staged in LDS), then
// one task each over the items' task range -- consecutive lanes read
// consecutive forward terms and MIS terms -- and leave each task's weight in
// LDS; then one item each again, drawing in candidate order from those
// weights (the same arithmetic, in the same order, as a lane that walks its
// item's candidates alone); then four lanes per item copy the winners'
// records, one float4 each, with the fields the shift rewrote (the same bits
// as decoding the record, patching it and encoding it again).
// ---------------------------------------------------------------------------
constexpr int kMergeWaves = 4;                   // waves per block of k_merge
constexpr int kMergeP4 = 2;                      // rounds of 16 records whose loads are issued together
// LDS of one merge wave, sized for the pass's K: per item its confidences
// (float4) and its selection (uint4), per task (64 (K + 1) at most) its
// weight and phat_q (float2), and under pairwise MIS per item the K
// neighbours' confidences (float)
__host__ __device__ __forceinline__ size_t merge_wave_lds(int K, bool pairwise) {
    return 64 * 16 + 64 * 16 + (size_t)64 * (K + 1) * 8 + (pairwise ? (size_t)64 * K * 4 : 0);
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// TPL: tasks a lane loads at once in the weight phase (the tile)
template <int TPL>
__global__ void __launch_bounds__(64 * kMergeWaves) k_merge(FrameArgs a, int mode, ResSet A, ResSet Bp,
                                                            const int* __restrict__ links,
                                                            const uint2* __restrict__ items,
                                                            const uint2* __restrict__ tasks,
                                                            const uint32_t* __restrict__ task0,
                                                            const uint32_t* __restrict__ count, uint32_t i0,
                                                            uint32_t ci, const uint32_t* __restrict__ win,
                                                            const float4* __restrict__ fwd,
                                                            const float* __restrict__ term,
                                                            const float4* __restrict__ shv, int round, ResSet out) {
    extern __shared__ __align__(16) unsigned char merge_lds[];
    const Sens& s = a.s;
    const int P = s.P;
    const int K = pass_K(s, mode);
    const int ncand = K + 1;
    const uint32_t ni = count[0];
    if (i0 >= ni) return;
    const uint32_t n = ni - i0 > ci ? i0 + ci : ni;
    const uint32_t tb = win[0];
    const int lane = (int)__lane_id();
    const int wv = (int)(threadIdx.x >> 6);
    const bool pw = mode == 1 && s.mis_mode == 1;
    unsigned char* lds = merge_lds + (size_t)wv * merge_wave_lds(K, pw);
    float4* s_it = (float4*)lds;                  // per item: M_q, M_tot, M_q / k_v, pairwise (1) or not (0)
    uint4* s_sel = (uint4*)(lds + 64 * 16);       // per item: source record, output record, task, W bits
    float2* s_w = (float2*)(lds + 2 * 64 * 16);   // per task: weight (-1: not a candidate), phat_q
    float* s_ml = (float*)(lds + 2 * 64 * 16 + (size_t)64 * (K + 1) * 8);   // per item: neighbour confidences (-1: no pixel)
    // wave-uniform loop (the shuffles below need every lane)
    for (uint32_t it0 = i0 + blockIdx.x * (64 * kMergeWaves) + 64 * (uint32_t)wv; it0 < n;
         it0 += gridDim.x * (64 * kMergeWaves)) {
        const uint32_t it = it0 + (uint32_t)lane;
        const bool have = it < n;
        // 1. one lane per item
        int pix = 0, pl = 0;
        uint32_t cm = 0, t0 = 0;
        if (have) {
            const uint2 item = items[it];
            pix = (int)item.x;
            pl = (int)(item.y & 0xFFFFu);
            cm = item.y >> 16;
            t0 = task0[it] - tb;
            const float mq = A.M[pix];
            // pairwise MIS: the neighbours' confidences and the canonical share
            float mtot = mq, mqk = mq;
            int kv = 0;
            if (pw) {
                for (int l = 0; l < K; ++l) {
                    const int dp = links[(size_t)l * P + pix];
                    const float ml = dp >= 0 ? A.M[dp] : -1.f;   // -1: no neighbour pixel
                    s_ml[lane * K + l] = ml;
                    if (dp >= 0) {
                        mtot += ml;
                        ++kv;
                    }
                }
                if (kv > 0) mqk = mq / (float)kv;
            }
            s_it[lane] = make_float4(mq, mtot, mqk, pw && kv > 0 ? 1.f : 0.f);
        }
        // the wave's task range: from its first item's first task to the end
        // of its last item's tasks
        const uint32_t tlo = __shfl(t0, 0, 64);
        const uint64_t live = __ballot(have);
        const int last = 63 - __clzll((long long)live);
        const uint32_t thi = __shfl(t0 + (uint32_t)__popc(cm), last, 64);
        const uint32_t nt = thi - tlo;
        wave_sync();
        // 2. one lane per task: its weight.  A lane takes TPL tasks at
        // a time and issues all their loads before it uses any of them, so
        // their memory latencies overlap.
        for (uint32_t j0 = 0; j0 < nt; j0 += 64 * TPL) {
            uint2 tk[TPL];
            float4 fw[TPL];
            float tm[TPL][kMaxK];
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const uint32_t j = j0 + 64 * (uint32_t)k + (uint32_t)lane;
                tk[k] = make_uint2(0u, 0u);
                fw[k] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int l = 0; l < kMaxK; ++l) tm[k][l] = 0.f;
                if (j < nt) {
                    const uint32_t t = tlo + j;
                    tk[k] = tasks[t];
                    fw[k] = fwd[t];
#pragma unroll
                    for (int l = 0; l < kMaxK; ++l)
                        if (l < K) tm[k][l] = term[(size_t)t * K + l];
                }
            }
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const uint32_t j = j0 + 64 * (uint32_t)k + (uint32_t)lane;
                if (j >= nt) continue;
                const int il = (int)(tk[k].x - it0), c = (int)tk[k].y;
                const float4 f4 = fw[k];
                const float phq = f4.x;
                float w = -1.f;
                if (c == 0 || phq > 0.f) {   // else the shift into q failed
                    const float4 iv = s_it[il];
                    const float mq = iv.x;
                    float m;
                    if (iv.w != 0.f) {   // pairwise
                        const float mtot = iv.y, mqk = iv.z;
                        const float* ml = &s_ml[il * K];
                        if (c == 0) {
                            m = 0.f;
                            const float qk = mqk * phq;
#pragma unroll
                            for (int l = 0; l < kMaxK; ++l)
                                if (l < K && ml[l] >= 0.f) m += (ml[l] + mqk) / mtot * (qk / (qk + tm[k][l]));
                        } else {
                            m = (ml[c - 1] + mqk) / mtot * (f4.z / (f4.z + mqk * phq));
                        }
                    } else {
                        float den = f4.z + mq * phq;
#pragma unroll
                        for (int l = 0; l < kMaxK; ++l)
                            if (l < K) den += tm[k][l];
                        m = (c == 0 ? mq * phq : f4.z) / den;
                    }
                    w = m * phq * f4.w * f4.y;
                    if (c > 0 && !(w > 0.f)) w = -1.f;
                }
                s_w[j] = make_float2(w, phq);
            }
        }
        wave_sync();
        // 3. one lane per item: the draw over its candidates in order
        uint32_t mkey = 0xFFFFFFFFu, mbit = 0u;   // mask word and bit this lane sets (none)
        if (have) {
            const uint64_t fp = full_pixel(s, pix);
            Draw ut;
            if (mode == 0) ut = philox(s.seed, fp, a.frame, PASS_TEMPORAL, 0, (uint64_t)pl);
            float ws = 0.f, sel_phat = 0.f;
            int sel = -1;
            uint32_t sel_t = 0;
            // one Philox draw serves four candidates; a group's draw is made
            // if any of its candidates has a weight.  The groups are drawn in
            // turn, each by every lane that needs it at once, so the wave
            // runs the generator once per group (the values do not depend
            // on when they are drawn).
            uint32_t need = 0;   // bit g: group g of four candidates has a weight
            for (int c = 0; c < ncand; ++c) {
                if (!((cm >> c) & 1u)) continue;
                const uint32_t t = t0 + (uint32_t)__popc(cm & ((1u << c) - 1u));
                if (s_w[t - tlo].x >= 0.f) need |= 1u << (c / 4);
            }
            auto group_draw = [&](int g) {
                if (mode == 0 || !((need >> g) & 1u)) return Draw{{0ull, 0ull, 0ull, 0ull}};
                return mode == 1 ? philox(s.seed, fp, a.frame, PASS_SPATIAL + (uint64_t)round, 2, (uint64_t)(pl * 2 + g))
                                 : philox(s.seed, fp, a.frame, PASS_BIN, 0, (uint64_t)(pl * 4 + g));
            };
            const Draw ug0 = group_draw(0), ug1 = group_draw(1), ug2 = group_draw(2);
            for (int c = 0; c < ncand; ++c) {
                if (!((cm >> c) & 1u)) continue;
                const uint32_t t = t0 + (uint32_t)__popc(cm & ((1u << c) - 1u));
                const float2 wp = s_w[t - tlo];
                const float w = wp.x;
                if (w < 0.f) continue;
                float u;
                if (mode == 0) {
                    u = ut.u_sel(c);
                } else {
                    const int g = c / 4, e4 = c % 4;
                    u = g == 0 ? ug0.u_sel(e4) : (g == 1 ? ug1.u_sel(e4) : ug2.u_sel(e4));
                }
                ws += w;
                if (u * ws < w) {
                    sel = c;
                    sel_phat = wp.y;
                    sel_t = t;
                }
            }
            // the winner: its record (plane-major index; bit 31 set for the
            // canonical one, whose fields stay), the output record, its task
            // and the new contribution weight; none: an empty output index
            uint4 wsel = make_uint4(0u, 0xFFFFFFFFu, 0u, 0u);
            if (sel >= 0 && ws > 0.f) {
                const uint32_t oidx = (uint32_t)pl * (uint32_t)P + (uint32_t)pix;
                const uint32_t sidx = sel == 0 ? (oidx | 0x80000000u)
                                               : (uint32_t)cand_plane(mode, pl, sel) * (uint32_t)P +
                                                     (uint32_t)cand_src(mode, links, P, pix, sel);
                wsel = make_uint4(sidx, oidx, sel_t, __float_as_uint(ws / sel_phat));
                mkey = (uint32_t)(pl >> 5) * (uint32_t)P + (uint32_t)pix;
                mbit = 1u << (pl & 31);
            }
            s_sel[lane] = wsel;
        } else {
            s_sel[lane] = make_uint4(0u, 0xFFFFFFFFu, 0u, 0u);
        }
        wave_sync();
        // 4. four lanes per item: float4 e of the winner's record, in four
        // rounds of 16 items; the loads of kMergeP4 rounds are issued before
        // any of their records is assembled (more would cost the registers
        // of a wave per SIMD); a lane reads only the parts its float4 needs.
        {
            const int e = lane & 3;
            const ResSet& srcset = mode == 0 ? Bp : A;
            for (int r0 = 0; r0 < 4; r0 += kMergeP4) {
                uint4 ws4[kMergeP4];
                float4 qv[kMergeP4], s0[kMergeP4], s1[kMergeP4];
                float phq[kMergeP4];
#pragma unroll
                for (int r = 0; r < kMergeP4; ++r) {
                    ws4[r] = s_sel[16 * (r0 + r) + (lane >> 2)];
                    qv[r] = s0[r] = s1[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                    phq[r] = 0.f;
                    if (ws4[r].y == 0xFFFFFFFFu) continue;
                    const bool canon = (ws4[r].x & 0x80000000u) != 0u;
                    const size_t si = canon ? (size_t)(ws4[r].x & 0x7FFFFFFFu) : (size_t)ws4[r].x;
                    const float4* q = (canon ? A : srcset).rec + si * kRecF4;
                    const size_t t = ws4[r].z;
                    if (canon || e == 1 || e == 3) qv[r] = q[e];
                    if (!canon) {
                        if (e == 0) {
                            s1[r] = shv[2 * t + 1];
                            phq[r] = fwd[t].x;
                        } else if (e == 1) {
                            s0[r] = shv[2 * t];
                        } else if (e == 2) {
                            s0[r] = shv[2 * t];
                            s1[r] = shv[2 * t + 1];
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < kMergeP4; ++r) {
                    if (ws4[r].y == 0xFFFFFFFFu) continue;
                    const bool canon = (ws4[r].x & 0x80000000u) != 0u;
                    const float Wn = __uint_as_float(ws4[r].w);
                    float4 v = qv[r];
                    if (canon) {
                        if (e == 0) v.x = Wn;
                    } else if (e == 0) {
                        v = make_float4(Wn, phq[r], s1[r].z, s1[r].w);
                    } else if (e == 1) {
                        // objects 0 and 1 of word 7 from the shift, object 2's low bits kept
                        const uint32_t w7 = (__float_as_uint(v.w) & 0xFF000000u) |
                                            ((uint32_t)__float_as_int(s0[r].x) & 0xFFFu) |
                                            (((uint32_t)__float_as_int(s0[r].w) & 0xFFFu) << 12);
                        v.w = __uint_as_float(w7);
                    } else if (e == 2) {
                        v = make_float4(s0[r].y, s0[r].z, s1[r].x, s1[r].y);
                    }
                    out.rec[(size_t)ws4[r].y * kRecF4 + e] = v;
                }
            }
        }
        // Items of one pixel are consecutive, so lanes that set bits of the
        // same mask word form runs: OR the bits down each run (a segmented
        // reduction over equal keys) and let its first lane write them with
        // one atomic instead of one per item.
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t k2 = __shfl_down(mkey, d, 64);
            const uint32_t b2 = __shfl_down(mbit, d, 64);
            if (lane + d < 64 && k2 == mkey) mbit |= b2;
        }
        const uint32_t kprev = __shfl_up(mkey, 1, 64);
        if (mbit && (lane == 0 || kprev != mkey)) atomicOr(out.mask + mkey, mbit);
        wave_sync();   // the next items' weights overwrite this wave's LDS
    }
}

// Shrink mapping (Sec. 4.4.2) of the gate reservoirs of pixels [p0, p0 + np):
// the winner x, drawn with the target f * 1[l in the wide gate], is moved by
// the path-length-aware shift of its own pixel with Delta l = (l - l0) / K +
// l0 - l; its contribution weight is multiplied by the shift's Jacobian / K.
// A path without a reconnection vertex (or under the naive shift) is kept
// only if it already lies in the gate.  A failed shrink, or a blocked
// visibility ray (which zeroes the record's W), leaves W = 0 for k_shrink_fin.
TOF_TRACE_KERNEL k_shrink(FrameArgs a, ResSet can, uint32_t p0, uint32_t np, RayQueue q) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, kStackDepth, st};
    const Sens& s = a.s;
    const int P = s.P, gp = s.n_bins;
    for (uint32_t t = blockIdx.x * kTB + threadIdx.x; t < np; t += gridDim.x * kTB) {
        const int pix = (int)(p0 + t);
        if (!mask_bit(can.mask, P, gp, pix)) continue;
        const size_t idx = (size_t)gp * P + pix;
        float W;
        Rec y = load_rec(can, idx, W);
        if (s.shift_mode != TOF_SHIFT_PATHLEN || y.k < 2) {
            if (!in_plane(s, gp, y.len)) rec_W(can, idx) = 0.f;
            continue;
        }
        const float l0 = s.gate_c, K = s.shrink_k, l = y.len;
        // (the shrink mapping is defined for path lengths only)
        const ShiftOut sh = shift_path<false>(s, a.S, a.F, tr, y, 0, pix, 0, pix, gp, (l - l0) / K + l0 - l, q,
                                       (uint32_t)pix * kRecWords);
        if (!sh.ok) {
            rec_W(can, idx) = 0.f;
            continue;
        }
        apply_shift(y, sh);
        y.phat = sh.phat;
        store_rec(can, idx, y, W * (sh.J / K));
    }
    flush_counters(st, a.counters);
}

// gate reservoirs left with W = 0 by the shrink mapping become empty
__global__ void k_shrink_fin(FrameArgs a, ResSet can) {
    const int P = a.s.P, gp = a.s.n_bins;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= P || !mask_bit(can.mask, P, gp, pix)) return;
    if (rec_W(can, (size_t)gp * P + pix) == 0.f)
        atomicAnd(can.mask + (size_t)(gp >> 5) * P + pix, ~(1u << (gp & 31)));
}

// ---------------------------------------------------------------------------
// Shrink mapping with R < 1 (Sec. 4.4.2): the gate's canonical reservoir
// (confidence M_n = M_init - M_w) and the wide-gate reservoir (M_w) are
// merged into the gate by GRIS with the generalized balance heuristic.
// k_shrink_mix shifts, per pixel of [p0, p0 + np): the gate sample into the
// wide gate (the expansion Delta l = K (l - l0) + l0 - l, the inverse of the
// shrink), whose |J| K p_hat gives the wide technique's density at it, and
// the wide sample into the gate (the shrink, |J| / K).  Paths that cannot be
// moved map by the identity where they lie in the gate.  scr[t] = (density
// of the wide technique at the gate sample, |J| of the shrunk wide sample,
// p_hat of the wide sample before the shrink); a blocked visibility ray of
// either shift zeroes its component (its owner).  After the rays,
// k_shrink_mix_fin forms the two resampling weights and selects one with a
// uniform of pass 17.
// ---------------------------------------------------------------------------
TOF_TRACE_KERNEL k_shrink_mix(FrameArgs a, ResSet can, ResSet wide, uint32_t p0, uint32_t np, RayQueue q,
                              float4* __restrict__ scr) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, kStackDepth, st};
    const Sens& s = a.s;
    const int P = s.P, gp = s.n_bins, wp = s.n_bins + 1;
    const float l0 = s.gate_c, K = s.shrink_k;
    for (uint32_t t = blockIdx.x * kTB + threadIdx.x; t < np; t += gridDim.x * kTB) {
        const int pix = (int)(p0 + t);
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        if (mask_bit(can.mask, P, gp, pix)) {   // the gate sample, expanded
            float W;
            const Rec y = load_rec(can, (size_t)gp * P + pix, W);
            if (s.shift_mode != TOF_SHIFT_PATHLEN || y.k < 2) {
                o.x = y.phat;
            } else {
                const float l = y.len;
                const ShiftOut e = shift_path<false>(s, a.S, a.F, tr, y, 0, pix, 0, pix, wp, K * (l - l0) + l0 - l, q,
                                                     4u * t);
                if (e.ok) o.x = e.phat * e.J * K;
            }
        }
        if (rec_W(wide, pix) > 0.f) {   // the wide sample, shrunk
            float W;
            Rec y = load_rec(wide, pix, W);
            o.z = y.phat;
            if (s.shift_mode != TOF_SHIFT_PATHLEN || y.k < 2) {
                if (in_plane(s, gp, y.len)) o.y = 1.f;
            } else {
                const float l = y.len;
                const ShiftOut sh = shift_path<false>(s, a.S, a.F, tr, y, 0, pix, 0, pix, gp, (l - l0) / K + l0 - l,
                                                      q, 4u * t + 1u);
                if (sh.ok) {
                    apply_shift(y, sh);
                    store_rec(wide, pix, y, W);
                    o.y = sh.J / K;
                }
            }
        }
        scr[t] = o;
    }
    flush_counters(st, a.counters);
}

__global__ void k_shrink_mix_fin(FrameArgs a, ResSet can, ResSet wide, uint32_t p0, uint32_t np,
                                 const float4* __restrict__ scr) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= np) return;
    const Sens& s = a.s;
    const int P = s.P, gp = s.n_bins;
    const int pix = (int)(p0 + t);
    const float Mw = (float)s.mw, Mn = (float)(s.m_init - s.mw);
    const float4 o = scr[t];
    const size_t ia = (size_t)gp * P + pix;
    const bool has_a = mask_bit(can.mask, P, gp, pix);
    float wa = 0.f, wb = 0.f, pa = 0.f, pb = 0.f;
    if (has_a) {
        pa = rec_phat(can, ia);
        wa = Mn * pa / (Mn * pa + Mw * o.x) * pa * rec_W(can, ia);
    }
    if (rec_W(wide, pix) > 0.f && o.y > 0.f) {
        pb = rec_phat(wide, pix);
        const float pw = o.z / o.y;   // the wide technique's density at the shrunk sample
        wb = Mw * pw / (Mn * pb + Mw * pw) * pb * rec_W(wide, pix) * o.y;
    }
    const float ws = wa + wb;
    uint32_t* mword = can.mask + (size_t)(gp >> 5) * P + pix;
    const uint32_t bit = 1u << (gp & 31);
    if (!(ws > 0.f)) {
        if (has_a) atomicAnd(mword, ~bit);
        return;
    }
    const Draw u = philox(s.seed, full_pixel(s, pix), a.frame, PASS_SHRINK_MIX, 0, 0);
    if (u.u(0) * ws < wb) {
        float W;
        const Rec y = load_rec(wide, pix, W);
        store_rec(can, ia, y, ws / pb);
        if (!has_a) atomicOr(mword, bit);
    } else {
        rec_W(can, ia) = ws / pa;
    }
}

// one plane passed through unchanged (the gate plane across the bin-axis pass)
__global__ void k_copy_plane(FrameArgs a, ResSet in, ResSet out, int pl) {
    const int P = a.s.P;
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= P || !mask_bit(in.mask, P, pl, pix)) return;
    const size_t i = (size_t)pl * P + pix;
#pragma unroll
    for (int e = 0; e < kRecF4; ++e) out.rec[kRecF4 * i + e] = in.rec[kRecF4 * i + e];
    atomicOr(out.mask + (size_t)(pl >> 5) * P + pix, 1u << (pl & 31));
}

// ---------------------------------------------------------------------------
// final shading (Sec. 3.2.4 step 4): I = phat(y) W per plane, divided by the
// gate/bin width; optional deterministic direct term; plain PT alongside.
// ---------------------------------------------------------------------------
// One thread per pixel and group of 32 planes (the planes of one mask word),
// the planes in turn: the pixel's mask word and direct term are read once,
// and at every plane the lanes of a wave read and write consecutive pixels.
// clear_pt: the deposits it reads are set back to zero (only the non-zero
// ones are written), so that the next frame finds the buffer cleared.
__global__ void __launch_bounds__(256) k_splat(FrameArgs a, ResSet shown, float* __restrict__ pt, int clear_pt,
                                               const float2* __restrict__ direct, float* __restrict__ out_image,
                                               float* __restrict__ out_hist, float* __restrict__ out_pt_image,
                                               float* __restrict__ out_pt_hist) {
    const Sens& s = a.s;
    const int P = s.P;
    const int pix = (int)(blockIdx.x * 256 + threadIdx.x);
    if (pix >= P) return;
    const int pl0 = 32 * (int)blockIdx.y, pl1 = min(s.B, pl0 + 32);
    const uint32_t mw = shown.mask[(size_t)blockIdx.y * P + pix];
    const float2 d = s.include_direct ? direct[pix] : make_float2(0.f, 0.f);
    for (int pl = pl0; pl < pl1; ++pl) {
        const size_t i = (size_t)pl * P + pix;
        float v = 0.f;
        if ((mw >> (pl - pl0)) & 1u) {
            const float2 wp = *(const float2*)(shown.rec + i * kRecF4);
            v = wp.x * wp.y;
        }
        float vp = pt[i];
        if (clear_pt && vp != 0.f) pt[i] = 0.f;
        if (s.include_direct && d.x > 0.f && in_plane(s, pl, d.y)) {
            v += d.x;
            vp += d.x;
        }
        const float inv = 1.0f / plane_width(s, pl);
        if (pl < s.n_bins) {
            if (out_hist) out_hist[i] = v * inv;
            if (out_pt_hist) out_pt_hist[i] = vp * inv;
        } else {
            if (out_image) out_image[pix] = v * inv;
            if (out_pt_image) out_pt_image[pix] = vp * inv;
        }
    }
}

inline unsigned grid_for(size_t n, unsigned bs, unsigned cap) {
    size_t g = (n + bs - 1) / bs;
    return (unsigned)std::max<size_t>(1, std::min<size_t>(g, cap));
}

}  // namespace

namespace tofh {

void launch_gbuffer(const FrameArgs& a, GBufOut out, hipStream_t st) {
    hipLaunchKernelGGL(k_gbuffer, dim3(grid_for(a.s.P, kTB, 1u << 30)), dim3(kTB), 0, st, a, out);
}
void launch_initial(const FrameArgs& a, ResSet can, ResSet wide, float* pt, float2* direct, hipStream_t st) {
    if (a.s.domain)
        hipLaunchKernelGGL(k_initial<true>, dim3(grid_for(a.s.P, kTB, 1u << 30)), dim3(kTB), 0, st, a, can, wide, pt,
                           direct);
    else
        hipLaunchKernelGGL(k_initial<false>, dim3(grid_for(a.s.P, kTB, 1u << 30)), dim3(kTB), 0, st, a, can, wide,
                           pt, direct);
}
void launch_reproject(const FrameArgs& a, const ResSet& can, const ResSet& prev, int* prev_pix, float* M_out,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_reproject, dim3(grid_for(a.s.P, 256, 1u << 30)), dim3(256), 0, st, a, can.M, prev.M,
                       prev_pix, M_out);
}
void launch_neighbours(const FrameArgs& a, int round, const ResSet& in, int* nb, float* M_out, hipStream_t st) {
    hipLaunchKernelGGL(k_neighbours, dim3(grid_for(a.s.P, 256, 1u << 30)), dim3(256), 0, st, a, round, in.M, nb,
                       M_out);
}
void launch_items(const FrameArgs& a, int mode, const ResSet& first, const ResSet& second, const int* links,
                  int ncand, uint2* items, uint32_t* task0, uint32_t* count, uint32_t* out_mask, uint32_t* wsum,
                  hipStream_t st) {
    // summaries for the passes over a pixel's own planes (temporal, spatial)
    // when the masks have at most 32 words; the bin-axis pass reads every word
    const int P = a.s.P;
    const uint32_t* s1 = nullptr;
    const uint32_t* s2 = nullptr;
    if (mode != 2 && a.s.mask_words <= 32 && wsum) {
        hipLaunchKernelGGL(k_word_sum, dim3(grid_for(P, 256, 1u << 30)), dim3(256), 0, st, first.mask, P,
                           a.s.mask_words, wsum);
        s1 = wsum;
        if (mode == 0) {
            hipLaunchKernelGGL(k_word_sum, dim3(grid_for(P, 256, 1u << 30)), dim3(256), 0, st, second.mask, P,
                               a.s.mask_words, wsum + P);
            s2 = wsum + P;
        }
    }
    hipLaunchKernelGGL(k_items, dim3(grid_for(P, 256, 1u << 30)), dim3(256), 0, st, a, mode, first.mask, second.mask,
                       links, ncand, items, task0, count, out_mask, s1, s2);
}
void launch_tasks(const uint2* items, const uint32_t* task0, const uint32_t* count, size_t i0, size_t ci,
                  uint2* tasks, uint32_t* win, hipStream_t st) {
    hipLaunchKernelGGL(k_tasks, dim3(grid_for(ci, 256, 16384)), dim3(256), 0, st, items, task0, count, (uint32_t)i0,
                       (uint32_t)ci, tasks, win);
}
void launch_fwd(const FrameArgs& a, int mode, const ResSet& A, const ResSet& Bp, const int* links,
                const uint2* items, const uint2* tasks, const uint32_t* win, float4* fwd, float4* shv,
                const RayQueue& q, unsigned grid, hipStream_t st) {
    if (a.s.domain)
        hipLaunchKernelGGL(k_fwd<true>, dim3(grid), dim3(kTB), 0, st, a, mode, A, Bp, links, items, tasks, win, fwd, shv,
                           q);
    else
        hipLaunchKernelGGL(k_fwd<false>, dim3(grid), dim3(kTB), 0, st, a, mode, A, Bp, links, items, tasks, win, fwd,
                           shv, q);
}
void launch_mis(const FrameArgs& a, int mode, const ResSet& A, const ResSet& Bp, const int* links,
                const uint2* items, const uint2* tasks, const uint32_t* win, const float4* fwd, const float4* shv,
                float* term, const IdxQueue& lq, const RayQueue& q, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_mis_list, dim3(grid), dim3(kTB), 0, st, a, mode, links, items, tasks, win, fwd, term, lq);
    if (a.s.domain)
        hipLaunchKernelGGL(k_mis<true>, dim3(grid), dim3(kTB), 0, st, a, mode, A, Bp, links, items, tasks, lq, fwd, shv,
                           term, q);
    else
        hipLaunchKernelGGL(k_mis<false>, dim3(grid), dim3(kTB), 0, st, a, mode, A, Bp, links, items, tasks, lq, fwd, shv,
                           term, q);
}
void launch_vis(const FrameArgs& a, int slot, const RayQueue& q, float* kill, unsigned grid, int waves,
                hipStream_t st) {
    if (a.S.n_tri >= kVisPersistentMinTris) {
        if (waves == 5)
            hipLaunchKernelGGL(k_vis<5>, dim3(grid), dim3(kTB), 0, st, a, slot, q, kill);
        else
            hipLaunchKernelGGL(k_vis<6>, dim3(grid), dim3(kTB), 0, st, a, slot, q, kill);
    } else
        hipLaunchKernelGGL(k_vis_lanes, dim3(std::min(grid, kShiftGrid)), dim3(kTB), 0, st, a, slot, q, kill);
}
void launch_merge(const FrameArgs& a, int mode, const ResSet& A, const ResSet& Bp, const int* links,
                  const uint2* items, const uint2* tasks, const uint32_t* task0, const uint32_t* count, size_t i0,
                  size_t ci,
                  const uint32_t* win, const float4* fwd, const float* term, const float4* shv, int round, ResSet out,
                  int tile, hipStream_t st) {
    const size_t lds = kMergeWaves * merge_wave_lds(pass_K(a.s, mode), mode == 1 && a.s.mis_mode == 1);
    const dim3 grid(grid_for(ci, 64 * kMergeWaves, 32768)), block(64 * kMergeWaves);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, block, lds, st, a, mode, A, Bp, links, items, tasks, task0, count,
                           (uint32_t)i0, (uint32_t)ci, win, fwd, term, shv, round, out);
    };
    if (tile == 1) go(k_merge<1>);
    else if (tile == 4) go(k_merge<4>);
    else go(k_merge<2>);
}
void launch_shrink(const FrameArgs& a, const ResSet& can, size_t p0, size_t np, const RayQueue& q, unsigned grid,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_shrink, dim3(grid), dim3(kTB), 0, st, a, can, (uint32_t)p0, (uint32_t)np, q);
}
void launch_shrink_mix(const FrameArgs& a, const ResSet& can, const ResSet& wide, size_t p0, size_t np,
                       const RayQueue& q, float4* scr, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_shrink_mix, dim3(grid), dim3(kTB), 0, st, a, can, wide, (uint32_t)p0, (uint32_t)np, q, scr);
}
void launch_shrink_mix_fin(const FrameArgs& a, const ResSet& can, const ResSet& wide, size_t p0, size_t np,
                           const float4* scr, hipStream_t st) {
    hipLaunchKernelGGL(k_shrink_mix_fin, dim3(grid_for(np, 256, 1u << 30)), dim3(256), 0, st, a, can, wide,
                       (uint32_t)p0, (uint32_t)np, scr);
}
void launch_shrink_fin(const FrameArgs& a, const ResSet& can, hipStream_t st) {
    hipLaunchKernelGGL(k_shrink_fin, dim3(grid_for(a.s.P, 256, 1u << 30)), dim3(256), 0, st, a, can);
}
void launch_copy_plane(const FrameArgs& a, const ResSet& in, const ResSet& out, int pl, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_plane, dim3(grid_for(a.s.P, 256, 1u << 30)), dim3(256), 0, st, a, in, out, pl);
}
void launch_splat(const FrameArgs& a, const ResSet& shown, float* pt, bool clear_pt, const float2* direct,
                  float* out_image, float* out_hist, float* out_pt_image, float* out_pt_hist, hipStream_t st) {
    const unsigned gx = (unsigned)((a.s.P + 255) / 256), gy = (unsigned)((a.s.B + 31) / 32);
    if (a.s.P > 0 && a.s.B > 0)
        hipLaunchKernelGGL(k_splat, dim3(gx, gy), dim3(256), 0, st, a, shown, pt, clear_pt ? 1 : 0, direct,
                           out_image, out_hist, out_pt_image, out_pt_hist);
}

}  // namespace tofh
