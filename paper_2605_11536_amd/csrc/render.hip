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

constexpr int kTB = 128;   // lanes per block of the tracing kernels (LDS stack: 64 x 128 x 4 B = 32 KB)

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
        if (traverse(a.S, G, o, dir, 3.0e38f, false, h, stk + threadIdx.x, kTB, st)) {
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
// and is splatted into the plain path-tracing buffer.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTB) k_initial(FrameArgs a, ResSet can, float* __restrict__ pt,
                                                 float2* __restrict__ direct) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, st};
    const Sens& s = a.s;
    const SceneDev& S = a.S;
    int pix = blockIdx.x * kTB + threadIdx.x;
    if (pix < s.P) {
        const SlotDev& G = a.F.g[0];
        const int P = s.P;
        for (int w = 0; w < s.mask_words; ++w) can.mask[(size_t)w * P + pix] = 0u;
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
                float beta = 1.0f, pdf = 1.0f, plen = camera_leg(s, G, g);
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
                            if (!tr.all_visible(G, &sg, 1)) C = 0.f;
                        }
                        float li = plen + dl;
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
                            float w = C / ((float)s.m_init * pdf);
                            int planes[2] = {bin_of(s, li), (s.gate_en && in_plane(s, s.n_bins, li)) ? s.n_bins : -1};
                            for (int q = 0; q < 2; ++q) {
                                int pl = planes[q];
                                if (pl < 0) continue;
                                size_t idx = (size_t)pl * P + pix;
                                pt[idx] += C / pdf / (float)s.m_init;
                                uint32_t* mw = can.mask + (size_t)(pl >> 5) * P + pix;
                                uint32_t bit = 1u << (pl & 31);
                                uint32_t m = *mw;
                                if (!(m & bit)) {   // first candidate of this plane: always selected
                                    *mw = m | bit;
                                    store_rec(can, idx, rec, w);
                                } else {
                                    float ws = can.W[idx] + w;
                                    if (u.u(q) * ws < w) store_rec(can, idx, rec, ws);
                                    else can.W[idx] = ws;
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
                    plen += len(nx.p - xi.p);
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
                    can.W[idx] = can.W[idx] / can.phat[idx];
                }
            }
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
// work lists: mode 0 (temporal) ORs the canonical mask and the previous
// frame's mask at the reprojected pixel; mode 1 (spatial) ORs the input mask
// of the pixel and of its neighbours.  Also clears the output mask.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t union_word(const FrameArgs& a, int mode, const uint32_t* m1, const uint32_t* m2,
                                               const int* links, int nlinks, int w, int pix) {
    const int P = a.s.P;
    uint32_t m = m1[(size_t)w * P + pix];
    if (mode == 0) {
        int q = links[pix];
        if (q >= 0) m |= m2[(size_t)w * P + q];
    } else {
        for (int l = 0; l < nlinks; ++l) {
            int q = links[(size_t)l * P + pix];
            if (q >= 0) m |= m1[(size_t)w * P + q];
        }
    }
    return m;
}

__global__ void __launch_bounds__(256) k_items(FrameArgs a, int mode, const uint32_t* __restrict__ m1,
                                               const uint32_t* __restrict__ m2, const int* __restrict__ links,
                                               int nlinks, uint2* __restrict__ items, uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ out_mask) {
    __shared__ uint32_t s_scan[256];
    __shared__ uint32_t s_base;
    const int P = a.s.P;
    int pix = blockIdx.x * 256 + threadIdx.x;
    bool valid = pix < P && a.F.g[0].gb_obj[pix] >= 0;
    uint32_t c = 0;
    if (pix < P)
        for (int w = 0; w < a.s.mask_words; ++w) out_mask[(size_t)w * P + pix] = 0u;
    if (valid)
        for (int w = 0; w < a.s.mask_words; ++w) c += __popc(union_word(a, mode, m1, m2, links, nlinks, w, pix));
    s_scan[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = (int)threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0u;
        __syncthreads();
        s_scan[threadIdx.x] += v;
        __syncthreads();
    }
    if (threadIdx.x == 255) s_base = atomicAdd(count, s_scan[255]);
    __syncthreads();
    uint32_t pos = s_base + s_scan[threadIdx.x] - c;
    if (valid && c) {
        for (int w = 0; w < a.s.mask_words; ++w) {
            uint32_t m = union_word(a, mode, m1, m2, links, nlinks, w, pix);
            while (m) {
                int b = __ffs(m) - 1;
                m &= m - 1;
                items[pos++] = make_uint2((uint32_t)pix, (uint32_t)(32 * w + b));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// temporal GRIS (Sec. 3.2.3-3.2.4): canonical + previous final reservoir,
// generalized balance heuristic with confidence M, M_prev capped.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTB) k_temporal(FrameArgs a, ResSet can, ResSet prev, const int* __restrict__ prev_pix,
                                                  const uint2* __restrict__ items, const uint32_t* __restrict__ count,
                                                  ResSet out) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, st};
    const Sens& s = a.s;
    const int P = s.P;
    const uint32_t n = *count;
    for (uint32_t it = blockIdx.x * kTB + threadIdx.x; it < n; it += gridDim.x * kTB) {
        const uint2 item = items[it];
        const int pix = (int)item.x, pl = (int)item.y;
        const int qp = prev_pix[pix];
        const float mc = can.M[pix];
        const float mp = qp >= 0 ? fminf(prev.M[qp], s.m_cap) : 0.f;
        const Draw u = philox(s.seed, full_pixel(s, pix), a.frame, PASS_TEMPORAL, 0, (uint64_t)pl);
        const size_t idx = (size_t)pl * P + pix;
        const bool hasc = mask_bit(can.mask, P, pl, pix);
        const bool hasp = qp >= 0 && mask_bit(prev.mask, P, pl, qp);
        float ws = 0.f;
        bool have = false;
        Rec sel;
        for (int cand = 0; cand < 2; ++cand) {
            if (cand == 0 ? !hasc : !hasp) continue;
            float Wx;
            Rec x = cand == 0 ? load_rec(can, idx, Wx) : load_rec(prev, (size_t)pl * P + qp, Wx);
            ShiftOut sh;
            sh.ok = false;
            if (cand == 1 || qp >= 0)
                sh = shift_path(s, a.S, a.F, tr, x, cand == 0 ? 0 : 1, cand == 0 ? pix : qp, cand == 0 ? 1 : 0,
                                cand == 0 ? qp : pix, pl, 0.f);
            float w;
            if (cand == 0) {
                float ph = x.phat;
                float den = mc * ph;
                if (sh.ok) den += mp * sh.phat * sh.J;
                w = (mc * ph / den) * ph * Wx;
            } else {
                if (!sh.ok) continue;
                float A = mp * x.phat / sh.J;
                float m = A / (A + mc * sh.phat);
                w = m * sh.phat * Wx * sh.J;
                x = sh.y;
            }
            ws += w;
            if (u.u(cand) * ws < w) {
                sel = x;
                have = true;
            }
        }
        if (have && ws > 0.f) {
            store_rec(out, idx, sel, ws / sel.phat);
            atomicOr(out.mask + (size_t)(pl >> 5) * P + pix, 1u << (pl & 31));
        }
    }
    flush_counters(st, a.counters);
}

// ---------------------------------------------------------------------------
// spatial GRIS round: canonical + k neighbours, generalized balance heuristic;
// empty neighbour domains still enter every denominator through their M.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTB) k_spatial(FrameArgs a, int round, ResSet in, const int* __restrict__ nb,
                                                 const uint2* __restrict__ items, const uint32_t* __restrict__ count,
                                                 ResSet out) {
    __shared__ uint32_t stk[kStackDepth * kTB];
    Counters st = {};
    Tracer tr{a.S, stk + threadIdx.x, kTB, st};
    const Sens& s = a.s;
    const int P = s.P;
    const int K = s.k;
    const uint32_t n = *count;
    for (uint32_t it = blockIdx.x * kTB + threadIdx.x; it < n; it += gridDim.x * kTB) {
        const uint2 item = items[it];
        const int pix = (int)item.x, pl = (int)item.y;
        int nbs[kMaxK];
        float ms[kMaxK];
        for (int l = 0; l < K; ++l) {
            nbs[l] = nb[(size_t)l * P + pix];
            ms[l] = nbs[l] >= 0 ? in.M[nbs[l]] : 0.f;
        }
        const float mq = in.M[pix];
        const uint64_t fp = full_pixel(s, pix);
        float ws = 0.f;
        bool have = false;
        Rec sel;
        for (int cand = 0; cand <= K; ++cand) {
            const int src = cand == 0 ? pix : nbs[cand - 1];
            if (src < 0 || !mask_bit(in.mask, P, pl, src)) continue;
            float Wx;
            const Rec x = load_rec(in, (size_t)pl * P + src, Wx);
            Rec y = x;
            float phq = x.phat, Jj = 1.0f;
            float den = mq * x.phat;
            bool fail = false;
            // step -1 brings a neighbour's sample into q; steps 0..K-1 shift the
            // sample from q into every other domain for the MIS denominator
            for (int step = (cand == 0 ? 0 : -1); step < K; ++step) {
                if (step >= 0 && (step == cand - 1 || nbs[step] < 0)) continue;
                ShiftOut sh = shift_path(s, a.S, a.F, tr, step < 0 ? x : y, 0, step < 0 ? src : pix, 0,
                                         step < 0 ? pix : nbs[step], pl, 0.f);
                if (step < 0) {
                    if (!sh.ok) {
                        fail = true;
                        break;
                    }
                    y = sh.y;
                    phq = sh.phat;
                    Jj = sh.J;
                    den = ms[cand - 1] * x.phat / Jj + mq * phq;
                } else if (sh.ok) {
                    den += ms[step] * sh.phat * sh.J;
                }
            }
            if (fail) continue;
            float w = cand == 0 ? (mq * phq / den) * phq * Wx : ((ms[cand - 1] * x.phat / Jj) / den) * phq * Wx * Jj;
            float uu = philox(s.seed, fp, a.frame, PASS_SPATIAL + (uint64_t)round, 2, (uint64_t)(pl * 2 + cand / 4))
                           .u(cand % 4);
            ws += w;
            if (uu * ws < w) {
                sel = y;
                have = true;
            }
        }
        if (have && ws > 0.f) {
            store_rec(out, (size_t)pl * P + pix, sel, ws / sel.phat);
            atomicOr(out.mask + (size_t)(pl >> 5) * P + pix, 1u << (pl & 31));
        }
    }
    flush_counters(st, a.counters);
}

// ---------------------------------------------------------------------------
// final shading (Sec. 3.2.4 step 4): I = phat(y) W per plane, divided by the
// gate/bin width; optional deterministic direct term; plain PT alongside.
// ---------------------------------------------------------------------------
__global__ void k_splat(FrameArgs a, ResSet shown, const float* __restrict__ pt, const float2* __restrict__ direct,
                        float* __restrict__ out_image, float* __restrict__ out_hist, float* __restrict__ out_pt_image,
                        float* __restrict__ out_pt_hist) {
    const Sens& s = a.s;
    const size_t total = (size_t)s.B * s.P;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int pl = (int)(i / (size_t)s.P);
        const int pix = (int)(i - (size_t)pl * s.P);
        float v = 0.f;
        if (mask_bit(shown.mask, s.P, pl, pix)) v = shown.W[i] * shown.phat[i];
        float vp = pt[i];
        if (s.include_direct) {
            float2 d = direct[pix];
            if (d.x > 0.f && in_plane(s, pl, d.y)) {
                v += d.x;
                vp += d.x;
            }
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
void launch_initial(const FrameArgs& a, ResSet can, float* pt, float2* direct, hipStream_t st) {
    hipLaunchKernelGGL(k_initial, dim3(grid_for(a.s.P, kTB, 1u << 30)), dim3(kTB), 0, st, a, can, pt, direct);
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
                  int nlinks, uint2* items, uint32_t* count, uint32_t* out_mask, hipStream_t st) {
    hipLaunchKernelGGL(k_items, dim3(grid_for(a.s.P, 256, 1u << 30)), dim3(256), 0, st, a, mode, first.mask,
                       second.mask, links, nlinks, items, count, out_mask);
}
void launch_temporal(const FrameArgs& a, const ResSet& can, const ResSet& prev, const int* prev_pix,
                     const uint2* items, const uint32_t* count, size_t max_items, ResSet out, hipStream_t st) {
    hipLaunchKernelGGL(k_temporal, dim3(grid_for(max_items, kTB, 16384)), dim3(kTB), 0, st, a, can, prev, prev_pix,
                       items, count, out);
}
void launch_spatial(const FrameArgs& a, int round, const ResSet& in, const int* nb, const uint2* items,
                    const uint32_t* count, size_t max_items, ResSet out, hipStream_t st) {
    hipLaunchKernelGGL(k_spatial, dim3(grid_for(max_items, kTB, 16384)), dim3(kTB), 0, st, a, round, in, nb, items,
                       count, out);
}
void launch_splat(const FrameArgs& a, const ResSet& shown, const float* pt, const float2* direct, float* out_image,
                  float* out_hist, float* out_pt_image, float* out_pt_hist, hipStream_t st) {
    size_t total = (size_t)a.s.B * a.s.P;
    hipLaunchKernelGGL(k_splat, dim3(grid_for(total, 256, 65536)), dim3(256), 0, st, a, shown, pt, direct, out_image,
                       out_hist, out_pt_image, out_pt_hist);
}

}  // namespace tofh
