// Per-frame geometry update on the GPU: object-space vertices to world space,
// triangles gathered into leaf order, and the 4-wide tree's boxes refit
// bottom-up, one launch per height level (the topology is built on the host:
// once per scene for the objects' trees, per frame for the small tree over
// the objects).  The world-space refit of a rigidly moving object keeps its
// tree valid and tight up to the rotation of the boxes.
#include "tof_device.h"
#include "tof_internal.h"

using namespace tofd;

namespace {

// wv = world positions (what the rays are traced against), wr = the vertices
// turned into world orientation about their object's origin (what the charts
// difference)
__global__ void k_world_verts(const float4* __restrict__ lv, const int* __restrict__ vobj,
                              const float* __restrict__ xf, float4* __restrict__ wv, float4* __restrict__ wr, int nv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    float4 q = lv[i];
    int o = vobj[i];
    if (o < 0) {   // vertex referenced by no object
        wv[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        wr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    V3 p = xf_point(xf + 12 * o, mk(q.x, q.y, q.z));
    V3 r = xf_dir(xf + 12 * o, mk(q.x, q.y, q.z));
    wv[i] = make_float4(p.x, p.y, p.z, 0.f);
    wr[i] = make_float4(r.x, r.y, r.z, 0.f);
}

// leaves[3s..3s+2] = world vertices of triangle leaf_tri[s] (w of the first = its id)
__global__ void k_leaf_gather(const int* __restrict__ leaf_tri, const int4* __restrict__ tv,
                              const float4* __restrict__ wv, int T, float4* __restrict__ leaves) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T) return;
    const int t = leaf_tri[s];
    const int4 v = tv[t];
    const float4 a = wv[v.x], b = wv[v.y], c = wv[v.z];
    leaves[3 * s] = make_float4(a.x, a.y, a.z, __int_as_float(t));
    leaves[3 * s + 1] = make_float4(b.x, b.y, b.z, 0.f);
    leaves[3 * s + 2] = make_float4(c.x, c.y, c.z, 0.f);
}

// boxes are widened by ~2^-20 relative (plus an absolute part) so that the
// FP32 slab test cannot reject a triangle lying on the box boundary
__device__ __forceinline__ float pad_lo(float x) { return x - (fabsf(x) + 1.0f) * 9.5367431640625e-7f; }
__device__ __forceinline__ float pad_hi(float x) { return x + (fabsf(x) + 1.0f) * 9.5367431640625e-7f; }

// smallest biased exponent b (scale 2^(b - 127)) with 255 * scale >= extent
__device__ __forceinline__ uint32_t quant_exp(float extent) {
    uint32_t b = 1;
    if (extent > 0.f) {
        const float need = extent * (1.0f / 255.0f);
        b = ((uint32_t)__float_as_int(need) >> 23) & 0xFFu;   // 2^(b-127) <= need (need normal, positive)
        if (__int_as_float((int)(b << 23)) < need) ++b;
        while (255.0f * __int_as_float((int)(b << 23)) < extent) ++b;   // the product rounds; at most a step
        b = b < 1 ? 1 : (b > 254 ? 254 : b);
    }
    return b;
}
// plane lo (down) or hi (up) of a child box in units of `scale` from org, 0..255
__device__ __forceinline__ uint32_t quant_lo(float x, float org, float scale) {
    const float q = floorf((x - org) / scale);
    float v = fminf(fmaxf(q, 0.f), 255.f);
    while (v > 0.f && fmaf(v, scale, org) > x) v -= 1.f;   // the decoded plane must not exceed x
    return (uint32_t)v;
}
__device__ __forceinline__ uint32_t quant_hi(float x, float org, float scale) {
    const float q = ceilf((x - org) / scale);
    float v = fminf(fmaxf(q, 0.f), 255.f);
    while (v < 255.f && fmaf(v, scale, org) < x) v += 1.f;   // the decoded plane must not fall below x
    return (uint32_t)v;
}

// one height level: every child box of the listed nodes from the level below;
// the exact boxes go to `nodes` (for the parents' refit), the quantized node
// that traversal reads to `nq`
__global__ void k_refit(Node4* nodes, NodeQ* __restrict__ nq, const uint32_t* __restrict__ order, int n,
                        const float4* __restrict__ leaves, int T) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Node4* nd = nodes + order[i];
    const int4 cc = nd->child;
    const int nc = nd->meta.x;
    const int ch[4] = {cc.x, cc.y, cc.z, cc.w};
    float lo[4][3], hi[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        for (int k = 0; k < 3; ++k) {
            lo[j][k] = 0.f;
            hi[j][k] = 0.f;
        }
        if (j >= nc) continue;
        float l[3] = {3e38f, 3e38f, 3e38f}, h[3] = {-3e38f, -3e38f, -3e38f};
        const uint32_t c = (uint32_t)ch[j];
        if (c & 0x80000000u) {
            const int first = (int)(c & 0x0FFFFFFFu), cnt = (int)((c >> 28) & 7u) + 1;
            for (int q = first; q < first + cnt && q < T; ++q)
                for (int v = 0; v < 3; ++v) {
                    const float4 p = leaves[3 * q + v];
                    l[0] = fminf(l[0], p.x);
                    l[1] = fminf(l[1], p.y);
                    l[2] = fminf(l[2], p.z);
                    h[0] = fmaxf(h[0], p.x);
                    h[1] = fmaxf(h[1], p.y);
                    h[2] = fmaxf(h[2], p.z);
                }
            for (int k = 0; k < 3; ++k) {
                l[k] = pad_lo(l[k]);
                h[k] = pad_hi(h[k]);
            }
        } else {
            const Node4& s = nodes[c];
            const int sn = s.meta.x;
            const float slx[4] = {s.lox.x, s.lox.y, s.lox.z, s.lox.w}, sly[4] = {s.loy.x, s.loy.y, s.loy.z, s.loy.w};
            const float slz[4] = {s.loz.x, s.loz.y, s.loz.z, s.loz.w}, shx[4] = {s.hix.x, s.hix.y, s.hix.z, s.hix.w};
            const float shy[4] = {s.hiy.x, s.hiy.y, s.hiy.z, s.hiy.w}, shz[4] = {s.hiz.x, s.hiz.y, s.hiz.z, s.hiz.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= sn) continue;
                l[0] = fminf(l[0], slx[q]);
                l[1] = fminf(l[1], sly[q]);
                l[2] = fminf(l[2], slz[q]);
                h[0] = fmaxf(h[0], shx[q]);
                h[1] = fmaxf(h[1], shy[q]);
                h[2] = fmaxf(h[2], shz[q]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            lo[j][k] = l[k];
            hi[j][k] = h[k];
        }
    }
    nd->lox = make_float4(lo[0][0], lo[1][0], lo[2][0], lo[3][0]);
    nd->loy = make_float4(lo[0][1], lo[1][1], lo[2][1], lo[3][1]);
    nd->loz = make_float4(lo[0][2], lo[1][2], lo[2][2], lo[3][2]);
    nd->hix = make_float4(hi[0][0], hi[1][0], hi[2][0], hi[3][0]);
    nd->hiy = make_float4(hi[0][1], hi[1][1], hi[2][1], hi[3][1]);
    nd->hiz = make_float4(hi[0][2], hi[1][2], hi[2][2], hi[3][2]);
    // quantized copy relative to the union of the children
    float org[3], sc[3];
    uint32_t eb[3], wl[3] = {0, 0, 0}, wh[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        float l = 3e38f, h = -3e38f;
        for (int j = 0; j < 4; ++j)
            if (j < nc) {
                l = fminf(l, lo[j][k]);
                h = fmaxf(h, hi[j][k]);
            }
        if (!(l <= h)) l = h = 0.f;
        org[k] = l;
        eb[k] = quant_exp(h - l);
        sc[k] = __int_as_float((int)(eb[k] << 23));
        for (int j = 0; j < 4; ++j) {
            const uint32_t ql = j < nc ? quant_lo(lo[j][k], l, sc[k]) : 0u;
            const uint32_t qh = j < nc ? quant_hi(hi[j][k], l, sc[k]) : 0u;
            wl[k] |= ql << (8 * j);
            wh[k] |= qh << (8 * j);
        }
    }
    NodeQ q;
    q.org = make_float4(org[0], org[1], org[2], 0.f);
    q.q0 = make_uint4(wl[0], wh[0], wl[1], wh[1]);
    q.q1 = make_uint4(wl[2], wh[2], eb[0] | (eb[1] << 8) | (eb[2] << 16), (uint32_t)nc);
    q.child = cc;
    nq[order[i]] = q;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

namespace tofh {

void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
    if (n == 0) return;
    unsigned g = (unsigned)std::min<size_t>(blocks_for(n, 256), 65536);
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, st, p, v, n);
}

void launch_world_verts(const float4* lv, const int* vobj, const float* xf, float4* wv, float4* wr, int nv,
                        hipStream_t st) {
    if (nv == 0) return;
    hipLaunchKernelGGL(k_world_verts, dim3(blocks_for(nv, 256)), dim3(256), 0, st, lv, vobj, xf, wv, wr, nv);
}

void launch_leaf_gather(const int* leaf_tri, const int4* tv, const float4* wv, int T, float4* leaves,
                        hipStream_t st) {
    if (T == 0) return;
    hipLaunchKernelGGL(k_leaf_gather, dim3(blocks_for(T, 256)), dim3(256), 0, st, leaf_tri, tv, wv, T, leaves);
}

void launch_refit(tofd::Node4* nodes, tofd::NodeQ* nq, const uint32_t* order, const std::vector<int>& level_off,
                  const float4* leaves, int T, hipStream_t st) {
    for (size_t l = 0; l + 1 < level_off.size(); ++l) {
        const int n = level_off[l + 1] - level_off[l];
        if (n <= 0) continue;
        hipLaunchKernelGGL(k_refit, dim3(blocks_for(n, 128)), dim3(128), 0, st, nodes, nq, order + level_off[l], n,
                           leaves, T);
    }
}

}  // namespace tofh
