// Linear BVH construction on the GPU for one frame's world-space triangles:
// centroid bounds -> 30-bit Morton codes -> 4-pass LSD radix sort (8-bit
// digits, ballot-ranked stable scatter) -> binary hierarchy from the sorted
// codes (Karras, HPG 2012) -> bottom-up refit with per-node arrival counters.
// The binary tree is then collapsed into a 4-wide tree (every node at even
// depth keeps its grandchildren) whose 128-byte nodes carry the four child
// boxes, halving the chain of dependent node fetches of a traversal.
#include "tof_device.h"
#include "tof_internal.h"

using namespace tofd;

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;

__global__ void k_world_verts(const float4* __restrict__ lv, const int* __restrict__ vobj,
                              const float* __restrict__ xf, float4* __restrict__ wv, int nv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    float4 q = lv[i];
    int o = vobj[i];
    if (o < 0) {   // vertex referenced by no object
        wv[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    V3 p = xf_point(xf + 12 * o, mk(q.x, q.y, q.z));
    wv[i] = make_float4(p.x, p.y, p.z, 0.f);
}

__device__ __forceinline__ void tri_world(const int4* tv, const float4* wv, int t, V3& a, V3& b, V3& c) {
    int4 v = tv[t];
    a = ld3(wv, v.x);
    b = ld3(wv, v.y);
    c = ld3(wv, v.z);
}

__global__ void __launch_bounds__(256) k_centroid_bounds(const int4* __restrict__ tv, const float4* __restrict__ wv,
                                                         int T, float* __restrict__ block_bounds) {
    __shared__ float red[6][256];
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    if (t < T) {
        V3 a, b, c;
        tri_world(tv, wv, t, a, b, c);
        V3 m = (1.0f / 3.0f) * (a + b + c);
        lo[0] = hi[0] = m.x;
        lo[1] = hi[1] = m.y;
        lo[2] = hi[2] = m.z;
    }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = lo[k];
        red[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + off]);
                red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) block_bounds[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_reduce_bounds(const float* __restrict__ bb, int nb, float* __restrict__ out) {
    __shared__ float red[6][256];
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], bb[6 * i + k]);
            hi[k] = fmaxf(hi[k], bb[6 * i + 3 + k]);
        }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = lo[k];
        red[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + off]);
                red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v = (v * 0x00010001u) & 0xFF0000FFu;
    v = (v * 0x00000101u) & 0x0F00F00Fu;
    v = (v * 0x00000011u) & 0xC30C30C3u;
    v = (v * 0x00000005u) & 0x49249249u;
    return v;
}

__global__ void k_morton(const int4* __restrict__ tv, const float4* __restrict__ wv, int T,
                         const float* __restrict__ bounds, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    V3 a, b, c;
    tri_world(tv, wv, t, a, b, c);
    V3 m = (1.0f / 3.0f) * (a + b + c);
    float q[3] = {m.x, m.y, m.z};
    uint32_t code = 0;
    for (int k = 0; k < 3; ++k) {
        float ext = bounds[3 + k] - bounds[k];
        float f = ext > 0.f ? (q[k] - bounds[k]) / ext : 0.5f;
        f = fminf(fmaxf(f, 0.f), 1.f);
        uint32_t iv = min((uint32_t)(f * 1024.0f), 1023u);
        code |= spread10(iv) << (2 - k);
    }
    keys[t] = code;
    vals[t] = (uint32_t)t;
}

__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                              uint32_t* __restrict__ hist, int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of hist[256 * nblocks] (digit-major), one block of 1024 threads
__global__ void __launch_bounds__(1024) k_radix_scan(uint32_t* __restrict__ hist, int total) {
    __shared__ uint32_t part[1024];
    int chunk = (total + 1023) / 1024;
    int s0 = threadIdx.x * chunk, s1 = min(s0 + chunk, total);
    uint32_t sum = 0;
    for (int i = s0; i < s1; ++i) sum += hist[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int i = s0; i < s1; ++i) {
        uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

// stable scatter: items of a tile are ranked in order (round, then lane)
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                                 const uint32_t* __restrict__ vin, int n, int shift,
                                                                 const uint32_t* __restrict__ offs, int nblocks,
                                                                 uint32_t* __restrict__ kout,
                                                                 uint32_t* __restrict__ vout) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wave[kWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s_base[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    const int base = blockIdx.x * kSortTile;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < kSortItems; ++r) {
        int i = base + r * kSortThreads + threadIdx.x;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u, val = valid ? vin[i] : 0u;
        uint32_t digit = (key >> shift) & 255u;
        uint64_t match = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((digit >> b) & 1u);
            match &= ((digit >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = __popcll(match & lt);
        uint32_t cnt = __popcll(match);
        for (int k = threadIdx.x; k < kWaves * 256; k += kSortThreads) (&s_wave[0][0])[k] = 0u;
        __syncthreads();
        if (valid && rank == 0) s_wave[wave][digit] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pre = s_base[digit];
            for (int w = 0; w < wave; ++w) pre += s_wave[w][digit];
            uint32_t pos = pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += s_wave[w][threadIdx.x];
        s_base[threadIdx.x] += add;
        __syncthreads();
    }
}

__device__ __forceinline__ int delta(const uint32_t* keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint32_t a = keys[i], b = keys[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

// internal node i of the hierarchy over sorted keys (Karras 2012)
__global__ void k_karras(const uint32_t* __restrict__ keys, int n, Node* __restrict__ nodes, int* __restrict__ parent) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, n, i, i - d);
    int lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = delta(keys, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + min(d, 0);
    int lo = min(i, j), hi = max(i, j);
    int c0 = (lo == gamma) ? (int)(0x80000000u | (uint32_t)gamma) : gamma;
    int c1 = (hi == gamma + 1) ? (int)(0x80000000u | (uint32_t)(gamma + 1)) : gamma + 1;
    nodes[i].c0 = c0;
    nodes[i].c1 = c1;
    if (c0 < 0) parent[(n - 1) + gamma] = i;
    else parent[gamma] = i;
    if (c1 < 0) parent[(n - 1) + gamma + 1] = i;
    else parent[gamma + 1] = i;
    if (i == 0) parent[0] = -1;
}

__device__ __forceinline__ float pad_lo(float x) { return x - (fabsf(x) + 1.0f) * 9.5367431640625e-7f; }
__device__ __forceinline__ float pad_hi(float x) { return x + (fabsf(x) + 1.0f) * 9.5367431640625e-7f; }

__global__ void k_leaves_refit(const uint32_t* __restrict__ vals, const int4* __restrict__ tv,
                               const float4* __restrict__ wv, int n, Node* nodes, const int* __restrict__ parent,
                               uint32_t* flags, float4* __restrict__ leaves) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int t = (int)vals[k];
    V3 a, b, c;
    tri_world(tv, wv, t, a, b, c);
    leaves[3 * k] = make_float4(a.x, a.y, a.z, __int_as_float(t));
    leaves[3 * k + 1] = make_float4(b.x, b.y, b.z, 0.f);
    leaves[3 * k + 2] = make_float4(c.x, c.y, c.z, 0.f);
    float lo[3] = {pad_lo(fminf(a.x, fminf(b.x, c.x))), pad_lo(fminf(a.y, fminf(b.y, c.y))),
                   pad_lo(fminf(a.z, fminf(b.z, c.z)))};
    float hi[3] = {pad_hi(fmaxf(a.x, fmaxf(b.x, c.x))), pad_hi(fmaxf(a.y, fmaxf(b.y, c.y))),
                   pad_hi(fmaxf(a.z, fmaxf(b.z, c.z)))};
    int child = (int)(0x80000000u | (uint32_t)k);
    int node = parent[(n - 1) + k];
    while (node >= 0) {
        volatile Node* vn = nodes + node;
        bool left = vn->c0 == child;
        for (int q = 0; q < 3; ++q) {
            if (left) {
                vn->lo0[q] = lo[q];
                vn->hi0[q] = hi[q];
            } else {
                vn->lo1[q] = lo[q];
                vn->hi1[q] = hi[q];
            }
        }
        __threadfence();
        uint32_t old = atomicAdd(&flags[node], 1u);
        if (old == 0u) break;   // the sibling finishes this node
        __threadfence();
        for (int q = 0; q < 3; ++q) {
            lo[q] = fminf(vn->lo0[q], vn->lo1[q]);
            hi[q] = fmaxf(vn->hi0[q], vn->hi1[q]);
        }
        child = node;
        node = parent[node];
    }
}

__device__ __forceinline__ int depth_of(const int* __restrict__ parent, int i) {
    int d = 0;   // bounded walk: a tree over 30-bit codes and 32-bit indices is < 64 deep
    for (int p = parent[i]; p >= 0 && d < 4096; p = parent[p]) ++d;
    return d;
}

// even[i] = 1 for binary internal nodes at even depth (they become 4-wide nodes)
__global__ void k_even_depth(const int* __restrict__ parent, int ni, uint32_t* __restrict__ even,
                             uint32_t* __restrict__ map) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    uint32_t e = (depth_of(parent, i) & 1) == 0 ? 1u : 0u;
    even[i] = e;
    map[i] = e;   // scanned in place into the 4-wide node index
}

// one 4-wide node per even-depth binary node: its children, with every
// internal child replaced by that child's two children
__global__ void k_collapse(const Node* __restrict__ nodes, int ni, const uint32_t* __restrict__ even,
                           const uint32_t* __restrict__ map, Node4* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || !even[i]) return;
    float lo[4][3], hi[4][3];
    int ch[4];
    int n = 0;
    const Node& b = nodes[i];
    for (int side = 0; side < 2; ++side) {
        const int c = side ? b.c1 : b.c0;
        const float* clo = side ? b.lo1 : b.lo0;
        const float* chi = side ? b.hi1 : b.hi0;
        if (c < 0) {
            for (int q = 0; q < 3; ++q) {
                lo[n][q] = clo[q];
                hi[n][q] = chi[q];
            }
            ch[n++] = c;
        } else {
            const Node& g = nodes[c];
            for (int gs = 0; gs < 2; ++gs) {
                const int gc = gs ? g.c1 : g.c0;
                const float* glo = gs ? g.lo1 : g.lo0;
                const float* ghi = gs ? g.hi1 : g.hi0;
                for (int q = 0; q < 3; ++q) {
                    lo[n][q] = glo[q];
                    hi[n][q] = ghi[q];
                }
                ch[n++] = gc < 0 ? gc : (int)map[gc];
            }
        }
    }
    for (int j = n; j < 4; ++j) {
        for (int q = 0; q < 3; ++q) {
            lo[j][q] = 0.f;
            hi[j][q] = 0.f;
        }
        ch[j] = -1;
    }
    Node4 o;
    o.lox = make_float4(lo[0][0], lo[1][0], lo[2][0], lo[3][0]);
    o.loy = make_float4(lo[0][1], lo[1][1], lo[2][1], lo[3][1]);
    o.loz = make_float4(lo[0][2], lo[1][2], lo[2][2], lo[3][2]);
    o.hix = make_float4(hi[0][0], hi[1][0], hi[2][0], hi[3][0]);
    o.hiy = make_float4(hi[0][1], hi[1][1], hi[2][1], hi[3][1]);
    o.hiz = make_float4(hi[0][2], hi[1][2], hi[2][2], hi[3][2]);
    o.child = make_int4(ch[0], ch[1], ch[2], ch[3]);
    o.meta = make_int4(n, 0, 0, 0);
    out[map[i]] = o;
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

void launch_world_verts(const float4* lv, const int* vobj, const float* xf, float4* wv, int nv, hipStream_t st) {
    if (nv == 0) return;
    hipLaunchKernelGGL(k_world_verts, dim3(blocks_for(nv, 256)), dim3(256), 0, st, lv, vobj, xf, wv, nv);
}

size_t bvh_scratch_bytes(int T) {
    int nb = (T + kSortTile - 1) / kSortTile;
    int cb = (T + 255) / 256;
    return sizeof(uint32_t) * (4 * (size_t)T + 256 * (size_t)std::max(nb, 1) + (size_t)T) +
           sizeof(float) * (6 * (size_t)std::max(cb, 1) + 6) + 256;
}

// Build the BVH of T >= 1 triangles: binary nodes[T-1] and parent[2T-1]
// (build state), leaves[3T] and the 4-wide traversal nodes nodes4[T-1].
void launch_bvh_build(const int4* tv, const float4* wv, int T, Node* nodes, Node4* nodes4, float4* leaves,
                      int* parent, void* scratch, hipStream_t st) {
    if (T < 1) return;
    int nb = (T + kSortTile - 1) / kSortTile;
    int cb = (T + 255) / 256;
    uint32_t* keys = (uint32_t*)scratch;
    uint32_t* vals = keys + T;
    uint32_t* keys2 = vals + T;
    uint32_t* vals2 = keys2 + T;
    uint32_t* hist = vals2 + T;
    uint32_t* flags = hist + 256 * (size_t)std::max(nb, 1);
    float* bb = (float*)(flags + T);
    float* bounds = bb + 6 * (size_t)std::max(cb, 1);
    hipLaunchKernelGGL(k_centroid_bounds, dim3(cb), dim3(256), 0, st, tv, wv, T, bb);
    hipLaunchKernelGGL(k_reduce_bounds, dim3(1), dim3(256), 0, st, bb, cb, bounds);
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(T, 256)), dim3(256), 0, st, tv, wv, T, bounds, keys, vals);
    for (int pass = 0; pass < 4; ++pass) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, st, keys, T, shift, hist, nb);
        hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, hist, 256 * nb);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortThreads), 0, st, keys, vals, T, shift, hist, nb, keys2,
                           vals2);
        std::swap(keys, keys2);
        std::swap(vals, vals2);
    }
    if (T >= 2) {
        hipLaunchKernelGGL(k_karras, dim3(blocks_for(T - 1, 256)), dim3(256), 0, st, keys, T, nodes, parent);
        launch_fill_u32(flags, 0u, (size_t)T, st);
    } else {
        launch_fill_u32((uint32_t*)parent, 0xFFFFFFFFu, 1, st);
    }
    hipLaunchKernelGGL(k_leaves_refit, dim3(blocks_for(T, 256)), dim3(256), 0, st, vals, tv, wv, T, nodes, parent,
                       flags, leaves);
    if (T >= 2) {
        // the sort buffers are free again: even-depth flags and their scan
        uint32_t* even = keys2;
        uint32_t* map = vals2;
        const int ni = T - 1;
        hipLaunchKernelGGL(k_even_depth, dim3(blocks_for(ni, 256)), dim3(256), 0, st, parent, ni, even, map);
        hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, map, ni);
        hipLaunchKernelGGL(k_collapse, dim3(blocks_for(ni, 256)), dim3(256), 0, st, nodes, ni, even, map, nodes4);
    }
}

}  // namespace tofh
