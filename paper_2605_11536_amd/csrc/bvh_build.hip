// Device construction of the objects' 4-wide trees (the alternative to the
// host's binned SAH in bvh_host.hip; the per-frame refit and the traversal
// are the same for both).  All mesh objects are built together:
//
//   1. per triangle, its object-space box; per object, the bounds of the
//      triangles' centroids (atomics on order-preserving integer images of
//      the floats);
//   2. keys (object ordinal << 30 | 30-bit Morton code of the centroid in its
//      object's centroid bounds, one scale for the three axes), sorted with a stable LSD radix sort, 8 bits
//      a pass (per-tile digit counts, a device-wide exclusive scan, a scatter
//      ranking each digit inside a wave from eight ballots);
//   3. agglomerative clustering in the sorted order (PLOC, Meister and
//      Bittner 2018): every cluster finds the cluster within R places, of the
//      same object, whose union box has the least surface area; mutual pairs
//      merge into a binary node, which takes the lower position; the array is
//      compacted by a scan; repeated until each object is one cluster.
//      Distances are symmetric and ties are broken by the pair's positions,
//      so the least pair of an object is always mutual and every round
//      merges;
//   4. at its creation each binary node takes the SAH-optimal collapse of
//      its subtree into 4-wide nodes from its children's (the host builder's
//      dynamic program: the least cost in up to j = 1..4 child slots, as a
//      leaf of at most 4 triangles, as a node, or spread over its children;
//      surface areas times triangle tests and node steps, 1 per step);
//   5. top-down, level by level, every 4-wide node takes the slots its
//      binary node's plan gives; children numbered by a scan, leaf slots
//      assigned in depth-first order so that each leaf's triangles are
//      contiguous.
//
// The host reads back only the small results (cluster counts per round, the
// 4-wide nodes' child links, their depths, the roots and object boxes);
// leaf_tri is written in place.
#include <chrono>

#include "tof_internal.h"

using namespace tofd;

#define HIP_TRY(expr)                \
    do {                             \
        if ((expr) != hipSuccess) {  \
            (void)hipGetLastError(); \
            return TOF_ERR_DEVICE;   \
        }                            \
    } while (0)

namespace {

constexpr int kTB = 256;            // threads per block of every kernel here
constexpr int kIPT = 8;             // elements per thread of the scan and sort tiles
constexpr int kTile = kTB * kIPT;   // 2048
constexpr int kRadius = 16;         // clustering window (places on either side; 32 and 64 were no better)
constexpr int kLeafMax = 4;         // triangles per leaf
constexpr float kNodeCost = 1.0f;   // a node step in triangle tests (the host builder's model)

__device__ __forceinline__ int fkey(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float fdec(int k) { return __int_as_float(k >= 0 ? k : k ^ 0x7FFFFFFF); }

__device__ __forceinline__ float box_area(float4 lo, float4 hi) {
    const float dx = fmaxf(hi.x - lo.x, 0.f), dy = fmaxf(hi.y - lo.y, 0.f), dz = fmaxf(hi.z - lo.z, 0.f);
    return 2.f * (dx * dy + dy * dz + dz * dx);
}
__device__ __forceinline__ float4 min4(float4 a, float4 b) {
    return make_float4(fminf(a.x, b.x), fminf(a.y, b.y), fminf(a.z, b.z), 0.f);
}
__device__ __forceinline__ float4 max4(float4 a, float4 b) {
    return make_float4(fmaxf(a.x, b.x), fmaxf(a.y, b.y), fmaxf(a.z, b.z), 0.f);
}

__device__ __forceinline__ void tri_box(const int4* __restrict__ tv, const float4* __restrict__ lv, int t, float4& lo,
                                        float4& hi) {
    const int4 v = tv[t];
    const float4 a = lv[v.x], b = lv[v.y], c = lv[v.z];
    lo = min4(min4(a, b), c);
    hi = max4(max4(a, b), c);
}

// mesh ordinal of slot s: the last m with m_slot[m] <= s (m_slot ascending, m_slot[M] = T)
__device__ __forceinline__ int ordinal_of(const int* __restrict__ m_slot, int M, int s) {
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m_slot[mid] <= s) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t expand10(uint32_t x) {
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of uint32 (tiles of kTile; the tile sums scanned
// by one block), the total left in total[0]
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_w, uint32_t* total) {
    const int lane = (int)__lane_id(), w = (int)(threadIdx.x >> 6);
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t off = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kTB / 64; ++k) {
        const uint32_t s = s_w[k];
        if (k < w) off += s;
        all += s;
    }
    __syncthreads();   // s_w may be reused by the caller
    *total = all;
    return off + x - v;
}

__global__ void __launch_bounds__(kTB) k_scan_partial(const uint32_t* __restrict__ in, size_t m,
                                                      uint32_t* __restrict__ part) {
    __shared__ uint32_t s_w[kTB / 64];
    const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kIPT;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k)
        if (base + k < m) s += in[base + k];
    uint32_t tot;
    (void)block_excl_scan(s, s_w, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// one block: part[0, nb) to its exclusive prefix, the sum to total[0]
__global__ void __launch_bounds__(kTB) k_scan_top(uint32_t* __restrict__ part, uint32_t nb,
                                                  uint32_t* __restrict__ total) {
    __shared__ uint32_t s_w[kTB / 64];
    const uint32_t per = (nb + kTB - 1) / kTB;
    const uint32_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    uint32_t s = 0;
    for (uint32_t b = b0; b < b1; ++b) s += part[b];
    uint32_t tot;
    uint32_t run = block_excl_scan(s, s_w, &tot);
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t v = part[b];
        part[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) total[0] = tot;
}

__global__ void __launch_bounds__(kTB) k_scan_final(const uint32_t* __restrict__ in, size_t m,
                                                    const uint32_t* __restrict__ part, uint32_t* __restrict__ out) {
    __shared__ uint32_t s_w[kTB / 64];
    const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kIPT;
    uint32_t v[kIPT], s = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        v[k] = base + k < m ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, s_w, &tot) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kIPT; ++k)
        if (base + k < m) {
            out[base + k] = run;
            run += v[k];
        }
}

// ---------------------------------------------------------------------------
// radix sort pieces (keys u64, values u32), digit (key >> shift) & 255;
// hist and offsets are digit-major: [digit * nb + tile]
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTB) k_rs_hist(const uint64_t* __restrict__ keys, size_t n, int shift,
                                                 uint32_t nb, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_c[256];
    s_c[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kTile;
#pragma unroll
    for (int r = 0; r < kIPT; ++r) {
        const size_t i = base + (size_t)r * kTB + threadIdx.x;
        if (i < n) atomicAdd(&s_c[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = s_c[threadIdx.x];
}

__global__ void __launch_bounds__(kTB) k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    size_t n, int shift, uint32_t nb, const uint32_t* __restrict__ offs,
                                                    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
    constexpr int kW = kTB / 64;
    __shared__ uint32_t s_base[256], s_run[256];
    __shared__ uint32_t s_wc[kW][256], s_wp[kW][256];
    const int lane = (int)__lane_id(), w = (int)(threadIdx.x >> 6);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    s_base[threadIdx.x] = offs[(size_t)threadIdx.x * nb + blockIdx.x];
    s_run[threadIdx.x] = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) s_wc[k][threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kTile;
    for (int r = 0; r < kIPT; ++r) {   // rounds in element order: the scatter is stable
        const size_t i = base + (size_t)r * kTB + threadIdx.x;
        const bool ok = i < n;
        uint64_t key = 0;
        uint32_t val = 0, d = 0;
        if (ok) {
            key = kin[i];
            val = vin[i];
            d = (uint32_t)(key >> shift) & 255u;
        }
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (ok && rank == 0) s_wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {   // per digit: the waves' starts in this round, then the running count
            const int dg = (int)threadIdx.x;
            uint32_t pre = s_run[dg];
#pragma unroll
            for (int k = 0; k < kW; ++k) {
                const uint32_t c = s_wc[k][dg];
                s_wp[k][dg] = pre;
                pre += c;
                s_wc[k][dg] = 0;
            }
            s_run[dg] = pre;
        }
        __syncthreads();
        if (ok) {
            const uint32_t dst = s_base[d] + s_wp[w][d] + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
    }
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
// per slot: the bounds of its object's centroids (6 ints per ordinal: lo xyz, hi xyz)
__global__ void __launch_bounds__(kTB) k_obj_bounds(const int4* __restrict__ tv, const float4* __restrict__ lv,
                                                    const int* __restrict__ m_slot, const int* __restrict__ m_tri,
                                                    int M, int T, int* __restrict__ ob) {
    const int s = blockIdx.x * kTB + threadIdx.x;
    if (s >= T) return;
    const int m = ordinal_of(m_slot, M, s);
    const int t = m_tri[m] + (s - m_slot[m]);
    float4 lo, hi;
    tri_box(tv, lv, t, lo, hi);
    const float c[3] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z)};
    int* o = ob + 6 * (size_t)m;
    for (int k = 0; k < 3; ++k) {
        atomicMin(o + k, fkey(c[k]));
        atomicMax(o + 3 + k, fkey(c[k]));
    }
}

__global__ void __launch_bounds__(kTB) k_morton(const int4* __restrict__ tv, const float4* __restrict__ lv,
                                                const int* __restrict__ m_slot, const int* __restrict__ m_tri, int M,
                                                int T, const int* __restrict__ ob, uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals) {
    const int s = blockIdx.x * kTB + threadIdx.x;
    if (s >= T) return;
    const int m = ordinal_of(m_slot, M, s);
    const int t = m_tri[m] + (s - m_slot[m]);
    float4 lo, hi;
    tri_box(tv, lv, t, lo, hi);
    const float c[3] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z)};
    const int* o = ob + 6 * (size_t)m;
    // one scale for the three axes (the largest extent): a flat object keeps
    // a flat curve instead of having its thin axis stretched to full range
    float e = 0.f;
    for (int k = 0; k < 3; ++k) e = fmaxf(e, fdec(o[3 + k]) - fdec(o[k]));
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        const float u = e > 0.f ? (c[k] - fdec(o[k])) / e : 0.f;
        q[k] = (uint32_t)fminf(fmaxf(u * 1024.f, 0.f), 1023.f);
    }
    const uint32_t code = (expand10(q[0]) << 2) | (expand10(q[1]) << 1) | expand10(q[2]);
    keys[s] = ((uint64_t)m << 30) | code;
    vals[s] = (uint32_t)t;
}

// ---------------------------------------------------------------------------
// clustering
// ---------------------------------------------------------------------------
struct Clusters {
    float4* lo;
    float4* hi;
    int* ref;   // >= 0 binary node, < 0: ~triangle
    int* obj;
};
struct BinTree {
    int2* child;
    float4* lo;
    float4* hi;
    int* count;
    float4* c;   // C(n, j), j = 1..4: least cost of the subtree in up to j child slots
    int* plan;   // bit 0: a node (else one leaf); bits 1-2: left child's slots as a node;
                 // bits 2j+1..2j+2 for j = 2..4: left child's slots when spread over j (0: one slot)
};

__global__ void __launch_bounds__(kTB) k_init_clusters(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals, int T,
                                                       const int4* __restrict__ tv, const float4* __restrict__ lv,
                                                       Clusters c) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= T) return;
    const int t = (int)vals[i];
    float4 lo, hi;
    tri_box(tv, lv, t, lo, hi);
    c.lo[i] = lo;
    c.hi[i] = hi;
    c.ref[i] = ~t;
    c.obj[i] = (int)(keys[i] >> 30);
}

__global__ void __launch_bounds__(kTB) k_nearest(Clusters c, int n, int* __restrict__ nn) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= n) return;
    const float4 li = c.lo[i], hi = c.hi[i];
    const int o = c.obj[i];
    float bd = 3.0e38f;
    int bj = -1;
    const int j0 = max(0, i - kRadius), j1 = min(n - 1, i + kRadius);
    for (int j = j0; j <= j1; ++j) {
        if (j == i || c.obj[j] != o) continue;
        const float d = box_area(min4(li, c.lo[j]), max4(hi, c.hi[j]));
        // the pair order (d, lower position, higher position): with i fixed,
        // a smaller partner position is a smaller pair in both cases
        bool better = d < bd;
        if (!better && d == bd && bj >= 0) {
            const int pa = min(i, j), qa = max(i, j), pb = min(i, bj), qb = max(i, bj);
            better = pa < pb || (pa == pb && qa < qb);
        }
        if (better) {
            bd = d;
            bj = j;
        }
    }
    nn[i] = bj;
}

// keep[i]: cluster i survives the round (a pair lives on at its lower
// position); make[i]: it is the lower end of a mutual pair
__global__ void __launch_bounds__(kTB) k_pairs(const int* __restrict__ nn, int n, uint32_t* __restrict__ keep,
                                               uint32_t* __restrict__ make) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= n) return;
    const int j = nn[i];
    const bool mutual = j >= 0 && j < n && nn[j] == i;
    keep[i] = (mutual && j < i) ? 0u : 1u;
    make[i] = (mutual && i < j) ? 1u : 0u;
}

// C(ref, j) for j = 1..4 (a triangle: a leaf of one, its area)
__device__ __forceinline__ float4 ref_cost(const BinTree& b, int ref, float area) {
    return ref < 0 ? make_float4(area, area, area, area) : b.c[ref];
}
__device__ __forceinline__ float cj(const float4& c, int j) {
    return j == 1 ? c.x : (j == 2 ? c.y : (j == 3 ? c.z : c.w));
}

__global__ void __launch_bounds__(kTB) k_merge_round(Clusters in, int n, const int* __restrict__ nn,
                                                     const uint32_t* __restrict__ keep,
                                                     const uint32_t* __restrict__ pos,
                                                     const uint32_t* __restrict__ make,
                                                     const uint32_t* __restrict__ mk_pos, int node_base, BinTree b,
                                                     Clusters out) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= n || !keep[i]) return;
    const uint32_t p = pos[i];
    float4 lo = in.lo[i], hi = in.hi[i];
    int ref = in.ref[i];
    if (make[i]) {
        const int j = nn[i];
        const int id = node_base + (int)mk_pos[i];
        const float4 lj = in.lo[j], hj = in.hi[j];
        const int rj = in.ref[j];
        const float4 ulo = min4(lo, lj), uhi = max4(hi, hj);
        const int cnt = (ref < 0 ? 1 : b.count[ref]) + (rj < 0 ? 1 : b.count[rj]);
        const float4 cl = ref_cost(b, ref, box_area(lo, hi)), cr = ref_cost(b, rj, box_area(lj, hj));
        // the SAH-optimal collapse into 4-wide nodes, one binary node at a
        // time (its children were made in earlier rounds): as one leaf, as a
        // node over its children spread into 4 slots, or (for a parent with
        // j >= 2 slots to give) spread itself
        const float A = box_area(ulo, uhi);
        auto spread = [&](int j, int& kb) {
            float best = 3.0e38f;
            kb = 0;
            for (int k = 1; k < j; ++k) {
                const float v = cj(cl, k) + cj(cr, j - k);
                if (v < best) {
                    best = v;
                    kb = k;
                }
            }
            return best;
        };
        int k4 = 0;
        const float as_node = A * kNodeCost + spread(4, k4);
        const float leaf = cnt <= kLeafMax ? A * (float)cnt : 3.0e38f;
        const bool node = as_node < leaf;
        const float c1 = node ? as_node : leaf;
        float cjs[3];
        int plan = (node ? 1 : 0) | (k4 << 1);
        for (int j = 2; j <= 4; ++j) {
            int k = 0;
            const float d = spread(j, k);
            cjs[j - 2] = d < c1 ? d : c1;
            plan |= (d < c1 ? k : 0) << (2 * j - 1 + 2);
        }
        b.child[id] = make_int2(ref, rj);
        b.lo[id] = ulo;
        b.hi[id] = uhi;
        b.count[id] = cnt;
        b.c[id] = make_float4(c1, cjs[0], cjs[1], cjs[2]);
        b.plan[id] = plan;
        lo = ulo;
        hi = uhi;
        ref = id;
    }
    out.lo[p] = lo;
    out.hi[p] = hi;
    out.ref[p] = ref;
    out.obj[p] = in.obj[i];
}

// ---------------------------------------------------------------------------
// 4-wide collapse
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool openable(const BinTree& b, int ref) { return ref >= 0 && (b.plan[ref] & 1); }
// left child's slots when ref's subtree is spread over j >= 2 slots (0: one slot)
__device__ __forceinline__ int spread_of(const BinTree& b, int ref, int j) {
    return ref < 0 ? 0 : (b.plan[ref] >> (2 * j + 1)) & 3;
}
__device__ __forceinline__ int ref_count(const BinTree& b, int ref) { return ref < 0 ? 1 : b.count[ref]; }

// children of a 4-wide node made from binary node r: its children spread
// over 4 slots as the collapse chose (left child k4 slots, the right one
// 4 - k4; a subtree given j >= 2 slots spreads further or takes one)
__device__ __forceinline__ int gather_kids(const BinTree& b, int r, int kids[4]) {
    const int2 c = b.child[r];
    const int k4 = (b.plan[r] >> 1) & 3;
    int st_ref[4], st_j[4], sp = 0, nk = 0;
    st_ref[sp] = c.y;   // right after left: a stack
    st_j[sp++] = 4 - k4;
    st_ref[sp] = c.x;
    st_j[sp++] = k4;
    while (sp > 0 && nk < 4) {
        const int x = st_ref[--sp], j = st_j[sp];
        const int k = j >= 2 ? spread_of(b, x, j) : 0;
        if (k == 0) {
            kids[nk++] = x;
        } else if (sp + 2 <= 4) {
            const int2 cx = b.child[x];
            st_ref[sp] = cx.y;
            st_j[sp++] = j - k;
            st_ref[sp] = cx.x;
            st_j[sp++] = k;
        }
    }
    return nk;
}

// the triangles of a leaf subtree into leaf_tri[first ...], left to right
__device__ __forceinline__ void emit_leaf(const BinTree& b, int ref, int first, int count, int* __restrict__ leaf_tri) {
    int stack[8];
    int sp = 0, k = 0;
    stack[sp++] = ref;
    while (sp > 0) {
        const int r = stack[--sp];
        if (r < 0) {
            if (k < count) leaf_tri[first + k] = ~r;
            ++k;
        } else if (sp + 2 <= 8) {
            const int2 c = b.child[r];
            stack[sp++] = c.y;
            stack[sp++] = c.x;
        }
    }
}

// per object's final cluster: a root that is one leaf gets its reference and
// its slots; others are marked for a node (need[m] = binary root + 1)
__global__ void __launch_bounds__(kTB) k_roots(Clusters c, int n, BinTree b, const int* __restrict__ m_slot,
                                               int* __restrict__ root, int* __restrict__ need,
                                               int* __restrict__ leaf_tri) {
    const int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= n) return;
    const int m = c.obj[i], ref = c.ref[i];
    const int first = m_slot[m];
    if (!openable(b, ref)) {
        const int cnt = ref_count(b, ref);
        root[m] = (int)(0x80000000u | ((uint32_t)(cnt - 1) << 28) | (uint32_t)first);
        need[m] = 0;
        emit_leaf(b, ref, first, cnt, leaf_tri);
    } else {
        root[m] = 0;
        need[m] = ref + 1;
    }
}

// frontier entry: (binary node, 4-wide node position, first leaf slot, 0)
__global__ void __launch_bounds__(kTB) k_collapse_count(const int4* __restrict__ F, int nf, BinTree b,
                                                        uint32_t* __restrict__ cnt) {
    const int e = blockIdx.x * kTB + threadIdx.x;
    if (e >= nf) return;
    int kids[4];
    const int nk = gather_kids(b, F[e].x, kids);
    uint32_t c = 0;
    for (int k = 0; k < nk; ++k) c += openable(b, kids[k]) ? 1u : 0u;
    cnt[e] = c;
}

__global__ void __launch_bounds__(kTB) k_collapse_write(const int4* __restrict__ F, int nf, BinTree b,
                                                        const uint32_t* __restrict__ off, int next_pos, int node_base,
                                                        int depth, int4* __restrict__ nd_child,
                                                        int* __restrict__ nd_nc, int* __restrict__ nd_depth,
                                                        int4* __restrict__ Fn, int* __restrict__ leaf_tri) {
    const int e = blockIdx.x * kTB + threadIdx.x;
    if (e >= nf) return;
    const int4 f = F[e];
    int kids[4];
    const int nk = gather_kids(b, f.x, kids);
    int refs[4] = {-1, -1, -1, -1};
    int slot = f.z;
    uint32_t r = 0;
    for (int k = 0; k < nk; ++k) {
        const int cn = ref_count(b, kids[k]);
        if (openable(b, kids[k])) {
            const uint32_t q = off[e] + r++;
            const int pos = next_pos + (int)q;
            refs[k] = node_base + pos;
            Fn[q] = make_int4(kids[k], pos, slot, 0);
        } else {
            refs[k] = (int)(0x80000000u | ((uint32_t)(cn - 1) << 28) | (uint32_t)slot);
            emit_leaf(b, kids[k], slot, cn, leaf_tri);
        }
        slot += cn;
    }
    nd_child[f.y] = make_int4(refs[0], refs[1], refs[2], refs[3]);
    nd_nc[f.y] = nk;
    nd_depth[f.y] = depth;
}

unsigned blocks_for(size_t n) { return (unsigned)std::max<size_t>(1, (n + kTB - 1) / kTB); }
unsigned tiles_for(size_t n) { return (unsigned)std::max<size_t>(1, (n + kTile - 1) / kTile); }

// carves the workspace front to back (256-byte aligned pieces)
struct Carve {
    char* p;
    size_t left;
    bool ok = true;
    template <typename T>
    T* take(size_t count) {
        const size_t bytes = (sizeof(T) * count + 255) & ~(size_t)255;
        if (bytes > left) {
            ok = false;
            return nullptr;
        }
        T* r = (T*)p;
        p += bytes;
        left -= bytes;
        return r;
    }
};

struct Scan {
    uint32_t* part;
    uint32_t* total;
    // out = exclusive prefix of in[0, m); returns the sum (a blocking read)
    hipError_t run(const uint32_t* in, size_t m, uint32_t* out, uint32_t* sum) {
        const unsigned nt = tiles_for(m);
        hipLaunchKernelGGL(k_scan_partial, dim3(nt), dim3(kTB), 0, 0, in, m, part);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTB), 0, 0, part, nt, total);
        hipLaunchKernelGGL(k_scan_final, dim3(nt), dim3(kTB), 0, 0, in, m, part, out);
        if (!sum) return hipGetLastError();
        return hipMemcpy(sum, total, sizeof(uint32_t), hipMemcpyDeviceToHost);
    }
};

}  // namespace

namespace tofh {

size_t blas_build_bytes(size_t T, size_t M) {
    const size_t nt = std::max<size_t>(1, (T + kTile - 1) / kTile);
    const size_t scan_max = std::max(T, 256 * nt);
    const size_t per_t = 2 * 8 + 2 * 4            // keys, values
                         + 2 * (16 + 16 + 4 + 4)  // clusters
                         + 4 + 4 * 4              // neighbours, keep, make and their scans
                         + 8 + 16 + 16 + 4 + 16 + 4  // binary nodes
                         + 2 * 16 + 4              // frontiers, child counts
                         + 16 + 4 + 4;             // 4-wide nodes
    return per_t * (T + 1) + 2 * 4 * 256 * nt + 4 * ((scan_max + kTile - 1) / kTile + 1) + 64 * (M + 1) +
           64 * 256 + 4096;
}

tof_status build_blas_device(void* work, size_t work_bytes, const int4* tv, const float4* lv,
                             const std::vector<int>& m_slot, const std::vector<int>& m_tri, int node_base,
                             int* leaf_tri, BlasResult& res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int M = (int)m_tri.size();
    const int T = m_slot.empty() ? 0 : m_slot.back();
    res.nodes.clear();
    res.heights.clear();
    res.roots.assign(M, -1);
    res.lbox.assign(6 * (size_t)M, 0.f);
    res.rounds = 0;
    if (T == 0) return TOF_OK;
    if (T >= (1 << 28) || M >= (1 << 24)) return TOF_ERR_INVALID_SCENE;
    const size_t nt = tiles_for(T);
    Carve cv{(char*)work, work_bytes};
    uint64_t* keys[2] = {cv.take<uint64_t>(T), cv.take<uint64_t>(T)};
    uint32_t* vals[2] = {cv.take<uint32_t>(T), cv.take<uint32_t>(T)};
    Clusters cl[2];
    for (auto& c : cl) {
        c.lo = cv.take<float4>(T);
        c.hi = cv.take<float4>(T);
        c.ref = cv.take<int>(T);
        c.obj = cv.take<int>(T);
    }
    int* nn = cv.take<int>(T);
    uint32_t* keep = cv.take<uint32_t>(T);
    uint32_t* make = cv.take<uint32_t>(T);
    uint32_t* pos = cv.take<uint32_t>(T);
    uint32_t* mk_pos = cv.take<uint32_t>(T);
    BinTree b;
    b.child = cv.take<int2>(T);
    b.lo = cv.take<float4>(T);
    b.hi = cv.take<float4>(T);
    b.count = cv.take<int>(T);
    b.c = cv.take<float4>(T);
    b.plan = cv.take<int>(T);
    int4* F[2] = {cv.take<int4>(T), cv.take<int4>(T)};
    uint32_t* fcnt = cv.take<uint32_t>(T);
    int4* nd_child = cv.take<int4>(T);
    int* nd_nc = cv.take<int>(T);
    int* nd_depth = cv.take<int>(T);
    uint32_t* hist = cv.take<uint32_t>(256 * nt);
    uint32_t* hoff = cv.take<uint32_t>(256 * nt);
    const size_t scan_max = std::max<size_t>(T, 256 * nt);
    Scan sc{cv.take<uint32_t>((scan_max + kTile - 1) / kTile + 1), cv.take<uint32_t>(16)};
    int* d_mslot = cv.take<int>(M + 1);
    int* d_mtri = cv.take<int>(M);
    int* ob = cv.take<int>(6 * (size_t)M);
    int* root = cv.take<int>(M);
    int* need = cv.take<int>(M);
    if (!cv.ok) return TOF_ERR_OUT_OF_MEMORY;

    // 1-2. object bounds and keys
    std::vector<int> ob0(6 * (size_t)M);
    for (int m = 0; m < M; ++m)
        for (int k = 0; k < 6; ++k) ob0[6 * (size_t)m + k] = k < 3 ? 0x7FFFFFFF : (int)0x80000000;
    HIP_TRY(hipMemcpy(d_mslot, m_slot.data(), sizeof(int) * (M + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_mtri, m_tri.data(), sizeof(int) * M, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ob, ob0.data(), sizeof(int) * ob0.size(), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_obj_bounds, dim3(blocks_for(T)), dim3(kTB), 0, 0, tv, lv, d_mslot, d_mtri, M, T, ob);
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(T)), dim3(kTB), 0, 0, tv, lv, d_mslot, d_mtri, M, T, ob, keys[0],
                       vals[0]);
    HIP_TRY(hipGetLastError());
    int obits = 0;
    while ((1 << obits) < M) ++obits;
    const int passes = (30 + obits + 7) / 8;
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nt), dim3(kTB), 0, 0, keys[cur], (size_t)T, 8 * p, (uint32_t)nt, hist);
        HIP_TRY(sc.run(hist, 256 * nt, hoff, nullptr));
        hipLaunchKernelGGL(k_rs_scatter, dim3(nt), dim3(kTB), 0, 0, keys[cur], vals[cur], (size_t)T, 8 * p,
                           (uint32_t)nt, hoff, keys[cur ^ 1], vals[cur ^ 1]);
        HIP_TRY(hipGetLastError());
        cur ^= 1;
    }
    // 3-4. clustering
    hipLaunchKernelGGL(k_init_clusters, dim3(blocks_for(T)), dim3(kTB), 0, 0, keys[cur], vals[cur], T, tv, lv, cl[0]);
    HIP_TRY(hipGetLastError());
    int n_obj = 0;   // objects with triangles: the clusters left at the end
    for (int m = 0; m < M; ++m) n_obj += m_slot[m + 1] > m_slot[m] ? 1 : 0;
    int n = T, cc = 0, made = 0;
    while (n > n_obj) {
        hipLaunchKernelGGL(k_nearest, dim3(blocks_for(n)), dim3(kTB), 0, 0, cl[cc], n, nn);
        hipLaunchKernelGGL(k_pairs, dim3(blocks_for(n)), dim3(kTB), 0, 0, nn, n, keep, make);
        uint32_t kept = 0, pairs = 0;
        HIP_TRY(sc.run(keep, n, pos, &kept));
        HIP_TRY(sc.run(make, n, mk_pos, &pairs));
        if (pairs == 0 || kept + pairs != (uint32_t)n || made + (int)pairs > T) return TOF_ERR_DEVICE;   // no progress
        hipLaunchKernelGGL(k_merge_round, dim3(blocks_for(n)), dim3(kTB), 0, 0, cl[cc], n, nn, keep, pos, make, mk_pos,
                           made, b, cl[cc ^ 1]);
        HIP_TRY(hipGetLastError());
        made += (int)pairs;
        n = (int)kept;
        cc ^= 1;
        ++res.rounds;
    }
    // roots and the objects' boxes
    hipLaunchKernelGGL(k_roots, dim3(blocks_for(n)), dim3(kTB), 0, 0, cl[cc], n, b, d_mslot, root, need, leaf_tri);
    HIP_TRY(hipGetLastError());
    std::vector<int> h_root(M), h_need(M), h_obj(n);
    std::vector<float4> h_lo(n), h_hi(n);
    HIP_TRY(hipMemcpy(h_root.data(), root, sizeof(int) * M, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(h_need.data(), need, sizeof(int) * M, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(h_obj.data(), cl[cc].obj, sizeof(int) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(h_lo.data(), cl[cc].lo, sizeof(float4) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(h_hi.data(), cl[cc].hi, sizeof(float4) * n, hipMemcpyDeviceToHost));
    std::vector<int4> f0;
    std::vector<char> seen(M, 0);
    for (int i = 0; i < n; ++i) {
        const int m = h_obj[i];
        if (m < 0 || m >= M || seen[m]) return TOF_ERR_DEVICE;
        seen[m] = 1;
        float* lb = &res.lbox[6 * (size_t)m];
        lb[0] = h_lo[i].x;
        lb[1] = h_lo[i].y;
        lb[2] = h_lo[i].z;
        lb[3] = h_hi[i].x;
        lb[4] = h_hi[i].y;
        lb[5] = h_hi[i].z;
    }
    for (int m = 0; m < M; ++m) {
        if (m_slot[m + 1] == m_slot[m]) continue;
        if (!seen[m]) return TOF_ERR_DEVICE;
        if (h_need[m]) {
            const int pos0 = (int)f0.size();
            f0.push_back(make_int4(h_need[m] - 1, pos0, m_slot[m], 0));
            res.roots[m] = node_base + pos0;
        } else {
            res.roots[m] = h_root[m];
        }
    }
    // 5. collapse, level by level
    int nf = (int)f0.size(), next_pos = nf, depth = 0, fc = 0;
    if (nf) HIP_TRY(hipMemcpy(F[0], f0.data(), sizeof(int4) * nf, hipMemcpyHostToDevice));
    while (nf > 0) {
        hipLaunchKernelGGL(k_collapse_count, dim3(blocks_for(nf)), dim3(kTB), 0, 0, F[fc], nf, b, fcnt);
        uint32_t total = 0;
        HIP_TRY(sc.run(fcnt, nf, pos, &total));
        if (next_pos + (int64_t)total > T) return TOF_ERR_DEVICE;
        hipLaunchKernelGGL(k_collapse_write, dim3(blocks_for(nf)), dim3(kTB), 0, 0, F[fc], nf, b, pos, next_pos,
                           node_base, depth, nd_child, nd_nc, nd_depth, F[fc ^ 1], leaf_tri);
        HIP_TRY(hipGetLastError());
        next_pos += (int)total;
        nf = (int)total;
        fc ^= 1;
        ++depth;
    }
    const int nb4 = next_pos;
    std::vector<int4> h_child(nb4);
    std::vector<int> h_nc(nb4), h_depth(nb4);
    if (nb4) {
        HIP_TRY(hipMemcpy(h_child.data(), nd_child, sizeof(int4) * nb4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(h_nc.data(), nd_nc, sizeof(int) * nb4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(h_depth.data(), nd_depth, sizeof(int) * nb4, hipMemcpyDeviceToHost));
    }
    res.nodes.assign(nb4, Node4{});
    res.heights.resize(nb4);
    const int dmax = depth - 1;
    for (int i = 0; i < nb4; ++i) {
        res.nodes[i].child = h_child[i];
        res.nodes[i].meta = make_int4(h_nc[i], 0, 0, 0);
        res.heights[i] = dmax - h_depth[i];   // deeper first: children refit before parents
    }
    res.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return TOF_OK;
}

}  // namespace tofh
