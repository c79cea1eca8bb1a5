// Host-side construction of 4-wide BVH topologies (binned SAH, then the
// SAH-optimal collapse of the binary tree into 4-wide nodes).  Used once per scene for
// every object's triangles (in object space; the device refits the boxes in
// world space each frame, which a rigid motion keeps tight) and once per frame
// for the top-level tree over the objects' world boxes.  Only child links and
// counts are produced; boxes are filled by the device refit.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "tof_internal.h"

namespace tofh {

namespace {

struct BinNode {
    float lo[3], hi[3];
    int left = -1, right = -1;   // binary children (-1: leaf)
    int first = 0, count = 0;    // leaf range in the primitive order
};

float area(const float lo[3], const float hi[3]) {
    const float dx = std::max(hi[0] - lo[0], 0.f), dy = std::max(hi[1] - lo[1], 0.f), dz = std::max(hi[2] - lo[2], 0.f);
    return 2.f * (dx * dy + dy * dz + dz * dx);
}

struct Bounds {
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    void grow(const float* l, const float* h) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], l[k]);
            hi[k] = std::max(hi[k], h[k]);
        }
    }
    void grow_pt(const float* p) { grow(p, p); }
};

constexpr int kBins = 16;

// Binned SAH over prims[first, first + count) (reordered in place).
void build_binary(const std::vector<BvhPrim>& prims, std::vector<int>& order, int leaf_max,
                  std::vector<BinNode>& out) {
    struct Job {
        int node, first, count;
    };
    out.clear();
    out.push_back(BinNode{});
    std::vector<Job> stack{{0, 0, (int)order.size()}};
    while (!stack.empty()) {
        const Job j = stack.back();
        stack.pop_back();
        Bounds b, cb;
        for (int i = j.first; i < j.first + j.count; ++i) {
            const BvhPrim& p = prims[order[i]];
            b.grow(p.lo, p.hi);
            float c[3] = {0.5f * (p.lo[0] + p.hi[0]), 0.5f * (p.lo[1] + p.hi[1]), 0.5f * (p.lo[2] + p.hi[2])};
            cb.grow_pt(c);
        }
        BinNode& nd = out[j.node];
        for (int k = 0; k < 3; ++k) {
            nd.lo[k] = b.lo[k];
            nd.hi[k] = b.hi[k];
        }
        nd.first = j.first;
        nd.count = j.count;
        if (j.count <= 1) continue;
        // best split over the three axes (cost in units of one triangle test;
        // a 4-wide node step costs about one: 0.25, 0.5, 1.5 and 2 gave
        // slower visibility on the glossy benchmark scene)
        const float parea = std::max(area(b.lo, b.hi), 1e-30f);
        float best = 3e38f;
        int best_axis = -1, best_bin = -1;
        for (int ax = 0; ax < 3; ++ax) {
            const float ext = cb.hi[ax] - cb.lo[ax];
            if (!(ext > 0.f)) continue;
            Bounds bb[kBins];
            int cnt[kBins] = {};
            for (int i = j.first; i < j.first + j.count; ++i) {
                const BvhPrim& p = prims[order[i]];
                const float c = 0.5f * (p.lo[ax] + p.hi[ax]);
                int k = (int)((c - cb.lo[ax]) / ext * kBins);
                k = std::min(std::max(k, 0), kBins - 1);
                bb[k].grow(p.lo, p.hi);
                ++cnt[k];
            }
            float ra[kBins];
            int rn[kBins];
            Bounds acc;
            int n = 0;
            for (int k = kBins - 1; k > 0; --k) {
                acc.grow(bb[k].lo, bb[k].hi);
                n += cnt[k];
                ra[k] = n ? area(acc.lo, acc.hi) : 0.f;
                rn[k] = n;
            }
            Bounds lacc;
            int ln = 0;
            for (int k = 0; k < kBins - 1; ++k) {
                lacc.grow(bb[k].lo, bb[k].hi);
                ln += cnt[k];
                if (ln == 0 || rn[k + 1] == 0) continue;
                const float cost = 1.0f + (area(lacc.lo, lacc.hi) * ln + ra[k + 1] * rn[k + 1]) / parea;
                if (cost < best) {
                    best = cost;
                    best_axis = ax;
                    best_bin = k;
                }
            }
        }
        if (j.count <= leaf_max && !(best < (float)j.count)) continue;   // a leaf is cheaper
        int mid;
        if (best_axis < 0) {   // all centroids coincide: split the range in half
            mid = j.first + j.count / 2;
        } else {
            const float ext = cb.hi[best_axis] - cb.lo[best_axis];
            auto it = std::partition(order.begin() + j.first, order.begin() + j.first + j.count, [&](int id) {
                const BvhPrim& p = prims[id];
                const float c = 0.5f * (p.lo[best_axis] + p.hi[best_axis]);
                int k = (int)((c - cb.lo[best_axis]) / ext * kBins);
                k = std::min(std::max(k, 0), kBins - 1);
                return k <= best_bin;
            });
            mid = (int)(it - order.begin());
            if (mid == j.first || mid == j.first + j.count) mid = j.first + j.count / 2;
        }
        const int l = (int)out.size(), r = l + 1;
        out.push_back(BinNode{});
        out.push_back(BinNode{});
        out[j.node].left = l;
        out[j.node].right = r;
        stack.push_back({r, mid, j.first + j.count - mid});
        stack.push_back({l, j.first, mid - j.first});
    }
}

}  // namespace

int32_t leaf_ref(int first, int count) {
    return (int32_t)(0x80000000u | ((uint32_t)(count - 1) << 28) | (uint32_t)first);
}

// Collapse of the binary tree into 4-wide nodes by dynamic programming over
// the SAH (the optimal collapse of a binary tree into a wide one, as in
// Ylitie, Karras and Laine 2017): C(n, j) is the least cost of n's subtree
// when it may occupy up to j child slots of a 4-wide node -- as one slot
// (a leaf of at most leaf_max triangles, cost A(n) * count, or a node, cost
// A(n) * node_cost + D(n, 4)) or, for j >= 2, spread over its binary
// children, D(n, j) = min over k of C(left, k) + C(right, j - k).  Costs are
// surface areas times the triangle tests and node steps they weigh, the
// units of the binned SAH above.
struct Collapse {
    float c[5];        // C(n, j), j = 1..4
    float d4;          // D(n, 4): the children of n as a node
    int8_t node;       // C(n, 1) as a node (1) or a leaf (0)
    int8_t spread[5];  // for j >= 2: 0 = one slot, k > 0 = left child takes k slots
    int8_t k4;         // left child's slots in D(n, 4)
};

// 4-wide tree over prims: nodes appended to `nodes` (global index = node_base
// + position), heights (1 + the highest internal child, leaves count 0)
// appended likewise, order = primitive indices in leaf order, leaf slots
// numbered from slot_base.  Returns the root reference.
int32_t build_bvh4(const std::vector<BvhPrim>& prims, int leaf_max, int node_base, int slot_base,
                   std::vector<tofd::Node4>& nodes, std::vector<int>& heights, std::vector<int>& order) {
    constexpr float kNodeCost = 1.0f;   // a node step in triangle tests, as in the split cost
    order.resize(prims.size());
    for (size_t i = 0; i < prims.size(); ++i) order[i] = (int)i;
    if (prims.empty()) return -1;
    const int lmax = std::min(leaf_max, 8);
    std::vector<BinNode> bin;
    build_binary(prims, order, lmax, bin);
    // children have larger indices than their parents: fill bottom-up
    std::vector<Collapse> dp(bin.size());
    for (size_t i = bin.size(); i-- > 0;) {
        const BinNode& b = bin[i];
        Collapse& q = dp[i];
        const float A = area(b.lo, b.hi);
        const float leaf = b.count <= lmax ? A * (float)b.count : 3e38f;
        if (b.left < 0) {   // a binary leaf is a leaf (count <= lmax by construction)
            for (int j = 1; j <= 4; ++j) {
                q.c[j] = leaf;
                q.spread[j] = 0;
            }
            q.node = 0;
            q.d4 = 3e38f;
            q.k4 = 0;
            continue;
        }
        const Collapse& l = dp[b.left];
        const Collapse& r = dp[b.right];
        auto distribute = [&](int j, int& kbest) {
            float best = 3e38f;
            kbest = 0;
            for (int k = 1; k < j; ++k) {
                const float v = l.c[k] + r.c[j - k];
                if (v < best) {
                    best = v;
                    kbest = k;
                }
            }
            return best;
        };
        int k4 = 0;
        q.d4 = distribute(4, k4);
        q.k4 = (int8_t)k4;
        const float as_node = A * kNodeCost + q.d4;
        q.node = as_node < leaf ? 1 : 0;
        q.c[1] = std::min(as_node, leaf);
        q.spread[1] = 0;
        for (int j = 2; j <= 4; ++j) {
            int k = 0;
            const float d = distribute(j, k);
            if (d < q.c[1]) {
                q.c[j] = d;
                q.spread[j] = (int8_t)k;
            } else {
                q.c[j] = q.c[1];
                q.spread[j] = 0;
            }
        }
    }
    if (!dp[0].node) return leaf_ref(slot_base + bin[0].first, bin[0].count);
    // the subtrees in the slots of n spread over j slots
    std::vector<int> kids;
    auto slots = [&](auto&& self, int n, int j) -> void {
        const int k = dp[n].spread[j];
        if (k == 0 || bin[n].left < 0) {
            kids.push_back(n);
        } else {
            self(self, bin[n].left, k);
            self(self, bin[n].right, j - k);
        }
    };
    const size_t base = nodes.size();
    struct Item {
        int bin;     // binary node of this 4-wide node
        int slot;    // its position in `nodes`
    };
    std::vector<Item> work{{0, (int)base}};
    nodes.push_back(tofd::Node4{});
    heights.push_back(0);
    std::vector<std::pair<int, int>> parent_of;   // (4-wide child position, 4-wide parent position)
    for (size_t w = 0; w < work.size(); ++w) {
        const Item it = work[w];
        kids.clear();
        const int k4 = dp[it.bin].k4;
        slots(slots, bin[it.bin].left, k4);
        slots(slots, bin[it.bin].right, 4 - k4);
        int ref[4] = {-1, -1, -1, -1};
        for (size_t k = 0; k < kids.size(); ++k) {
            const BinNode& b = bin[kids[k]];
            if (b.left < 0 || !dp[kids[k]].node) {
                ref[k] = leaf_ref(slot_base + b.first, b.count);
            } else {
                const int pos = (int)nodes.size();
                nodes.push_back(tofd::Node4{});
                heights.push_back(0);
                ref[k] = node_base + (pos - (int)base);
                work.push_back({kids[k], pos});
                parent_of.push_back({pos, it.slot});
            }
        }
        tofd::Node4& nd = nodes[it.slot];
        nd.child = make_int4(ref[0], ref[1], ref[2], ref[3]);
        nd.meta = make_int4((int)kids.size(), 0, 0, 0);
    }
    // heights: children are always created after their parent
    for (size_t k = parent_of.size(); k-- > 0;) {
        const int c = parent_of[k].first, p = parent_of[k].second;
        heights[p] = std::max(heights[p], heights[c] + 1);
    }
    return node_base;
}

}  // namespace tofh
