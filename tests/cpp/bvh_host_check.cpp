// Structural checks of the host 4-wide tree builder on random triangle boxes:
// every primitive in exactly one leaf of at most leaf_max, every node reached
// once from the root, 1..4 children per node, heights above the children's.
#include <cstdio>
#include <random>
#include <vector>

#include "tof_internal.h"

static int check(int n, int leaf_max, unsigned seed) {
    std::mt19937 rng(seed);
    std::uniform_real_distribution<float> u(-5.f, 5.f), s(0.001f, 0.3f);
    std::vector<tofh::BvhPrim> prims(n);
    for (auto& p : prims)
        for (int k = 0; k < 3; ++k) {
            const float c = (k == 1 && seed % 2) ? 0.f : u(rng);   // odd seeds: a flat layer
            p.lo[k] = c - s(rng);
            p.hi[k] = c + s(rng);
        }
    std::vector<tofd::Node4> nodes;
    std::vector<int> heights, order;
    const int base = 7, slot_base = 11;
    const int32_t root = tofh::build_bvh4(prims, leaf_max, base, slot_base, nodes, heights, order);
    std::vector<int> seen(n, 0), node_refs(nodes.size(), 0);
    std::vector<int> stack;
    auto visit_leaf = [&](int32_t ref) -> bool {
        const int first = (int)((uint32_t)ref & 0x0FFFFFFFu) - slot_base, cnt = (int)(((uint32_t)ref >> 28) & 7u) + 1;
        if (cnt > leaf_max || first < 0 || first + cnt > n) return false;
        for (int i = first; i < first + cnt; ++i) seen[order[i]]++;
        return true;
    };
    if (root < 0) {
        if (!visit_leaf(root)) return 1;
    } else {
        if (root != base) return 2;
        stack.push_back(0);
        node_refs[0]++;
    }
    while (!stack.empty()) {
        const int i = stack.back();
        stack.pop_back();
        const tofd::Node4& nd = nodes[i];
        const int nc = nd.meta.x;
        if (nc < 1 || nc > 4) return 3;
        const int ch[4] = {nd.child.x, nd.child.y, nd.child.z, nd.child.w};
        for (int j = 0; j < nc; ++j) {
            if (ch[j] < 0) {
                if (!visit_leaf(ch[j])) return 4;
            } else {
                const int k = ch[j] - base;
                if (k <= 0 || k >= (int)nodes.size()) return 5;
                if (heights[i] <= heights[k]) return 6;
                node_refs[k]++;
                stack.push_back(k);
            }
        }
    }
    for (int v : seen)
        if (v != 1) return 7;
    for (int v : node_refs)
        if (v != 1) return 8;
    return 0;
}

int main() {
    const int sizes[] = {1, 2, 3, 5, 17, 100, 1000, 5000};
    for (int n : sizes)
        for (int leaf_max : {1, 4})
            for (unsigned seed = 0; seed < 3; ++seed) {
                const int e = check(n, leaf_max, seed);
                if (e) {
                    std::printf("FAIL n=%d leaf_max=%d seed=%u code=%d\n", n, leaf_max, seed, e);
                    return 1;
                }
            }
    std::printf("ok\n");
    return 0;
}
