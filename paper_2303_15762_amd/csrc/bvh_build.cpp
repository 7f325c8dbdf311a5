// Binned SAH build (16 bins per axis, all three axes) of a binary BVH over triangle bounds,
// then a greedy collapse to 4-wide nodes (repeatedly open the child with the largest surface
// area).  Node boxes are widened by a relative 1e-6 so that the FP32 slab test of the
// traversal is conservative.
#include "bvh_build.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace grw {
namespace {

struct Box {
    float lo[3] = {std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity(),
                   std::numeric_limits<float>::infinity()};
    float hi[3] = {-std::numeric_limits<float>::infinity(), -std::numeric_limits<float>::infinity(),
                   -std::numeric_limits<float>::infinity()};
    void grow(const Box& b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    void grow(const float* p) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    float area() const {
        float d[3];
        for (int a = 0; a < 3; ++a) d[a] = std::max(0.0f, hi[a] - lo[a]);
        return 2.0f * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
    bool empty() const { return lo[0] > hi[0]; }
};

struct BNode {
    Box box;
    int left = -1, right = -1;
    int first = 0, count = 0;
};

struct Builder {
    const float* verts;
    const int32_t* tris;
    std::vector<Box> pbox;
    std::vector<float> cen;     // [nt][3]
    std::vector<int32_t> idx;
    std::vector<BNode> nodes;
    int max_leaf_seen = 0;

    void build(int64_t nt) {
        pbox.resize(nt);
        cen.resize(3 * nt);
        idx.resize(nt);
        for (int64_t t = 0; t < nt; ++t) {
            Box b;
            for (int c = 0; c < 3; ++c) b.grow(verts + 3 * (int64_t)tris[3 * t + c]);
            pbox[t] = b;
            for (int a = 0; a < 3; ++a) cen[3 * t + a] = 0.5f * (b.lo[a] + b.hi[a]);
            idx[t] = (int32_t)t;
        }
        nodes.reserve(2 * nt / 2 + 16);
        struct Item { int node, first, count, depth; };
        std::vector<Item> stack;
        nodes.push_back(BNode());
        stack.push_back({0, 0, (int)nt, 0});
        constexpr int NB = 16;
        while (!stack.empty()) {
            Item it = stack.back();
            stack.pop_back();
            Box nb, cb;
            for (int i = it.first; i < it.first + it.count; ++i) {
                nb.grow(pbox[idx[i]]);
                cb.grow(&cen[3 * (int64_t)idx[i]]);
            }
            nodes[it.node].box = nb;
            nodes[it.node].first = it.first;
            nodes[it.node].count = it.count;
            if (it.count <= 1) {
                max_leaf_seen = std::max(max_leaf_seen, it.count);
                continue;
            }
            int best_axis = -1, best_split = -1;
            float best_cost = std::numeric_limits<float>::infinity();
            const float leaf_cost = (float)it.count;
            const float parent_area = std::max(nb.area(), 1e-30f);
            const bool force_median = it.depth >= 48;
            if (!force_median) {
                for (int a = 0; a < 3; ++a) {
                    const float ext = cb.hi[a] - cb.lo[a];
                    if (!(ext > 0.0f)) continue;
                    Box bb[NB];
                    int bc[NB] = {0};
                    const float sc = NB / ext;
                    for (int i = it.first; i < it.first + it.count; ++i) {
                        int b = (int)((cen[3 * (int64_t)idx[i] + a] - cb.lo[a]) * sc);
                        b = std::min(std::max(b, 0), NB - 1);
                        bb[b].grow(pbox[idx[i]]);
                        bc[b]++;
                    }
                    float ra[NB];
                    int rc[NB];
                    Box acc;
                    int cnt = 0;
                    for (int b = NB - 1; b > 0; --b) {
                        acc.grow(bb[b]);
                        cnt += bc[b];
                        ra[b] = acc.empty() ? 0.0f : acc.area();
                        rc[b] = cnt;
                    }
                    acc = Box();
                    cnt = 0;
                    for (int b = 0; b < NB - 1; ++b) {
                        acc.grow(bb[b]);
                        cnt += bc[b];
                        if (cnt == 0 || rc[b + 1] == 0) continue;
                        const float cost = 1.2f + (acc.area() * cnt + ra[b + 1] * rc[b + 1]) / parent_area;
                        if (cost < best_cost) {
                            best_cost = cost;
                            best_axis = a;
                            best_split = b;
                        }
                    }
                }
            }
            if (!force_median && it.count <= kMaxLeaf && leaf_cost <= best_cost) {
                max_leaf_seen = std::max(max_leaf_seen, it.count);
                continue;
            }
            int mid;
            if (best_axis >= 0 && !force_median) {
                const int a = best_axis;
                const float sc = NB / (cb.hi[a] - cb.lo[a]);
                auto pit = std::partition(idx.begin() + it.first, idx.begin() + it.first + it.count,
                                          [&](int32_t t) {
                                              int b = (int)((cen[3 * (int64_t)t + a] - cb.lo[a]) * sc);
                                              b = std::min(std::max(b, 0), NB - 1);
                                              return b <= best_split;
                                          });
                mid = (int)(pit - idx.begin());
            } else {
                // degenerate centroids or depth cap: object median on the widest axis
                int a = 0;
                float e = -1.0f;
                for (int q = 0; q < 3; ++q)
                    if (nb.hi[q] - nb.lo[q] > e) { e = nb.hi[q] - nb.lo[q]; a = q; }
                mid = it.first + it.count / 2;
                std::nth_element(idx.begin() + it.first, idx.begin() + mid,
                                 idx.begin() + it.first + it.count, [&](int32_t x, int32_t y) {
                                     const float cx = cen[3 * (int64_t)x + a], cy = cen[3 * (int64_t)y + a];
                                     return cx < cy || (cx == cy && x < y);
                                 });
            }
            if (mid == it.first || mid == it.first + it.count) mid = it.first + it.count / 2;
            const int l = (int)nodes.size();
            nodes.push_back(BNode());
            nodes.push_back(BNode());
            nodes[it.node].left = l;
            nodes[it.node].right = l + 1;
            stack.push_back({l + 1, mid, it.first + it.count - mid, it.depth + 1});
            stack.push_back({l, it.first, mid - it.first, it.depth + 1});
        }
    }
};

float widen_lo(float x) {
    return std::nextafter(x - 1e-6f * std::fabs(x) - 1e-12f, -std::numeric_limits<float>::infinity());
}
float widen_hi(float x) {
    return std::nextafter(x + 1e-6f * std::fabs(x) + 1e-12f, std::numeric_limits<float>::infinity());
}

struct Collapser {
    const Builder& B;
    BuiltBVH& out;
    int max_depth = 0;

    int32_t leaf_code(const BNode& n) const {
        return (int32_t)(0x80000000u | ((uint32_t)(n.count - 1) << 28) | (uint32_t)n.first);
    }

    // Emit the 4-wide node for binary node b (an inner node); returns its index.
    int emit(int b, int depth) {
        max_depth = std::max(max_depth, depth);
        int kids[4];
        int nk = 0;
        const BNode& bn = B.nodes[b];
        if (bn.left < 0) {
            kids[nk++] = b;   // the root itself is a leaf: one leaf child
        } else {
            kids[nk++] = bn.left;
            kids[nk++] = bn.right;
            while (nk < 4) {
                int pick = -1;
                float best = -1.0f;
                for (int i = 0; i < nk; ++i) {
                    const BNode& c = B.nodes[kids[i]];
                    if (c.left >= 0 && c.box.area() > best) { best = c.box.area(); pick = i; }
                }
                if (pick < 0) break;
                const BNode& c = B.nodes[kids[pick]];
                kids[pick] = c.left;
                kids[nk++] = c.right;
            }
        }
        const int id = (int)out.nodes.size();
        out.nodes.push_back(BVH4Node());
        for (int i = 0; i < 4; ++i) {
            BVH4Node& N = out.nodes[id];
            if (i >= nk) {
                // unused slot: a box at +infinity on every axis fails the slab test for any
                // ray direction, and the child code is the sentinel the traversal skips
                N.lox[i] = N.loy[i] = N.loz[i] = std::numeric_limits<float>::infinity();
                N.hix[i] = N.hiy[i] = N.hiz[i] = std::numeric_limits<float>::infinity();
                N.child[i] = kEmptyChild;
                continue;
            }
            const BNode& c = B.nodes[kids[i]];
            N.lox[i] = widen_lo(c.box.lo[0]);
            N.loy[i] = widen_lo(c.box.lo[1]);
            N.loz[i] = widen_lo(c.box.lo[2]);
            N.hix[i] = widen_hi(c.box.hi[0]);
            N.hiy[i] = widen_hi(c.box.hi[1]);
            N.hiz[i] = widen_hi(c.box.hi[2]);
            if (c.left < 0) {
                N.child[i] = leaf_code(c);
            } else {
                const int cid = emit(kids[i], depth + 1);
                out.nodes[id].child[i] = cid;
            }
        }
        for (int i = 0; i < 4; ++i) out.nodes[id].pad[i] = 0;
        return id;
    }
};

// Renumber the nodes so that the first kTopNodes inner nodes met breadth-first from the root
// come first, in that order (the traversal keeps them in LDS); the rest keep their depth-first
// order.  A node is met only after its parent, and no node after them has a child among them
// (the breadth-first prefix holds all nodes of a level before any of the next), so child
// indices stay above their parents'.
void top_levels_first(std::vector<BVH4Node>& nodes) {
    const int n = (int)nodes.size();
    std::vector<int> bfs;
    bfs.reserve(kTopNodes);
    bfs.push_back(0);
    for (size_t h = 0; h < bfs.size() && (int)bfs.size() < kTopNodes; ++h)
        for (int i = 0; i < 4 && (int)bfs.size() < kTopNodes; ++i) {
            const int32_t c = nodes[bfs[h]].child[i];
            if (c >= 0 && c != kEmptyChild) bfs.push_back(c);
        }
    std::vector<int32_t> id(n, -1);
    for (size_t i = 0; i < bfs.size(); ++i) id[bfs[i]] = (int32_t)i;
    int32_t next = (int32_t)bfs.size();
    for (int i = 0; i < n; ++i)
        if (id[i] < 0) id[i] = next++;
    std::vector<BVH4Node> out(n);
    for (int i = 0; i < n; ++i) {
        BVH4Node N = nodes[i];
        for (int j = 0; j < 4; ++j)
            if (N.child[j] >= 0 && N.child[j] != kEmptyChild) N.child[j] = id[N.child[j]];
        out[id[i]] = N;
    }
    nodes.swap(out);
}

}  // namespace

BuiltBVH build_bvh4(const float* verts, const int32_t* tris, int64_t nt) {
    Builder B{verts, tris, {}, {}, {}, {}, 0};
    B.build(nt);
    BuiltBVH out;
    out.nodes.reserve(B.nodes.size() / 3 + 4);
    Collapser C{B, out, 0};
    C.emit(0, 0);
    top_levels_first(out.nodes);
    out.tri_order = B.idx;
    out.depth = C.max_depth;
    out.max_leaf = B.max_leaf_seen;
    return out;
}

}  // namespace grw
