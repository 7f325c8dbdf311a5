// Host-side bounding-volume hierarchy for the triangle scene: binned surface-area-heuristic
// binary build, collapsed into a 4-wide tree whose nodes are one 128-byte cache line.
#pragma once

#include <cstdint>
#include <vector>

namespace grw {

// 4-wide node, structure-of-arrays over the children so one lane reads 7 x 16 bytes.
// child[i] >= 0: index of an inner node; child[i] < 0: leaf with triangles
// [first, first + count) where first = child & 0x0FFFFFFF, count = ((child >> 28) & 7) + 1.
// Unused slots have child = kEmptyChild and a box at +infinity.
struct alignas(128) BVH4Node {
    float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
    int32_t child[4];
    int32_t pad[4];
};
static_assert(sizeof(BVH4Node) == 128, "BVH4Node must be one 128-byte line");

constexpr int kMaxLeaf = 8;
constexpr int32_t kEmptyChild = 0x7FFFFFFF;

struct BuiltBVH {
    std::vector<BVH4Node> nodes;     // root at index 0
    std::vector<int32_t> tri_order;  // leaf order -> original triangle index
    int depth = 0;                   // deepest inner-node level (root = 0)
    int max_leaf = 0;
};

// verts: [nv][3] floats; tris: [nt][3] indices (validated by the caller).
BuiltBVH build_bvh4(const float* verts, const int32_t* tris, int64_t nt);

}  // namespace grw
