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
// The first kTopNodes inner nodes of the tree in breadth-first order (root, its children,
// theirs, ...) take indices 0 .. kTopNodes - 1; every other node keeps the depth-first
// pre-order of the collapse, after them.  Every child index stays above its parent's.
constexpr int kTopNodes = 64;

struct BuiltBVH {
    std::vector<BVH4Node> nodes;     // root at index 0; the top levels first (kTopNodes)
    std::vector<int32_t> tri_order;  // leaf order -> original triangle index
    int depth = 0;                   // deepest inner-node level (root = 0)
    int max_leaf = 0;
};

// verts: [nv][3] floats; tris: [nt][3] indices (validated by the caller).
BuiltBVH build_bvh4(const float* verts, const int32_t* tris, int64_t nt);

}  // namespace grw

namespace grw {

// Material boundaries of a triangle mesh, for composite interactions: every mesh edge
// (unordered vertex-index pair) used by exactly two triangles of different materials, and for
// each triangle the boundary edges of its own material that lie within `reach` metres of it
// (candidates: the exact distance test runs at the hit).
struct BuiltBoundaries {
    std::vector<float> edges;        // [n][16]: p0, mat a (int bits), p1, mat b, third vertex of a (+pad), of b (+pad)
    std::vector<uint32_t> first;     // per triangle: first entry in idx
    std::vector<uint32_t> count;     // per triangle: number of entries
    std::vector<float> gap;          // per triangle: a lower bound of its distance to its listed edges
    std::vector<uint32_t> idx;       // boundary edge ids, ascending per triangle
    int64_t n_edges = 0;
};

// verts [nv][3], tris [nt][3] (validated), tri_mat [nt].  Fails (returns false) when the lists
// would exceed 2^32 entries.
bool build_boundaries(const float* verts, const int32_t* tris, const int32_t* tri_mat, int64_t nt, float reach,
                      BuiltBoundaries& out);

// Coefficients a_1 .. a_n of Weideman's rational approximation of the Faddeeva function with
// n terms, and its parameter L = sqrt(n / sqrt(2)).
void weideman_coefficients(int n, float* a, float* L);

}  // namespace grw
