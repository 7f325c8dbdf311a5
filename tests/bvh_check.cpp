// Host-side check of the 4-wide BVH builder used by libgrwave: structural invariants and a
// replay of the traversal's push/pop discipline in FP32 on the CPU, against brute force.
// Input (stdin): nv nt, then nv lines "x y z", then nt lines "a b c", then nr rays "o d".
// Output: "OK depth max_stack nodes" or "FAIL reason".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

#include "../paper_2303_15762_amd/csrc/bvh_build.hpp"

using namespace grw;

static bool tri_hit(const float* o, const float* d, const float* a, const float* b, const float* c,
                    float& t) {
    // plain Moller-Trumbore in double for the reference
    double e1[3], e2[3], p[3], s[3], q[3];
    for (int i = 0; i < 3; ++i) { e1[i] = b[i] - a[i]; e2[i] = c[i] - a[i]; s[i] = o[i] - a[i]; }
    p[0] = d[1] * e2[2] - d[2] * e2[1]; p[1] = d[2] * e2[0] - d[0] * e2[2]; p[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0) return false;
    double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) / det;
    if (u < 0 || u > 1) return false;
    q[0] = s[1] * e1[2] - s[2] * e1[1]; q[1] = s[2] * e1[0] - s[0] * e1[2]; q[2] = s[0] * e1[1] - s[1] * e1[0];
    double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) / det;
    if (v < 0 || u + v > 1) return false;
    t = (float)((e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) / det);
    return t > 1e-7f;
}

int main() {
    long nv, nt;
    if (std::scanf("%ld %ld", &nv, &nt) != 2) return 2;
    std::vector<float> V(3 * nv);
    std::vector<int32_t> T(3 * nt);
    for (long i = 0; i < 3 * nv; ++i) std::scanf("%f", &V[i]);
    for (long i = 0; i < 3 * nt; ++i) std::scanf("%d", &T[i]);
    BuiltBVH B = build_bvh4(V.data(), T.data(), nt);
    const long nn = (long)B.nodes.size();
    std::vector<int> seen(nt, 0);
    // structure
    for (long n = 0; n < nn; ++n) {
        const BVH4Node& N = B.nodes[n];
        for (int i = 0; i < 4; ++i) {
            int32_t c = N.child[i];
            if (c == kEmptyChild) continue;
            if (c >= 0) {
                if (c <= n || c >= nn) { std::printf("FAIL child index %d at node %ld\n", c, n); return 1; }
                // nested boxes: every box of the child node lies inside the slot's box (the
                // traversal skips a popped node whose slot box starts beyond the closest hit,
                // which is exact only if no box below starts nearer)
                const BVH4Node& C = B.nodes[c];
                for (int k = 0; k < 4; ++k) {
                    if (C.child[k] == kEmptyChild) continue;
                    if (C.lox[k] < N.lox[i] || C.hix[k] > N.hix[i] || C.loy[k] < N.loy[i] ||
                        C.hiy[k] > N.hiy[i] || C.loz[k] < N.loz[i] || C.hiz[k] > N.hiz[i]) {
                        std::printf("FAIL child box outside its slot box at node %ld\n", n);
                        return 1;
                    }
                }
            } else {
                int first = c & 0x0FFFFFFF, cnt = ((c >> 28) & 7) + 1;
                if (first + cnt > nt) { std::printf("FAIL leaf range\n"); return 1; }
                for (int j = first; j < first + cnt; ++j) {
                    seen[j]++;
                    int t = B.tri_order[j];
                    for (int k = 0; k < 3; ++k) {
                        const float* p = &V[3 * (long)T[3 * t + k]];
                        if (p[0] < N.lox[i] || p[0] > N.hix[i] || p[1] < N.loy[i] || p[1] > N.hiy[i] ||
                            p[2] < N.loz[i] || p[2] > N.hiz[i]) {
                            std::printf("FAIL triangle outside its leaf box\n");
                            return 1;
                        }
                    }
                }
            }
        }
    }
    for (long j = 0; j < nt; ++j)
        if (seen[j] != 1) { std::printf("FAIL triangle %ld referenced %d times\n", j, seen[j]); return 1; }
    // the top levels come first, breadth-first: the k-th inner node met from the root, level by
    // level and in child-slot order, has index k for k < kTopNodes
    {
        std::vector<int32_t> q(1, 0);
        for (size_t h = 0; h < q.size() && (long)q.size() < kTopNodes; ++h)
            for (int i = 0; i < 4 && (long)q.size() < kTopNodes; ++i) {
                const int32_t c = B.nodes[q[h]].child[i];
                if (c >= 0 && c != kEmptyChild) q.push_back(c);
            }
        for (size_t k = 0; k < q.size(); ++k)
            if (q[k] != (int32_t)k) { std::printf("FAIL top node %zu at index %d\n", k, q[k]); return 1; }
    }
    const int stack_cap = 3 * (B.depth + 1) + 1;
    // traversal replay
    long nr;
    if (std::scanf("%ld", &nr) != 1) nr = 0;
    int max_sp = 0;
    for (long r = 0; r < nr; ++r) {
        float o[3], d[3];
        for (int i = 0; i < 3; ++i) std::scanf("%f", &o[i]);
        for (int i = 0; i < 3; ++i) std::scanf("%f", &d[i]);
        float inv[3];
        for (int i = 0; i < 3; ++i) inv[i] = 1.0f / (std::fabs(d[i]) > 1e-30f ? d[i] : std::copysign(1e-30f, d[i]));
        float best = std::numeric_limits<float>::max();
        int besti = -1;
        std::vector<int> stk;
        int cur = 0;
        while (true) {
            if (cur >= 0) {
                const BVH4Node& N = B.nodes[cur];
                float k[4];
                int c[4];
                for (int i = 0; i < 4; ++i) {
                    c[i] = N.child[i];
                    float t0x = (N.lox[i] - o[0]) * inv[0], t1x = (N.hix[i] - o[0]) * inv[0];
                    float t0y = (N.loy[i] - o[1]) * inv[1], t1y = (N.hiy[i] - o[1]) * inv[1];
                    float t0z = (N.loz[i] - o[2]) * inv[2], t1z = (N.hiz[i] - o[2]) * inv[2];
                    float tn = std::fmax(std::fmax(std::fmin(t0x, t1x), std::fmin(t0y, t1y)), std::fmax(std::fmin(t0z, t1z), 1e-7f));
                    float tf = std::fmin(std::fmin(std::fmax(t0x, t1x), std::fmax(t0y, t1y)), std::fmin(std::fmax(t0z, t1z), best));
                    k[i] = (tn <= tf && c[i] != kEmptyChild) ? tn : std::numeric_limits<float>::max();
                }
                for (int a = 0; a < 4; ++a)
                    for (int b = a + 1; b < 4; ++b)
                        if (k[a] < k[b]) { std::swap(k[a], k[b]); std::swap(c[a], c[b]); }
                for (int i = 0; i < 3; ++i)
                    if (k[i] != std::numeric_limits<float>::max()) stk.push_back(c[i]);
                max_sp = std::max(max_sp, (int)stk.size());
                if ((int)stk.size() > stack_cap) { std::printf("FAIL stack %zu > %d\n", stk.size(), stack_cap); return 1; }
                if (k[3] != std::numeric_limits<float>::max()) { cur = c[3]; continue; }
            } else {
                int first = cur & 0x0FFFFFFF, cnt = ((cur >> 28) & 7) + 1;
                for (int j = first; j < first + cnt; ++j) {
                    int t = B.tri_order[j];
                    float th;
                    if (tri_hit(o, d, &V[3 * (long)T[3 * t]], &V[3 * (long)T[3 * t + 1]], &V[3 * (long)T[3 * t + 2]], th) && th < best) {
                        best = th;
                        besti = t;
                    }
                }
            }
            if (stk.empty()) break;
            cur = stk.back();
            stk.pop_back();
        }
        // brute force
        float bb = std::numeric_limits<float>::max();
        int bi = -1;
        for (long t = 0; t < nt; ++t) {
            float th;
            if (tri_hit(o, d, &V[3 * (long)T[3 * t]], &V[3 * (long)T[3 * t + 1]], &V[3 * (long)T[3 * t + 2]], th) && th < bb) {
                bb = th;
                bi = (int)t;
            }
        }
        if (bi != besti && bb != best) { std::printf("FAIL ray %ld: bvh %d brute %d\n", r, besti, bi); return 1; }
    }
    std::printf("OK %d %d %ld\n", B.depth, max_sp, nn);
    return 0;
}
