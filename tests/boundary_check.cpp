// Host-side check of libgrwave's material-boundary lists (composite interactions): for points
// on triangles, the nearest boundary edge of the triangle's material within the reach, found
// through the triangle's candidate list, against brute force over every boundary edge; and
// the triangle's distance bound below every listed edge's distance.
// Input (stdin): nv nt reach, nv lines "x y z", nt lines "a b c m", nq, nq lines "t u v".
// Output: "OK n_edges n_found total_list_entries" or "FAIL reason".
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../paper_2303_15762_amd/csrc/bvh_build.hpp"

using namespace grw;

static double seg_dist(const double* P, const float* a, const float* b) {
    double ab[3], ap[3], l2 = 0, t = 0;
    for (int i = 0; i < 3; ++i) { ab[i] = (double)b[i] - a[i]; ap[i] = P[i] - a[i]; l2 += ab[i] * ab[i]; t += ap[i] * ab[i]; }
    t = l2 > 0 ? std::fmin(1.0, std::fmax(0.0, t / l2)) : 0.0;
    double s = 0;
    for (int i = 0; i < 3; ++i) { const double d = ap[i] - t * ab[i]; s += d * d; }
    return std::sqrt(s);
}

int main() {
    long nv, nt;
    float reach;
    if (scanf("%ld %ld %f", &nv, &nt, &reach) != 3) { printf("FAIL input\n"); return 1; }
    std::vector<float> v(3 * nv);
    std::vector<int32_t> t(3 * nt), m(nt);
    for (long i = 0; i < nv; ++i) if (scanf("%f %f %f", &v[3 * i], &v[3 * i + 1], &v[3 * i + 2]) != 3) return 1;
    for (long i = 0; i < nt; ++i) if (scanf("%d %d %d %d", &t[3 * i], &t[3 * i + 1], &t[3 * i + 2], &m[i]) != 4) return 1;
    BuiltBoundaries B;
    if (!build_boundaries(v.data(), t.data(), m.data(), nt, reach, B)) { printf("FAIL build\n"); return 0; }
    long nq;
    if (scanf("%ld", &nq) != 1) return 1;
    long found = 0;
    for (long q = 0; q < nq; ++q) {
        long ti; double u, w;
        if (scanf("%ld %lf %lf", &ti, &u, &w) != 3) return 1;
        double P[3];
        for (int k = 0; k < 3; ++k)
            P[k] = (1 - u - w) * v[3 * t[3 * ti] + k] + u * v[3 * t[3 * ti + 1] + k] + w * v[3 * t[3 * ti + 2] + k];
        // brute force
        long bb = -1; double bd = reach;
        for (long e = 0; e < B.n_edges; ++e) {
            const float* r = &B.edges[16 * e];
            int32_t ma, mb;
            std::memcpy(&ma, &r[3], 4); std::memcpy(&mb, &r[7], 4);
            if (ma != m[ti] && mb != m[ti]) continue;
            const double d = seg_dist(P, r, r + 4);
            if (d < bd) { bd = d; bb = e; }
        }
        // through the list
        long lb = -1; double ld = reach;
        for (uint32_t i = 0; i < B.count[ti]; ++i) {
            const uint32_t e = B.idx[B.first[ti] + i];
            if (i > 0 && e <= B.idx[B.first[ti] + i - 1]) { printf("FAIL list not ascending\n"); return 0; }
            const float* r = &B.edges[16 * e];
            const double d = seg_dist(P, r, r + 4);
            if (d < (double)B.gap[ti]) { printf("FAIL query %ld: edge %u at %g below the bound %g\n", q, e, d, (double)B.gap[ti]); return 0; }
            if (d < ld) { ld = d; lb = e; }
        }
        if (lb != bb) { printf("FAIL query %ld: list %ld brute %ld (%g %g)\n", q, lb, bb, ld, bd); return 0; }
        if (bb >= 0) ++found;
    }
    printf("OK %ld %ld %zu\n", (long)B.n_edges, found, B.idx.size());
    return 0;
}
