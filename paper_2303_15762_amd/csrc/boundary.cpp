// Host side of composite interactions: material boundaries of the uploaded mesh, per-triangle
// candidate lists, and the constants of the device's Faddeeva approximation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "bvh_build.hpp"

namespace grw {

namespace {

struct Box {
    float lo[3], hi[3];
};

// squared distance between two axis-aligned boxes
double box_gap2(const Box& a, const Box& b) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double g = std::max({0.0, (double)a.lo[i] - b.hi[i], (double)b.lo[i] - a.hi[i]});
        s += g * g;
    }
    return s;
}

}  // namespace

bool build_boundaries(const float* verts, const int32_t* tris, const int32_t* tri_mat, int64_t nt, float reach,
                      BuiltBoundaries& out) {
    out = BuiltBoundaries{};
    // edges by vertex-index pair
    std::vector<std::pair<uint64_t, int64_t>> keys;   // (key, 3 * triangle + local edge)
    keys.reserve((size_t)(3 * nt));
    for (int64_t t = 0; t < nt; ++t)
        for (int e = 0; e < 3; ++e) {
            uint64_t a = (uint32_t)tris[3 * t + e], b = (uint32_t)tris[3 * t + (e + 1) % 3];
            if (a > b) std::swap(a, b);
            keys.push_back({(a << 32) | b, 3 * t + e});
        }
    std::sort(keys.begin(), keys.end());
    std::vector<Box> eboxes;
    std::vector<int32_t> emat;   // two per edge
    for (size_t i = 0; i < keys.size();) {
        size_t j = i;
        while (j < keys.size() && keys[j].first == keys[i].first) ++j;
        if (j - i == 2) {
            const int64_t t0 = keys[i].second / 3, t1 = keys[i + 1].second / 3;
            const int e0 = (int)(keys[i].second % 3), e1 = (int)(keys[i + 1].second % 3);
            if (tri_mat[t0] != tri_mat[t1]) {
                const float* p0 = verts + 3 * (int64_t)tris[3 * t0 + e0];
                const float* p1 = verts + 3 * (int64_t)tris[3 * t0 + (e0 + 1) % 3];
                const float* q0 = verts + 3 * (int64_t)tris[3 * t0 + (e0 + 2) % 3];
                const float* q1 = verts + 3 * (int64_t)tris[3 * t1 + (e1 + 2) % 3];
                float rec[16];
                const int32_t ma = tri_mat[t0], mb = tri_mat[t1];
                for (int k = 0; k < 3; ++k) {
                    rec[k] = p0[k];
                    rec[4 + k] = p1[k];
                    rec[8 + k] = q0[k];
                    rec[12 + k] = q1[k];
                }
                std::memcpy(&rec[3], &ma, 4);
                std::memcpy(&rec[7], &mb, 4);
                rec[11] = rec[15] = 0.0f;
                out.edges.insert(out.edges.end(), rec, rec + 16);
                Box b;
                for (int k = 0; k < 3; ++k) {
                    b.lo[k] = std::min(p0[k], p1[k]);
                    b.hi[k] = std::max(p0[k], p1[k]);
                }
                eboxes.push_back(b);
                emat.push_back(ma);
                emat.push_back(mb);
            }
        }
        i = j;
    }
    const int64_t ne = (int64_t)eboxes.size();
    out.n_edges = ne;
    out.first.assign((size_t)nt, 0u);
    out.count.assign((size_t)nt, 0u);
    out.gap.assign((size_t)nt, 0.0f);
    if (ne == 0) return true;
    // uniform grid over the edges, hashed by cell coordinates: each edge is listed in every
    // cell that its box widened by reach touches, so a triangle within reach of it shares a
    // cell with it.  Cells at least reach and one mean edge extent wide.
    double ext = 0.0;
    for (const Box& b : eboxes)
        ext += std::max({b.hi[0] - b.lo[0], b.hi[1] - b.lo[1], b.hi[2] - b.lo[2]});
    const double h = std::max({(double)reach, ext / (double)ne, 1e-9});
    double org[3] = {1e300, 1e300, 1e300};
    for (const Box& b : eboxes)
        for (int k = 0; k < 3; ++k) org[k] = std::min(org[k], (double)b.lo[k] - (double)reach - h);
    auto cell = [&](double x, int k) { return (int64_t)std::floor((x - org[k]) / h); };
    auto key3 = [](int64_t x, int64_t y, int64_t z) {
        return ((uint64_t)(x & 0x1FFFFF) << 42) | ((uint64_t)(y & 0x1FFFFF) << 21) | (uint64_t)(z & 0x1FFFFF);
    };
    std::vector<std::pair<uint64_t, uint32_t>> cells;
    for (int64_t e = 0; e < ne; ++e) {
        const Box& b = eboxes[e];
        int64_t lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = cell((double)b.lo[k] - (double)reach, k);
            hi[k] = cell((double)b.hi[k] + (double)reach, k);
        }
        for (int64_t x = lo[0]; x <= hi[0]; ++x)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
                for (int64_t z = lo[2]; z <= hi[2]; ++z) cells.push_back({key3(x, y, z), (uint32_t)e});
    }
    std::sort(cells.begin(), cells.end());
    std::unordered_map<uint64_t, std::pair<size_t, size_t>> range;
    range.reserve(cells.size() / 2 + 1);
    for (size_t i = 0; i < cells.size();) {
        size_t j = i;
        while (j < cells.size() && cells[j].first == cells[i].first) ++j;
        range[cells[i].first] = {i, j};
        i = j;
    }
    const double r2 = (double)reach * (double)reach;
    std::vector<uint32_t> cand;
    for (int64_t t = 0; t < nt; ++t) {
        Box tb;
        for (int k = 0; k < 3; ++k) {
            tb.lo[k] = 3.4e38f;
            tb.hi[k] = -3.4e38f;
        }
        for (int c = 0; c < 3; ++c) {
            const float* p = verts + 3 * (int64_t)tris[3 * t + c];
            for (int k = 0; k < 3; ++k) {
                tb.lo[k] = std::min(tb.lo[k], p[k]);
                tb.hi[k] = std::max(tb.hi[k], p[k]);
            }
        }
        int64_t lo[3], hi[3];
        bool outside = false;
        for (int k = 0; k < 3; ++k) {
            lo[k] = cell(tb.lo[k], k);
            hi[k] = cell(tb.hi[k], k);
            if (hi[k] < 0) outside = true;
        }
        out.first[(size_t)t] = (uint32_t)out.idx.size();
        if (outside) continue;
        cand.clear();
        const int32_t m = tri_mat[t];
        for (int64_t x = std::max<int64_t>(lo[0], 0); x <= hi[0]; ++x)
            for (int64_t y = std::max<int64_t>(lo[1], 0); y <= hi[1]; ++y)
                for (int64_t z = std::max<int64_t>(lo[2], 0); z <= hi[2]; ++z) {
                    auto it = range.find(key3(x, y, z));
                    if (it == range.end()) continue;
                    for (size_t i = it->second.first; i < it->second.second; ++i) {
                        const uint32_t e = cells[i].second;
                        if (emat[2 * e] != m && emat[2 * e + 1] != m) continue;
                        if (box_gap2(tb, eboxes[e]) <= r2) cand.push_back(e);
                    }
                }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        // the smallest box gap to a listed edge bounds every hit's distance from below
        double g2 = 1e300;
        for (uint32_t e : cand) g2 = std::min(g2, box_gap2(tb, eboxes[e]));
        // rounded down to float, so that the bound stays a bound
        out.gap[(size_t)t] = cand.empty() ? 0.0f : std::nextafter((float)std::sqrt(g2), 0.0f);
        if (out.idx.size() + cand.size() >= (1ull << 32)) return false;
        out.idx.insert(out.idx.end(), cand.begin(), cand.end());
        out.count[(size_t)t] = (uint32_t)cand.size();
    }
    return true;
}

void weideman_coefficients(int n, float* a, float* L) {
    // f(theta) = exp(-t^2) (L^2 + t^2), t = L tan(theta / 2), is even in theta; its Fourier
    // cosine coefficients by the trapezoidal rule on 2M = 4n points (f vanishes at theta = pi)
    const double l = std::sqrt((double)n / std::sqrt(2.0));
    const int M = 2 * n;
    for (int k = 1; k <= n; ++k) {
        double s = 0.0;
        for (int j = -M + 1; j <= M - 1; ++j) {
            const double th = M_PI * (double)j / (double)M;
            const double t = l * std::tan(0.5 * th);
            s += std::exp(-t * t) * (l * l + t * t) * std::cos((double)k * th);
        }
        a[k - 1] = (float)(s / (2.0 * M));
    }
    *L = (float)l;
}

}  // namespace grw
