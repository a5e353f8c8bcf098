// Host-side RWG table, mesh validation and flagged-pair list.
//
// RWG functions without edge-length normalisation (Sec. II): one unknown per
// interior edge; on triangle p of f_m, f_m = s_p (r - v_p)/(2 A_p), with
// s_p = +1 on c+ and -1 on c-, v_p the free vertex (Sec. VI-A sketch).
// Numbering reading: edges sorted by (lower, higher vertex index); c+
// traverses the edge from the lower to the higher index.
#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>

#include "bie_internal.hpp"

namespace bie {

namespace {

struct HalfEdge {
    int32_t lo, hi;   // undirected key
    int32_t tri;      // owning triangle
    int8_t slot;      // local slot a = vertex opposite the edge
    int8_t forward;   // 1 if the triangle traverses lo -> hi
};

}  // namespace

Mesh build_mesh(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double near_factor)
{
    if (nv < 3 || nt < 1) throw Error(BIE_EMESH, "mesh needs at least 3 vertices and 1 triangle");
    if (nt > (int64_t(1) << 30)) throw Error(BIE_EINVAL, "too many triangles");
    Mesh M;
    M.nv = nv;
    M.F = nt;
    M.V.assign(verts, verts + 3 * nv);
    M.T.assign(tris, tris + 3 * nt);
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(M.V[i])) throw Error(BIE_EMESH, "non-finite vertex coordinate");
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (M.T[i] < 0 || M.T[i] >= nv) throw Error(BIE_EMESH, "vertex index out of range");

    const int64_t F = nt;
    M.area.resize(F);
    M.cent.resize(3 * F);
    M.longest.resize(F);
    for (int64_t t = 0; t < F; ++t) {
        const double *a = &M.V[3 * M.T[3 * t]], *b = &M.V[3 * M.T[3 * t + 1]], *c = &M.V[3 * M.T[3 * t + 2]];
        double e1[3], e2[3], e3[3];
        for (int d = 0; d < 3; ++d) { e1[d] = b[d] - a[d]; e2[d] = c[d] - a[d]; e3[d] = c[d] - b[d]; }
        double cr[3] = { e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0] };
        double tw = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(tw > 0.0)) throw Error(BIE_EMESH, "zero-area triangle " + std::to_string(t));
        M.area[t] = 0.5 * tw;
        for (int d = 0; d < 3; ++d) M.cent[3 * t + d] = (a[d] + b[d] + c[d]) / 3.0;
        auto len = [](const double *v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); };
        M.longest[t] = std::max(len(e1), std::max(len(e2), len(e3)));
    }

    // Half-edges sorted by undirected key, then direction; a closed,
    // consistently oriented 2-manifold has exactly one forward and one
    // backward half-edge per key.
    std::vector<HalfEdge> he;
    he.reserve(3 * F);
    for (int64_t t = 0; t < F; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t i = M.T[3 * t + k], j = M.T[3 * t + (k + 1) % 3];
            if (i == j) throw Error(BIE_EMESH, "degenerate triangle");
            HalfEdge h;
            h.lo = std::min(i, j);
            h.hi = std::max(i, j);
            h.tri = int32_t(t);
            h.slot = int8_t((k + 2) % 3);
            h.forward = i < j ? 1 : 0;
            he.push_back(h);
        }
    std::sort(he.begin(), he.end(), [](const HalfEdge &x, const HalfEdge &y) {
        if (x.lo != y.lo) return x.lo < y.lo;
        if (x.hi != y.hi) return x.hi < y.hi;
        return x.forward > y.forward;
    });
    if (he.size() % 2) throw Error(BIE_EMESH, "open mesh");
    const int64_t N = int64_t(he.size() / 2);
    M.N = N;
    M.edges.resize(4 * N);
    M.slot_m.assign(3 * F, -1);
    M.slot_s.assign(3 * F, 0);
    for (int64_t m = 0; m < N; ++m) {
        const HalfEdge &p = he[2 * m], &q = he[2 * m + 1];
        if (p.lo != q.lo || p.hi != q.hi)
            throw Error(BIE_EMESH, "open or non-manifold mesh at edge (" + std::to_string(p.lo) + "," +
                                       std::to_string(p.hi) + ")");
        if (!(p.forward == 1 && q.forward == 0))
            throw Error(BIE_EMESH, "inconsistent orientation at edge (" + std::to_string(p.lo) + "," +
                                       std::to_string(p.hi) + ")");
        if (m + 1 < N && he[2 * m + 2].lo == p.lo && he[2 * m + 2].hi == p.hi)
            throw Error(BIE_EMESH, "non-manifold edge");
        M.edges[4 * m + 0] = p.lo;
        M.edges[4 * m + 1] = p.hi;
        M.edges[4 * m + 2] = p.tri;
        M.edges[4 * m + 3] = q.tri;
        M.slot_m[3 * p.tri + p.slot] = int32_t(m);
        M.slot_s[3 * p.tri + p.slot] = 1;
        M.slot_m[3 * q.tri + q.slot] = int32_t(m);
        M.slot_s[3 * q.tri + q.slot] = -1;
    }
    for (int64_t i = 0; i < 3 * F; ++i)
        if (M.slot_m[i] < 0) throw Error(BIE_EMESH, "edge without two triangles");

    // Flagged pairs: share a vertex, or centroid distance^2 < (f * max longest)^2.
    // Uniform grid over centroids with cell size >= the largest threshold.
    double Lmax = 0.0;
    for (double l : M.longest) Lmax = std::max(Lmax, l);
    const double cell = near_factor * Lmax;
    double lo[3] = { 1e300, 1e300, 1e300 };
    for (int64_t t = 0; t < F; ++t)
        for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], M.cent[3 * t + d]);
    auto key = [&](int64_t ix, int64_t iy, int64_t iz) { return (ix * 1000003LL + iy) * 1000033LL + iz; };
    std::unordered_map<int64_t, std::vector<int32_t>> grid;
    std::vector<std::array<int64_t, 3>> cellof(F);
    for (int64_t t = 0; t < F; ++t) {
        std::array<int64_t, 3> c;
        for (int d = 0; d < 3; ++d) c[d] = int64_t(std::floor((M.cent[3 * t + d] - lo[d]) / cell));
        cellof[t] = c;
        grid[key(c[0], c[1], c[2])].push_back(int32_t(t));
    }
    // vertex -> triangles, for the touching test
    std::vector<std::vector<int32_t>> vt(nv);
    for (int64_t t = 0; t < F; ++t)
        for (int k = 0; k < 3; ++k) vt[M.T[3 * t + k]].push_back(int32_t(t));
    std::vector<int32_t> cand;
    for (int64_t p = 0; p < F; ++p) {
        cand.clear();
        for (int k = 0; k < 3; ++k)
            for (int32_t q : vt[M.T[3 * p + k]])
                if (q >= p) cand.push_back(q);
        const auto &c = cellof[p];
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = grid.find(key(c[0] + dx, c[1] + dy, c[2] + dz));
                    if (it == grid.end()) continue;
                    for (int32_t q : it->second) {
                        if (q < p) continue;
                        double dd[3];
                        for (int d = 0; d < 3; ++d) dd[d] = M.cent[3 * p + d] - M.cent[3 * q + d];
                        double d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
                        double thr = near_factor * std::max(M.longest[p], M.longest[q]);
                        if (d2 < thr * thr) cand.push_back(q);
                    }
                }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int32_t q : cand) {
            M.near.push_back(int32_t(p));
            M.near.push_back(q);
        }
    }
    return M;
}

}  // namespace bie
