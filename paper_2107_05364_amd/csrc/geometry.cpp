// Geometry ingest: canonical hash and face-neighbour search (host side).
//
// Tiles are axis-aligned cuboids (paper Sec. 3).  Two tiles are exchange
// neighbours when they touch along one axis and share a face patch of
// positive area; the exchange operator uses the shared area S_ab and the
// centre distance d_ab along the normal (a two-point flux that equals the
// 3-point finite-difference Laplacian on a Cartesian mesh, Sec. 3).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace tmag {

// FNV-1a over the canonical bytes: n as int64, then every centre and edge as
// float64 with -0.0 folded into +0.0.
uint64_t geometry_hash(int64_t n, const double* centers, const double* sizes) {
    uint64_t h = 0xcbf29ce484222325ull;
    auto eat = [&h](const void* p, size_t len) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < len; ++i) {
            h ^= b[i];
            h *= 0x100000001b3ull;
        }
    };
    eat(&n, sizeof(n));
    for (int64_t i = 0; i < 3 * n; ++i) {
        double v = centers[i] == 0.0 ? 0.0 : centers[i];
        eat(&v, sizeof(v));
    }
    for (int64_t i = 0; i < 3 * n; ++i) {
        double v = sizes[i] == 0.0 ? 0.0 : sizes[i];
        eat(&v, sizeof(v));
    }
    return h;
}

namespace {
struct FaceRef {
    double key;    // face plane coordinate
    double lo1, hi1, lo2, hi2;
    int32_t tile;
};
}  // namespace

void find_faces(Geom& g) {
    const int64_t n = g.n;
    const double* c = g.centers.data();
    const double* s = g.sizes.data();
    double smin = s[0], smax = s[0];
    for (int64_t i = 0; i < 3 * n; ++i) {
        smin = std::min(smin, s[i]);
        smax = std::max(smax, s[i]);
    }
    const double tol = 1e-9 * smin;
    std::vector<std::vector<std::pair<int32_t, std::pair<double, double>>>> adj(n);
    for (int d = 0; d < 3; ++d) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        std::vector<FaceRef> up(n), dn(n);
        for (int64_t a = 0; a < n; ++a) {
            FaceRef f;
            f.lo1 = c[3 * a + e1] - 0.5 * s[3 * a + e1];
            f.hi1 = c[3 * a + e1] + 0.5 * s[3 * a + e1];
            f.lo2 = c[3 * a + e2] - 0.5 * s[3 * a + e2];
            f.hi2 = c[3 * a + e2] + 0.5 * s[3 * a + e2];
            f.tile = static_cast<int32_t>(a);
            f.key = c[3 * a + d] + 0.5 * s[3 * a + d];
            up[a] = f;
            f.key = c[3 * a + d] - 0.5 * s[3 * a + d];
            dn[a] = f;
        }
        // lower faces sorted by (plane, lo1) so that one plane's candidates
        // along e1 form a contiguous, searchable run
        auto by_plane_lo1 = [](const FaceRef& x, const FaceRef& y) {
            return x.key < y.key || (x.key == y.key && x.lo1 < y.lo1);
        };
        std::sort(dn.begin(), dn.end(), by_plane_lo1);
        for (int64_t a = 0; a < n; ++a) {
            const FaceRef& u = up[a];
            // all lower faces whose plane is within tol of u's plane
            auto first = std::lower_bound(dn.begin(), dn.end(), u.key - tol,
                                          [](const FaceRef& x, double v) { return x.key < v; });
            auto it = first;
            while (it != dn.end() && it->key <= u.key + tol) {
                // one run of identical plane keys, sorted by lo1: only faces
                // starting in (u.lo1 - smax, u.hi1) can overlap u along e1
                const double k = it->key;
                auto run_end = std::upper_bound(it, dn.end(), k,
                                                [](double v, const FaceRef& x) { return v < x.key; });
                auto q = std::lower_bound(it, run_end, u.lo1 - smax - tol,
                                          [](const FaceRef& x, double v) { return x.lo1 < v; });
                for (; q != run_end && q->lo1 < u.hi1 - tol; ++q) {
                    if (q->hi1 <= u.lo1 + tol) continue;
                    double o1 = std::min(u.hi1, q->hi1) - std::max(u.lo1, q->lo1);
                    double o2 = std::min(u.hi2, q->hi2) - std::max(u.lo2, q->lo2);
                    double t1 = 1e-9 * std::min(u.hi1 - u.lo1, q->hi1 - q->lo1);
                    double t2 = 1e-9 * std::min(u.hi2 - u.lo2, q->hi2 - q->lo2);
                    if (o1 <= t1 || o2 <= t2) continue;
                    const int32_t b = q->tile;
                    if (b == a) continue;
                    double area = o1 * o2;
                    double dist = std::fabs(c[3 * a + d] - c[3 * b + d]);
                    adj[a].push_back({b, {area, dist}});
                    adj[b].push_back({static_cast<int32_t>(a), {area, dist}});
                }
                it = run_end;
            }
        }
    }
    g.nbr_ptr.assign(n + 1, 0);
    for (int64_t a = 0; a < n; ++a) {
        std::sort(adj[a].begin(), adj[a].end(),
                  [](const auto& x, const auto& y) { return x.first < y.first; });
        g.nbr_ptr[a + 1] = g.nbr_ptr[a] + static_cast<int32_t>(adj[a].size());
    }
    g.nbr_idx.resize(g.nbr_ptr[n]);
    g.nbr_area.resize(g.nbr_ptr[n]);
    g.nbr_dist.resize(g.nbr_ptr[n]);
    for (int64_t a = 0; a < n; ++a) {
        int32_t o = g.nbr_ptr[a];
        for (size_t j = 0; j < adj[a].size(); ++j) {
            g.nbr_idx[o + j] = adj[a][j].first;
            g.nbr_area[o + j] = adj[a][j].second.first;
            g.nbr_dist[o + j] = adj[a][j].second.second;
        }
    }
}

}  // namespace tmag
