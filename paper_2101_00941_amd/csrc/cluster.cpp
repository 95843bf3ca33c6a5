// Cross-DM candidate clustering on the host (friends of friends): candidates of one beam
// whose trials differ by at most dm_radius and whose starts differ by at most t_radius
// are linked, and each connected component is reported once, by its highest-S/N member.
// Candidate lists are short next to the planes they come from (they cross PCIe anyway),
// and the grouping is irregular, so this runs in host code after the D2H copy.
//
// Method: sort by (beam, trial, start); for each candidate, link it to its predecessor
// in its own row when within t_radius (within a row, consecutive members within the
// radius connect the same components as all pairs do), and to every candidate of the
// dm_radius rows below it whose start lies within t_radius (binary search per row).
// Union-find with path halving keeps the smallest index as the root.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "aa_internal.h"

using namespace aa;

namespace {
struct Key {
    int32_t beam, dm;
    int64_t t;
};
bool key_less(const Key& a, const Key& b) {
    if (a.beam != b.beam) return a.beam < b.beam;
    if (a.dm != b.dm) return a.dm < b.dm;
    return a.t < b.t;
}
}  // namespace

extern "C" int aa_cluster(const aa_candidate_t* h_cand, int64_t n, int32_t dm_radius, int64_t t_radius,
                          aa_cluster_t* h_out, int64_t cap, int64_t* n_clusters) {
    if (n < 0 || (n > 0 && !h_cand) || dm_radius < 0 || t_radius < 0 || cap < 0 || (cap > 0 && !h_out) || !n_clusters)
        return fail(AA_EINVAL, "aa_cluster: bad argument");
    *n_clusters = 0;
    if (n == 0) return AA_OK;
    try {
        std::vector<int64_t> ord(static_cast<size_t>(n));
        std::iota(ord.begin(), ord.end(), 0);
        auto key = [&](int64_t i) { return Key{h_cand[i].beam, h_cand[i].dm_idx, h_cand[i].t}; };
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
            const Key ka = key(a), kb = key(b);
            if (key_less(ka, kb)) return true;
            if (key_less(kb, ka)) return false;
            return a < b;
        });
        // sorted copy of the keys and the start of each (beam, trial) row
        std::vector<Key> k(static_cast<size_t>(n));
        for (int64_t i = 0; i < n; ++i) k[i] = key(ord[i]);
        std::vector<int64_t> row_start;   // positions where a new (beam, dm) row starts
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || k[i].beam != k[i - 1].beam || k[i].dm != k[i - 1].dm) row_start.push_back(i);
        row_start.push_back(n);
        std::vector<int64_t> parent(static_cast<size_t>(n));
        std::iota(parent.begin(), parent.end(), 0);
        auto find = [&](int64_t i) {
            while (parent[i] != i) {
                parent[i] = parent[parent[i]];
                i = parent[i];
            }
            return i;
        };
        auto unite = [&](int64_t a, int64_t b) {
            a = find(a);
            b = find(b);
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        };
        const int64_t nrows = static_cast<int64_t>(row_start.size()) - 1;
        for (int64_t r = 0; r < nrows; ++r) {
            const int64_t r0 = row_start[r], r1 = row_start[r + 1];
            for (int64_t i = r0 + 1; i < r1; ++i)
                if (k[i].t - k[i - 1].t <= t_radius) unite(i, i - 1);
            // rows below within dm_radius (same beam), newest first
            for (int64_t q = r - 1; q >= 0; --q) {
                const int64_t q0 = row_start[q], q1 = row_start[q + 1];
                if (k[q0].beam != k[r0].beam || static_cast<int64_t>(k[r0].dm) - k[q0].dm > dm_radius) break;
                for (int64_t i = r0; i < r1; ++i) {
                    const int64_t lo_t = k[i].t - t_radius, hi_t = k[i].t + t_radius;
                    int64_t a = q0, b = q1;   // first position with t >= lo_t
                    while (a < b) {
                        const int64_t m = (a + b) / 2;
                        if (k[m].t < lo_t) a = m + 1; else b = m;
                    }
                    for (int64_t j = a; j < q1 && k[j].t <= hi_t; ++j) unite(i, j);
                }
            }
        }
        // one cluster per root: peak (highest S/N, then smallest trial, then start), size, extent
        std::vector<int64_t> slot(static_cast<size_t>(n), -1);
        std::vector<aa_cluster_t> cl;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t root = find(i);
            if (slot[root] < 0) {
                slot[root] = static_cast<int64_t>(cl.size());
                aa_cluster_t c{};
                c.peak = h_cand[ord[i]];
                c.members = 0;
                c.dm_lo = c.dm_hi = k[i].dm;
                c.t_lo = c.t_hi = k[i].t;
                cl.push_back(c);
            }
            aa_cluster_t& c = cl[slot[root]];
            const aa_candidate_t& x = h_cand[ord[i]];
            ++c.members;
            c.dm_lo = std::min(c.dm_lo, x.dm_idx);
            c.dm_hi = std::max(c.dm_hi, x.dm_idx);
            c.t_lo = std::min(c.t_lo, x.t);
            c.t_hi = std::max(c.t_hi, x.t);
            const bool better = x.snr > c.peak.snr ||
                                (x.snr == c.peak.snr && (x.dm_idx < c.peak.dm_idx ||
                                                         (x.dm_idx == c.peak.dm_idx && x.t < c.peak.t)));
            if (better) c.peak = x;
        }
        std::sort(cl.begin(), cl.end(), [](const aa_cluster_t& a, const aa_cluster_t& b) {
            if (a.peak.beam != b.peak.beam) return a.peak.beam < b.peak.beam;
            if (a.peak.dm_idx != b.peak.dm_idx) return a.peak.dm_idx < b.peak.dm_idx;
            return a.peak.t < b.peak.t;
        });
        *n_clusters = static_cast<int64_t>(cl.size());
        const int64_t m = std::min<int64_t>(cap, static_cast<int64_t>(cl.size()));
        if (m > 0) std::memcpy(h_out, cl.data(), static_cast<size_t>(m) * sizeof(aa_cluster_t));
        return static_cast<int64_t>(cl.size()) > cap ? fail(AA_EOVERFLOW, "aa_cluster: more clusters than cap") : AA_OK;
    } catch (const std::bad_alloc&) {
        return fail(AA_ENOMEM, "aa_cluster: out of host memory");
    }
}
