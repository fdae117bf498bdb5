// CH-partitioning by simulated annealing (host).
//
// The cost of a partition is eq. (4): C = sum_k s_k^3, s_k = c_k + h_k, the
// size of part k's core plus its one-hop halo in the undirected graph.  The
// paper's graph-theory section names simulated annealing on this cost as an
// alternative to METIS that usually lowers C further.  This refines a given
// partition by single-vertex moves with Metropolis acceptance:
//
//  * a move takes a vertex v from its part p to a part q, chosen among the
//    parts that hold a neighbour of v, or (one proposal in eight, and always
//    for a vertex with no neighbour outside p) among all other parts, so that
//    every partition is reachable; p must keep at least one vertex (the
//    number of parts is fixed: the paper reports that letting SA dissolve
//    parts hurt the load balance);
//  * the change of C is exact and local.  With n_k(w) the number of
//    neighbours of w in part k (before the move):
//        s_p' = s_p - 1 + [n_p(v) > 0] - #{w ~ v : part(w) != p, n_p(w) = 1}
//        s_q' = s_q + 1 - [n_q(v) > 0] + #{w ~ v : part(w) != q, n_q(w) = 0}
//    (v leaves p's core and may join p's halo; neighbours whose only link
//    into p was v leave p's halo; v leaves q's halo for q's core; neighbours
//    with no link into q before join q's halo);
//  * a move with change D is taken when D <= 0 or u < exp(-D / T), u uniform
//    from a seeded counter-based generator (splitmix64); T starts at t0
//    times 3 (C / n_parts)^(2/3), the change of C when a part of mean cost
//    grows by one vertex, and is multiplied by `cooling` after every sweep;
//  * the best partition seen at the end of a sweep (or the one given) is
//    returned.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <utility>
#include <vector>

#include "gsp2_internal.hpp"

namespace gsp2 {

namespace {

uint64_t splitmix64(uint64_t &state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &state) { return (double)(splitmix64(state) >> 11) * 0x1p-53; }

int64_t cube(int64_t s) { return s * s * s; }

// Neighbour counts of one vertex per part, as a short list of (part, count).
struct PartCounts {
    std::vector<std::pair<int32_t, int32_t>> v;
    int32_t get(int32_t k) const {
        for (const auto &e : v)
            if (e.first == k) return e.second;
        return 0;
    }
    void add(int32_t k, int32_t d) {
        for (auto &e : v)
            if (e.first == k) {
                e.second += d;
                return;
            }
        v.emplace_back(k, d);
    }
};

}  // namespace

AnnealResult anneal_partition(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col, int32_t n_parts,
                              int32_t *part, int32_t sweeps, double t0, double cooling, uint64_t seed) {
    // undirected, deduplicated neighbour lists without self loops
    std::vector<std::vector<int32_t>> nb(n);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = adj_ptr[u]; e < adj_ptr[u + 1]; ++e) {
            const int32_t w = adj_col[e];
            if (w == u) continue;
            nb[u].push_back(w);
            nb[w].push_back(u);
        }
    for (auto &l : nb) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    std::vector<PartCounts> cnt(n);
    std::vector<int64_t> core(n_parts, 0), halo(n_parts, 0);
    for (int32_t v = 0; v < n; ++v) {
        core[part[v]]++;
        for (int32_t w : nb[v]) cnt[v].add(part[w], 1);
    }
    for (int32_t v = 0; v < n; ++v)
        for (const auto &e : cnt[v].v)
            if (e.first != part[v] && e.second > 0) halo[e.first]++;
    auto size = [&](int32_t k) { return core[k] + halo[k]; };
    int64_t cost = 0;
    for (int32_t k = 0; k < n_parts; ++k) cost += cube(size(k));
    AnnealResult res{cost, cost, 0};
    std::vector<int32_t> best(part, part + n);
    int64_t best_cost = cost;
    uint64_t rng = seed;
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<int32_t> targets;
    double temp = t0 * 3.0 * std::pow((double)cost / n_parts, 2.0 / 3.0);
    for (int32_t sweep = 0; sweep < sweeps; ++sweep) {
        // a seeded shuffle of the visiting order
        for (int32_t i = n - 1; i > 0; --i) {
            const int32_t j = (int32_t)(splitmix64(rng) % (uint64_t)(i + 1));
            std::swap(order[i], order[j]);
        }
        for (int32_t v : order) {
            const int32_t p = part[v];
            if (core[p] <= 1) continue;
            if (n_parts < 2) break;
            targets.clear();
            for (const auto &e : cnt[v].v)
                if (e.first != p && e.second > 0) targets.push_back(e.first);
            int32_t q;
            if (targets.empty() || (splitmix64(rng) & 7u) == 0u) {
                q = (int32_t)(splitmix64(rng) % (uint64_t)(n_parts - 1));
                if (q >= p) ++q;
            } else {
                std::sort(targets.begin(), targets.end());
                q = targets[splitmix64(rng) % targets.size()];
            }
            int64_t dp = -1 + (cnt[v].get(p) > 0 ? 1 : 0);
            int64_t dq = 1 - (cnt[v].get(q) > 0 ? 1 : 0);
            for (int32_t w : nb[v]) {
                if (part[w] != p && cnt[w].get(p) == 1) dp -= 1;
                if (part[w] != q && cnt[w].get(q) == 0) dq += 1;
            }
            const int64_t sp = size(p), sq = size(q);
            const int64_t delta = cube(sp + dp) - cube(sp) + cube(sq + dq) - cube(sq);
            if (delta > 0 && !(temp > 0.0 && uniform01(rng) < std::exp(-(double)delta / temp))) continue;
            // apply: halo bookkeeping follows the same rules as the change of cost
            if (cnt[v].get(p) > 0) halo[p]++;
            if (cnt[v].get(q) > 0) halo[q]--;
            for (int32_t w : nb[v]) {
                if (part[w] != p && cnt[w].get(p) == 1) halo[p]--;
                if (part[w] != q && cnt[w].get(q) == 0) halo[q]++;
                cnt[w].add(p, -1);
                cnt[w].add(q, 1);
            }
            core[p]--;
            core[q]++;
            part[v] = q;
            cost += delta;
            res.moves++;
        }
        if (cost < best_cost) {
            best_cost = cost;
            std::copy(part, part + n, best.begin());
        }
        temp *= cooling;
    }
    std::copy(best.begin(), best.end(), part);
    res.cost_after = best_cost;
    return res;
}

}  // namespace gsp2

// ---------------------------------------------------------------------------
// Locality construction of the graph (host).
//
// The paper's graph-theory section notes that sub-problems can also be built
// from locality: beyond a localization radius the elements of P are taken as
// zero.  Here orbitals u != v are adjacent when their atoms lie closer than
// `radius` (minimum image in a cubic periodic box of edge `box`, or open
// boundaries for box <= 0); orbitals of one atom are always adjacent.  Atom
// pairs come from a cell list with cells no smaller than the radius (27
// neighbouring cells; a direct double loop when the box holds fewer than
// three cells per edge).
// ---------------------------------------------------------------------------
namespace gsp2 {

void locality_graph(int32_t n_orb, const int32_t *orbital_atom, int32_t n_atoms, const double *xyz, double radius,
                    double box, std::vector<int64_t> &adj_ptr, std::vector<int32_t> &adj_col) {
    const bool periodic = box > 0.0;
    const double r2 = radius * radius;
    auto dist2 = [&](int32_t a, int32_t b) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            double x = xyz[3 * b + d] - xyz[3 * a + d];
            if (periodic) x -= box * std::nearbyint(x / box);
            s += x * x;
        }
        return s;
    };
    // atom neighbour lists (both orientations), strict distance < radius
    std::vector<std::vector<int32_t>> anb(n_atoms);
    const int nc = periodic ? (int)std::floor(box / radius) : 0;
    if (periodic && nc >= 3) {
        auto cell_of = [&](int32_t a, int d) {
            double x = xyz[3 * a + d] - box * std::floor(xyz[3 * a + d] / box);   // wrap into [0, box)
            int c = (int)(x / box * nc);
            return c >= nc ? nc - 1 : c;
        };
        std::vector<std::vector<int32_t>> cells((size_t)nc * nc * nc);
        std::vector<int> cx(n_atoms), cy(n_atoms), cz(n_atoms);
        for (int32_t a = 0; a < n_atoms; ++a) {
            cx[a] = cell_of(a, 0); cy[a] = cell_of(a, 1); cz[a] = cell_of(a, 2);
            cells[((size_t)cx[a] * nc + cy[a]) * nc + cz[a]].push_back(a);
        }
        for (int32_t a = 0; a < n_atoms; ++a)
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int x = (cx[a] + dx + nc) % nc, y = (cy[a] + dy + nc) % nc, z = (cz[a] + dz + nc) % nc;
                        for (int32_t b : cells[((size_t)x * nc + y) * nc + z])
                            if (b != a && dist2(a, b) < r2) anb[a].push_back(b);
                    }
    } else {
        for (int32_t a = 0; a < n_atoms; ++a)
            for (int32_t b = 0; b < n_atoms; ++b)
                if (b != a && dist2(a, b) < r2) anb[a].push_back(b);
    }
    // orbitals of every atom
    std::vector<int64_t> aptr(n_atoms + 1, 0);
    for (int32_t u = 0; u < n_orb; ++u) aptr[orbital_atom[u] + 1]++;
    for (int32_t a = 0; a < n_atoms; ++a) aptr[a + 1] += aptr[a];
    std::vector<int32_t> aorb(n_orb);
    {
        std::vector<int64_t> fill(aptr.begin(), aptr.end() - 1);
        for (int32_t u = 0; u < n_orb; ++u) aorb[fill[orbital_atom[u]]++] = u;
    }
    adj_ptr.assign(n_orb + 1, 0);
    adj_col.clear();
    std::vector<int32_t> row;
    for (int32_t u = 0; u < n_orb; ++u) {
        const int32_t a = orbital_atom[u];
        row.clear();
        for (int64_t i = aptr[a]; i < aptr[a + 1]; ++i)
            if (aorb[i] != u) row.push_back(aorb[i]);
        for (int32_t b : anb[a])
            for (int64_t i = aptr[b]; i < aptr[b + 1]; ++i) row.push_back(aorb[i]);
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        adj_col.insert(adj_col.end(), row.begin(), row.end());
        adj_ptr[u + 1] = (int64_t)adj_col.size();
    }
}

}  // namespace gsp2
