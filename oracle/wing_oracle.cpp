// Sequential CPU oracle for per-edge butterfly counts, wing decomposition and
// k-tip extraction on bipartite graphs.
//
// TEST INFRASTRUCTURE ONLY.  Like tip_oracle.cpp it is the checker the GPU
// path is compared against; the product library never links, loads or calls
// it, and it shares no code, header or helper with the product.
//
// What it computes (Lakhotia et al., "RECEIPT", arXiv 2010.08695):
//   * the butterflies containing each edge (the edge analogue of the
//     per-vertex counts of Section 2.1): for e = (u, v), every u' != u
//     adjacent to v closes a butterfly with e through each common neighbour
//     v' != v of u and u', so the count is the sum over u' in N_v, u' != u,
//     of (|N_u intersect N_u'| - 1);
//   * wing numbers by sequential bottom-up edge peeling (the edge-peeling
//     extension named in the Extensions section: the k-wing is the edge analogue of
//     the k-tip, every edge in at least k butterflies of the subgraph): edges
//     leave in order of least support, each with the support it has when it
//     leaves (never less than any earlier wing number); every butterfly it
//     closed with remaining edges is lost by the other three edges;
//   * k-tips (Def. 1): for one side, the maximal vertex sets in which every
//     vertex has at least k butterflies and every two vertices are joined by
//     a chain of butterflies; they are the butterfly-connected components of
//     {x : theta_x >= k} (a vertex's butterfly partners inside that set all
//     lie in its component, so its count there is at least k), found here by
//     breadth-first search over pairs sharing two or more neighbours.
//
// Edges are reported in canonical order: duplicates merged, sorted by (u, v).
//
// Build: compiled together with tip_oracle.cpp into liboracle.so.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

struct EdgeGraph {
    int32_t n_u = 0, n_v = 0;
    std::vector<int32_t> eu, ev;                                // canonical edges
    std::vector<std::vector<std::pair<int32_t, int64_t>>> nu;  // N_u: (v, edge id)
    std::vector<std::vector<std::pair<int32_t, int64_t>>> nv;  // N_v: (u, edge id)
};

bool build_edges(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev, EdgeGraph& g) {
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve(static_cast<size_t>(m));
    for (int64_t i = 0; i < m; ++i) {
        if (eu[i] < 0 || eu[i] >= n_u || ev[i] < 0 || ev[i] >= n_v) return false;
        e.emplace_back(eu[i], ev[i]);
    }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    g.n_u = n_u;
    g.n_v = n_v;
    g.eu.resize(e.size());
    g.ev.resize(e.size());
    g.nu.assign(n_u, {});
    g.nv.assign(n_v, {});
    for (size_t i = 0; i < e.size(); ++i) {
        g.eu[i] = e[i].first;
        g.ev[i] = e[i].second;
        g.nu[e[i].first].emplace_back(e[i].second, (int64_t)i);
        g.nv[e[i].second].emplace_back(e[i].first, (int64_t)i);
    }
    return true;
}

bool args_ok(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev) {
    return n_u >= 0 && n_v >= 0 && m >= 0 && (m == 0 || (eu && ev));
}

}  // namespace

extern "C" {

// Canonical edges (duplicates merged, sorted by (u, v)): cu, cv [m] may be
// NULL; *m_unique receives their number.  Returns 0, or -1 on bad input.
int oracle_canonical_edges(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
                           int32_t* cu, int32_t* cv, int64_t* m_unique) {
    if (!args_ok(n_u, n_v, m, eu, ev) || !m_unique) return -1;
    EdgeGraph g;
    if (!build_edges(n_u, n_v, m, eu, ev, g)) return -1;
    *m_unique = (int64_t)g.eu.size();
    if (cu) std::memcpy(cu, g.eu.data(), sizeof(int32_t) * g.eu.size());
    if (cv) std::memcpy(cv, g.ev.data(), sizeof(int32_t) * g.ev.size());
    return 0;
}

// Butterflies containing each canonical edge.  cnt has m_unique entries.
int oracle_edge_count(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev, int64_t* cnt) {
    if (!args_ok(n_u, n_v, m, eu, ev) || (m > 0 && !cnt)) return -1;
    EdgeGraph g;
    if (!build_edges(n_u, n_v, m, eu, ev, g)) return -1;
    std::vector<int32_t> co(n_u, 0);  // |N_u intersect N_u'| for the current u
    std::vector<int32_t> met;
    for (int32_t u = 0; u < n_u; ++u) {
        met.clear();
        for (auto& yv : g.nu[u])
            for (auto& xu : g.nv[yv.first])
                if (xu.first != u && co[xu.first]++ == 0) met.push_back(xu.first);
        for (auto& yv : g.nu[u]) {
            int64_t s = 0;
            for (auto& xu : g.nv[yv.first])
                if (xu.first != u) s += co[xu.first] - 1;
            cnt[yv.second] = s;
        }
        for (int32_t w : met) co[w] = 0;
    }
    return 0;
}

// Wing numbers of the canonical edges by bottom-up edge peeling.
//   psi    [m_unique] output
//   order  [m_unique] optional: edge ids in the order they left the graph
//   wedges optional: number of (u', v') pairs examined while removing edges
// The edges wait in a bucket queue keyed by support (stale entries are
// skipped); the smallest key is the level, and an edge lowered to the level
// joins the level's bag.
int oracle_wing(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev, int64_t* psi,
                int64_t* order, int64_t* wedges) {
    if (!args_ok(n_u, n_v, m, eu, ev) || (m > 0 && !psi)) return -1;
    EdgeGraph g;
    if (!build_edges(n_u, n_v, m, eu, ev, g)) return -1;
    const int64_t ne = (int64_t)g.eu.size();
    std::vector<int64_t> supp(ne);
    if (oracle_edge_count(n_u, n_v, m, eu, ev, supp.data()) != 0) return -1;

    std::map<int64_t, std::vector<int64_t>> queue;
    for (int64_t e = 0; e < ne; ++e) queue[supp[e]].push_back(e);
    int64_t filed = ne;
    std::vector<char> gone(ne, 0);
    std::vector<int64_t> tag(n_v, -1);  // tag[v'] = id of the remaining edge (u, v') of the edge leaving
    std::vector<int64_t> rest(ne);         // every edge still in the graph, and some that left
    for (int64_t e = 0; e < ne; ++e) rest[e] = e;
    int64_t examined = 0, left_graph = 0;

    while (!queue.empty()) {
        const int64_t level = queue.begin()->first;
        std::vector<int64_t> bag = std::move(queue.begin()->second);
        queue.erase(queue.begin());
        filed -= (int64_t)bag.size();
        for (size_t i = 0; i < bag.size(); ++i) {
            const int64_t e = bag[i];
            if (gone[e] || supp[e] != level) continue;  // stale entry
            gone[e] = 1;
            psi[e] = level;
            if (order) order[left_graph] = e;
            ++left_graph;
            const int32_t u = g.eu[e], v = g.ev[e];
            auto lower = [&](int64_t f) {
                const int64_t lowered = std::max(level, supp[f] - 1);
                if (lowered == supp[f]) return;
                supp[f] = lowered;
                if (lowered == level) {
                    bag.push_back(f);
                } else {
                    queue[lowered].push_back(f);
                    ++filed;
                }
            };
            for (auto& yv : g.nu[u])
                if (!gone[yv.second]) tag[yv.first] = yv.second;
            for (auto& xu : g.nv[v]) {
                const int32_t u2 = xu.first;
                const int64_t e3 = xu.second;  // (u', v)
                if (u2 == u || gone[e3]) continue;
                for (auto& yv : g.nu[u2]) {
                    const int64_t e4 = yv.second;  // (u', v')
                    ++examined;
                    if (yv.first == v || gone[e4] || tag[yv.first] < 0) continue;
                    // butterfly {u, u'} x {v, v'}: its other three edges lose it
                    lower(tag[yv.first]);
                    lower(e3);
                    lower(e4);
                }
            }
            for (auto& yv : g.nu[u]) tag[yv.first] = -1;

            const int64_t remaining = ne - left_graph;
            if (filed > 4 * remaining + 4096) {
                queue.clear();
                filed = 0;
                size_t k = 0;
                for (int64_t f : rest)
                    if (!gone[f]) rest[k++] = f;
                rest.resize(k);
                for (int64_t f : rest)
                    if (supp[f] > level) {
                        queue[supp[f]].push_back(f);
                        ++filed;
                    }
            }
        }
    }
    if (wedges) *wedges = examined;
    return 0;
}

// k-tips of side `side` (0 = U, 1 = V) given its tip numbers: comp[x] = the
// smallest vertex id of x's k-tip, or -1 when theta[x] < k.
int oracle_ktip(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev, int32_t side,
                const int64_t* theta, int64_t k, int32_t* comp) {
    if (!args_ok(n_u, n_v, m, eu, ev) || !theta || !comp || (side != 0 && side != 1)) return -1;
    EdgeGraph g;
    if (!build_edges(n_u, n_v, m, eu, ev, g)) return -1;
    const int32_t n = side == 0 ? n_u : n_v;
    const auto& own = side == 0 ? g.nu : g.nv;    // x -> other side
    const auto& other = side == 0 ? g.nv : g.nu;  // other side -> x
    std::vector<int32_t> co(n, 0), met, stack;
    for (int32_t x = 0; x < n; ++x) comp[x] = -1;
    for (int32_t s = 0; s < n; ++s) {
        if (theta[s] < k || comp[s] >= 0) continue;
        // the search visits vertices in any order; the label is fixed to the
        // smallest id of the component afterwards
        std::vector<int32_t> members{s};
        comp[s] = s;
        stack.assign(1, s);
        while (!stack.empty()) {
            const int32_t x = stack.back();
            stack.pop_back();
            met.clear();
            for (auto& y : own[x])
                for (auto& w : other[y.first])
                    if (w.first != x && theta[w.first] >= k && co[w.first]++ == 0) met.push_back(w.first);
            for (int32_t w : met) {
                if (co[w] >= 2 && comp[w] < 0) {  // x and w share a butterfly
                    comp[w] = s;
                    members.push_back(w);
                    stack.push_back(w);
                }
                co[w] = 0;
            }
        }
        const int32_t lo = *std::min_element(members.begin(), members.end());
        for (int32_t x : members) comp[x] = lo;
    }
    return 0;
}

}  // extern "C"
