// Sequential CPU oracle for bipartite butterfly counting and tip decomposition.
//
// TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU path is compared
// against.  Only the tests, the smoke check and the benchmark's CPU-baseline
// leg may load it; the product library never links, loads or calls it, and it
// shares no code, header or helper with the product.
//
// What it computes (Lakhotia et al., "RECEIPT", arXiv 2010.08695):
//   * per-vertex butterfly counts by the plain definition: for u on one side,
//     the support is the sum over same-side w != u of C(c(u,w), 2), where
//     c(u,w) = |N_u intersect N_w| (notation table; Alg. 2 "update" computes
//     the same shared-butterfly term).  The counting-specific vertex-priority
//     trick of Alg. 1 is deliberately NOT used here, so the oracle stays
//     independent of the GPU's counting method.
//   * tip numbers by sequential bottom-up peeling (Alg. 2, BUP, Section 2.2):
//     vertices leave the graph in order of least support; each gets the
//     support it has when it leaves (never less than any earlier tip number)
//     as its tip number, and the vertices that remain lose the butterflies
//     they shared with it.
//   * f_u(S): the butterflies of u inside the subgraph induced on S and the
//     whole other side, for sampled property checks at any size; also for
//     the three sets a tip-number array defines around u at once (all of the
//     side, theta >= theta_u, theta > theta_u).
//
// Readings of the paper taken here:
//   * Vertices already peeled are not updated (the update has no effect on
//     them; Lemma 2 makes the same remark for the parallel case).
//   * Among vertices of equal least support, the one filed first leaves
//     first; tip numbers do not depend on that order.
//   * Duplicate input edges are merged (the datasets are simple graphs).
//   * All counts are exact 64-bit integers.
//
// Build: g++ -O2 -std=c++17 -shared -fPIC tip_oracle.cpp -o liboracle.so
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

struct Adjacency {
    // adjacency of the side being examined ("A") and of the other side ("B")
    int32_t n_a = 0, n_b = 0;
    std::vector<std::vector<int32_t>> a_to_b;  // N_x for x in A
    std::vector<std::vector<int32_t>> b_to_a;  // N_y for y in B
};

int64_t choose2(int64_t c) { return c * (c - 1) / 2; }

// Builds the simple graph (duplicates merged) with side `side` as A.
// Returns false if any id is out of range.
bool build(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
           int32_t side, Adjacency& g) {
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve(static_cast<size_t>(m));
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = eu[i], v = ev[i];
        if (u < 0 || u >= n_u || v < 0 || v >= n_v) return false;
        if (side == 0) e.emplace_back(u, v);
        else e.emplace_back(v, u);
    }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    g.n_a = side == 0 ? n_u : n_v;
    g.n_b = side == 0 ? n_v : n_u;
    g.a_to_b.assign(g.n_a, {});
    g.b_to_a.assign(g.n_b, {});
    for (auto& p : e) {
        g.a_to_b[p.first].push_back(p.second);
        g.b_to_a[p.second].push_back(p.first);
    }
    return true;
}

// Support of every vertex of A: sum over w != x of C(c(x,w), 2).  Each
// unordered pair {x, w} is visited once (w > x) and credited to both ends.
void count_side(const Adjacency& g, int64_t* out) {
    std::vector<int32_t> cnt(g.n_a, 0);
    std::vector<int32_t> touched;
    for (int32_t x = 0; x < g.n_a; ++x) out[x] = 0;
    for (int32_t x = 0; x < g.n_a; ++x) {
        touched.clear();
        for (int32_t y : g.a_to_b[x])
            for (int32_t w : g.b_to_a[y])
                if (w > x) {
                    if (cnt[w] == 0) touched.push_back(w);
                    ++cnt[w];
                }
        for (int32_t w : touched) {
            int64_t b = choose2(cnt[w]);
            out[x] += b;
            out[w] += b;
            cnt[w] = 0;
        }
    }
}

}  // namespace

extern "C" {

// Per-vertex butterfly counts of both sides and the total number of
// butterflies B (each butterfly has two vertices per side, so B is half the
// sum of either side's counts).  Returns 0, or -1 on an invalid argument.
int oracle_count(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
                 int64_t* bfly_u, int64_t* bfly_v, int64_t* total) {
    if (n_u < 0 || n_v < 0 || m < 0 || (m > 0 && (!eu || !ev))) return -1;
    Adjacency gu, gv;
    if (!build(n_u, n_v, m, eu, ev, 0, gu)) return -1;
    if (!build(n_u, n_v, m, eu, ev, 1, gv)) return -1;
    std::vector<int64_t> bu(n_u), bv(n_v);
    count_side(gu, bu.data());
    count_side(gv, bv.data());
    int64_t s = 0;
    for (int64_t x : bu) s += x;
    if (bfly_u) std::memcpy(bfly_u, bu.data(), sizeof(int64_t) * n_u);
    if (bfly_v) std::memcpy(bfly_v, bv.data(), sizeof(int64_t) * n_v);
    if (total) *total = s / 2;
    return 0;
}

// Per-vertex butterfly counts of side `side` only (0 = U, 1 = V): the same
// plain definition as oracle_count, for graphs whose other side would take
// far longer to count.  Returns 0, or -1 on an invalid argument.
int oracle_count_side(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
                      int32_t side, int64_t* bfly) {
    if (n_u < 0 || n_v < 0 || m < 0 || (m > 0 && (!eu || !ev)) || !bfly) return -1;
    if (side != 0 && side != 1) return -1;
    Adjacency g;
    if (!build(n_u, n_v, m, eu, ev, side, g)) return -1;
    count_side(g, bfly);
    return 0;
}

// Tip numbers of side `side` (0 = U, 1 = V) by sequential bottom-up peeling
// (Alg. 2, Section 2.2).
//
// The vertices of the side wait in a bucket queue keyed by support: `queue`
// maps a support value to the vertices filed under it.  An entry is stale
// once its vertex has left the graph or been re-filed under a smaller value;
// only entries whose key equals the vertex's present support count.  The
// smallest key is the current level.  Vertices at the level leave the graph
// one at a time, each with tip number = level.  When x leaves, every vertex
// w that remains loses the butterflies it shared with x: C(co[w], 2), where
// co[w] is the co-degree |N_x intersect N_w| gathered by walking x's 2-hop
// neighbourhood.  A support never drops below the level (the tip number just
// assigned), so a vertex lowered that far joins the level's own bag and
// leaves later in the same level.
//
//   theta  [n_side]  output tip numbers
//   order  [n_side]  optional: vertices in the order they left the graph
//   wedges           optional: number of (x, y, w) paths with w != x walked
//                    while removing vertices
// Returns 0, or -1 on an invalid argument.
int oracle_bup(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
               int32_t side, int64_t* theta, int32_t* order, int64_t* wedges) {
    if (n_u < 0 || n_v < 0 || m < 0 || (m > 0 && (!eu || !ev)) || !theta) return -1;
    if (side != 0 && side != 1) return -1;
    Adjacency g;
    if (!build(n_u, n_v, m, eu, ev, side, g)) return -1;
    const int32_t n = g.n_a;

    // every vertex starts with its butterfly count in the whole graph
    std::vector<int64_t> supp(n);
    count_side(g, supp.data());

    std::map<int64_t, std::vector<int32_t>> queue;
    for (int32_t x = 0; x < n; ++x) queue[supp[x]].push_back(x);
    int64_t filed = n;  // entries held by `queue`, stale ones included

    std::vector<char> gone(n, 0);
    std::vector<int32_t> co(n, 0);
    std::vector<int32_t> met;  // vertices with co > 0 for the vertex leaving
    std::vector<int32_t> rest(n);  // every vertex still in the graph, and some that left
    for (int32_t x = 0; x < n; ++x) rest[x] = x;
    int64_t walked = 0;
    int32_t left_graph = 0;

    while (!queue.empty()) {
        const int64_t level = queue.begin()->first;
        std::vector<int32_t> bag = std::move(queue.begin()->second);
        queue.erase(queue.begin());
        filed -= static_cast<int64_t>(bag.size());
        for (size_t i = 0; i < bag.size(); ++i) {
            const int32_t x = bag[i];
            if (gone[x] || supp[x] != level) continue;  // stale entry
            gone[x] = 1;
            theta[x] = level;
            if (order) order[left_graph] = x;
            ++left_graph;

            met.clear();
            for (int32_t y : g.a_to_b[x])
                for (int32_t w : g.b_to_a[y]) {
                    if (w == x) continue;
                    ++walked;
                    if (co[w]++ == 0) met.push_back(w);
                }
            for (int32_t w : met) {
                const int64_t shared = choose2(co[w]);
                co[w] = 0;
                if (gone[w] || shared == 0) continue;
                const int64_t lowered = std::max(level, supp[w] - shared);
                if (lowered == supp[w]) continue;
                supp[w] = lowered;
                if (lowered == level) {
                    bag.push_back(w);
                } else {
                    queue[lowered].push_back(w);
                    ++filed;
                }
            }

            // Bound the queue's memory: once stale entries dominate, file
            // every remaining vertex above the level afresh (those at the
            // level are already in the bag).  `rest` drops the vertices that
            // left, so this costs time in proportion to what remains.
            const int64_t remaining = static_cast<int64_t>(n) - left_graph;
            if (filed > 4 * remaining + 4096) {
                queue.clear();
                filed = 0;
                size_t k = 0;
                for (int32_t z : rest)
                    if (!gone[z]) rest[k++] = z;
                rest.resize(k);
                for (int32_t z : rest)
                    if (supp[z] > level) {
                        queue[supp[z]].push_back(z);
                        ++filed;
                    }
            }
        }
    }
    if (wedges) *wedges = walked;
    return 0;
}

// f_x(S) for each query vertex x of side `side`: the sum over w in S, w != x,
// of C(c(x,w), 2).  `member[w]` != 0 marks S.  With S = the whole side this is
// the butterfly count of x.  Returns 0, or -1 on an invalid argument.
int oracle_support_in(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu,
                      const int32_t* ev, int32_t side, const uint8_t* member,
                      const int32_t* query, int64_t n_query, int64_t* out) {
    if (n_u < 0 || n_v < 0 || m < 0 || (m > 0 && (!eu || !ev)) || !member || !out) return -1;
    if (side != 0 && side != 1) return -1;
    if (n_query > 0 && !query) return -1;
    Adjacency g;
    if (!build(n_u, n_v, m, eu, ev, side, g)) return -1;
    std::vector<int32_t> cnt(g.n_a, 0);
    std::vector<int32_t> touched;
    for (int64_t q = 0; q < n_query; ++q) {
        const int32_t x = query[q];
        if (x < 0 || x >= g.n_a) return -1;
        touched.clear();
        for (int32_t y : g.a_to_b[x])
            for (int32_t w : g.b_to_a[y])
                if (w != x && member[w]) {
                    if (cnt[w] == 0) touched.push_back(w);
                    ++cnt[w];
                }
        int64_t s = 0;
        for (int32_t w : touched) {
            s += choose2(cnt[w]);
            cnt[w] = 0;
        }
        out[q] = s;
    }
    return 0;
}

// For each query x, three values of f_x(S) from one walk of x's wedges:
// out[3q] with S = all of side A, out[3q+1] with S = {w : theta[w] >= theta[x]}
// and out[3q+2] with S = {w : theta[w] > theta[x]} (x itself never counts).
int oracle_support_levels(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu,
                          const int32_t* ev, int32_t side, const int64_t* theta,
                          const int32_t* query, int64_t n_query, int64_t* out) {
    if (n_u < 0 || n_v < 0 || m < 0 || (m > 0 && (!eu || !ev)) || !theta || !out) return -1;
    if (side != 0 && side != 1) return -1;
    if (n_query > 0 && !query) return -1;
    Adjacency g;
    if (!build(n_u, n_v, m, eu, ev, side, g)) return -1;
    std::vector<int32_t> cnt(g.n_a, 0);
    std::vector<int32_t> touched;
    for (int64_t q = 0; q < n_query; ++q) {
        const int32_t x = query[q];
        if (x < 0 || x >= g.n_a) return -1;
        touched.clear();
        for (int32_t y : g.a_to_b[x])
            for (int32_t w : g.b_to_a[y])
                if (w != x) {
                    if (cnt[w] == 0) touched.push_back(w);
                    ++cnt[w];
                }
        int64_t all = 0, ge = 0, gt = 0;
        for (int32_t w : touched) {
            const int64_t f = choose2(cnt[w]);
            all += f;
            if (theta[w] >= theta[x]) ge += f;
            if (theta[w] > theta[x]) gt += f;
            cnt[w] = 0;
        }
        out[3 * q] = all;
        out[3 * q + 1] = ge;
        out[3 * q + 2] = gt;
    }
    return 0;
}

}  // extern "C"
