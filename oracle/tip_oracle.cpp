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
//     repeatedly take the remaining vertex of minimum support, record its
//     support as its tip number, and lower every remaining vertex u' by the
//     butterflies it shares with it, never below the recorded value.
//   * f_u(S): the butterflies of u inside the subgraph induced on S and the
//     whole other side, for sampled property checks at any size; also for
//     the three sets a tip-number array defines around u at once (all of the
//     side, theta >= theta_u, theta > theta_u).
//
// Readings of the paper taken here:
//   * Vertices already peeled are not updated (the update has no effect on
//     them; Lemma 2 makes the same remark for the parallel case).
//   * Ties in the minimum support are broken by vertex id; tip numbers do not
//     depend on the tie order.
//   * Duplicate input edges are merged (the datasets are simple graphs).
//   * All counts are exact 64-bit integers.
//
// Build: g++ -O2 -std=c++17 -shared -fPIC tip_oracle.cpp -o liboracle.so
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <queue>
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

// Tip numbers of side `side` (0 = U, 1 = V) by bottom-up peeling, Alg. 2.
//   theta  [n_side]  output tip numbers
//   order  [n_side]  optional: vertices in the order they were peeled
//   wedges           optional: number of (u, v, u') triples with u' != u that
//                    the update routine visited
// Returns 0, or -1 on an invalid argument.
int oracle_bup(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
               int32_t side, int64_t* theta, int32_t* order, int64_t* wedges) {
    if (n_u < 0 || n_v < 0 || m < 0 || (m > 0 && (!eu || !ev)) || !theta) return -1;
    if (side != 0 && side != 1) return -1;
    Adjacency g;
    if (!build(n_u, n_v, m, eu, ev, side, g)) return -1;
    const int32_t n = g.n_a;

    // Initial count (Alg. 2 first line).
    std::vector<int64_t> support(n);
    count_side(g, support.data());

    // Minimum-support retrieval: a binary heap of (support, id) entries; an
    // entry is current only if it matches the vertex's present support.
    using Entry = std::pair<int64_t, int32_t>;
    std::priority_queue<Entry, std::vector<Entry>, std::greater<Entry>> heap;
    for (int32_t x = 0; x < n; ++x) heap.emplace(support[x], x);

    std::vector<char> remaining(n, 1);
    std::vector<int32_t> wdg_arr(n, 0);
    std::vector<int32_t> touched;
    int64_t visited = 0;
    int32_t peeled = 0;

    while (!heap.empty()) {
        Entry top = heap.top();
        heap.pop();
        const int32_t u = top.second;
        if (!remaining[u] || top.first != support[u]) continue;  // stale entry
        // theta_u <- support_u; remove u from U
        const int64_t theta_u = support[u];
        theta[u] = theta_u;
        remaining[u] = 0;
        if (order) order[peeled] = u;
        ++peeled;

        // update(u, theta_u): aggregate wedge counts over the 2-hop
        // neighbourhood of u ...
        touched.clear();
        for (int32_t v : g.a_to_b[u])
            for (int32_t w : g.b_to_a[v]) {
                if (w == u) continue;
                ++visited;
                if (wdg_arr[w] == 0) touched.push_back(w);
                ++wdg_arr[w];
            }
        // ... then lower each remaining neighbour by the shared butterflies,
        // never below theta_u.
        for (int32_t w : touched) {
            const int64_t shared = choose2(wdg_arr[w]);
            wdg_arr[w] = 0;
            if (!remaining[w] || shared == 0) continue;
            const int64_t lowered = std::max(theta_u, support[w] - shared);
            if (lowered != support[w]) {
                support[w] = lowered;
                heap.emplace(lowered, w);
            }
        }
        // Keep the heap's memory bounded: once stale entries dominate,
        // rebuild it with one current entry per remaining vertex.
        const int64_t left = static_cast<int64_t>(n) - peeled;
        if (static_cast<int64_t>(heap.size()) > 4 * left + 4096) {
            std::vector<Entry> fresh;
            fresh.reserve(static_cast<size_t>(left));
            for (int32_t x = 0; x < n; ++x)
                if (remaining[x]) fresh.emplace_back(support[x], x);
            heap = decltype(heap)(decltype(heap)::value_compare(), std::move(fresh));
        }
    }
    if (wedges) *wedges = visited;
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
