// Edge peeling (wing decomposition) and k-tip extraction.
//
// Wing numbers are the edge analogue of tip numbers: the k-wing is the
// largest subgraph in which every edge lies in at least k butterflies, and
// an edge's wing number is the largest k whose k-wing holds it.  The paper's
// Extensions section names parallel edge peeling as the extension of its method and
// its one difficulty: several edges of one butterfly can be peeled in the
// same round, and the butterfly must then be taken out of the survivors'
// supports exactly once.  Here every peeling round takes ALL live edges of
// support at most the current level (level-synchronous bottom-up peeling;
// by the same argument as for vertices, Q1, the order inside a level does
// not change any wing number), and a butterfly with several edges in the
// round is handled only by the one of smallest edge id (the priority order).
//
// Per-edge butterfly counts: the butterflies of e = (x, y) are, for every x'
// != x adjacent to y, the common neighbours of x and x' other than y, so with
// c(x, x') gathered over x's 2-hop neighbourhood the count of each edge of x
// is the sum over x' in N_y \ {x} of c(x, x') - 1.
//
// k-tips (Def. 1): the butterfly-connected components of {theta >= k}; two
// vertices are joined when they share at least two neighbours.  Components
// are found with a lock-free union-find over those pairs.
//
// Every workgroup handles one vertex or one peeled edge at a time; keys go
// to an LDS hash table when there are few of them, else to a per-workgroup
// direct-address array in HBM (the spill arena, all zero between uses).
#include <cstring>

#include "kern_util.h"
#include "wing.h"

namespace tip {
namespace {

constexpr int kWT = 256;                // threads per workgroup
constexpr int kWNW = kWT / kWave;
constexpr int kWHashSlots = 4096;       // LDS hash slots (64-bit)
constexpr int64_t kWHashMax = 2048;     // the hash takes at most this many keys (half full)
constexpr int kWGroup = kWT;            // list entries staged per pass

// One side's adjacency as seen from its vertices: list of x = adj[off[x],
// off[x+1]); eid maps a list position to the edge id (CSR position of the
// edge), or is null when positions are edge ids.
struct SideView {
    const int64_t* off;
    const int32_t* adj;
    const int32_t* eid;
    __device__ inline int64_t id(int64_t p) const { return eid ? (int64_t)eid[p] : p; }
};

struct WLds {
    unsigned long long tab[kWHashSlots];
    int64_t sbeg[kWGroup];
    int64_t pre[kWGroup + 1];
    int64_t acc[kWGroup];
    int64_t aux[kWGroup];
    int64_t red[kWNW];
    int64_t item;
};

// ---- LDS hash: slot = (key + 1) << 32 | value ------------------------------

__device__ inline void h_count(WLds& L, uint32_t k) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & (kWHashSlots - 1);
#pragma unroll 1
    for (;;) {
        unsigned long long* slot = &L.tab[h];
        unsigned long long cur = __atomic_load_n(slot, __ATOMIC_RELAXED);
        if (cur == 0) {
            const unsigned long long prev = atomicCAS(slot, 0ull, tag | 1ull);
            if (prev == 0) return;
            cur = prev;
        }
        if ((cur & 0xffffffff00000000ull) == tag) {
            atomicAdd(slot, 1ull);
            return;
        }
        h = (h + 1) & (kWHashSlots - 1);
    }
}

// Inserts a key that is not in the table yet with value v < 2^32.
__device__ inline void h_put(WLds& L, uint32_t k, uint32_t v) {
    const unsigned long long e = ((unsigned long long)(k + 1) << 32) | v;
    uint32_t h = hash32(k) & (kWHashSlots - 1);
#pragma unroll 1
    while (atomicCAS(&L.tab[h], 0ull, e) != 0ull) h = (h + 1) & (kWHashSlots - 1);
}

// Value of key k, or -1.
__device__ inline int64_t h_get(const WLds& L, uint32_t k) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & (kWHashSlots - 1);
#pragma unroll 1
    for (int p = 0; p < kWHashSlots; ++p) {
        const unsigned long long cur = L.tab[h];
        if (cur == 0) return -1;
        if ((cur & 0xffffffff00000000ull) == tag) return (int64_t)(cur & 0xffffffffull);
        h = (h + 1) & (kWHashSlots - 1);
    }
    return -1;
}

__device__ inline void h_clear(WLds& L) {
    for (int i = threadIdx.x; i < kWHashSlots; i += kWT) L.tab[i] = 0;
}

// ---- workgroup helpers ----------------------------------------------------

__device__ inline int64_t wg_next(WLds& L, unsigned long long* head) {
    __syncthreads();
    if (threadIdx.x == 0) L.item = (int64_t)atomicAdd(head, 1ull);
    __syncthreads();
    return L.item;
}

// Exclusive scan of the lengths held by threads j < gs into L.pre; returns
// the total.
__device__ inline int64_t wg_scan(WLds& L, int gs, int64_t len) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int64_t x = tid < gs ? len : 0;
    const int64_t inc = wave_incl_scan_i64<kWT>(x);
    __syncthreads();
    if (lane == kWave - 1) L.red[wid] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWNW; ++w) {
        const int64_t v = L.red[w];
        off += w < wid ? v : 0;
        tot += v;
    }
    if (tid < gs) L.pre[tid] = off + inc - x;
    if (tid == 0) L.pre[gs] = tot;
    __syncthreads();
    return tot;
}

__device__ inline int wg_slice(const WLds& L, int gs, int64_t i) {
    int lo = 0, hi = gs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// For the entries q in [q0, q1) of list view A, group by group: thread j of
// the group calls keep(j, q, y) for y = A.adj[q] (it may write L.acc[j] and
// L.aux[j]); the lists B.adj[B.off[y] .. B.off[y + 1]) of the kept entries
// are then walked by the whole workgroup, calling f(j, pos, z) for every
// position pos of those lists (z = B.adj[pos]); after each group,
// end(g0, gs) runs on every thread.  Returns the number of (j, pos) visited
// (the same value on every thread).
template <class Keep, class F, class End>
__device__ inline int64_t staged_two_hop(WLds& L, const SideView& A, int64_t q0, int64_t q1, const SideView& B,
                                         Keep&& keep, F&& f, End&& end) {
    const int tid = threadIdx.x;
    int64_t visited = 0;
    for (int64_t g0 = q0; g0 < q1; g0 += kWGroup) {
        const int gs = (int)min<int64_t>(kWGroup, q1 - g0);
        int64_t len = 0;
        if (tid < gs) {
            const int64_t q = g0 + tid;
            const int32_t y = A.adj[q];
            int64_t beg = 0;
            if (keep(tid, q, y)) {
                beg = B.off[y];
                len = B.off[y + 1] - beg;
            }
            L.sbeg[tid] = beg;
        }
        const int64_t total = wg_scan(L, gs, len);
        visited += total;
        for (int64_t i = tid; i < total; i += kWT) {
            const int j = wg_slice(L, gs, i);
            const int64_t pos = L.sbeg[j] + (i - L.pre[j]);
            f(j, pos, B.adj[pos]);
        }
        __syncthreads();
        end(g0, gs);
        __syncthreads();
    }
    return visited;
}

struct NoEnd {
    __device__ inline void operator()(int64_t, int) const {}
};
struct KeepAll {
    __device__ inline bool operator()(int, int64_t, int32_t) const { return true; }
};

// ---- set-up kernels ---------------------------------------------------------

// Edge id of every CSC position: the CSR position of the same edge.
__global__ void k_eid_b(DevGraph g, int32_t* eid_b) {
    GRID_STRIDE(q, g.m) eid_b[q] = (int32_t)(g.a_off[g.b_adj[q]] + g.b_rev[q]);
}

// w[x] = sum over y in N_x of (d_y - 1), one wave per row.
__global__ void k_wsum(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t n,
                       const int64_t* __restrict__ off_other, int64_t* w) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t x = wave; x < n; x += nwaves) {
        int64_t s = 0;
        for (int64_t p = off[x] + lane; p < off[x + 1]; p += kWave) {
            const int32_t y = adj[p];
            s += off_other[y + 1] - off_other[y] - 1;
        }
        s = wave_sum_i64(s);
        if (lane == 0) w[x] = s;
    }
}

__global__ void k_sum_i64_to(const int64_t* __restrict__ a, int32_t n, int64_t* out) {
    __shared__ long long r[1024];
    long long t = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) t += a[i];
    r[threadIdx.x] = t;
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) r[threadIdx.x] += r[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = r[0];
}

__device__ inline void add_stat(unsigned long long* p, int64_t v) {
    if (threadIdx.x == 0 && v) atomicAdd(p, (unsigned long long)v);
}

// ---- per-edge butterfly counts ----------------------------------------------

// cnt[edge] for every edge of every x of side X: c(x, z) over the 2-hop
// neighbourhood first, then, per edge (x, y), the sum of c(x, z) - 1 over
// z in N_y \ {x}.
__global__ void __launch_bounds__(kWT) k_edge_count(SideView X, SideView Y, int32_t n_x, const int64_t* __restrict__ wx,
                                                    int64_t* cnt, SpillArena spa, unsigned long long* head,
                                                    unsigned long long* wedges) {
    __shared__ WLds L;
    const int tid = threadIdx.x;
    int32_t* dense = spa.dense + (int64_t)blockIdx.x * spa.stride;
    h_clear(L);
    int64_t wl = 0;
    for (;;) {
        const int64_t x = wg_next(L, head);
        if (x >= n_x) break;
        const int64_t q0 = X.off[x], q1 = X.off[x + 1];
        if (wx[x] == 0) {
            for (int64_t q = q0 + tid; q < q1; q += kWT) cnt[X.id(q)] = 0;
            continue;
        }
        const bool hashed = wx[x] <= kWHashMax;
        wl += staged_two_hop(L, X, q0, q1, Y, KeepAll{}, [&](int, int64_t, int32_t z) {
            if (z == (int32_t)x) return;
            if (hashed) h_count(L, (uint32_t)z);
            else atomicAdd(&dense[z], 1);
        }, NoEnd{});
        staged_two_hop(L, X, q0, q1, Y,
            [&](int j, int64_t, int32_t) {
                L.acc[j] = 0;
                return true;
            },
            [&](int j, int64_t, int32_t z) {
                if (z == (int32_t)x) return;
                const int64_t c = hashed ? h_get(L, (uint32_t)z) : (int64_t)dense[z];
                if (c > 1) atomicAdd(reinterpret_cast<unsigned long long*>(&L.acc[j]), (unsigned long long)(c - 1));
            },
            [&](int64_t g0, int gs) {
                if (tid < gs) cnt[X.id(g0 + tid)] = L.acc[tid];
            });
        if (hashed) {
            h_clear(L);
        } else {
            staged_two_hop(L, X, q0, q1, Y, KeepAll{}, [&](int, int64_t, int32_t z) { dense[z] = 0; }, NoEnd{});
        }
    }
    add_stat(wedges, wl);
}

// ---- edge peeling -----------------------------------------------------------

struct WingState {
    int32_t* state;        // [m] -1 live, else the round that peeled the edge
    int64_t* supp;         // [m] raw supports
    int64_t* psi;          // [m] wing numbers
    const int32_t* erow;   // [m] U end of each edge (CSR row)
    const int32_t* ecol;   // [m] V end of each edge (CSR column)
};



__device__ inline bool alive_at(const int32_t* state, int64_t f, int32_t round) {
    const int32_t st = state[f];
    return st < 0 || st == round;
}

// The round's peeled edges (frontier) remove their butterflies from the
// surviving edges' supports.  Peeled edge e = (u, v): with x the end whose
// other end y has the cheaper 2-hop walk, the live edges (x, y') go to a
// table keyed by y'; then for every live (x', y), x' != x, and every live
// (x', y'') with y'' in the table, {x, x'} x {y, y''} is a butterfly of live
// edges.  It is applied by its peeled edge of smallest id only; each of its
// surviving edges loses one, and an edge whose support drops to the level
// joins the next frontier.
__global__ void __launch_bounds__(kWT) k_wing_update(SideView U, SideView V, const int64_t* __restrict__ wu,
                                                     const int64_t* __restrict__ wv, WingState ws,
                                                     const int32_t* __restrict__ front, int32_t* next,
                                                     int32_t round, WingCtl* ctl, SpillArena spa) {
    __shared__ WLds L;
    const int tid = threadIdx.x;
    int32_t* tag = spa.dense + (int64_t)blockIdx.x * spa.stride;
    const int32_t n_front = ctl->n_front;
    const int64_t level = ctl->level;
    h_clear(L);
    int64_t walked = 0, decs = 0;
    for (;;) {
        const int64_t i = wg_next(L, &ctl->head);
        if (i >= n_front) break;
        const int64_t e = front[i];
        const int32_t u = ws.erow[e], v = ws.ecol[e];
        // orientation: x's list is tabled, y's 2-hop walked
        const bool xu = wv[v] <= wu[u];
        const SideView X = xu ? U : V, Y = xu ? V : U;
        const int32_t x = xu ? u : v, y = xu ? v : u;
        const int64_t q0 = X.off[x], q1 = X.off[x + 1];
        const bool hashed = q1 - q0 <= kWHashMax;
        for (int64_t q = q0 + tid; q < q1; q += kWT) {
            const int32_t y2 = X.adj[q];
            const int64_t f = X.id(q);
            if (y2 == y || !alive_at(ws.state, f, round)) continue;
            if (hashed) h_put(L, (uint32_t)y2, (uint32_t)f);
            else tag[y2] = (int32_t)(f + 1);
        }
        __syncthreads();
        walked += staged_two_hop(L, Y, Y.off[y], Y.off[y + 1], X,
            [&](int j, int64_t q, int32_t x2) {
                const int64_t e3 = Y.id(q);
                L.aux[j] = e3;
                return x2 != x && alive_at(ws.state, e3, round);
            },
            [&](int j, int64_t pos, int32_t y2) {
                if (y2 == y) return;
                const int64_t e2 = hashed ? h_get(L, (uint32_t)y2) : (int64_t)tag[y2] - 1;
                if (e2 < 0) return;
                const int64_t e4 = X.id(pos);
                if (!alive_at(ws.state, e4, round)) return;
                const int64_t e3 = L.aux[j];
                const int64_t o[3] = {e2, e3, e4};
                // the butterfly belongs to its peeled edge of smallest id
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (o[k] < e && ws.state[o[k]] == round) return;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (ws.state[o[k]] != -1) continue;
                    const int64_t old = atomic_add_i64_ret(&ws.supp[o[k]], -1);
                    ++decs;
                    if (old == level + 1) next[atomicAdd(&ctl->n_next, 1)] = (int32_t)o[k];
                }
            },
            NoEnd{});
        if (hashed) {
            h_clear(L);
        } else {
            for (int64_t q = q0 + tid; q < q1; q += kWT) tag[X.adj[q]] = 0;
        }
    }
    add_stat(&ctl->wedges_peel, walked);
    decs = wave_sum_i64(decs);
    if ((tid & (kWave - 1)) == 0 && decs) atomicAdd(&ctl->decrements, (unsigned long long)decs);
}

// Level start: the live list without the edges peeled since, and the least
// support among them.
__global__ void k_wing_compact(const int32_t* __restrict__ live_in, int32_t n_in, const int32_t* __restrict__ state,
                               const int64_t* __restrict__ supp, int32_t* live_out, WingCtl* ctl) {
    unsigned long long mn = ~0ull;
    UNIFORM_STRIDE(base, (int64_t)n_in) {
        const int64_t i = base + threadIdx.x;
        bool keep = false;
        int32_t e = 0;
        if (i < n_in) {
            e = live_in[i];
            keep = state[e] < 0;
            if (keep) mn = min(mn, (unsigned long long)supp[e]);
        }
        wave_append(keep, e, live_out, &ctl->n_live);
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(mn, d, kWave);
        mn = o < mn ? o : mn;
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && mn != ~0ull) atomicMin(&ctl->min_supp, mn);
}

__global__ void k_wing_level(WingCtl* ctl) {
    if (ctl->n_live > 0 && (long long)ctl->min_supp > ctl->level) ctl->level = (long long)ctl->min_supp;
    ctl->levels += ctl->n_live > 0 ? 1 : 0;
    ctl->n_front = 0;
}

__global__ void k_wing_front(const int32_t* __restrict__ live, const int64_t* __restrict__ supp, int32_t* front,
                             WingCtl* ctl) {
    const int32_t n = ctl->n_live;
    const long long level = ctl->level;
    UNIFORM_STRIDE(base, (int64_t)n) {
        const int64_t i = base + threadIdx.x;
        bool take = false;
        int32_t e = 0;
        if (i < n) {
            e = live[i];
            take = supp[e] <= level;
        }
        wave_append(take, e, front, &ctl->n_front);
    }
}

// Marks the round's frontier peeled (wing number = level) and resets the
// counters of the round.
__global__ void k_wing_mark(const int32_t* __restrict__ front, WingState ws, int32_t round, WingCtl* ctl) {
    const int32_t n = ctl->n_front;
    const long long level = ctl->level;
    GRID_STRIDE(i, (int64_t)n) {
        const int32_t e = front[i];
        ws.state[e] = round;
        ws.psi[e] = level;
    }
}

__global__ void k_wing_round_reset(WingCtl* ctl) {
    ctl->head = 0;
    ctl->n_next = 0;
    ctl->rounds += 1;
}

__global__ void k_wing_swap(WingCtl* ctl) { ctl->n_front = ctl->n_next; }

// ---- k-tips -----------------------------------------------------------------

__device__ inline int32_t uf_find(int32_t* p, int32_t x) {
    for (;;) {
        const int32_t px = __hip_atomic_load(&p[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (px == x) return x;
        const int32_t gx = __hip_atomic_load(&p[px], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gx != px) __hip_atomic_store(&p[x], gx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gx;
    }
}

__device__ inline void uf_union(int32_t* p, int32_t a, int32_t b) {
    for (;;) {
        a = uf_find(p, a);
        b = uf_find(p, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // link the larger root under the smaller one
        if (atomicCAS(&p[b], b, a) == b) return;
    }
}

// For every x with theta >= k, the pairs {x, z} (z > x, theta_z >= k) that
// share two or more neighbours are joined.
__global__ void __launch_bounds__(kWT) k_ktip_pairs(SideView X, SideView Y, int32_t n_x, const int64_t* __restrict__ wx,
                                                    const int64_t* __restrict__ theta, long long k, int32_t* parent,
                                                    SpillArena spa, unsigned long long* head, unsigned long long* wedges) {
    __shared__ WLds L;
    const int tid = threadIdx.x;
    int32_t* dense = spa.dense + (int64_t)blockIdx.x * spa.stride;
    h_clear(L);
    int64_t wl = 0;
    for (;;) {
        const int64_t x = wg_next(L, head);
        if (x >= n_x) break;
        if (theta[x] < k || wx[x] == 0) continue;
        const int64_t q0 = X.off[x], q1 = X.off[x + 1];
        const bool hashed = wx[x] <= kWHashMax;
        wl += staged_two_hop(L, X, q0, q1, Y, KeepAll{}, [&](int, int64_t, int32_t z) {
            if (z <= (int32_t)x || theta[z] < k) return;
            if (hashed) h_count(L, (uint32_t)z);
            else atomicAdd(&dense[z], 1);
        }, NoEnd{});
        if (hashed) {
            for (int i = tid; i < kWHashSlots; i += kWT) {
                const unsigned long long e = L.tab[i];
                if (e != 0 && (e & 0xffffffffull) >= 2) uf_union(parent, (int32_t)x, (int32_t)((e >> 32) - 1));
            }
            __syncthreads();
            h_clear(L);
        } else {
            staged_two_hop(L, X, q0, q1, Y, KeepAll{}, [&](int, int64_t, int32_t z) {
                if (z <= (int32_t)x || theta[z] < k) return;
                if (dense[z] >= 2) uf_union(parent, (int32_t)x, z);
                dense[z] = 0;
            }, NoEnd{});
        }
    }
    add_stat(wedges, wl);
}

__global__ void k_ktip_min_id(int32_t* parent, const int64_t* __restrict__ theta, long long k,
                              const int32_t* __restrict__ orig, int32_t n, int32_t* min_id) {
    GRID_STRIDE(x, (int64_t)n) {
        if (theta[x] >= k) atomicMin(&min_id[uf_find(parent, (int32_t)x)], orig[x]);
    }
}

__global__ void k_ktip_label(int32_t* parent, const int64_t* __restrict__ theta, long long k,
                             const int32_t* __restrict__ orig, int32_t n, const int32_t* __restrict__ min_id,
                             int32_t* comp_orig) {
    GRID_STRIDE(x, (int64_t)n) {
        comp_orig[orig[x]] = theta[x] >= k ? min_id[uf_find(parent, (int32_t)x)] : -1;
    }
}

__global__ void k_theta_by_rank(const int64_t* __restrict__ theta_orig, const int32_t* __restrict__ orig, int32_t n,
                                int64_t* theta_rank) {
    GRID_STRIDE(x, (int64_t)n) theta_rank[x] = theta_orig[orig[x]];
}

// ---- output in input order --------------------------------------------------

// out[i] = per_edge[CSR position of input edge i] (duplicates share one).
__global__ void k_edges_to_input(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev, int64_t m,
                                 const int32_t* __restrict__ rank_u, const int32_t* __restrict__ rank_v, DevGraph g,
                                 const int64_t* __restrict__ per_edge, int64_t* out) {
    GRID_STRIDE(i, m) {
        const int32_t ru = rank_u[eu[i]], rv = rank_v[ev[i]];
        const int64_t p = lower_bound_i32(g.a_adj, g.a_off[ru], g.a_off[ru + 1], rv);
        out[i] = per_edge[p];
    }
}

int wing_occupancy() {
    int a = 0, b = 0, c = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_wing_update, kWT, 0));
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_edge_count, kWT, 0));
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_ktip_pairs, kWT, 0));
    return std::max(1, std::min(a, std::min(b, c)));
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int wing_slots() {
    int dev = 0, cus = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    TIP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(1, cus) * wing_occupancy();
}

void wing_plan(Arena& ar, int32_t n_u, int32_t n_v, int64_t m, int slots, bool ktip, WingWork& w) {
    const int64_t mm = std::max<int64_t>(m, 1), nu = std::max<int32_t>(n_u, 1), nv = std::max<int32_t>(n_v, 1);
    ingest_alloc(ar, n_u, n_v, m, w.ib);
    graph_alloc(ar, n_u, n_v, m, w.g, w.aux);
    w.eid_b = ar.take<int32_t>(mm);
    w.wu = ar.take<int64_t>(nu);
    w.wv = ar.take<int64_t>(nv);
    if (ktip) {
        w.theta_orig = ar.take<int64_t>(nu);
        w.theta_rank = ar.take<int64_t>(nu);
        w.parent = ar.take<int32_t>(nu);
        w.min_id = ar.take<int32_t>(nu);
        w.comp = ar.take<int32_t>(nu);
    } else {
        w.supp = ar.take<int64_t>(mm);
        w.psi = ar.take<int64_t>(mm);
        w.state = ar.take<int32_t>(mm);
        for (int i = 0; i < 2; ++i) w.live[i] = ar.take<int32_t>(mm);
        for (int i = 0; i < 2; ++i) w.front[i] = ar.take<int32_t>(mm);
        w.out = ar.take<int64_t>(mm);
    }
    w.ctl = ar.take<WingCtl>(1);
    const int64_t keys = std::max<int64_t>(std::max(nu, nv), 64);
    w.spill.stride = (keys + 63) & ~int64_t(63);
    w.spill.slots = slots;
    w.spill.dense = ar.take<int32_t>(w.spill.stride * slots);
    w.spill.list = nullptr;
}

namespace {

WingCtl read_wctl(const WingWork& w, hipStream_t s) {
    WingCtl h;
    TIP_HIP_TRY(hipMemcpyAsync(&h, w.ctl, sizeof(WingCtl), hipMemcpyDeviceToHost, s));
    TIP_HIP_TRY(hipStreamSynchronize(s));
    return h;
}

// Ingest (U as side A) and the set-up every call shares.
bool wing_ingest(WingWork& w, const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                 hipStream_t s) {
    TIP_HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(WingCtl), s));
    if (!ingest(d_eu, d_ev, n_u, n_v, m, true, w.ib, w.g, w.aux, s)) return false;
    fill_i32(w.spill.dense, 0, w.spill.stride * w.spill.slots, s);
    const DevGraph& g = w.g;
    if (g.m > 0) {
        k_eid_b<<<grid1(g.m), kT, 0, s>>>(g, w.eid_b);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (n_u > 0) {
        k_wsum<<<grid1((int64_t)n_u * kWave), kT, 0, s>>>(g.a_off, g.a_adj, n_u, g.b_off, w.wu);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (n_v > 0) {
        k_wsum<<<grid1((int64_t)n_v * kWave), kT, 0, s>>>(g.b_off, g.b_adj, n_v, g.a_off, w.wv);
        TIP_HIP_TRY(hipGetLastError());
    }
    return true;
}

}  // namespace

tip_status wing_run(WingWork& w, const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                    bool decompose, int64_t* d_out, tip_stats* st, hipStream_t s) {
    if (!wing_ingest(w, d_eu, d_ev, n_u, n_v, m, s)) {
        set_error("an edge endpoint id is out of range");
        return TIP_EINVAL;
    }
    const DevGraph& g = w.g;
    const int slots = w.spill.slots;
    const SideView U{g.a_off, g.a_adj, nullptr};
    const SideView V{g.b_off, g.b_adj, w.eid_b};
    // per-edge counts from the side with fewer wedges to walk
    int64_t wsum[2] = {0, 0};
    if (g.m > 0) {
        // the two wedge totals decide the side; both are sums of d(d - 1)
        // over the other side, read back once
        int64_t* tmp = w.supp;  // free until the counts are written
        k_sum_i64_to<<<1, 1024, 0, s>>>(w.wu, n_u, tmp);
        k_sum_i64_to<<<1, 1024, 0, s>>>(w.wv, n_v, tmp + 1);
        TIP_HIP_TRY(hipGetLastError());
        TIP_HIP_TRY(hipMemcpyAsync(wsum, tmp, sizeof(wsum), hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        const bool from_u = wsum[0] <= wsum[1];
        TIP_HIP_TRY(hipMemsetAsync(&w.ctl->head, 0, sizeof(unsigned long long), s));
        k_edge_count<<<slots, kWT, 0, s>>>(from_u ? U : V, from_u ? V : U, from_u ? n_u : n_v, from_u ? w.wu : w.wv,
                                           w.supp, w.spill, &w.ctl->head, &w.ctl->wedges_count);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (!decompose) {
        if (m > 0) {
            k_edges_to_input<<<grid1(m), kT, 0, s>>>(d_eu, d_ev, m, w.ib.rank_a, w.ib.rank_b, g, w.supp, d_out);
            TIP_HIP_TRY(hipGetLastError());
        }
    } else if (g.m > 0) {
        const WingState ws{w.state, w.supp, w.psi, g.a_row, g.a_adj};
        fill_i32(w.state, -1, g.m, s);
        iota_i32(w.live[0], g.m, s);
        int cur = 0;
        int32_t n_live = (int32_t)g.m;
        int32_t round = 0;
        for (;;) {
            // level start: compact, least support, level, frontier
            TIP_HIP_TRY(hipMemsetAsync(&w.ctl->n_live, 0, sizeof(int32_t), s));
            TIP_HIP_TRY(hipMemsetAsync(&w.ctl->min_supp, 0xff, sizeof(unsigned long long), s));
            k_wing_compact<<<grid1(n_live, 4096), kT, 0, s>>>(w.live[cur], n_live, w.state, w.supp, w.live[cur ^ 1],
                                                             w.ctl);
            cur ^= 1;
            k_wing_level<<<1, 1, 0, s>>>(w.ctl);
            k_wing_front<<<grid1(n_live, 4096), kT, 0, s>>>(w.live[cur], w.supp, w.front[0], w.ctl);
            TIP_HIP_TRY(hipGetLastError());
            WingCtl c = read_wctl(w, s);
            n_live = c.n_live;
            if (n_live == 0) break;
            int fb = 0;
            int32_t n_front = c.n_front;
            while (n_front > 0) {
                k_wing_mark<<<grid1(n_front), kT, 0, s>>>(w.front[fb], ws, round, w.ctl);
                k_wing_round_reset<<<1, 1, 0, s>>>(w.ctl);
                k_wing_update<<<slots, kWT, 0, s>>>(U, V, w.wu, w.wv, ws, w.front[fb], w.front[fb ^ 1], round, w.ctl,
                                                    w.spill);
                k_wing_swap<<<1, 1, 0, s>>>(w.ctl);
                TIP_HIP_TRY(hipGetLastError());
                fb ^= 1;
                ++round;
                n_front = read_wctl(w, s).n_front;
            }
        }
        k_edges_to_input<<<grid1(m), kT, 0, s>>>(d_eu, d_ev, m, w.ib.rank_a, w.ib.rank_b, g, w.psi, d_out);
        TIP_HIP_TRY(hipGetLastError());
    }
    const WingCtl c = read_wctl(w, s);
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->wedges_count = (int64_t)c.wedges_count;
        st->wedges_cd = (int64_t)c.wedges_peel;
        st->pair_updates = (int64_t)c.decrements;
        st->rounds = (int64_t)c.rounds;
        st->fd_levels = (int64_t)c.levels;
        st->m_unique = g.m;
    }
    return TIP_OK;
}

tip_status ktip_run(WingWork& w, const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                    int32_t side, const int64_t* theta_host, int64_t k, int32_t* d_comp, hipStream_t s) {
    const bool a_is_u = side == TIP_SIDE_U;
    const int32_t n_a = a_is_u ? n_u : n_v, n_b = a_is_u ? n_v : n_u;
    TIP_HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(WingCtl), s));
    if (!ingest(a_is_u ? d_eu : d_ev, a_is_u ? d_ev : d_eu, n_a, n_b, m, a_is_u, w.ib, w.g, w.aux, s)) {
        set_error("an edge endpoint id is out of range");
        return TIP_EINVAL;
    }
    if (n_a <= 0) return TIP_OK;
    const DevGraph& g = w.g;
    fill_i32(w.spill.dense, 0, w.spill.stride * w.spill.slots, s);
    TIP_HIP_TRY(hipMemcpyAsync(w.theta_orig, theta_host, sizeof(int64_t) * n_a, hipMemcpyHostToDevice, s));
    k_theta_by_rank<<<grid1(n_a), kT, 0, s>>>(w.theta_orig, g.a_orig, n_a, w.theta_rank);
    k_wsum<<<grid1((int64_t)n_a * kWave), kT, 0, s>>>(g.a_off, g.a_adj, n_a, g.b_off, w.wu);
    iota_i32(w.parent, n_a, s);
    fill_i32(w.min_id, INT32_MAX, n_a, s);
    TIP_HIP_TRY(hipGetLastError());
    const SideView X{g.a_off, g.a_adj, nullptr};
    const SideView Y{g.b_off, g.b_adj, nullptr};
    k_ktip_pairs<<<w.spill.slots, kWT, 0, s>>>(X, Y, n_a, w.wu, w.theta_rank, (long long)k, w.parent, w.spill,
                                               &w.ctl->head, &w.ctl->wedges_count);
    k_ktip_min_id<<<grid1(n_a), kT, 0, s>>>(w.parent, w.theta_rank, (long long)k, g.a_orig, n_a, w.min_id);
    k_ktip_label<<<grid1(n_a), kT, 0, s>>>(w.parent, w.theta_rank, (long long)k, g.a_orig, n_a, w.min_id, d_comp);
    TIP_HIP_TRY(hipGetLastError());
    return TIP_OK;
}

}  // namespace tip
