// Counting, coarse-grained (CD) and fine-grained (FD) decomposition kernels.
//
// Supports are stored raw (uncapped) and decremented with 64-bit atomics; the
// cap of the paper's update (never below the current level) is applied when a
// support is read: the effective support is max(level, raw).  A live vertex's
// raw support is exactly its butterflies with the other live vertices, so it
// never underflows.
#include "agg.h"
#include "tip_kernels.h"

namespace tip {
namespace {

constexpr int kT = 256;

inline unsigned grid1(int64_t n, int64_t cap = 262144) {
    int64_t g = (n + kT - 1) / kT;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// Loop with a trip count that is uniform across each wave (for wave_append).
#define UNIFORM_STRIDE(base, n) \
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < (n); base += (int64_t)gridDim.x * blockDim.x)

__device__ inline void atomic_add_i64(int64_t* p, int64_t v) {
    atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}
__device__ inline int64_t atomic_add_i64_ret(int64_t* p, int64_t v) {
    return (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

// ===========================================================================
// Per-vertex butterfly counting (Alg. 1)
// ===========================================================================
//
// Start vertex x on side X, middle vertex y in N_x, end vertex z in N_y with
// z before both x and y in the joint degree order.  Since every list is sorted
// by rank, the admissible z of the edge (x, y) are the first
// min(cut[y], pos of x in N_y) entries of N_y.  With c = number of wedges from
// x ending at z: x and z each gain C(c, 2) and y gains c - 1 per wedge.

struct SideView {
    const int64_t* own_off;
    const int32_t* own_adj;
    const int32_t* own_rev;
    const int64_t* oth_off;
    const int32_t* oth_adj;
    const int32_t* oth_cut;
    int64_t* own_bfly;
    int64_t* oth_bfly;
};

__device__ inline SideView side_view(const DevGraph& g, bool side_b, int64_t* bfly_a, int64_t* bfly_b) {
    SideView v;
    if (!side_b) {
        v = {g.a_off, g.a_adj, g.a_rev, g.b_off, g.b_adj, g.b_cut, bfly_a, bfly_b};
    } else {
        v = {g.b_off, g.b_adj, g.b_rev, g.a_off, g.a_adj, g.a_cut, bfly_b, bfly_a};
    }
    return v;
}

__global__ void k_count_work(DevGraph g, int64_t* work) {
    GRID_STRIDE(p, g.m) {
        const int32_t x = g.a_row[p], y = g.a_adj[p];
        const int64_t l1 = min(g.b_cut[y], g.a_rev[p]);
        if (l1) atomic_add_i64(&work[x], l1);
        const int32_t yb = g.b_row[p], xb = g.b_adj[p];
        const int64_t l2 = min(g.a_cut[xb], g.b_rev[p]);
        if (l2) atomic_add_i64(&work[(int64_t)g.n_a + yb], l2);
    }
}

__global__ void k_count_bins(const int64_t* __restrict__ work, int64_t n, int32_t* small, int32_t* big, Ctl* ctl) {
    unsigned long long tot = 0;
    UNIFORM_STRIDE(base, n) {
        const int64_t i = base + threadIdx.x;
        const int64_t w = i < n ? work[i] : 0;
        tot += (unsigned long long)w;
        wave_append(w > 0 && w <= kSmallMaxWedges, (int32_t)i, small, &ctl->n_items[0]);
        wave_append(w > kSmallMaxWedges, (int32_t)i, big, &ctl->n_items[1]);
    }
    tot = (unsigned long long)wave_sum_i64((int64_t)tot);
    if ((threadIdx.x & (kWave - 1)) == 0 && tot) atomicAdd(&ctl->wedges_count, tot);
}

__global__ void __launch_bounds__(kSmallThreads)
k_count_small(DevGraph g, const int32_t* __restrict__ items, const Ctl* ctl, int64_t* bfly_a, int64_t* bfly_b) {
    __shared__ WaveLds WL[kSmallThreads / kWave];
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    WaveLds& W = WL[wid];
    for (int s = lane; s < kSmallSlots; s += kWave) W.tab[s] = 0;
    wave_sync();
    const int64_t n_items = ctl->n_items[0];
    const int nw = kSmallThreads / kWave;
    for (int64_t it = (int64_t)blockIdx.x * nw + wid; it < n_items; it += (int64_t)gridDim.x * nw) {
        const int32_t item = items[it];
        const bool side_b = item >= g.n_a;
        const int32_t x = side_b ? item - g.n_a : item;
        const SideView sv = side_view(g, side_b, bfly_a, bfly_b);
        const int64_t e0 = sv.own_off[x], d = sv.own_off[x + 1] - e0;
        // pass 1: wedge counts c(x, z)
        for (int64_t g0 = 0; g0 < d; g0 += kWave) {
            const int gs = (int)min<int64_t>(kWave, d - g0);
            int64_t len = 0;
            if (lane < gs) {
                const int64_t e = e0 + g0 + lane;
                const int32_t y = sv.own_adj[e];
                W.sbeg[lane] = sv.oth_off[y];
                len = min(sv.oth_cut[y], sv.own_rev[e]);
            }
            const int64_t tot = wave_scan_lengths(W, len);
            for (int64_t i = lane; i < tot; i += kWave) {
                const int j = wave_find_slice(W, gs, i);
                wave_insert(W, (uint32_t)sv.oth_adj[W.sbeg[j] + (i - W.pre[j])]);
            }
            wave_sync();
        }
        // pass 2: middle vertices gain c - 1 per wedge
        for (int64_t g0 = 0; g0 < d; g0 += kWave) {
            const int gs = (int)min<int64_t>(kWave, d - g0);
            int64_t len = 0;
            int32_t y = 0;
            if (lane < gs) {
                const int64_t e = e0 + g0 + lane;
                y = sv.own_adj[e];
                W.sbeg[lane] = sv.oth_off[y];
                len = min(sv.oth_cut[y], sv.own_rev[e]);
            }
            W.acc[lane] = 0;
            const int64_t tot = wave_scan_lengths(W, len);
            for (int64_t i = lane; i < tot; i += kWave) {
                const int j = wave_find_slice(W, gs, i);
                const int32_t c = wave_lookup(W, (uint32_t)sv.oth_adj[W.sbeg[j] + (i - W.pre[j])]);
                if (c > 1) atomicAdd(reinterpret_cast<unsigned long long*>(&W.acc[j]), (unsigned long long)(c - 1));
            }
            wave_sync();
            if (lane < gs && W.acc[lane]) atomic_add_i64(&sv.oth_bfly[y], W.acc[lane]);
            wave_sync();
        }
        // pass 3: start and end vertices gain C(c, 2)
        int64_t local = 0;
        for (int s = lane; s < kSmallSlots; s += kWave) {
            const unsigned long long v = W.tab[s];
            if (v) {
                const int64_t c = (int64_t)(v & 0xffffffffull);
                if (c >= 2) {
                    const int64_t b = choose2(c);
                    atomic_add_i64(&sv.own_bfly[(int64_t)(v >> 32) - 1], b);
                    local += b;
                }
                W.tab[s] = 0;
            }
        }
        local = wave_sum_i64(local);
        if (lane == 0 && local) atomic_add_i64(&sv.own_bfly[x], local);
        wave_sync();
    }
}

// Slice of the counting wedges of edge e restricted to keys [klo, khi).
struct CountSlice {
    __device__ static inline void get(const SideView& sv, int64_t e, bool multi, int32_t klo, int32_t khi,
                                      int64_t& s0, int64_t& len) {
        const int32_t y = sv.own_adj[e];
        int64_t a = sv.oth_off[y];
        int64_t b = a + min(sv.oth_cut[y], sv.own_rev[e]);
        if (multi) {
            a = lower_bound_i32(sv.oth_adj, a, b, klo);
            b = lower_bound_i32(sv.oth_adj, a, b, khi);
        }
        s0 = a;
        len = b - a;
    }
};

__global__ void __launch_bounds__(kBigThreads)
k_count_big(DevGraph g, const int32_t* __restrict__ items, const Ctl* ctl, int64_t* bfly_a, int64_t* bfly_b,
            SpillArena spa, Ctl* ctl_rw) {
    __shared__ BigLds L;
    constexpr int NT = kBigThreads;
    const int tid = threadIdx.x;
    bm_clear<NT>(L, kBmBits);
    if (tid == 0) L.spill_n = 0;
    __syncthreads();
    const Spill sp{spa.dense + (int64_t)blockIdx.x * spa.stride, spa.list + (int64_t)blockIdx.x * spa.stride};
    const int64_t n_items = ctl->n_items[1];
    unsigned long long spills = 0;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int32_t item = items[it];
        const bool side_b = item >= g.n_a;
        const int32_t x = side_b ? item - g.n_a : item;
        const SideView sv = side_view(g, side_b, bfly_a, bfly_b);
        const int64_t e0 = sv.own_off[x], d = sv.own_off[x + 1] - e0;
        const bool multi = x > kBmBits;
        for (int32_t klo = 0; klo < x; klo += kBmBits) {
            const int32_t khi = (int32_t)min<int64_t>(x, (int64_t)klo + kBmBits);
            // pass 1
            for (int64_t g0 = 0; g0 < d; g0 += kGroup) {
                const int gs = (int)min<int64_t>(kGroup, d - g0);
                int64_t len = 0;
                if (tid < gs) {
                    int64_t s0;
                    CountSlice::get(sv, e0 + g0 + tid, multi, klo, khi, s0, len);
                    L.sbeg[tid] = s0;
                }
                const int64_t tot = block_scan_lengths<NT>(L, gs, len);
                for (int64_t i = tid; i < tot; i += NT) {
                    const int j = find_slice(L, gs, i);
                    bm_mark(L, sp, (uint32_t)(sv.oth_adj[L.sbeg[j] + (i - L.pre[j])] - klo));
                }
                __syncthreads();
            }
            const bool spilled = L.spill_n > 0;
            // pass 2
            for (int64_t g0 = 0; g0 < d; g0 += kGroup) {
                const int gs = (int)min<int64_t>(kGroup, d - g0);
                int64_t len = 0;
                if (tid < gs) {
                    int64_t s0;
                    CountSlice::get(sv, e0 + g0 + tid, multi, klo, khi, s0, len);
                    L.sbeg[tid] = s0;
                    L.acc[tid] = 0;
                }
                const int64_t tot = block_scan_lengths<NT>(L, gs, len);
                for (int64_t i = tid; i < tot; i += NT) {
                    const int j = find_slice(L, gs, i);
                    const uint32_t k = (uint32_t)(sv.oth_adj[L.sbeg[j] + (i - L.pre[j])] - klo);
                    const int32_t c = rep_lookup(L, sp, spilled, k);
                    if (c > 1) atomicAdd(reinterpret_cast<unsigned long long*>(&L.acc[j]), (unsigned long long)(c - 1));
                }
                __syncthreads();
                if (tid < gs && L.acc[tid]) atomic_add_i64(&sv.oth_bfly[sv.own_adj[e0 + g0 + tid]], L.acc[tid]);
                __syncthreads();
            }
            // pass 3
            int64_t local = 0;
            for (int s = tid; s < kRepSlots; s += NT) {
                const unsigned long long v = L.rep[s];
                if (v) {
                    const int64_t c = 1 + (int64_t)(v & 0xffffffffull);
                    const int64_t b = choose2(c);
                    atomic_add_i64(&sv.own_bfly[klo + (int64_t)(v >> 32) - 1], b);
                    local += b;
                }
            }
            const int32_t nsp = L.spill_n;
            spills += (tid == 0) ? (unsigned long long)nsp : 0ull;
            for (int32_t i = tid; i < nsp; i += NT) {
                const int32_t k = sp.list[i];
                const int64_t b = choose2(1 + (int64_t)sp.dense[k]);
                atomic_add_i64(&sv.own_bfly[klo + (int64_t)k], b);
                local += b;
                sp.dense[k] = 0;
            }
            const int64_t total = block_sum_i64<NT>(L, local);
            if (tid == 0 && total) atomic_add_i64(&sv.own_bfly[x], total);
            bm_clear<NT>(L, khi - klo);
            if (tid == 0) L.spill_n = 0;
            __syncthreads();
        }
    }
    if (tid == 0 && spills) atomicAdd(&ctl_rw->spills, spills);
}

// ===========================================================================
// Coarse-grained decomposition (Alg. 3)
// ===========================================================================

// w[u]: wedges of G with endpoint u (the range-sizing proxy), i.e. the sum
// over v in N_u of d_v - 1.
__global__ void k_wproxy(DevGraph g, const int32_t* __restrict__ deg_b, int64_t* wprox) {
    GRID_STRIDE(p, g.m) {
        const int32_t dv = deg_b[g.a_adj[p]];
        if (dv > 1) atomic_add_i64(&wprox[g.a_row[p]], dv - 1);
    }
}

__global__ void k_ctl_begin_range(Ctl* ctl) {
    ctl->n_live_next = 0;
    ctl->max_supp = 0;
    ctl->w_rem = 0;
    ctl->w_range = 0;
    ctl->n_front[0] = ctl->n_front[1] = 0;
    ctl->n_next[0] = ctl->n_next[1] = 0;
}

// Compacts the live list, snapshots the supports of the live vertices
// (Alg. 3 support init) and reduces the maximum support and the wedge proxy
// of the remaining vertices.
__global__ void k_range_start(const int32_t* __restrict__ live_in, int32_t n_in, int32_t* live_out,
                              const int32_t* __restrict__ state, const int64_t* __restrict__ supp, int64_t* init,
                              const int64_t* __restrict__ wprox, Ctl* ctl) {
    unsigned long long mx = 0;
    long long ws = 0;
    UNIFORM_STRIDE(base, (int64_t)n_in) {
        const int64_t j = base + threadIdx.x;
        int32_t u = 0;
        bool keep = false;
        if (j < n_in) {
            u = live_in[j];
            keep = state[u] == kLive;
        }
        if (keep) {
            const int64_t su = supp[u];
            init[u] = su;
            mx = max(mx, (unsigned long long)su);
            ws += wprox[u];
        }
        wave_append(keep, u, live_out, &ctl->n_live_next);
    }
    __shared__ unsigned long long smx[kT / kWave];
    __shared__ long long sws[kT / kWave];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(mx, d, kWave);
        mx = o > mx ? o : mx;
    }
    ws = wave_sum_i64(ws);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        smx[wid] = mx;
        sws[wid] = ws;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m2 = 0;
        long long w2 = 0;
        for (int w = 0; w < kT / kWave; ++w) {
            m2 = smx[w] > m2 ? smx[w] : m2;
            w2 += sws[w];
        }
        if (m2) atomicMax(&ctl->max_supp, m2);
        if (w2) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->w_rem), (unsigned long long)w2);
    }
}

__global__ void k_ctl_select_init(Ctl* ctl, long long tgt) {
    ctl->sel_prefix = 0;
    ctl->sel_cum = 0;
    ctl->sel_found = 1;
    ctl->sel_tgt = tgt;
}

// findHi as a weighted radix select: one 8-bit digit per pass, most
// significant first.  The histogram adds w[u] over live u whose support
// matches the prefix chosen so far.
__global__ void k_select_hist(const int32_t* __restrict__ live, int32_t n_live, const int64_t* __restrict__ supp,
                              const int64_t* __restrict__ wprox, int shift, const Ctl* ctl, int64_t* hist) {
    if (!ctl->sel_found) return;
    __shared__ unsigned long long h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = ctl->sel_prefix;
    const int hs = shift + 8;
    GRID_STRIDE(j, (int64_t)n_live) {
        const int32_t u = live[j];
        const uint64_t key = (uint64_t)supp[u];
        if (hs >= 64 || (key >> hs) == (prefix >> hs))
            atomicAdd(&h[(key >> shift) & 255], (unsigned long long)wprox[u]);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(reinterpret_cast<unsigned long long*>(&hist[threadIdx.x]), h[threadIdx.x]);
}

__global__ void k_select_pick(int shift, Ctl* ctl, int64_t* hist) {
    __shared__ long long hh[256];
    hh[threadIdx.x] = hist[threadIdx.x];
    hist[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && ctl->sel_found) {
        long long run = ctl->sel_cum;
        const long long tgt = ctl->sel_tgt;
        int chosen = -1;
        for (int d = 0; d < 256; ++d) {
            if (run + hh[d] >= tgt) {
                chosen = d;
                break;
            }
            run += hh[d];
        }
        if (chosen < 0) {
            ctl->sel_found = 0;
        } else {
            ctl->sel_cum = run;
            ctl->sel_prefix |= (unsigned long long)chosen << shift;
        }
    }
}

// First activeSet of a range: live vertices with support below the upper
// bound.  They are assigned to the subset here; vertices with zero support
// share no butterfly with any live vertex and need no update.
__global__ void k_frontier_init(const int32_t* __restrict__ live, int32_t n_live, const int64_t* __restrict__ supp,
                                int32_t* state, const int64_t* __restrict__ wprox, long long hi, int32_t label,
                                int32_t* f_small, int32_t* f_big, Ctl* ctl) {
    long long ws = 0;
    unsigned long long skipped = 0;
    UNIFORM_STRIDE(base, (int64_t)n_live) {
        const int64_t j = base + threadIdx.x;
        bool pred = false, zero = false;
        int32_t u = 0;
        int64_t wu = 0;
        if (j < n_live) {
            u = live[j];
            const int64_t su = supp[u];
            pred = su < hi;
            if (pred) {
                state[u] = label;
                zero = su == 0;
                wu = wprox[u];
                ws += wu;
                skipped += zero;
            }
        }
        wave_append(pred && !zero && wu <= kSmallMaxWedges, u, f_small, &ctl->n_front[0]);
        wave_append(pred && !zero && wu > kSmallMaxWedges, u, f_big, &ctl->n_front[1]);
    }
    ws = wave_sum_i64(ws);
    skipped = (unsigned long long)wave_sum_i64((int64_t)skipped);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (ws) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->w_range), (unsigned long long)ws);
        if (skipped) atomicAdd(&ctl->skipped, skipped);
    }
}

// Applies the decrement of a (peeled u, live w) pair and appends w to the
// next activeSet when its support crosses below the range's upper bound.
struct CdApply {
    int64_t* supp;
    const int32_t* state;
    const int64_t* wprox;
    long long hi;
    int32_t* n_small;
    int32_t* n_big;
    int32_t* l_small;
    int32_t* l_big;

    // Must be reached by all lanes of the wave.
    __device__ inline void apply(bool valid, int32_t w, int64_t c, unsigned long long& pairs) const {
        bool cross = false;
        int64_t ww = 0;
        if (valid && c >= 2 && state[w] == kLive) {
            const int64_t dec = choose2(c);
            const int64_t old = atomic_add_i64_ret(&supp[w], -dec);
            cross = old >= hi && old - dec < hi;
            ++pairs;
            if (cross) ww = wprox[w];
        }
        wave_append(cross && ww <= kSmallMaxWedges, w, l_small, n_small);
        wave_append(cross && ww > kSmallMaxWedges, w, l_big, n_big);
    }
};

__global__ void __launch_bounds__(kSmallThreads)
k_peel_small(DevGraph g, const int32_t* __restrict__ front, const int32_t* n_front_p, CdApply ap, Ctl* ctl) {
    __shared__ WaveLds WL[kSmallThreads / kWave];
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    WaveLds& W = WL[wid];
    for (int s = lane; s < kSmallSlots; s += kWave) W.tab[s] = 0;
    wave_sync();
    const int64_t n_front = *n_front_p;
    const int nw = kSmallThreads / kWave;
    unsigned long long wedges = 0, pairs = 0, skipped = 0;
    for (int64_t it = (int64_t)blockIdx.x * nw + wid; it < n_front; it += (int64_t)gridDim.x * nw) {
        const int32_t u = front[it];
        if (ap.supp[u] == 0) {
            skipped += lane == 0;
            continue;
        }
        const int64_t e0 = g.a_off[u], d = g.a_off[u + 1] - e0;
        for (int64_t g0 = 0; g0 < d; g0 += kWave) {
            const int gs = (int)min<int64_t>(kWave, d - g0);
            int64_t len = 0;
            if (lane < gs) {
                const int32_t v = g.a_adj[e0 + g0 + lane];
                W.sbeg[lane] = g.b_off[v];
                len = g.b_off[v + 1] - W.sbeg[lane];
            }
            const int64_t tot = wave_scan_lengths(W, len);
            for (int64_t i = lane; i < tot; i += kWave) {
                const int j = wave_find_slice(W, gs, i);
                const int32_t w = g.b_adj[W.sbeg[j] + (i - W.pre[j])];
                if (w != u) wave_insert(W, (uint32_t)w);
            }
            if (lane == 0) wedges += (unsigned long long)(tot - gs);
            wave_sync();
        }
        for (int s = lane; s < kSmallSlots; s += kWave) {
            const unsigned long long v = W.tab[s];
            if (v) W.tab[s] = 0;
            ap.apply(v != 0, (int32_t)((v >> 32) - 1), (int64_t)(v & 0xffffffffull), pairs);
        }
        wave_sync();
    }
    wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
    pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
    skipped = (unsigned long long)wave_sum_i64((int64_t)skipped);
    if (lane == 0) {
        if (wedges) atomicAdd(&ctl->wedges_cd, wedges);
        if (pairs) atomicAdd(&ctl->pair_updates, pairs);
        if (skipped) atomicAdd(&ctl->skipped, skipped);
    }
}

__global__ void __launch_bounds__(kBigThreads)
k_peel_big(DevGraph g, const int32_t* __restrict__ front, const int32_t* n_front_p, CdApply ap,
           SpillArena spa, Ctl* ctl) {
    __shared__ BigLds L;
    constexpr int NT = kBigThreads;
    const int tid = threadIdx.x;
    bm_clear<NT>(L, kBmBits);
    if (tid == 0) L.spill_n = 0;
    __syncthreads();
    const Spill sp{spa.dense + (int64_t)blockIdx.x * spa.stride, spa.list + (int64_t)blockIdx.x * spa.stride};
    const int64_t n_front = *n_front_p;
    const bool multi = g.n_a > kBmBits;
    unsigned long long wedges = 0, pairs = 0, skipped = 0, spills = 0;
    for (int64_t it = blockIdx.x; it < n_front; it += gridDim.x) {
        const int32_t u = front[it];
        if (ap.supp[u] == 0) {
            skipped += tid == 0;
            continue;
        }
        const int64_t e0 = g.a_off[u], d = g.a_off[u + 1] - e0;
        for (int32_t klo = 0; klo < g.n_a; klo += kBmBits) {
            const int32_t khi = (int32_t)min<int64_t>(g.n_a, (int64_t)klo + kBmBits);
            const bool self_in = u >= klo && u < khi;
            for (int64_t g0 = 0; g0 < d; g0 += kGroup) {
                const int gs = (int)min<int64_t>(kGroup, d - g0);
                int64_t len = 0;
                if (tid < gs) {
                    const int32_t v = g.a_adj[e0 + g0 + tid];
                    int64_t a = g.b_off[v], b = g.b_off[v + 1];
                    if (multi) {
                        a = lower_bound_i32(g.b_adj, a, b, klo);
                        b = lower_bound_i32(g.b_adj, a, b, khi);
                    }
                    L.sbeg[tid] = a;
                    len = b - a;
                }
                const int64_t tot = block_scan_lengths<NT>(L, gs, len);
                for (int64_t i = tid; i < tot; i += NT) {
                    const int j = find_slice(L, gs, i);
                    const int32_t w = g.b_adj[L.sbeg[j] + (i - L.pre[j])];
                    if (w != u) bm_mark(L, sp, (uint32_t)(w - klo));
                }
                if (tid == 0) wedges += (unsigned long long)(tot - (self_in ? gs : 0));
                __syncthreads();
            }
            for (int s = tid; s < kRepSlots; s += NT) {
                const unsigned long long v = L.rep[s];
                ap.apply(v != 0, klo + (int32_t)((v >> 32) - 1), 1 + (int64_t)(v & 0xffffffffull), pairs);
            }
            const int32_t nsp = L.spill_n;
            if (tid == 0) spills += (unsigned long long)nsp;
            for (int32_t b0 = 0; b0 < nsp; b0 += NT) {
                const int32_t i = b0 + tid;
                int32_t k = 0, r = 0;
                if (i < nsp) {
                    k = sp.list[i];
                    r = sp.dense[k];
                    sp.dense[k] = 0;
                }
                ap.apply(i < nsp, klo + k, 1 + (int64_t)r, pairs);
            }
            __syncthreads();
            bm_clear<NT>(L, khi - klo);
            if (tid == 0) L.spill_n = 0;
            __syncthreads();
        }
    }
    wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
    pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
    skipped = (unsigned long long)wave_sum_i64((int64_t)skipped);
    spills = (unsigned long long)wave_sum_i64((int64_t)spills);
    if ((tid & (kWave - 1)) == 0) {
        if (wedges) atomicAdd(&ctl->wedges_cd, wedges);
        if (pairs) atomicAdd(&ctl->pair_updates, pairs);
        if (skipped) atomicAdd(&ctl->skipped, skipped);
        if (spills) atomicAdd(&ctl->spills, spills);
    }
}

// Vertices that crossed below the upper bound during the round become the
// next activeSet: assign them to the subset before any of them is peeled.
__global__ void k_round_end(const int32_t* __restrict__ l_small, const int32_t* __restrict__ l_big,
                            const int32_t* n_next, int32_t* state, const int64_t* __restrict__ wprox, int32_t label,
                            Ctl* ctl) {
    const int64_t ns = n_next[0], nb = n_next[1];
    long long ws = 0;
    GRID_STRIDE(j, ns + nb) {
        const int32_t u = j < ns ? l_small[j] : l_big[j - ns];
        state[u] = label;
        ws += wprox[u];
    }
    ws = wave_sum_i64(ws);
    if ((threadIdx.x & (kWave - 1)) == 0 && ws)
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->w_range), (unsigned long long)ws);
}

__global__ void k_ctl_swap_front(Ctl* ctl) {
    ctl->n_front[0] = ctl->n_next[0];
    ctl->n_front[1] = ctl->n_next[1];
    ctl->n_next[0] = ctl->n_next[1] = 0;
}

__global__ void k_assign_live(const int32_t* __restrict__ live, int32_t n_live, int32_t* state, int32_t label) {
    GRID_STRIDE(j, (int64_t)n_live) state[live[j]] = label;
}

// ===========================================================================
// Fine-grained decomposition (Alg. 4)
// ===========================================================================

__global__ void k_fd_vertex_keys(const int32_t* __restrict__ state, int32_t n_a, uint64_t* keys, int32_t* vals,
                                 int64_t* sub_cnt) {
    GRID_STRIDE(u, (int64_t)n_a) {
        const int32_t s = state[u];
        keys[u] = (uint64_t)s;
        vals[u] = (int32_t)u;
        atomic_add_i64(&sub_cnt[s], 1);
    }
}

__global__ void k_fd_positions(const int32_t* __restrict__ fd_vert, int32_t n_a, int32_t* fd_pos) {
    GRID_STRIDE(p, (int64_t)n_a) fd_pos[fd_vert[p]] = (int32_t)p;
}

// Partitioned CSC: key (row, subset of the entry), value = entry's index
// inside its subset.  The stable sort keeps each (row, subset) run ascending.
__global__ void k_fd_csc_keys(DevGraph g, const int32_t* __restrict__ state, const int32_t* __restrict__ fd_pos,
                              const int64_t* __restrict__ sub_off, int32_t S, uint64_t* keys, int32_t* vals) {
    GRID_STRIDE(q, g.m) {
        const int32_t w = g.b_adj[q];
        const int32_t s = state[w];
        keys[q] = (uint64_t)g.b_row[q] * (uint64_t)S + (uint64_t)s;
        vals[q] = (int32_t)(fd_pos[w] - sub_off[s]);
    }
}

__device__ inline int64_t lower_bound_u64(const uint64_t* __restrict__ a, int64_t lo, int64_t hi, uint64_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// For every CSR edge (u, v): the run of N_v inside u's own subset, i.e. the
// edges of the induced subgraph G_i seen from v (Alg. 4 induced subgraph).
__global__ void k_fd_slices(DevGraph g, const int32_t* __restrict__ state, const uint64_t* __restrict__ pkeys,
                            int32_t S, int64_t* fd_beg, int32_t* fd_len, int64_t* task_w) {
    GRID_STRIDE(p, g.m) {
        const int32_t u = g.a_row[p], v = g.a_adj[p];
        const int32_t s = state[u];
        const uint64_t k0 = (uint64_t)v * (uint64_t)S + (uint64_t)s;
        const int64_t lo = lower_bound_u64(pkeys, g.b_off[v], g.b_off[v + 1], k0);
        const int64_t hi = lower_bound_u64(pkeys, lo, g.b_off[v + 1], k0 + 1);
        fd_beg[p] = lo;
        fd_len[p] = (int32_t)(hi - lo);
        if (hi - lo > 1) atomic_add_i64(&task_w[s], hi - lo - 1);
    }
}

// Workload-aware schedule: subsets in decreasing order of induced wedges
// (ties by subset id).
__global__ void k_fd_order(const int64_t* __restrict__ task_w, int32_t S, int32_t* order) {
    for (int32_t i = threadIdx.x; i < S; i += blockDim.x) {
        const int64_t wi = task_w[i];
        int32_t r = 0;
        for (int32_t j = 0; j < S; ++j) {
            const int64_t wj = task_w[j];
            r += (wj > wi) || (wj == wi && j < i);
        }
        order[r] = i;
    }
}

__global__ void k_fd_reset_head(Ctl* ctl) { ctl->fd_head = 0; }

template <int NT>
__device__ inline int32_t block_excl_scan_i32(BigLds& L, int32_t x, int32_t& total) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t inc = wave_incl_scan_i64<NT>(x);
    __syncthreads();
    if (lane == kWave - 1) L.red[wid] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        const int64_t v = L.red[w];
        off += w < wid ? v : 0;
        tot += v;
    }
    total = (int32_t)tot;
    __syncthreads();
    return (int32_t)(off + inc - x);
}

// One workgroup peels one subset at a time, taking subsets from the
// workload-sorted queue (dynamic allocation).  Inside a subset it runs
// bottom-up peeling level by level: the level is max(level, minimum live
// support), and every live vertex whose support is at most the level is
// peeled at that level (equal to one-at-a-time peeling, whatever the order).
__global__ void __launch_bounds__(kBigThreads)
k_fd_peel(DevGraph g, FdBuffers fb, const int64_t* __restrict__ init, int32_t S, SpillArena spa, Ctl* ctl) {
    __shared__ BigLds L;
    constexpr int NT = kBigThreads;
    const int tid = threadIdx.x;
    bm_clear<NT>(L, kBmBits);
    if (tid == 0) L.spill_n = 0;
    __syncthreads();
    const Spill sp{spa.dense + (int64_t)blockIdx.x * spa.stride, spa.list + (int64_t)blockIdx.x * spa.stride};
    unsigned long long wedges = 0, pairs = 0, levels = 0, spills = 0;
    for (;;) {
        if (tid == 0) L.flag = atomicAdd(&ctl->fd_head, 1);
        __syncthreads();
        const int32_t t = L.flag;
        __syncthreads();
        if (t >= S) break;
        const int32_t sub = fb.order[t];
        const int64_t P0 = fb.sub_off[sub];
        const int32_t n_i = (int32_t)(fb.sub_off[sub + 1] - P0);
        if (n_i == 0) continue;
        int32_t* lc = fb.lst[0] + P0;
        int32_t* ln = fb.lst[1] + P0;
        int32_t* pl = fb.lst[2] + P0;
        int64_t* sup = fb.supp_fd + P0;
        int32_t* alive = fb.alive + P0;
        const int32_t* vert = fb.fd_vert + P0;
        for (int32_t j = tid; j < n_i; j += NT) {
            lc[j] = j;
            sup[j] = init[vert[j]];
            alive[j] = 1;
        }
        __syncthreads();
        const bool multi = n_i > kBmBits;
        int32_t n_live = n_i;
        int64_t level = 0;
        while (n_live > 0) {
            int64_t mn = INT64_MAX;
            for (int32_t j = tid; j < n_live; j += NT) {
                const int64_t s = sup[lc[j]];
                mn = s < mn ? s : mn;
            }
            mn = block_min_i64<NT>(L, mn);
            level = mn > level ? mn : level;
            int32_t n_peel = 0, n_keep = 0;
            for (int32_t b0 = 0; b0 < n_live; b0 += NT) {
                const int32_t j = b0 + tid;
                int32_t x = 0;
                bool pe = false, ke = false;
                if (j < n_live) {
                    x = lc[j];
                    pe = sup[x] <= level;
                    ke = !pe;
                }
                int32_t tp, tk;
                const int32_t op = block_excl_scan_i32<NT>(L, pe ? 1 : 0, tp);
                const int32_t ok = block_excl_scan_i32<NT>(L, ke ? 1 : 0, tk);
                if (pe) {
                    pl[n_peel + op] = x;
                    alive[x] = 0;
                    fb.theta[vert[x]] = level;
                }
                if (ke) ln[n_keep + ok] = x;
                n_peel += tp;
                n_keep += tk;
            }
            __syncthreads();
            levels += tid == 0;
            for (int32_t q = 0; q < n_peel; ++q) {
                const int32_t x = pl[q];
                if (sup[x] == 0) continue;
                const int32_t ux = vert[x];
                const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
                for (int32_t klo = 0; klo < n_i; klo += kBmBits) {
                    const int32_t khi = (int32_t)min<int64_t>(n_i, (int64_t)klo + kBmBits);
                    const bool self_in = x >= klo && x < khi;
                    for (int64_t g0 = 0; g0 < d; g0 += kGroup) {
                        const int gs = (int)min<int64_t>(kGroup, d - g0);
                        int64_t len = 0;
                        if (tid < gs) {
                            const int64_t e = e0 + g0 + tid;
                            int64_t a = fb.fd_beg[e], b = a + fb.fd_len[e];
                            if (multi) {
                                a = lower_bound_i32(fb.pcsc, a, b, klo);
                                b = lower_bound_i32(fb.pcsc, a, b, khi);
                            }
                            L.sbeg[tid] = a;
                            len = b - a;
                        }
                        const int64_t tot = block_scan_lengths<NT>(L, gs, len);
                        for (int64_t i = tid; i < tot; i += NT) {
                            const int j = find_slice(L, gs, i);
                            const int32_t w = fb.pcsc[L.sbeg[j] + (i - L.pre[j])];
                            if (w != x) bm_mark(L, sp, (uint32_t)(w - klo));
                        }
                        if (tid == 0) wedges += (unsigned long long)(tot - (self_in ? gs : 0));
                        __syncthreads();
                    }
                    for (int s = tid; s < kRepSlots; s += NT) {
                        const unsigned long long v = L.rep[s];
                        if (v) {
                            const int32_t w = klo + (int32_t)((v >> 32) - 1);
                            if (alive[w]) {
                                atomic_add_i64(&sup[w], -choose2(1 + (int64_t)(v & 0xffffffffull)));
                                ++pairs;
                            }
                        }
                    }
                    const int32_t nsp = L.spill_n;
                    if (tid == 0) spills += (unsigned long long)nsp;
                    for (int32_t i = tid; i < nsp; i += NT) {
                        const int32_t k = sp.list[i];
                        const int32_t w = klo + k;
                        if (alive[w]) {
                            atomic_add_i64(&sup[w], -choose2(1 + (int64_t)sp.dense[k]));
                            ++pairs;
                        }
                        sp.dense[k] = 0;
                    }
                    __syncthreads();
                    bm_clear<NT>(L, khi - klo);
                    if (tid == 0) L.spill_n = 0;
                    __syncthreads();
                }
            }
            int32_t* tmp = lc;
            lc = ln;
            ln = tmp;
            n_live = n_keep;
        }
    }
    wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
    pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
    levels = (unsigned long long)wave_sum_i64((int64_t)levels);
    spills = (unsigned long long)wave_sum_i64((int64_t)spills);
    if ((tid & (kWave - 1)) == 0) {
        if (wedges) atomicAdd(&ctl->wedges_fd, wedges);
        if (pairs) atomicAdd(&ctl->pair_updates, pairs);
        if (levels) atomicAdd(&ctl->fd_levels, levels);
        if (spills) atomicAdd(&ctl->spills, spills);
    }
}

__global__ void k_scatter_i64(const int64_t* __restrict__ by_rank, const int32_t* __restrict__ orig, int32_t n,
                              int64_t* out) {
    GRID_STRIDE(r, (int64_t)n) out[orig[r]] = by_rank[r];
}

int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

}  // namespace

// ===========================================================================
// Launch wrappers
// ===========================================================================

int big_kernel_occupancy() {
    int n = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_peel_big, kBigThreads, 0));
    int n2 = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, k_count_big, kBigThreads, 0));
    int n3 = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n3, k_fd_peel, kBigThreads, 0));
    return std::max(1, std::min(n, std::min(n2, n3)));
}

void launch_count(const DevGraph& g, CountBuffers& cb, Ctl* ctl, const SpillArena& spill, int big_grid, hipStream_t s) {
    const int64_t n_tot = (int64_t)g.n_a + g.n_b;
    fill_i64(cb.bfly_a, 0, g.n_a, s);
    fill_i64(cb.bfly_b, 0, g.n_b, s);
    fill_i64(cb.work, 0, n_tot, s);
    if (g.m == 0) return;
    k_count_work<<<grid1(g.m), kT, 0, s>>>(g, cb.work);
    TIP_HIP_TRY(hipGetLastError());
    k_count_bins<<<grid1(n_tot, 4096), kT, 0, s>>>(cb.work, n_tot, cb.items_small, cb.items_big, ctl);
    TIP_HIP_TRY(hipGetLastError());
    k_count_small<<<2048, kSmallThreads, 0, s>>>(g, cb.items_small, ctl, cb.bfly_a, cb.bfly_b);
    TIP_HIP_TRY(hipGetLastError());
    k_count_big<<<big_grid, kBigThreads, 0, s>>>(g, cb.items_big, ctl, cb.bfly_a, cb.bfly_b, spill, ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_wproxy(const DevGraph& g, const int32_t* deg_b_rank, int64_t* wprox, hipStream_t s) {
    fill_i64(wprox, 0, g.n_a, s);
    if (g.m == 0) return;
    k_wproxy<<<grid1(g.m), kT, 0, s>>>(g, deg_b_rank, wprox);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_range_start(PeelBuffers& pb, int cur_live, int32_t n_live, Ctl* ctl, hipStream_t s) {
    k_ctl_begin_range<<<1, 1, 0, s>>>(ctl);
    TIP_HIP_TRY(hipGetLastError());
    if (n_live <= 0) return;
    k_range_start<<<grid1(n_live, 4096), kT, 0, s>>>(pb.live[cur_live], n_live, pb.live[1 - cur_live], pb.state,
                                                      pb.supp, pb.init, pb.wprox, ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_select(PeelBuffers& pb, int cur_live, int32_t n_live, uint64_t max_supp, int64_t tgt, Ctl* ctl,
                   hipStream_t s) {
    k_ctl_select_init<<<1, 1, 0, s>>>(ctl, (long long)tgt);
    TIP_HIP_TRY(hipGetLastError());
    const int bits = bits_for(max_supp);
    const int passes = (bits + 7) / 8;
    for (int p = passes - 1; p >= 0; --p) {
        const int shift = 8 * p;
        k_select_hist<<<grid1(n_live, 2048), kT, 0, s>>>(pb.live[cur_live], n_live, pb.supp, pb.wprox, shift, ctl,
                                                          pb.sel_hist);
        TIP_HIP_TRY(hipGetLastError());
        k_select_pick<<<1, 256, 0, s>>>(shift, ctl, pb.sel_hist);
        TIP_HIP_TRY(hipGetLastError());
    }
}

void launch_frontier_init(PeelBuffers& pb, int cur_live, int32_t n_live, int64_t hi, int32_t label, int cur_front,
                          Ctl* ctl, hipStream_t s) {
    if (n_live <= 0) return;
    k_frontier_init<<<grid1(n_live, 4096), kT, 0, s>>>(pb.live[cur_live], n_live, pb.supp, pb.state, pb.wprox,
                                                        (long long)hi, label, pb.front[cur_front][0],
                                                        pb.front[cur_front][1], ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_peel_round(const DevGraph& g, PeelBuffers& pb, int cur_front, int32_t n_small, int32_t n_big,
                       int64_t hi, Ctl* ctl, const SpillArena& spill, int big_grid, hipStream_t s) {
    const int nxt = 1 - cur_front;
    CdApply ap{pb.supp, pb.state, pb.wprox, (long long)hi, &ctl->n_next[0], &ctl->n_next[1],
               pb.front[nxt][0], pb.front[nxt][1]};
    if (n_small > 0) {
        const int nw = kSmallThreads / kWave;
        int64_t blocks = (n_small + nw - 1) / nw;
        if (blocks > 8192) blocks = 8192;
        k_peel_small<<<(unsigned)blocks, kSmallThreads, 0, s>>>(g, pb.front[cur_front][0], &ctl->n_front[0], ap,
                                                                 ctl);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (n_big > 0) {
        const int grid = (int)std::min<int64_t>(n_big, big_grid);
        k_peel_big<<<grid, kBigThreads, 0, s>>>(g, pb.front[cur_front][1], &ctl->n_front[1], ap, spill, ctl);
        TIP_HIP_TRY(hipGetLastError());
    }
}

void launch_round_end(PeelBuffers& pb, int next_front, int32_t n_small, int32_t n_big, int32_t label, Ctl* ctl,
                      hipStream_t s) {
    if (n_small + n_big > 0) {
        k_round_end<<<grid1((int64_t)n_small + n_big, 4096), kT, 0, s>>>(
            pb.front[next_front][0], pb.front[next_front][1], ctl->n_next, pb.state, pb.wprox, label, ctl);
        TIP_HIP_TRY(hipGetLastError());
    }
    k_ctl_swap_front<<<1, 1, 0, s>>>(ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_assign_live(PeelBuffers& pb, int cur_live, int32_t n_live, int32_t label, hipStream_t s) {
    if (n_live <= 0) return;
    k_assign_live<<<grid1(n_live), kT, 0, s>>>(pb.live[cur_live], n_live, pb.state, label);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_fd(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, Ctl* ctl, const SpillArena& spill,
               int big_grid, uint64_t* tmp_keys, int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp,
               uint64_t* keys_scratch, int32_t* vals_scratch, hipStream_t s) {
    const int32_t n_a = g.n_a;
    if (n_a <= 0) return;
    // vertices grouped by subset, ascending rank inside each subset
    fill_i64(fb.sub_cnt, 0, (int64_t)S + 1, s);
    k_fd_vertex_keys<<<grid1(n_a), kT, 0, s>>>(pb.state, n_a, keys_scratch, fb.fd_vert, fb.sub_cnt);
    TIP_HIP_TRY(hipGetLastError());
    radix_sort_pairs(keys_scratch, fb.fd_vert, tmp_keys, tmp_vals, n_a, bits_for((uint64_t)S), hist, scan_tmp, s);
    scan_exclusive_i64(fb.sub_cnt, fb.sub_off, (int64_t)S + 1, scan_tmp, s);
    k_fd_positions<<<grid1(n_a), kT, 0, s>>>(fb.fd_vert, n_a, fb.fd_pos);
    TIP_HIP_TRY(hipGetLastError());
    fill_i64(fb.task_w, 0, S, s);
    if (g.m > 0) {
        k_fd_csc_keys<<<grid1(g.m), kT, 0, s>>>(g, pb.state, fb.fd_pos, fb.sub_off, S, fb.pkeys, fb.pcsc);
        TIP_HIP_TRY(hipGetLastError());
        radix_sort_pairs(fb.pkeys, fb.pcsc, tmp_keys, tmp_vals, g.m,
                         bits_for((uint64_t)g.n_b * (uint64_t)S), hist, scan_tmp, s);
        k_fd_slices<<<grid1(g.m), kT, 0, s>>>(g, pb.state, fb.pkeys, S, fb.fd_beg, fb.fd_len, fb.task_w);
        TIP_HIP_TRY(hipGetLastError());
    }
    k_fd_order<<<1, 1024, 0, s>>>(fb.task_w, S, fb.order);
    TIP_HIP_TRY(hipGetLastError());
    k_fd_reset_head<<<1, 1, 0, s>>>(ctl);
    TIP_HIP_TRY(hipGetLastError());
    const int grid = std::max(1, std::min<int>(S, big_grid));
    k_fd_peel<<<grid, kBigThreads, 0, s>>>(g, fb, pb.init, S, spill, ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_scatter_i64(const int64_t* by_rank, const int32_t* orig, int32_t n, int64_t* out, hipStream_t s) {
    if (n <= 0) return;
    k_scatter_i64<<<grid1(n), kT, 0, s>>>(by_rank, orig, n, out);
    TIP_HIP_TRY(hipGetLastError());
}

}  // namespace tip
