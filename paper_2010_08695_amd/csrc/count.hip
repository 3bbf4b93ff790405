// Per-vertex butterfly counting (Alg. 1) on the device.
#include "kern_util.h"

namespace tip {
namespace {
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

// The highest-degree vertices of each side (the smallest ids, since ids are
// ranks by descending degree) end most butterflies' priority wedges, so their
// counts take a large share of all increments.  Each workgroup accumulates
// the increments of ids below kCountHot in LDS and adds them to HBM once at
// its end; one address in HBM takes only ~1e8 atomics per second.
constexpr int kCountHot = 112;

struct HotCounts {
    unsigned long long v[2][kCountHot];

    __device__ inline void clear() {
        for (int i = threadIdx.x; i < 2 * kCountHot; i += blockDim.x) v[i / kCountHot][i % kCountHot] = 0;
    }
    __device__ inline void add(int64_t* bfly, int side, int64_t id, int64_t x) {
        if (id < kCountHot) atomicAdd(&v[side][id], (unsigned long long)x);
        else atomic_add_i64(&bfly[id], x);
    }
    // after a barrier that every thread of the workgroup reaches
    __device__ inline void flush(int64_t* bfly_a, int64_t* bfly_b) const {
        for (int i = threadIdx.x; i < 2 * kCountHot; i += blockDim.x) {
            const unsigned long long x = v[i / kCountHot][i % kCountHot];
            if (x) atomic_add_i64(i < kCountHot ? &bfly_a[i] : &bfly_b[i - kCountHot], (int64_t)x);
        }
    }
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

// Sum over the lanes of a wave that hold the same row (rows are sorted, so
// equal rows are adjacent): the last lane of each run adds it to out[row].
__device__ inline void wave_row_add(int32_t row, int64_t x, int64_t* out) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(x, d, kWave);
        const int32_t ry = __shfl_up(row, d, kWave);
        if (lane >= d && ry == row) x += y;
    }
    const int32_t rn = __shfl_down(row, 1, kWave);
    if (row >= 0 && (lane == kWave - 1 || rn != row) && x) atomic_add_i64(&out[row], x);
}

// Counting wedges of every start vertex; CSR rows are contiguous, so the
// per-edge terms are summed per row inside each wave before the atomic.
__global__ void k_count_work(DevGraph g, int64_t* work) {
    UNIFORM_STRIDE(base, g.m) {
        const int64_t p = base + threadIdx.x;
        int32_t x = -1, yb = -1;
        int64_t l1 = 0, l2 = 0;
        if (p < g.m) {
            x = g.a_row[p];
            l1 = min(g.b_cut[g.a_adj[p]], g.a_rev[p]);
            yb = g.b_row[p];
            l2 = min(g.a_cut[g.b_adj[p]], g.b_rev[p]);
        }
        wave_row_add(x, l1, work);
        wave_row_add(yb, l2, work + g.n_a);
    }
}

// Start vertices by work item kind.  Almost every vertex is appended to one
// of the two lists, so the list counters are reserved once per workgroup
// for its whole contiguous chunk (counted in a first pass): per-wave appends
// would queue tens of thousands of atomics on the two counters.
constexpr int kBinsThreads = 256;

__global__ void __launch_bounds__(kBinsThreads)
k_count_bins(const int64_t* __restrict__ work, int64_t n, int32_t* small, int32_t* big, Ctl* ctl) {
    constexpr int NW = kBinsThreads / kWave;
    __shared__ int32_t wcnt[2][NW];
    __shared__ int32_t base_l[2];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = (int64_t)blockIdx.x * chunk, c1 = min(n, c0 + chunk);
    int32_t ns = 0, nb = 0;
    unsigned long long tot = 0;
    for (int64_t i = c0 + tid; i < c1; i += kBinsThreads) {
        const int64_t w = work[i];
        tot += (unsigned long long)w;
        ns += (w > 0 && w <= kSmallMaxWedges) ? 1 : 0;
        nb += w > kSmallMaxWedges ? 1 : 0;
    }
    tot = (unsigned long long)wave_sum_i64((int64_t)tot);
    if (lane == 0 && tot) atomicAdd(&ctl->wedges_count, tot);
    ns = (int32_t)wave_sum_i64(ns);
    nb = (int32_t)wave_sum_i64(nb);
    if (lane == 0) {
        wcnt[0][wid] = ns;
        wcnt[1][wid] = nb;
    }
    __syncthreads();
    if (tid < 2) {
        int32_t t = 0;
        for (int w = 0; w < NW; ++w) t += wcnt[tid][w];
        base_l[tid] = t ? atomicAdd(&ctl->n_items[tid], t) : 0;
    }
    __syncthreads();
    // second pass: positions in chunk order, one running offset per wave
    // (waves take consecutive 64-entry slices in turn)
    int32_t off_s = base_l[0], off_b = base_l[1];
    for (int64_t b0 = c0; b0 < c1; b0 += kBinsThreads) {
        const int64_t i = b0 + tid;
        const int64_t w = i < c1 ? work[i] : 0;
        const bool is_s = w > 0 && w <= kSmallMaxWedges, is_b = w > kSmallMaxWedges;
        const uint64_t ms = __ballot(is_s), mb = __ballot(is_b);
        if (lane == 0) {
            wcnt[0][wid] = (int32_t)__popcll(ms);
            wcnt[1][wid] = (int32_t)__popcll(mb);
        }
        __syncthreads();
        int32_t ps = off_s, pb = off_b;
        for (int w2 = 0; w2 < wid; ++w2) {
            ps += wcnt[0][w2];
            pb += wcnt[1][w2];
        }
        if (is_s) small[ps + (int32_t)__popcll(ms & lanemask_lt())] = (int32_t)i;
        if (is_b) big[pb + (int32_t)__popcll(mb & lanemask_lt())] = (int32_t)i;
        for (int w2 = 0; w2 < NW; ++w2) {
            off_s += wcnt[0][w2];
            off_b += wcnt[1][w2];
        }
        __syncthreads();  // wcnt is rewritten by the next slice
    }
}

__global__ void __launch_bounds__(kSmallThreads)
k_count_small(DevGraph g, const int32_t* __restrict__ items, const Ctl* ctl, const int64_t* __restrict__ work,
              int64_t* bfly_a, int64_t* bfly_b, const int32_t* __restrict__ live_a) {
    // live_a (re-count of the live graph, HUC): only when the round asks for
    // it; side-A vertices count only while live, side-B counts are not kept
    if (live_a && !ctl->huc_now) return;
    __shared__ WaveLds WL[kSmallThreads / kWave];
    __shared__ HotCounts hot;
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    WaveLds& W = WL[wid];
    for (int s = lane; s < kSmallSlots; s += kWave) W.tab[s] = 0;
    hot.clear();
    __syncthreads();
    const int64_t n_items = ctl->n_items[0];
    const int nw = kSmallThreads / kWave;
    for (int64_t it = (int64_t)blockIdx.x * nw + wid; it < n_items; it += (int64_t)gridDim.x * nw) {
        const int32_t item = items[it];
        const bool side_b = item >= g.n_a;
        const int own = side_b ? 1 : 0;
        const int32_t x = side_b ? item - g.n_a : item;
        if (live_a && !side_b && live_a[x] != kLive) continue;
        const SideView sv = side_view(g, side_b, bfly_a, bfly_b);
        const int64_t e0 = sv.own_off[x], d = sv.own_off[x + 1] - e0;
        const uint32_t slots = wave_slots(work[item]);
        const uint32_t mask = slots - 1;
        const bool mid_dead_check = live_a && side_b;   // middle vertices on side A
        const bool end_dead_check = live_a && !side_b;  // end vertices on side A
        // pass 1: wedge counts c(x, z)
        for (int64_t g0 = 0; g0 < d; g0 += kWave) {
            const int gs = (int)min<int64_t>(kWave, d - g0);
            int64_t len = 0;
            if (lane < gs) {
                const int64_t e = e0 + g0 + lane;
                const int32_t y = sv.own_adj[e];
                W.sbeg[lane] = sv.oth_off[y];
                len = (mid_dead_check && live_a[y] != kLive) ? 0 : min(sv.oth_cut[y], sv.own_rev[e]);
            }
            const int64_t tot = wave_scan_lengths(W, len);
            int j = 0;
            for (int64_t i = lane; i < tot; i += kWave) {
                while (j + 1 < gs && W.pre[j + 1] <= i) ++j;
                const uint32_t z = (uint32_t)sv.oth_adj[W.sbeg[j] + (i - W.pre[j])];
                if (!end_dead_check || live_a[z] == kLive) wave_insert(W, z, mask);
            }
            wave_sync();
        }
        // pass 2: middle vertices gain c - 1 per wedge; with one chunk of
        // neighbours the runs staged by pass 1 are still in LDS
        const bool one_chunk = d <= kWave;
        for (int64_t g0 = 0; g0 < (end_dead_check ? 0 : d); g0 += kWave) {
            const int gs = (int)min<int64_t>(kWave, d - g0);
            int64_t len = 0;
            int32_t y = 0;
            int64_t tot;
            if (one_chunk) {
                if (lane < gs) y = sv.own_adj[e0 + lane];
                tot = W.pre[gs];
            } else {
                if (lane < gs) {
                    const int64_t e = e0 + g0 + lane;
                    y = sv.own_adj[e];
                    W.sbeg[lane] = sv.oth_off[y];
                    len = (mid_dead_check && live_a[y] != kLive) ? 0 : min(sv.oth_cut[y], sv.own_rev[e]);
                }
                tot = wave_scan_lengths(W, len);
            }
            W.acc[lane] = 0;
            wave_sync();
            int j = 0;
            for (int64_t i = lane; i < tot; i += kWave) {
                while (j + 1 < gs && W.pre[j + 1] <= i) ++j;
                const int32_t c = wave_lookup(W, (uint32_t)sv.oth_adj[W.sbeg[j] + (i - W.pre[j])], mask);
                if (c > 1) atomicAdd(reinterpret_cast<unsigned long long*>(&W.acc[j]), (unsigned long long)(c - 1));
            }
            wave_sync();
            if (lane < gs && W.acc[lane]) hot.add(sv.oth_bfly, 1 - own, y, W.acc[lane]);
            wave_sync();
        }
        // pass 3: start and end vertices gain C(c, 2)
        int64_t local = 0;
        for (uint32_t s = lane; s < slots; s += kWave) {
            const unsigned long long v = W.tab[s];
            if (v) {
                const int64_t c = (int64_t)(v & 0xffffffffull);
                if (c >= 2 && !mid_dead_check) {
                    const int64_t b = choose2(c);
                    hot.add(sv.own_bfly, own, (int64_t)(v >> 32) - 1, b);
                    local += b;
                }
                W.tab[s] = 0;
            }
        }
        local = wave_sum_i64(local);
        if (lane == 0 && local) hot.add(sv.own_bfly, own, x, local);
        wave_sync();
    }
    __syncthreads();
    hot.flush(bfly_a, bfly_b);
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
            SpillArena spa, Ctl* ctl_rw, const int32_t* __restrict__ live_a) {
    if (live_a && !ctl->huc_now) return;
    __shared__ BigLds L;
    __shared__ HotCounts hot;
    constexpr int NT = kBigThreads;
    const int tid = threadIdx.x;
    hot.clear();
    bm_clear<NT>(L, kBmBits);
    if (tid == 0) L.spill_n = 0;
    __syncthreads();
    const Spill sp{spa.dense + (int64_t)blockIdx.x * spa.stride, spa.list + (int64_t)blockIdx.x * spa.stride};
    const int64_t n_items = ctl->n_items[1];
    unsigned long long spills = 0;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int32_t item = items[it];
        const bool side_b = item >= g.n_a;
        const int own = side_b ? 1 : 0;
        const int32_t x = side_b ? item - g.n_a : item;
        if (live_a && !side_b && live_a[x] != kLive) continue;
        const SideView sv = side_view(g, side_b, bfly_a, bfly_b);
        const int64_t e0 = sv.own_off[x], d = sv.own_off[x + 1] - e0;
        const bool multi = x > kBmBits;
        const bool mid_dead_check = live_a && side_b;
        const bool end_dead_check = live_a && !side_b;
        for (int32_t klo = 0; klo < x; klo += kBmBits) {
            const int32_t khi = (int32_t)min<int64_t>(x, (int64_t)klo + kBmBits);
            // pass 1
            for (int64_t g0 = 0; g0 < d; g0 += kGroup) {
                const int gs = (int)min<int64_t>(kGroup, d - g0);
                int64_t len = 0;
                if (tid < gs) {
                    int64_t s0;
                    CountSlice::get(sv, e0 + g0 + tid, multi, klo, khi, s0, len);
                    if (mid_dead_check && live_a[sv.own_adj[e0 + g0 + tid]] != kLive) len = 0;
                    L.sbeg[tid] = s0;
                }
                const int64_t tot = block_scan_lengths<NT>(L, gs, len);
                for (int64_t i = tid; i < tot; i += NT) {
                    const int j = find_slice(L, gs, i);
                    const int32_t z = sv.oth_adj[L.sbeg[j] + (i - L.pre[j])];
                    if (!end_dead_check || live_a[z] == kLive) bm_mark(L, sp, (uint32_t)(z - klo));
                }
                __syncthreads();
            }
            const bool spilled = L.spill_n > 0;
            // pass 2; with one group of neighbours the runs staged by pass 1
            // are still in LDS
            const bool one_group = d <= kGroup;
            for (int64_t g0 = 0; g0 < (end_dead_check ? 0 : d); g0 += kGroup) {
                const int gs = (int)min<int64_t>(kGroup, d - g0);
                int64_t len = 0;
                int64_t tot;
                if (one_group) {
                    if (tid < gs) L.acc[tid] = 0;
                    tot = L.pre[gs];
                    __syncthreads();
                } else {
                    if (tid < gs) {
                        int64_t s0;
                        CountSlice::get(sv, e0 + g0 + tid, multi, klo, khi, s0, len);
                        if (mid_dead_check && live_a[sv.own_adj[e0 + g0 + tid]] != kLive) len = 0;
                        L.sbeg[tid] = s0;
                        L.acc[tid] = 0;
                    }
                    tot = block_scan_lengths<NT>(L, gs, len);
                }
                for (int64_t i = tid; i < tot; i += NT) {
                    const int j = find_slice(L, gs, i);
                    const uint32_t k = (uint32_t)(sv.oth_adj[L.sbeg[j] + (i - L.pre[j])] - klo);
                    const int32_t c = rep_lookup(L, sp, spilled, k);
                    if (c > 1) atomicAdd(reinterpret_cast<unsigned long long*>(&L.acc[j]), (unsigned long long)(c - 1));
                }
                __syncthreads();
                if (tid < gs && L.acc[tid]) hot.add(sv.oth_bfly, 1 - own, sv.own_adj[e0 + g0 + tid], L.acc[tid]);
                __syncthreads();
            }
            // pass 3
            int64_t local = 0;
            for (int s = tid; s < kRepSlots; s += NT) {
                const unsigned long long v = L.rep[s];
                if (v && !mid_dead_check) {
                    const int64_t c = 1 + (int64_t)(v & 0xffffffffull);
                    const int64_t b = choose2(c);
                    hot.add(sv.own_bfly, own, klo + (int64_t)(v >> 32) - 1, b);
                    local += b;
                }
            }
            const int32_t nsp = L.spill_n;
            spills += (tid == 0) ? (unsigned long long)nsp : 0ull;
            for (int32_t i = tid; i < nsp; i += NT) {
                const int32_t k = sp.list[i];
                if (!mid_dead_check) {
                    const int64_t b = choose2(1 + (int64_t)sp.dense[k]);
                    hot.add(sv.own_bfly, own, klo + (int64_t)k, b);
                    local += b;
                }
                sp.dense[k] = 0;
            }
            const int64_t total = block_sum_i64<NT>(L, local);
            if (tid == 0 && total) hot.add(sv.own_bfly, own, x, total);
            bm_clear<NT>(L, khi - klo);
            if (tid == 0) L.spill_n = 0;
            __syncthreads();
        }
    }
    if (tid == 0 && spills) atomicAdd(&ctl_rw->spills, spills);
    __syncthreads();
    hot.flush(bfly_a, bfly_b);
}

}  // namespace

int count_occupancy() {
    int n = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_count_big, kBigThreads, 0));
    return std::max(1, n);
}

void launch_count(const DevGraph& g, CountBuffers& cb, Ctl* ctl, const SpillArena& spill, int big_grid, hipStream_t s) {
    const int64_t n_tot = (int64_t)g.n_a + g.n_b;
    fill_i64(cb.bfly_a, 0, g.n_a, s);
    fill_i64(cb.bfly_b, 0, g.n_b, s);
    fill_i64(cb.work, 0, n_tot, s);
    if (g.m == 0) return;
    k_count_work<<<grid1(g.m), kT, 0, s>>>(g, cb.work);
    TIP_HIP_TRY(hipGetLastError());
    k_count_bins<<<(unsigned)std::min<int64_t>(256, std::max<int64_t>(1, (n_tot + kBinsThreads - 1) / kBinsThreads)),
                   kBinsThreads, 0, s>>>(cb.work, n_tot, cb.items_small, cb.items_big, ctl);
    TIP_HIP_TRY(hipGetLastError());
    k_count_small<<<2048, kSmallThreads, 0, s>>>(g, cb.items_small, ctl, cb.work, cb.bfly_a, cb.bfly_b, nullptr);
    TIP_HIP_TRY(hipGetLastError());
    k_count_big<<<big_grid, kBigThreads, 0, s>>>(g, cb.items_big, ctl, cb.bfly_a, cb.bfly_b, spill, ctl, nullptr);
    TIP_HIP_TRY(hipGetLastError());
}

// HUC (Section 4.1): when the control block says so for this round, the
// side-A counts are computed again on the graph of live side-A vertices
// (state == kLive) and all of side B, into bfly_a, which then holds every
// live vertex's support.  Reuses the work items of the first count; every
// kernel returns at once otherwise, so the launches can sit in a captured
// round.
__global__ void k_clear_if_huc(int64_t* a, int64_t n, const Ctl* ctl) {
    if (!ctl->huc_now) return;
    GRID_STRIDE(i, n) a[i] = 0;
}

void launch_recount(const DevGraph& g, CountBuffers& cb, const int32_t* state, Ctl* ctl, const SpillArena& spill,
                    int big_grid, hipStream_t s) {
    if (g.m == 0) return;
    k_clear_if_huc<<<grid1(g.n_a, 1024), kT, 0, s>>>(cb.bfly_a, g.n_a, ctl);
    TIP_HIP_TRY(hipGetLastError());
    k_count_small<<<2048, kSmallThreads, 0, s>>>(g, cb.items_small, ctl, cb.work, cb.bfly_a, cb.bfly_b, state);
    TIP_HIP_TRY(hipGetLastError());
    k_count_big<<<big_grid, kBigThreads, 0, s>>>(g, cb.items_big, ctl, cb.bfly_a, cb.bfly_b, spill, ctl, state);
    TIP_HIP_TRY(hipGetLastError());
}

}  // namespace tip
