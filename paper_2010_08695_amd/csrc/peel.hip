// Coarse-grained decomposition (Alg. 3): range bounds, activeSets and the
// delete-update peeling kernels.
//
// Supports are stored raw (uncapped) and decremented with 64-bit atomics; the
// cap of the paper's update (never below the current level) is applied when a
// support is read: the effective support is max(level, raw).  A live vertex's
// raw support is exactly its butterflies with the other live vertices, so it
// never underflows.
//
// Every live vertex starts a round with support >= the range's upper bound
// (those below it form the round's activeSet), so the next activeSet is the
// set of live vertices whose support is below the bound after the round: it
// is found by one scan of the live list, and the update kernels decrement
// without waiting for the atomics' old values.
//
// A peeled vertex u's update aggregates c(u, w) over its 2-hop neighbourhood
// (Alg. 2, update).  Three kernels share the work by the size of that
// neighbourhood (w[u], the wedges of u in the original graph):
//   * wave path: a few hundred wedges, one wavefront per vertex with its own
//     LDS hash table of every key;
//   * bitmap path: one workgroup per vertex, one LDS bit per key of a key
//     tile, keys reached again go to an LDS table of repeat counts;
//   * dense path: 2-hop neighbourhoods that cover a large share of the key
//     space; one workgroup per (vertex, key tiles) with a 2- to 32-bit
//     counter per key, so a heavy vertex is spread over many workgroups.
// All lists of the other side are sorted, so the part of N_v inside a key
// tile is a contiguous run whose bounds come from a per-list table.
#include "kern_util.h"

#include <type_traits>

namespace tip {
namespace {

// ---------------------------------------------------------------------------
// Shared staging of neighbour-list runs and unit-wise traversal
// ---------------------------------------------------------------------------

// Staging of up to NR runs (one per thread j < NR) for a workgroup of NT
// threads.
template <int NT, int NR = NT>
struct Stage {
    int64_t sbeg[NR];
    int32_t len[NR];
    int32_t upre[NR + 1];
    int64_t red[NT / kWave];
    int64_t item;
};

// Work items of a round are taken from a per-kernel counter, so workgroups
// that drew cheap items go on to the next instead of idling behind one that
// drew an expensive one.  (Taking the next index early does not pay: vector
// memory results return in order, so every later load would wait for it.)
// All threads of the workgroup must call.
template <int NT, int NR>
__device__ inline int64_t next_item(Stage<NT, NR>& S, unsigned long long* head) {
    __syncthreads();
    if (threadIdx.x == 0) S.item = (int64_t)atomicAdd(head, 1ull);
    __syncthreads();
    return S.item;
}

// Stages the runs held by threads j < gs <= NR (one run per thread: start,
// length) and returns the number of traversal units (kUnit entries of one
// run).
template <int NT, int NR>
__device__ inline int32_t stage_units(Stage<NT, NR>& S, int gs, int64_t s0, int32_t len) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int32_t units = tid < gs ? (len + kUnit - 1) / kUnit : 0;
    if (tid < gs) {
        S.sbeg[tid] = s0;
        S.len[tid] = len;
    }
    const int64_t inc = wave_incl_scan_i64<NT>(units);
    __syncthreads();
    if (lane == kWave - 1) S.red[wid] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        const int64_t v = S.red[w];
        off += w < wid ? v : 0;
        tot += v;
    }
    if (tid < gs) S.upre[tid] = (int32_t)(off + inc - units);
    if (tid == 0) S.upre[gs] = (int32_t)tot;
    __syncthreads();
    return (int32_t)tot;
}

// Every wave takes units in turn (k = wave, wave + NW, ...); a unit is read
// with coalesced loads.  A wave's unit indices only grow, so the run holding
// a unit is found by stepping forward from the previous one.  kUnitsInFlight
// units are loaded before any is consumed, so 2 * kUnitsInFlight loads per
// lane are in flight together.
template <int NT, int NR>
__device__ inline int advance_run(const Stage<NT, NR>& S, int j, int gs, int32_t k) {
    while (j + 1 < gs && S.upre[j + 1] <= k) ++j;
    return j;
}

constexpr int kUnitsInFlight = 4;

template <int NT, int NR, class F>
__device__ inline void traverse_units(const Stage<NT, NR>& S, int gs, int32_t nunits,
                                      const int32_t* __restrict__ adj, F&& f) {
    constexpr int NW = NT / kWave;
    constexpr int R = kUnitsInFlight;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int j = 0;
    for (int32_t k0 = wid; k0 < nunits; k0 += R * NW) {
        int32_t x[2 * R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t k = k0 + r * NW;
            int32_t n = 0;
            const int32_t* p = adj;
            if (k < nunits) {
                j = advance_run(S, j, gs, k);
                const int32_t off = (k - S.upre[j]) * kUnit;
                n = min(kUnit, S.len[j] - off);
                p = adj + S.sbeg[j] + off;
            }
            x[2 * r] = lane < n ? p[lane] : -1;
            x[2 * r + 1] = lane + kWave < n ? p[lane + kWave] : -1;
        }
#pragma unroll
        for (int r = 0; r < 2 * R; ++r)
            if (x[r] >= 0) f(x[r]);
    }
}

// ---------------------------------------------------------------------------
// Range set-up kernels
// ---------------------------------------------------------------------------

// w[u]: wedges of G with endpoint u (the range-sizing proxy), i.e. the sum
// over v in N_u of d_v - 1.  CSR rows are contiguous, so the terms are summed
// per row inside each wave and one atomic goes out per row piece (a hub row
// would otherwise take one atomic per edge on one address).
__global__ void k_wproxy(DevGraph g, const int32_t* __restrict__ deg_b, int64_t* wprox) {
    const int lane = threadIdx.x & (kWave - 1);
    UNIFORM_STRIDE(base, g.m) {
        const int64_t p = base + threadIdx.x;
        int32_t u = -1;
        int64_t x = 0;
        if (p < g.m) {
            u = g.a_row[p];
            const int32_t dv = deg_b[g.a_adj[p]];
            x = dv > 1 ? dv - 1 : 0;
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t y = __shfl_up(x, d, kWave);
            const int32_t uy = __shfl_up(u, d, kWave);
            if (lane >= d && uy == u) x += y;
        }
        const int32_t un = __shfl_down(u, 1, kWave);
        if (u >= 0 && (lane == kWave - 1 || un != u) && x) atomic_add_i64(&wprox[u], x);
    }
}

// Which update kernel peels u, by its wedge count w[u] and degree: the wave
// kernel for a few hundred wedges; the bitmap kernel while the repeat keys
// (a few percent of the wedges) fit its LDS table, i.e. up to bm_max wedges;
// above that the dense kernel, unless its counter bytes (n_a * bits / 8,
// bits from the degree so that c(u, w) <= d_u fits) are large against the
// wedges (w <= n_a * bits / dense_div), or one table tile of its counters
// does not fit the workgroup's LDS (16-bit counters on sides of more than
// 64M keys, 32-bit ones above 8M keys).  With 16- or 32-bit counters an item
// covers one list tile, so every pass stages all of u's
// neighbours again: such a vertex takes the dense path only when its wedges
// are at least kDense16Stage times its degree times the passes, or when they
// are more than one bitmap workgroup takes without spilling (late hubs whose
// live wedges have shrunk would otherwise run on one workgroup).  A dense
// vertex is heavy when a light-sized item (item_keys[kind] keys) would hold
// more than kItemWedges of its wedges.
struct ItemKeys {
    int64_t k[kDenseKinds];
};

__global__ void k_peel_bins(const int64_t* __restrict__ a_off, const int64_t* __restrict__ wprox, int32_t n_a,
                            int64_t dense_div, int64_t bm_max, ItemKeys ik, const Ctl* ctl, uint8_t* bin) {
    // keys the update can touch: all of side A, or below the live bound
    const int64_t nk = ctl ? max<int64_t>(1, ctl->key_hi) : max<int32_t>(1, n_a);
    GRID_STRIDE(u, (int64_t)n_a) {
        const int64_t w = wprox[u];
        const int64_t d = a_off[u + 1] - a_off[u];
        const int bits = dense_bits(d);
        uint8_t b = kBinBitmap;
        if (w <= kSmallMaxWedges) {
            b = kBinWave;
        } else if (bits && ik.k[dense_kind(bits)] * bits <= (int64_t)kDenseLdsBytes * 8 &&
                   w > max<int64_t>(bm_max, nk * bits / dense_div) &&
                   (bits < 16 || w > kBmHubWedges ||
                    w >= kDense16Stage * d * ((nk + ik.k[dense_kind(bits)] - 1) / ik.k[dense_kind(bits)]))) {
            const bool heavy = (double)w * (double)ik.k[dense_kind(bits)] > (double)kItemWedges * (double)nk;
            b = (uint8_t)dense_bin(bits, heavy);
        }
        bin[u] = b;
    }
}

// tb[v * (ntt + 1) + t] = offset in N_v of the first entry >= t * tk.
__global__ void k_tile_bounds(const int64_t* __restrict__ b_off, const int32_t* __restrict__ b_adj, int32_t n_b,
                              int32_t tk, int32_t ntt, int32_t* tb) {
    const int64_t n = (int64_t)n_b * (ntt + 1);
    GRID_STRIDE(i, n) {
        const int64_t v = i / (ntt + 1);
        const int32_t t = (int32_t)(i % (ntt + 1));
        const int64_t lo = b_off[v], hi = b_off[v + 1];
        int64_t pos = hi;
        if (t < ntt) pos = lower_bound_i32(b_adj, lo, hi, (int32_t)min<int64_t>((int64_t)t * tk, INT32_MAX));
        tb[i] = (int32_t)(pos - lo);
    }
}

__global__ void k_ctl_begin_range(Ctl* ctl) {
    ctl->n_live_next = 0;
    ctl->w_range = 0;
    for (int i = 0; i < kSpread; ++i) {
        ctl->spread[i][kScWRange] = 0;
        ctl->spread[i][kScWRem] = 0;
        ctl->spread_max[i] = 0;
    }
    for (int b = 0; b < kBins; ++b) ctl->n_front[b] = ctl->n_next[b] = ctl->head[b] = 0;
}

// Workgroup size of the scans over a live list.
constexpr int kScanThreads = 512;

// Appends val, for every thread with pred, to list b (b < NB) with one
// atomic per list per workgroup: the appends of a scan go to a handful of
// counters, and one address takes only about 1e8 atomics per second.  All
// threads of the workgroup must call.
template <int NB>
__device__ inline void block_append(bool pred, int32_t val, int b, int32_t* const* lists, int32_t* counts) {
    constexpr int NW = kScanThreads / kWave;
    __shared__ int32_t s_off[NB][NW];
    __shared__ int32_t s_base[NB];
    if (!__syncthreads_or(pred)) return;  // one barrier when nothing is appended
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    uint64_t mine = 0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const uint64_t m = __ballot(pred && b == k);
        if (lane == 0) s_off[k][wid] = __popcll(m);
        if (pred && b == k) mine = m;
    }
    __syncthreads();
    if (tid < NB) {
        int32_t tot = 0;
        for (int w = 0; w < NW; ++w) {
            const int32_t c = s_off[tid][w];
            s_off[tid][w] = tot;
            tot += c;
        }
        s_base[tid] = tot ? atomicAdd(&counts[tid], tot) : 0;
    }
    __syncthreads();
    if (pred) lists[b][s_base[b] + s_off[b][wid] + __popcll(mine & lanemask_lt())] = val;
    __syncthreads();
}

inline unsigned scan_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(512, (n + kScanThreads - 1) / kScanThreads));
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
        block_append<1>(keep, u, 0, &live_out, &ctl->n_live_next);
    }
    __shared__ unsigned long long smx[kScanThreads / kWave];
    __shared__ long long sws[kScanThreads / kWave];
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
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            m2 = smx[w] > m2 ? smx[w] : m2;
            w2 += sws[w];
        }
        if (m2) atomicMax(&ctl->spread_max[blockIdx.x & (kSpread - 1)], m2);
        if (w2) spread_add(ctl, kScWRem, (unsigned long long)w2);
    }
}

__global__ void k_ctl_select_init(Ctl* ctl, long long tgt) {
    ctl->sel_prefix = 0;
    ctl->sel_cum = 0;
    ctl->sel_found = 1;
    ctl->sel_tgt = tgt;
}

// findHi as a weighted radix select: one kSelBits-bit digit per pass, most
// significant first.  The histogram adds w[u] over live u whose support
// matches the prefix chosen so far.  kT threads.
__global__ void k_select_hist(const int32_t* __restrict__ live, int32_t n_live, const int64_t* __restrict__ supp,
                              const int64_t* __restrict__ wprox, int shift, const Ctl* ctl, int64_t* hist) {
    if (!ctl->sel_found) return;
    __shared__ unsigned long long h[kSelBins];
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t prefix = ctl->sel_prefix;
    const int hs = shift + kSelBits;
    const int lane = threadIdx.x & (kWave - 1);
    // the supports of a range cluster, so a wave's keys often share the
    // digit: then one LDS atomic adds the wave's sum
    UNIFORM_STRIDE(base, (int64_t)n_live) {
        const int64_t j = base + threadIdx.x;
        bool ok = false;
        uint32_t dg = 0;
        unsigned long long w = 0;
        if (j < n_live) {
            const int32_t u = live[j];
            const uint64_t key = (uint64_t)supp[u];
            if (hs >= 64 || (key >> hs) == (prefix >> hs)) {
                ok = true;
                dg = (uint32_t)((key >> shift) & (kSelBins - 1));
                w = (unsigned long long)wprox[u];
            }
        }
        const uint64_t act = __ballot(ok);
        if (act == 0) continue;
        const int first = __ffsll((unsigned long long)act) - 1;
        const uint32_t d0 = (uint32_t)__shfl((int)dg, first, kWave);
        if (__ballot(ok && dg != d0) == 0) {
            const unsigned long long tot = (unsigned long long)wave_sum_i64((int64_t)(ok ? w : 0));
            if (lane == first) atomicAdd(&h[d0], tot);
        } else if (ok) {
            atomicAdd(&h[dg], w);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x)
        if (h[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&hist[i]), h[i]);
}

// The digit of this pass: the first d with sel_cum + hist[0..d] >= target.
// Thread t holds bins [t * PER, (t + 1) * PER); a block scan of their sums
// finds the one thread whose bins cross the target, which walks them.  The
// histogram is left zero for the next pass.  kT threads.
__global__ void k_select_pick(int shift, Ctl* ctl, int64_t* hist) {
    constexpr int PER = kSelBins / kT;
    static_assert(PER * kT == kSelBins, "bins split evenly over the threads");
    __shared__ long long wsum[kT / kWave];
    __shared__ int chosen;
    __shared__ long long chosen_run;
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    long long v[PER], s = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        v[i] = hist[t * PER + i];
        hist[t * PER + i] = 0;
        s += v[i];
    }
    const long long inc = wave_incl_scan_i64<kT>(s);
    if (lane == kWave - 1) wsum[wid] = inc;
    if (t == 0) chosen = -1;
    __syncthreads();
    const bool found = ctl->sel_found != 0;
    if (found) {
        const long long tgt = ctl->sel_tgt;
        long long before = ctl->sel_cum + inc - s;
        for (int w = 0; w < wid; ++w) before += wsum[w];
        // prefix sums never decrease, so one thread crosses (thread 0 also
        // when sel_cum alone reaches the target)
        if ((t == 0 || before < tgt) && before + s >= tgt) {
            long long run = before;
            for (int i = 0; i < PER; ++i) {
                if (run + v[i] >= tgt) {
                    chosen = t * PER + i;
                    chosen_run = run;
                    break;
                }
                run += v[i];
            }
        }
    }
    __syncthreads();
    if (t == 0 && found) {
        if (chosen < 0) {
            ctl->sel_found = 0;
        } else {
            ctl->sel_cum = chosen_run;
            ctl->sel_prefix |= (unsigned long long)chosen << shift;
        }
    }
}

struct Fronts {
    int32_t* list[kBins];
    int32_t* count;  // [kBins]
};

// Both frontier buffers; kernels pick the current one from the control block.
struct FrontSet {
    int32_t* list[2][kBins];
};

// Appends u to the frontier list of its bin; all lanes of the wave must call.
// (Appends are sparse after a range's first round; per-workgroup batching
// measured slower here than in the range start.)
__device__ inline void append_binned(bool pred, int32_t u, uint8_t b, const Fronts& f) {
#pragma unroll
    for (int k = 0; k < kBins; ++k) wave_append(pred && b == k, u, f.list[k], &f.count[k]);
}

// activeSet of a round: live vertices with support below the range's upper
// bound.  They are assigned to the subset here (before any of them is
// peeled); vertices with zero support share no butterfly with any live
// vertex and need no update.  next = 0: the range's first activeSet, into
// the current buffer; next = 1: after a round, into the other buffer (and
// nothing to do when the round's activeSet was empty).
__global__ void k_frontier_scan(FrontSet fs, const int32_t* live0, const int32_t* live1,
                                const int64_t* __restrict__ supp, int32_t* state, const int64_t* __restrict__ wprox,
                                const uint8_t* __restrict__ bin, const int64_t* __restrict__ a_off, int next,
                                Ctl* ctl) {
    if (next) {
        int32_t any = 0;
#pragma unroll
        for (int b = 0; b < kBins; ++b) any |= ctl->n_front[b];
        if (!any) return;
    }
    const int32_t* __restrict__ live = ctl->range_live ? live1 : live0;
    const int32_t n_live = ctl->range_n_live;
    const long long hi = ctl->range_hi;
    const int32_t label = ctl->range_label;
    const int buf = next ? 1 - ctl->front_buf : ctl->front_buf;
    Fronts fr;
#pragma unroll
    for (int b = 0; b < kBins; ++b) fr.list[b] = fs.list[buf][b];
    fr.count = next ? ctl->n_next : ctl->n_front;
    long long ws = 0;
    unsigned long long skipped = 0, dead = 0;
    UNIFORM_STRIDE(base, (int64_t)n_live) {
        const int64_t j = base + threadIdx.x;
        bool pred = false;
        int32_t u = 0;
        uint8_t b = 0;
        if (j < n_live) {
            u = live[j];
            const int64_t su = supp[u];
            if (su < hi && state[u] == kLive) {
                state[u] = label;
                ws += wprox[u];
                dead += (unsigned long long)(a_off[u + 1] - a_off[u]);
                if (su == 0) ++skipped;
                else {
                    pred = true;
                    b = bin[u];
                }
            }
        }
        append_binned(pred, u, b, fr);
    }
    ws = wave_sum_i64(ws);
    skipped = (unsigned long long)wave_sum_i64((int64_t)skipped);
    dead = (unsigned long long)wave_sum_i64((int64_t)dead);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (ws) spread_add(ctl, kScWRange, (unsigned long long)ws);
        if (skipped) spread_add(ctl, kScSkipped, skipped);
        if (dead) spread_add(ctl, kScDeadEdges, dead);
    }
}

// hi < 0: the bound is the select's result, read here on the device so that
// the host need not wait for it (findHi's answer, or max_supp + 1 when no
// prefix reached the target).
__global__ void k_set_range(Ctl* ctl, long long hi, long long max_supp, int32_t label, int32_t live,
                            int32_t n_live) {
    if (hi < 0) hi = ctl->sel_found ? (long long)ctl->sel_prefix + 1 : max_supp + 1;
    ctl->huc_now = 0;
    ctl->huc_w_prev = 0;
    ctl->range_hi = hi;
    ctl->range_label = label;
    ctl->range_live = live;
    ctl->range_n_live = n_live;
    ctl->front_buf = 0;
    for (int b = 0; b < kBins; ++b) ctl->n_front[b] = ctl->n_next[b] = ctl->head[b] = 0;
}

// ---------------------------------------------------------------------------
// Delete-update
// ---------------------------------------------------------------------------

// Up to B (key, c) pairs held by one lane in registers: every index is a
// compile-time constant after unrolling, so nothing goes to private memory.
template <int B>
struct PairBuf {
    int32_t key[B];
    int32_t cnt[B];
    int n = 0;

    __device__ inline void push(int32_t k, int32_t c) {
#pragma unroll
        for (int i = 0; i < B; ++i)
            if (i == n) {
                key[i] = k;
                cnt[i] = c;
            }
        ++n;
    }
};

// Applies the decrement C(c, 2) of (peeled u, w) pairs.  It goes to every w,
// live or not: the support of a vertex that is no longer live is never read
// again (rounds and range starts read live vertices only, and the fine-grained
// step starts from the range's snapshot), so no liveness load has to come
// before the atomic.  Decrements of vertices peeled in the same round can
// bring their support to 0, which is why zero-support vertices are left out
// by the frontier scan only (at that point no decrement of the round has
// happened) and not again by the update kernels.
struct CdApply {
    int64_t* supp;

    // Applies and empties the lane's buffered pairs (all with c >= 2); the
    // decrements do not return a value, so nothing waits on them.
    template <int B>
    __device__ inline void flush(PairBuf<B>& pb, unsigned long long& pairs) const {
#pragma unroll
        for (int i = 0; i < B; ++i)
            if (i < pb.n) {
                atomic_add_i64(&supp[pb.key[i]], -choose2(pb.cnt[i]));
                ++pairs;
            }
        pb.n = 0;
    }
};

struct PeelCounters {
    unsigned long long wedges = 0, pairs = 0, skipped = 0, spills = 0, edges = 0;

    __device__ inline void flush(Ctl* ctl, bool big) {
        wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
        pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
        skipped = (unsigned long long)wave_sum_i64((int64_t)skipped);
        spills = (unsigned long long)wave_sum_i64((int64_t)spills);
        edges = (unsigned long long)wave_sum_i64((int64_t)edges);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            if (wedges) spread_add(ctl, kScWedgesCd, wedges);
            if (pairs) spread_add(ctl, kScPairs, pairs);
            if (skipped) spread_add(ctl, kScSkipped, skipped);
            if (spills) spread_add(ctl, kScSpills, spills);
            if (big) {
                if (wedges) spread_add(ctl, kScBigWedges, wedges);
                if (pairs) spread_add(ctl, kScBigPairs, pairs);
                if (edges) spread_add(ctl, kScBigEdges, edges);
            }
        }
    }
};

// Wave path: one wavefront per vertex, every 2-hop key in a per-wave LDS hash
// table sized to the vertex's wedge count.
__global__ void __launch_bounds__(kSmallThreads)
k_peel_wave(DevGraph g, FrontSet fs, const int64_t* __restrict__ wprox, CdApply ap, Ctl* ctl) {
    const int64_t n_front = ctl->n_front[kBinWave];
    if (n_front == 0 || ctl->huc_now) return;
    const int32_t* __restrict__ front = fs.list[ctl->front_buf][kBinWave];
    __shared__ WaveLds WL[kSmallThreads / kWave];
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    WaveLds& W = WL[wid];
    for (int s = lane; s < kSmallSlots; s += kWave) W.tab[s] = 0;
    wave_sync();
    const int nw = kSmallThreads / kWave;
    PeelCounters pc;
    for (int64_t it = (int64_t)blockIdx.x * nw + wid; it < n_front; it += (int64_t)gridDim.x * nw) {
        const int32_t u = front[it];
        const int64_t e0 = g.a_off[u], d = g.a_off[u + 1] - e0;
        const uint32_t slots = wave_slots(wprox[u]);
        for (int64_t g0 = 0; g0 < d; g0 += kWave) {
            const int gs = (int)min<int64_t>(kWave, d - g0);
            int64_t len = 0;
            if (lane < gs) {
                const int32_t v = g.a_adj[e0 + g0 + lane];
                W.sbeg[lane] = g.b_off[v];
                len = g.b_off[v + 1] - W.sbeg[lane];
            }
            const int64_t tot = wave_scan_lengths(W, len);
            int j = 0;
            for (int64_t i = lane; i < tot; i += kWave) {
                while (j + 1 < gs && W.pre[j + 1] <= i) ++j;
                const int32_t w = g.b_adj[W.sbeg[j] + (i - W.pre[j])];
                if (w != u) wave_insert(W, (uint32_t)w, slots - 1);
            }
            if (lane == 0) pc.wedges += (unsigned long long)(tot - gs);
            wave_sync();
        }
        // slots is a multiple of the wave size, so the loop is wave-uniform
        PairBuf<4> pbuf;
        for (uint32_t s = lane; s < slots; s += kWave) {
            const unsigned long long v = W.tab[s];
            if (v) W.tab[s] = 0;
            const int32_t c = (int32_t)(v & 0xffffffffull);
            if (c >= 2) pbuf.push((int32_t)((v >> 32) - 1), c);
            if (__ballot(pbuf.n == 4)) ap.flush(pbuf, pc.pairs);
        }
        ap.flush(pbuf, pc.pairs);
        wave_sync();
    }
    pc.flush(ctl, false);
}

// Bitmap path LDS: one bit per key of a kBmTile-key tile, a table of repeat
// counts, staging.
struct BmLds {
    uint32_t bm[kBmTile / 32];
    unsigned long long rep[kBmRep];
    Stage<kBmThreads, kBmRuns> st;
    int32_t spill_n;
};

__device__ inline void bm_rep_insert(BmLds& L, const Spill& sp, uint32_t k) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    const uint32_t h = hash32(k) & (kBmRep - 1);
#pragma unroll 1
    for (int p = 0; p < kRepProbe; ++p) {
        unsigned long long* slot = &L.rep[(h + p) & (kBmRep - 1)];
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
    }
    if (atomicAdd(&sp.dense[k], 1) == 0) {
        const int32_t idx = atomicAdd(&L.spill_n, 1);
        sp.list[idx] = (int32_t)k;
    }
}

__global__ void __launch_bounds__(kBmThreads)
k_peel_bitmap(DevGraph g, const int32_t* __restrict__ tb, int32_t tk, int32_t ntt, FrontSet fs, CdApply ap,
              SpillArena spa, Ctl* ctl) {
    const int64_t n_front = ctl->n_front[kBinBitmap];
    if (n_front == 0 || ctl->huc_now) return;
    const int32_t* __restrict__ front = fs.list[ctl->front_buf][kBinBitmap];
    __shared__ BmLds L;
    constexpr int NT = kBmThreads;
    constexpr int kPer = kBmRep / NT;  // repeat slots scanned by each thread
    static_assert(kBmRep % NT == 0 && kPer >= 1 && kPer <= 32, "repeat slots per thread");
    const int tid = threadIdx.x;
    for (int w = tid; w < kBmTile / 32; w += NT) L.bm[w] = 0;
    for (int s = tid; s < kBmRep; s += NT) L.rep[s] = 0;
    if (tid == 0) L.spill_n = 0;
    __syncthreads();
    // a tile never holds more than min(kBmTile, stride) keys, so workgroups
    // are packed that far apart in the spill arena
    const int64_t sp_gap = min<int64_t>(kBmTile, spa.stride);
    const Spill sp{spa.dense + (int64_t)blockIdx.x * sp_gap, spa.list + (int64_t)blockIdx.x * sp_gap};
    const int32_t sub = kBmTile / tk;  // table tiles per bitmap tile
    const int32_t key_hi = ctl->key_hi;
    PeelCounters pc;
    for (;;) {
        const int64_t it = next_item(L.st, &ctl->head[kBinBitmap]);
        if (it >= n_front) break;
        const int32_t u = front[it];
        const int64_t e0 = g.a_off[u], d = g.a_off[u + 1] - e0;
        if (tid == 0) pc.edges += (unsigned long long)d;
        for (int32_t klo = 0; klo < key_hi; klo += kBmTile) {
            const int32_t khi = (int32_t)min<int64_t>(key_hi, (int64_t)klo + kBmTile);
            const int32_t t0 = klo / tk, t1 = min(t0 + sub, ntt);
            for (int64_t g0 = 0; g0 < d; g0 += kBmRuns) {
                const int gs = (int)min<int64_t>(kBmRuns, d - g0);
                int64_t s0 = 0;
                int32_t len = 0;
                if (tid < gs) {
                    const int32_t v = g.a_adj[e0 + g0 + tid];
                    const int32_t* row = tb + (int64_t)v * (ntt + 1);
                    const int32_t a = row[t0];
                    s0 = g.b_off[v] + a;
                    len = row[t1] - a;
                }
                const int32_t nu = stage_units(L.st, gs, s0, len);
                unsigned long long wl = 0;
                traverse_units(L.st, gs, nu, g.b_adj, [&](int32_t w) {
                    if (w != u) {
                        ++wl;
                        const uint32_t k = (uint32_t)(w - klo);
                        const uint32_t bit = 1u << (k & 31);
                        if (atomicOr(&L.bm[k >> 5], bit) & bit) bm_rep_insert(L, sp, k);
                    }
                });
                pc.wedges += wl;
                __syncthreads();
            }
            // repeat keys: each thread owns kPer slots, applied in batches
            PairBuf<kApplyBatch> pbuf;
            for (int q = 0; q < kPer; ++q) {
                const unsigned long long v = L.rep[tid + q * NT];
                if (v) pbuf.push(klo + (int32_t)((v >> 32) - 1), 1 + (int32_t)(v & 0xffffffffull));
                if (__ballot(pbuf.n == kApplyBatch)) ap.flush(pbuf, pc.pairs);
            }
            ap.flush(pbuf, pc.pairs);
            const int32_t nsp = L.spill_n;
            if (tid == 0) pc.spills += (unsigned long long)nsp;
            for (int32_t b0 = 0; b0 < nsp; b0 += NT) {
                const int32_t i = b0 + tid;
                if (i < nsp) {
                    const int32_t k = sp.list[i];
                    const int32_t r = sp.dense[k];
                    sp.dense[k] = 0;
                    pbuf.push(klo + k, 1 + r);
                }
                if (__ballot(pbuf.n == kApplyBatch)) ap.flush(pbuf, pc.pairs);
            }
            ap.flush(pbuf, pc.pairs);
            __syncthreads();
            const int32_t words = (khi - klo + 31) >> 5;
            for (int w = tid; w < words; w += NT) L.bm[w] = 0;
            for (int s = tid; s < kBmRep; s += NT) L.rep[s] = 0;
            if (tid == 0) L.spill_n = 0;
            __syncthreads();
        }
    }
    pc.flush(ctl, false);
}

// Counters of value >= 2 in a word of BITS-bit counters: the top bit of
// every such field is set in the result.
template <int BITS>
__device__ inline uint32_t ge2_mask(uint32_t x) {
    if (BITS == 32) return x >= 2 ? 0x80000000u : 0u;
    if (BITS == 2) return x & 0xaaaaaaaau;
    if (BITS == 4) {
        const uint32_t t = x & 0xeeeeeeeeu;
        return (((t & 0x77777777u) + 0x77777777u) | t) & 0x88888888u;
    }
    if (BITS == 8) {
        const uint32_t t = x & 0xfefefefeu;
        return (((t & 0x7f7f7f7fu) + 0x7f7f7f7fu) | t) & 0x80808080u;
    }
    const uint32_t t = x & 0xfffefffeu;
    return (((t & 0x7fff7fffu) + 0x7fff7fffu) | t) & 0x80008000u;
}

// Dense path: a work item is (frontier vertex, table tiles [t_begin, t_end)):
// one workgroup counts the 2-hop keys of one vertex inside that key range
// with one BITS-bit LDS counter per key (the bins guarantee c(u, w) <= d_u
// fits), then applies C(c, 2) for every key with c >= 2.  Counters are all
// zero between items: an item clears every word it read.
template <int BITS>
__device__ inline void dense_item(const DevGraph& g, const int32_t* __restrict__ tb, int32_t tk, int32_t ntt,
                                  int32_t u, int32_t t_begin, int32_t t_end, int32_t gpass, uint32_t* cnt,
                                  Stage<kDenseThreads>& S, const CdApply& ap, PeelCounters& pc) {
    constexpr int NT = kDenseThreads;
    constexpr int PER_WORD = 32 / BITS;          // counters per 32-bit word
    constexpr uint32_t FMASK = BITS == 32 ? 0xffffffffu : BITS == 16 ? 0xffffu : ((1u << (BITS % 32)) - 1);
    constexpr int32_t kStageWords = 4 * kWave;  // one quad per lane of the wave
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    uint4* cnt4 = reinterpret_cast<uint4*>(cnt);
    const int64_t e0 = g.a_off[u], d = g.a_off[u + 1] - e0;
    if (tid == 0 && t_begin == 0) pc.edges += (unsigned long long)d;
    // with at most NT neighbours, their list offsets and the tile bounds of
    // every pass of the item (at most kDensePasses + 1) are loaded once and
    // stay in registers; bnd[0] and bnd[1] bound the current pass
    //
    // With at most kWave neighbours (every vertex of the 2- and 4-bit
    // counters, most of the 8-bit ones) every wave loads all of them, lane l
    // neighbour l, and finds each traversal unit's run with a ballot over its
    // own lanes: a pass then needs no staging in LDS and no barrier before
    // its traversal.
    const bool one = d <= NT;
    const bool narrow = d <= kWave;
    int64_t bo1 = 0;
    int32_t bnd[kDensePasses + 1];
#pragma unroll
    for (int k = 0; k <= kDensePasses; ++k) bnd[k] = 0;
    const int nb_idx = narrow ? lane : tid;  // the neighbour this thread holds
    if (one && nb_idx < d) {
        const int32_t v1 = g.a_adj[e0 + nb_idx];
        bo1 = g.b_off[v1];
        const int32_t* row = tb + (int64_t)v1 * (ntt + 1);
#pragma unroll
        for (int k = 0; k <= kDensePasses; ++k) bnd[k] = row[min(t_end, t_begin + k * gpass)];
    }
    // one pass per gpass tiles: count in LDS, then apply and clear
    for (int32_t p0 = t_begin; p0 < t_end; p0 += gpass) {
        const int32_t p1 = min(t_end, p0 + gpass);
        const int32_t klo = p0 * tk;
        if (narrow) {
            constexpr int NW = NT / kWave;
            constexpr int R = kUnitsInFlight;
            const int wid = tid / kWave;
            int64_t s0 = 0;
            int32_t len = 0;
            if (lane < d) {
                s0 = bo1 + bnd[0];
                len = bnd[1] - bnd[0];
            }
            const int32_t units = (len + kUnit - 1) / kUnit;
            const int32_t incl = wave_incl_scan_i32(units);
            const int32_t nu = __shfl(incl, kWave - 1, kWave);
            const int32_t pre = incl - units;  // lanes past d: nu
            unsigned long long wl = 0;
            for (int32_t k0 = wid; k0 < nu; k0 += R * NW) {
                int32_t x[2 * R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int32_t k = k0 + r * NW;
                    int32_t n = 0;
                    const int32_t* pp = g.b_adj;
                    if (k < nu) {
                        // the unit's run: the last lane whose first unit is <= k
                        const uint64_t le = __ballot(pre <= k);
                        const int j = kWave - 1 - __clzll((long long)le);
                        const int64_t sj = __shfl(s0, j, kWave);
                        const int32_t lj = __shfl(len, j, kWave), pj = __shfl(pre, j, kWave);
                        const int32_t off = (k - pj) * kUnit;
                        n = min(kUnit, lj - off);
                        pp = g.b_adj + sj + off;
                    }
                    x[2 * r] = lane < n ? pp[lane] : -1;
                    x[2 * r + 1] = lane + kWave < n ? pp[lane + kWave] : -1;
                }
#pragma unroll
                for (int r = 0; r < 2 * R; ++r) {
                    const int32_t w = x[r];
                    if (w >= 0 && w != u) {
                        ++wl;
                        const uint32_t k = (uint32_t)(w - klo);
                        atomicAdd(&cnt[k / PER_WORD], 1u << ((k % PER_WORD) * BITS));
                    }
                }
            }
            pc.wedges += wl;
            __syncthreads();
        }
        for (int64_t g0 = 0; !narrow && g0 < d; g0 += NT) {
            const int gs = (int)min<int64_t>(NT, d - g0);
            int64_t s0 = 0;
            int32_t len = 0;
            if (tid < gs) {
                if (one) {
                    s0 = bo1 + bnd[0];
                    len = bnd[1] - bnd[0];
                } else {
                    const int32_t v = g.a_adj[e0 + g0 + tid];
                    const int32_t* row = tb + (int64_t)v * (ntt + 1);
                    const int32_t a = row[p0];
                    s0 = g.b_off[v] + a;
                    len = row[p1] - a;
                }
            }
            const int32_t nu = stage_units(S, gs, s0, len);
            unsigned long long wl = 0;
            traverse_units(S, gs, nu, g.b_adj, [&](int32_t w) {
                if (w != u) {
                    ++wl;
                    const uint32_t k = (uint32_t)(w - klo);
                    atomicAdd(&cnt[k / PER_WORD], 1u << ((k % PER_WORD) * BITS));
                }
            });
            pc.wedges += wl;
            __syncthreads();
        }
        // keys with c >= 2 are applied in key order from consecutive lanes, so
        // that an atomic instruction touches few 128-byte lines of supports:
        // with at most one pair per lane through one cross-lane permute, else
        // staged in the 64 counter quads the wave has just read (256 packed
        // (key offset, c) words per round); then the quads are cleared.  n4
        // is a multiple of 256 (tk is a multiple of 16K keys); with n4 < NT
        // the threads past n4 read quads outside this pass, inside the
        // counter array and zero, so their waves stage nothing.
        const int32_t n4 = (int32_t)((int64_t)(p1 - p0) * tk / PER_WORD / 4);
        for (int32_t base = 0; base < n4; base += NT) {
            const int32_t w4 = base + tid;
            const uint4 x = cnt4[w4];
            const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
            uint32_t msk[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) msk[q] = ge2_mask<BITS>(xs[q]);
            const int32_t mine0 = __popc(msk[0]) + __popc(msk[1]) + __popc(msk[2]) + __popc(msk[3]);
            const uint64_t has = __ballot(mine0 > 0);
            if (has != 0 && __ballot(mine0 > 1) == 0) {
                // at most one pair per lane (the common case): one permute
                // moves the pairs, in key order, to the first lanes
                int32_t key = 0;
                uint32_t c = 0;
                if (mine0 == 1) {
                    const int q = msk[0] ? 0 : msk[1] ? 1 : msk[2] ? 2 : 3;
                    const uint32_t m = q == 0 ? msk[0] : q == 1 ? msk[1] : q == 2 ? msk[2] : msk[3];
                    const uint32_t xq = q == 0 ? xs[0] : q == 1 ? xs[1] : q == 2 ? xs[2] : xs[3];
                    const int f = (__ffs(m) - 1) / BITS;
                    key = klo + w4 * 4 * PER_WORD + q * PER_WORD + f;
                    c = (xq >> (f * BITS)) & FMASK;
                }
                // lanes with a pair go to their rank among them, the others
                // to the lanes after those: a permutation of the wave
                const int32_t n_has = __popcll(has);
                const uint64_t lt = lanemask_lt();
                const int dst = mine0 == 1 ? __popcll(has & lt) : n_has + __popcll(~has & lt);
                const int32_t k2 = __builtin_amdgcn_ds_permute(dst << 2, key);
                const int32_t c2v = __builtin_amdgcn_ds_permute(dst << 2, (int32_t)c);
                if (lane < n_has) {
                    atomic_add_i64(&ap.supp[k2], -choose2(c2v));
                    ++pc.pairs;
                }
            } else if (has != 0 && BITS == 32) {
                // 32-bit counts do not fit the window's 16-bit field: each
                // lane applies its own quad (consecutive keys across lanes)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (xs[q] >= 2) {
                        atomic_add_i64(&ap.supp[klo + w4 * 4 + q], -choose2((int64_t)xs[q]));
                        ++pc.pairs;
                    }
            } else if (has != 0) {
                // denser: stage the pairs through the quad window
                uint32_t* win = reinterpret_cast<uint32_t*>(cnt4 + (w4 - lane));
                const int32_t kwin = klo + (w4 - lane) * 4 * PER_WORD;
                const uint32_t koff = (uint32_t)lane * 4 * PER_WORD;
                for (;;) {
                    const int32_t mine = __popc(msk[0]) + __popc(msk[1]) + __popc(msk[2]) + __popc(msk[3]);
                    const int32_t incl = wave_incl_scan_i32(mine);
                    const int32_t total = __shfl(incl, kWave - 1, kWave);
                    if (total == 0) break;
                    int32_t pos = incl - mine;
                    wave_sync();  // every lane has read its quad before the window is written
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        while (msk[q] && pos < kStageWords) {
                            const int bit = __ffs(msk[q]) - 1;
                            msk[q] &= msk[q] - 1;
                            const int f = bit / BITS;
                            win[pos++] = ((koff + (uint32_t)(q * PER_WORD + f)) << 16) | ((xs[q] >> (f * BITS)) & FMASK);
                        }
                    }
                    wave_sync();
                    const int32_t n_st = min(total, kStageWords);
#pragma unroll
                    for (int i = 0; i < kStageWords / kWave; ++i) {
                        const int32_t j = lane + i * kWave;
                        if (j < n_st) {
                            const uint32_t e = win[j];
                            atomic_add_i64(&ap.supp[kwin + (int32_t)(e >> 16)], -choose2((int32_t)(e & 0xffffu)));
                            ++pc.pairs;
                        }
                    }
                    wave_sync();  // the window is read before the next round rewrites it
                }
            }
            cnt4[w4] = make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kDensePasses; ++k) bnd[k] = bnd[k + 1];
    }
}

// Item layout of one dense launch: counter widths 16, 8, 4, 2 bits in that
// order (most wedges per vertex first), each heavy vertices (items of gh
// tiles) then light ones (items of gl tiles).
struct DensePlan {
    int64_t end[kDenseKinds];      // cumulative item counts
    int64_t n_heavy[kDenseKinds];  // heavy items of each width
    int32_t gl[kDenseKinds], gh[kDenseKinds], ngl[kDenseKinds], ngh[kDenseKinds], np[kDenseKinds];
};

constexpr int kDenseOrder[kDenseKinds] = {4, 3, 2, 1, 0};  // kinds of 32, 16, 8, 4, 2 bits

// One launch for every dense vertex of the round, whatever its counter
// width: a single work queue, one tail.  g_max[kind]: widest light item
// (tiles) the LDS allows for that width.  LDS: kDenseLdsBytes of counters +
// staging.
__global__ void __launch_bounds__(kDenseThreads)
k_peel_dense(DevGraph g, const int32_t* __restrict__ tb, int32_t tk, int32_t ntt, FrontSet fs, ItemKeys g_max,
             int64_t slots, CdApply ap, Ctl* ctl) {
    constexpr int NT = kDenseThreads;
    if (ctl->huc_now) return;
    // only tiles below the live key bound can hold a key to update; ntt
    // itself stays the row stride of the tile-bound table
    const int32_t ntk = min(ntt, (int32_t)((max(ctl->key_hi, 1) + (int64_t)tk - 1) / tk));
    __shared__ DensePlan pl;   // identical in every thread; kept in LDS so it is indexed without scratch
    int64_t total = 0;
    for (int o = 0; o < kDenseKinds; ++o) {
        const int k = kDenseOrder[o];
        const int32_t n_l = ctl->n_front[dense_bin_of_kind(k, false)], n_h = ctl->n_front[dense_bin_of_kind(k, true)];
        // light items span gl tiles, heavy ones gh = gl / kHeavySplit; a
        // light item makes np passes of gl tiles.  np shrinks first (to
        // about two items per resident workgroup), then gl (to about one):
        // every item pays its staging, scans and barriers and one atomic on
        // the shared item counter, so small rounds gain from fewer, larger
        // items
        const auto n_items_of = [&](int32_t l, int32_t np) {
            const int32_t h = max(1, l / kHeavySplit);
            const int64_t span = (int64_t)l * np;
            return (int64_t)n_l * ((ntk + span - 1) / span) + (int64_t)n_h * ((ntk + h - 1) / h);
        };
        int32_t gl = (int32_t)min<int64_t>(g_max.k[k], ntk);
        int32_t np = kDensePasses;
        while (np > 1 && n_items_of(gl, np) < 2 * slots) np >>= 1;
        while (np == 1 && gl > 1 && n_items_of(gl, 1) < slots) gl = (gl + 1) / 2;
        const int32_t gh = max(1, gl / kHeavySplit);
        const int32_t ngl = (int32_t)((ntk + (int64_t)gl * np - 1) / ((int64_t)gl * np));
        const int32_t ngh = (ntk + gh - 1) / gh;
        const int64_t nh_items = (int64_t)n_h * ngh;
        total += nh_items + (int64_t)n_l * ngl;
        if (threadIdx.x == 0) {
            pl.np[o] = np;
            pl.gl[o] = gl;
            pl.gh[o] = gh;
            pl.ngl[o] = ngl;
            pl.ngh[o] = ngh;
            pl.n_heavy[o] = nh_items;
            pl.end[o] = total;
        }
    }
    if (total == 0) return;
    extern __shared__ __align__(16) uint32_t dyn[];
    uint32_t* cnt = dyn;
    Stage<NT>& S = *reinterpret_cast<Stage<NT>*>(dyn + kDenseLdsBytes / 4);
    const int tid = threadIdx.x;
    {
        uint4* cnt4 = reinterpret_cast<uint4*>(cnt);
        for (int w = tid; w < kDenseLdsBytes / 16; w += NT) cnt4[w] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    const int32_t buf = ctl->front_buf;
    PeelCounters pc;
    for (;;) {
        const int64_t it = next_item(S, &ctl->head[dense_bin_of_kind(0, false)]);
        if (it >= total) break;
        int o = 0;
        while (it >= pl.end[o]) ++o;
        const int k = kDenseOrder[o];
        const int64_t r = it - (o ? pl.end[o - 1] : 0);
        int32_t u, t_begin, t_end, gpass;
        if (r < pl.n_heavy[o]) {
            u = fs.list[buf][dense_bin_of_kind(k, true)][r / pl.ngh[o]];
            gpass = pl.gh[o];
            t_begin = (int32_t)(r % pl.ngh[o]) * gpass;
            t_end = min(ntk, t_begin + gpass);
        } else {
            const int64_t q = r - pl.n_heavy[o];
            u = fs.list[buf][dense_bin_of_kind(k, false)][q / pl.ngl[o]];
            gpass = pl.gl[o];
            t_begin = (int32_t)(q % pl.ngl[o]) * gpass * pl.np[o];
            t_end = min(ntk, t_begin + gpass * pl.np[o]);
        }
        switch (k) {
            case 4: dense_item<32>(g, tb, tk, ntt, u, t_begin, t_end, gpass, cnt, S, ap, pc); break;
            case 3: dense_item<16>(g, tb, tk, ntt, u, t_begin, t_end, gpass, cnt, S, ap, pc); break;
            case 2: dense_item<8>(g, tb, tk, ntt, u, t_begin, t_end, gpass, cnt, S, ap, pc); break;
            case 1: dense_item<4>(g, tb, tk, ntt, u, t_begin, t_end, gpass, cnt, S, ap, pc); break;
            default: dense_item<2>(g, tb, tk, ntt, u, t_begin, t_end, gpass, cnt, S, ap, pc); break;
        }
    }
    pc.flush(ctl, true);
}

size_t dense_lds_bytes() { return (size_t)kDenseLdsBytes + sizeof(Stage<kDenseThreads>); }

void launch_dense(const DevGraph& g, PeelBuffers& pb, const FrontSet& fs, CdApply ap, Ctl* ctl, hipStream_t s) {
    int dev = 0, cus = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    TIP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ItemKeys g_max;
    for (int k = 0; k < kDenseKinds; ++k) g_max.k[k] = dense_item_tiles(2 << k, pb.tk, pb.ntt);
    const size_t lds = dense_lds_bytes();
    int occ = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_peel_dense, kDenseThreads, lds));
    const int64_t slots = (int64_t)cus * std::max(1, occ);
    k_peel_dense<<<(unsigned)slots, kDenseThreads, lds, s>>>(g, pb.tb, pb.tk, pb.ntt, fs, g_max, slots, ap, ctl);
    TIP_HIP_TRY(hipGetLastError());
}

// HUC (Section 4.1): the round about to run re-counts the live supports
// instead of peeling when the peel work of its activeSet (its wedge proxy,
// added to the range by the frontier scan) exceeds huc_pct percent of the
// re-count work, estimated as the counting wedges scaled by the share of
// side A still live at the range start.  Either way the supports after the
// round are the same.
__device__ inline void huc_decide(Ctl* ctl) {
    unsigned long long w = 0;
    for (int i = 0; i < kSpread; ++i) w += ctl->spread[i][kScWRange];
    const unsigned long long peel = w - ctl->huc_w_prev;
    ctl->huc_w_prev = w;
    const double rcnt = (double)ctl->wedges_count * (double)ctl->range_n_live / (double)max(ctl->huc_n_a, 1);
    ctl->huc_now = (ctl->huc_pct > 0 && peel > 0 && (double)peel * 100.0 > (double)ctl->huc_pct * rcnt) ? 1 : 0;
    ctl->huc_rounds += (unsigned long long)ctl->huc_now;
}

__global__ void k_huc_decide(Ctl* ctl) { huc_decide(ctl); }

__global__ void k_set_huc(Ctl* ctl, long long pct, int32_t n_a) {
    ctl->huc_pct = pct;
    ctl->huc_n_a = n_a;
    ctl->huc_now = 0;
}

__global__ void k_ctl_swap_front(Ctl* ctl) {
    int32_t any = 0;
    for (int b = 0; b < kBins; ++b) {
        any |= ctl->n_front[b];
        ctl->n_front[b] = ctl->n_next[b];
        ctl->n_next[b] = 0;
        ctl->head[b] = 0;
    }
    if (any) {
        ++ctl->rounds_done;
        ctl->front_buf ^= 1;
    }
    if (ctl->huc_pct > 0) huc_decide(ctl);
}

__global__ void k_assign_live(const int32_t* __restrict__ live, int32_t n_live, int32_t* state, int32_t label) {
    GRID_STRIDE(j, (int64_t)n_live) state[live[j]] = label;
}

// ---------------------------------------------------------------------------
// List compaction (DGM): vertices that are no longer live are removed from
// the lists the coarse-grained update traverses.  c(u, w) for live w is
// unchanged, so results are too; only dead entries stop being read.
// ---------------------------------------------------------------------------

__global__ void k_dgm_flags(const int32_t* __restrict__ adj, int64_t n, const int32_t* __restrict__ state,
                            int64_t* flag) {
    GRID_STRIDE(q, n) flag[q] = state[adj[q]] == kLive ? 1 : 0;
}

__global__ void k_dgm_scatter(const int32_t* __restrict__ adj, const int32_t* __restrict__ row, int64_t n,
                              const int64_t* __restrict__ flag, const int64_t* __restrict__ pos, int32_t* nadj,
                              int32_t* nrow) {
    GRID_STRIDE(q, n) {
        if (flag[q]) {
            nadj[pos[q]] = adj[q];
            nrow[pos[q]] = row[q];
        }
    }
}

// New offsets; the new entry count goes to ctl->cd_m and the dead-entry
// counter restarts.
__global__ void k_dgm_offsets(const int64_t* __restrict__ off, int32_t n_b, int64_t n, const int64_t* __restrict__ flag,
                              const int64_t* __restrict__ pos, int64_t* noff, Ctl* ctl) {
    const int64_t total = n > 0 ? pos[n - 1] + flag[n - 1] : 0;
    GRID_STRIDE(v, (int64_t)n_b + 1) {
        const int64_t o = off[v];
        noff[v] = o < n ? pos[o] : total;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->cd_m = total;
        for (int i = 0; i < kSpread; ++i) ctl->spread[i][kScDeadEdges] = 0;
    }
}

// Tile bounds of the compacted lists without searching: entry q of N_v is
// the first entry >= t * tk for every tile t after the previous entry's
// tile, up to its own.
__global__ void k_dgm_tiles(const int64_t* __restrict__ off, const int32_t* __restrict__ adj,
                            const int32_t* __restrict__ row, const long long* n_p, int32_t tk, int32_t ntt,
                            int32_t* tb) {
    const int64_t n = *n_p;
    GRID_STRIDE(q, n) {
        const int32_t v = row[q];
        const int64_t o = off[v];
        const int32_t t = adj[q] / tk;
        const int32_t tp = q == o ? -1 : adj[q - 1] / tk;
        int32_t* r = tb + (int64_t)v * (ntt + 1);
        for (int32_t x = tp + 1; x <= t; ++x) r[x] = (int32_t)(q - o);
    }
}

// Tiles after a list's last entry (every tile of an empty list) point to its end.
__global__ void k_dgm_tiles_tail(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t n_b,
                                 int32_t tk, int32_t ntt, int32_t* tb) {
    const int64_t tot = (int64_t)n_b * (ntt + 1);
    GRID_STRIDE(i, tot) {
        const int64_t v = i / (ntt + 1);
        const int32_t t = (int32_t)(i % (ntt + 1));
        const int64_t lo = off[v], hi = off[v + 1];
        const int32_t tl = hi > lo ? adj[hi - 1] / tk : -1;
        if (t > tl) tb[i] = (int32_t)(hi - lo);
    }
}

// Wedges of each u over the current CD lists (u's own entry excluded): a
// wave-level segmented sum over the CSR positions (rows are contiguous), one
// atomic per row segment of a wave.  wlive must be zero.
__global__ void k_wlive(const int32_t* __restrict__ a_row, const int32_t* __restrict__ a_adj, int64_t m,
                        const int64_t* __restrict__ cd_off, int64_t* wlive) {
    const int lane = threadIdx.x & (kWave - 1);
    UNIFORM_STRIDE(base, m) {
        const int64_t p = base + threadIdx.x;
        int32_t u = -1;
        int64_t x = 0;
        if (p < m) {
            u = a_row[p];
            const int32_t v = a_adj[p];
            const int64_t l = cd_off[v + 1] - cd_off[v];
            x = l > 1 ? l - 1 : 0;
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t y = __shfl_up(x, d, kWave);
            const int32_t uy = __shfl_up(u, d, kWave);
            if (lane >= d && uy == u) x += y;
        }
        const int32_t un = __shfl_down(u, 1, kWave);
        if (u >= 0 && (lane == kWave - 1 || un != u) && x) atomic_add_i64(&wlive[u], x);
    }
}

__global__ void k_set_key_hi(Ctl* ctl, int32_t v) { ctl->key_hi = v; }

// Largest live rank + 1: every key the update can still touch is below it.
__global__ void k_key_hi(const int32_t* __restrict__ state, int32_t n_a, Ctl* ctl) {
    __shared__ int32_t bhi;
    if (threadIdx.x == 0) bhi = 0;
    __syncthreads();
    int32_t hi = 0;
    GRID_STRIDE(u, (int64_t)n_a)
        if (state[u] == kLive) hi = (int32_t)u + 1;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) hi = max(hi, __shfl_xor(hi, d, kWave));
    // one atomic per workgroup on the single address
    if ((threadIdx.x & (kWave - 1)) == 0 && hi) atomicMax(&bhi, hi);
    __syncthreads();
    if (threadIdx.x == 0 && bhi) atomicMax(&ctl->key_hi, bhi);
}

__global__ void k_set_cd_m(Ctl* ctl, long long m, int32_t n_a) {
    ctl->cd_m = m;
    for (int i = 0; i < kSpread; ++i) ctl->spread[i][kScDeadEdges] = 0;
    ctl->key_hi = n_a;
}

ItemKeys item_keys(const PeelBuffers& pb) {
    ItemKeys ik;
    for (int k = 0; k < kDenseKinds; ++k) ik.k[k] = (int64_t)dense_item_tiles(2 << k, pb.tk, pb.ntt) * pb.tk;
    return ik;
}

FrontSet front_set(PeelBuffers& pb) {
    FrontSet f;
    for (int i = 0; i < 2; ++i)
        for (int b = 0; b < kBins; ++b) f.list[i][b] = pb.front[i][b];
    return f;
}

}  // namespace

int peel_occupancy() {
    int a = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_peel_bitmap, kBmThreads, 0));
    return std::max(1, a);
}

void launch_peel_setup(const DevGraph& g, const int32_t* deg_b_rank, PeelBuffers& pb, const Tune& tune, Ctl* ctl,
                       hipStream_t s) {
    fill_i64(pb.wprox, 0, g.n_a, s);
    // the select histogram is cleared after every use, so it starts cleared
    fill_i64(pb.sel_hist, 0, kSelBins, s);
    if (g.m > 0) {
        k_wproxy<<<grid1(g.m), kT, 0, s>>>(g, deg_b_rank, pb.wprox);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (g.n_a > 0) {
        k_peel_bins<<<grid1(g.n_a), kT, 0, s>>>(g.a_off, pb.wprox, g.n_a, tune.dense_div, tune.bitmap_max,
                                                item_keys(pb), nullptr, pb.bin);
        TIP_HIP_TRY(hipGetLastError());
        TIP_HIP_TRY(hipMemcpyAsync(pb.wlive, pb.wprox, sizeof(int64_t) * g.n_a, hipMemcpyDeviceToDevice, s));
    }
    // the CD lists start as a copy of the CSC
    TIP_HIP_TRY(hipMemcpyAsync(pb.cd_off, g.b_off, sizeof(int64_t) * ((size_t)g.n_b + 1), hipMemcpyDeviceToDevice, s));
    if (g.m > 0) {
        TIP_HIP_TRY(hipMemcpyAsync(pb.cd_adj, g.b_adj, sizeof(int32_t) * g.m, hipMemcpyDeviceToDevice, s));
        TIP_HIP_TRY(hipMemcpyAsync(pb.cd_row, g.b_row, sizeof(int32_t) * g.m, hipMemcpyDeviceToDevice, s));
    }
    k_set_huc<<<1, 1, 0, s>>>(ctl, (long long)tune.huc_pct, g.n_a);
    TIP_HIP_TRY(hipGetLastError());
    k_set_cd_m<<<1, 1, 0, s>>>(ctl, (long long)g.m, g.n_a);
    TIP_HIP_TRY(hipGetLastError());
    const int64_t n_tb = (int64_t)g.n_b * (pb.ntt + 1);
    if (n_tb > 0) {
        k_tile_bounds<<<grid1(n_tb), kT, 0, s>>>(g.b_off, g.b_adj, g.n_b, pb.tk, pb.ntt, pb.tb);
        TIP_HIP_TRY(hipGetLastError());
    }
}

void launch_compact(const DevGraph& g, PeelBuffers& pb, const CompactScratch& cs, int64_t cd_m, const Tune& tune,
                    Ctl* ctl, hipStream_t s) {
    if (cd_m <= 0) return;
    k_dgm_flags<<<grid1(cd_m), kT, 0, s>>>(pb.cd_adj, cd_m, pb.state, cs.flag);
    TIP_HIP_TRY(hipGetLastError());
    scan_exclusive_i64(cs.flag, cs.pos, cd_m, cs.scan_tmp, s);
    k_dgm_scatter<<<grid1(cd_m), kT, 0, s>>>(pb.cd_adj, pb.cd_row, cd_m, cs.flag, cs.pos, cs.adj, cs.row);
    TIP_HIP_TRY(hipGetLastError());
    k_dgm_offsets<<<grid1((int64_t)g.n_b + 1), kT, 0, s>>>(pb.cd_off, g.n_b, cd_m, cs.flag, cs.pos, pb.cd_tmp_off,
                                                           ctl);
    TIP_HIP_TRY(hipGetLastError());
    // back to the fixed addresses the (possibly graph-captured) rounds read
    TIP_HIP_TRY(hipMemcpyAsync(pb.cd_adj, cs.adj, sizeof(int32_t) * cd_m, hipMemcpyDeviceToDevice, s));
    TIP_HIP_TRY(hipMemcpyAsync(pb.cd_row, cs.row, sizeof(int32_t) * cd_m, hipMemcpyDeviceToDevice, s));
    TIP_HIP_TRY(hipMemcpyAsync(pb.cd_off, pb.cd_tmp_off, sizeof(int64_t) * ((size_t)g.n_b + 1),
                               hipMemcpyDeviceToDevice, s));
    k_dgm_tiles<<<grid1(cd_m), kT, 0, s>>>(pb.cd_off, pb.cd_adj, pb.cd_row, &ctl->cd_m, pb.tk, pb.ntt, pb.tb);
    TIP_HIP_TRY(hipGetLastError());
    const int64_t n_tb = (int64_t)g.n_b * (pb.ntt + 1);
    if (n_tb > 0) {
        k_dgm_tiles_tail<<<grid1(n_tb), kT, 0, s>>>(pb.cd_off, pb.cd_adj, g.n_b, pb.tk, pb.ntt, pb.tb);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (g.n_a > 0) {
        fill_i64(pb.wlive, 0, g.n_a, s);
        k_wlive<<<grid1(g.m, 8192), kT, 0, s>>>(g.a_row, g.a_adj, g.m, pb.cd_off, pb.wlive);
        TIP_HIP_TRY(hipGetLastError());
        k_set_key_hi<<<1, 1, 0, s>>>(ctl, 0);
        TIP_HIP_TRY(hipGetLastError());
        k_key_hi<<<grid1(g.n_a, 512), kT, 0, s>>>(pb.state, g.n_a, ctl);
        TIP_HIP_TRY(hipGetLastError());
        k_peel_bins<<<grid1(g.n_a), kT, 0, s>>>(g.a_off, pb.wlive, g.n_a, tune.dense_div, tune.bitmap_max,
                                                item_keys(pb), ctl, pb.bin);
        TIP_HIP_TRY(hipGetLastError());
    }
}

void launch_range_start(PeelBuffers& pb, int cur_live, int32_t n_live, Ctl* ctl, hipStream_t s) {
    k_ctl_begin_range<<<1, 1, 0, s>>>(ctl);
    TIP_HIP_TRY(hipGetLastError());
    if (n_live <= 0) return;
    k_range_start<<<scan_grid(n_live), kScanThreads, 0, s>>>(pb.live[cur_live], n_live, pb.live[1 - cur_live], pb.state,
                                                      pb.supp, pb.init, pb.wprox, ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_select(PeelBuffers& pb, int cur_live, int32_t n_live, uint64_t max_supp, int64_t tgt, Ctl* ctl,
                   hipStream_t s) {
    k_ctl_select_init<<<1, 1, 0, s>>>(ctl, (long long)tgt);
    TIP_HIP_TRY(hipGetLastError());
    const int bits = bits_for(max_supp);
    const int passes = (bits + kSelBits - 1) / kSelBits;
    for (int p = passes - 1; p >= 0; --p) {
        const int shift = kSelBits * p;
        k_select_hist<<<grid1(n_live, 256), kT, 0, s>>>(pb.live[cur_live], n_live, pb.supp, pb.wprox, shift, ctl,
                                                          pb.sel_hist);
        TIP_HIP_TRY(hipGetLastError());
        k_select_pick<<<1, kT, 0, s>>>(shift, ctl, pb.sel_hist);
        TIP_HIP_TRY(hipGetLastError());
    }
}

void launch_range_begin(const DevGraph& g, PeelBuffers& pb, int cur_live, int32_t n_live, int64_t hi,
                        uint64_t max_supp, int32_t label, Ctl* ctl, hipStream_t s, bool huc) {
    k_set_range<<<1, 1, 0, s>>>(ctl, (long long)hi, (long long)max_supp, label, cur_live, n_live);
    TIP_HIP_TRY(hipGetLastError());
    if (n_live <= 0) return;
    k_frontier_scan<<<grid1(n_live, 1024), kT, 0, s>>>(front_set(pb), pb.live[0], pb.live[1], pb.supp, pb.state,
                                                        pb.wprox, pb.bin, g.a_off, 0, ctl);
    TIP_HIP_TRY(hipGetLastError());
    if (huc) {
        k_huc_decide<<<1, 1, 0, s>>>(ctl);
        TIP_HIP_TRY(hipGetLastError());
    }
}

// Resident workgroups of the bitmap-path kernel on the current device.
int bitmap_grid() {
    int dev = 0, cus = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    TIP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(1, cus) * peel_occupancy();
}

void launch_round(const DevGraph& g, PeelBuffers& pb, Ctl* ctl, const SpillArena& spill, int big_grid,
                  hipStream_t s, hipEvent_t* ev_big, const int32_t* n_cur, CountBuffers* cb) {
    const CdApply ap{pb.supp};
    const FrontSet fs = front_set(pb);
    if (g.n_a <= 0) return;
    // the update traverses the CD copy of the lists N_v
    DevGraph gc = g;
    gc.b_off = pb.cd_off;
    gc.b_adj = pb.cd_adj;
    // grids are fixed; every kernel reads its work from the control block and
    // returns at once when it has none.  With the frontier sizes known on the
    // host (n_cur), kernels without work are not launched at all.
    const auto has = [&](int b) { return !n_cur || n_cur[b] > 0; };
    // HUC: a round the control block marks re-counts (the update kernels
    // below then return at once); uses the original lists and their cuts
    if (cb) launch_recount(g, *cb, pb.state, ctl, spill, big_grid, s);
    if (has(kBinWave)) {
        k_peel_wave<<<1024, kSmallThreads, 0, s>>>(gc, fs, pb.wlive, ap, ctl);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (has(kBinBitmap)) {
        // workgroups the spill arena can hold at the bitmap path's spacing
        const int64_t gap = std::min<int64_t>(kBmTile, spill.stride);
        const int64_t fit = (int64_t)spill.slots * (spill.stride / std::max<int64_t>(gap, 1));
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(bitmap_grid(), fit));
        k_peel_bitmap<<<grid, kBmThreads, 0, s>>>(gc, pb.tb, pb.tk, pb.ntt, fs, ap, spill, ctl);
        TIP_HIP_TRY(hipGetLastError());
    }
    bool any_dense = false;
    for (int b = dense_bin(2, false); b < kBins; ++b) any_dense = any_dense || has(b);
    if (any_dense) {
        if (ev_big) TIP_HIP_TRY(hipEventRecord(ev_big[0], s));
        launch_dense(gc, pb, fs, ap, ctl, s);
        if (ev_big) TIP_HIP_TRY(hipEventRecord(ev_big[1], s));
    }
    k_frontier_scan<<<grid1(g.n_a, 1024), kT, 0, s>>>(fs, pb.live[0], pb.live[1], pb.supp, pb.state, pb.wprox,
                                                       pb.bin, g.a_off, 1, ctl);
    TIP_HIP_TRY(hipGetLastError());
    k_ctl_swap_front<<<1, 1, 0, s>>>(ctl);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_assign_live(PeelBuffers& pb, int cur_live, int32_t n_live, int32_t label, hipStream_t s) {
    if (n_live <= 0) return;
    k_assign_live<<<grid1(n_live), kT, 0, s>>>(pb.live[cur_live], n_live, pb.state, label);
    TIP_HIP_TRY(hipGetLastError());
}

}  // namespace tip
