// Fine-grained decomposition (Alg. 4) and output scatter.
#include "kern_util.h"

#include <cstdlib>
#include <mutex>

namespace tip {
namespace {
// ===========================================================================
// Fine-grained decomposition (Alg. 4)
// ===========================================================================

// Sort keys of the vertices by subset and the subsets' sizes.  With lds_hist
// the sizes are counted in LDS per workgroup (S bins) and added to HBM once
// per workgroup and subset: a million atomics on a few hundred addresses
// would queue up at those addresses.
__global__ void k_fd_vertex_keys(const int32_t* __restrict__ state, int32_t n_a, int32_t S, uint64_t* keys,
                                 int32_t* vals, int64_t* sub_cnt, int lds_hist) {
    extern __shared__ int32_t hist_s[];  // [S] when lds_hist
    if (lds_hist) {
        for (int32_t i = threadIdx.x; i < S; i += blockDim.x) hist_s[i] = 0;
        __syncthreads();
    }
    GRID_STRIDE(u, (int64_t)n_a) {
        const int32_t s = state[u];
        keys[u] = (uint64_t)s;
        vals[u] = (int32_t)u;
        if (lds_hist) atomicAdd(&hist_s[s], 1);
        else atomic_add_i64(&sub_cnt[s], 1);
    }
    if (lds_hist) {
        __syncthreads();
        for (int32_t i = threadIdx.x; i < S; i += blockDim.x)
            if (hist_s[i]) atomic_add_i64(&sub_cnt[i], hist_s[i]);
    }
}

__global__ void k_fd_positions(const int32_t* __restrict__ fd_vert, int32_t n_a, int32_t* fd_pos) {
    GRID_STRIDE(p, (int64_t)n_a) fd_pos[fd_vert[p]] = (int32_t)p;
}

// Partitioned CSC: key (row, subset of the entry), value = the entry's CSC
// position (replaced after the sort by the entry's index inside its subset).
// The stable sort keeps each (row, subset) run ascending.
__global__ void k_fd_csc_keys(DevGraph g, const int32_t* __restrict__ state, int32_t S, uint64_t* keys,
                              int32_t* vals) {
    GRID_STRIDE(q, g.m) {
        keys[q] = (uint64_t)g.b_row[q] * (uint64_t)S + (uint64_t)state[g.b_adj[q]];
        vals[q] = (int32_t)q;
    }
}

// Entry q of the sorted partitioned CSC starts a (row, subset) run.
__device__ inline bool fd_run_start(const uint64_t* __restrict__ pkeys, int64_t q) {
    return q == 0 || pkeys[q] != pkeys[q - 1];
}

// The run of every sorted entry of the partitioned CSC: pos = exclusive scan
// of the run-start flags, so entry i lies in run pos[i] + start(i) - 1;
// run_lo[r] = the first entry of run r.
__global__ void k_fd_run_lo(const uint64_t* __restrict__ pkeys, int64_t m, const int64_t* __restrict__ pos,
                            int64_t* run_lo) {
    GRID_STRIDE(i, m) if (fd_run_start(pkeys, i)) run_lo[pos[i]] = i;
}

// Every sorted entry i of the partitioned CSC is an edge (w, v) with w in
// subset s: the CSR edge (w, v) gets the run [lo, hi) of N_v inside s (the
// edges of the induced subgraph G_i seen from v, Alg. 4), and the entry's
// value becomes w's index inside s.
__global__ void k_fd_run_scatter(DevGraph g, const int32_t* __restrict__ state, const uint64_t* __restrict__ pkeys,
                                 const int64_t* __restrict__ pos, const int64_t* __restrict__ run_lo,
                                 const int32_t* __restrict__ fd_pos, const int64_t* __restrict__ sub_off,
                                 int32_t* pcsc, int64_t* fd_beg, int32_t* fd_len) {
    const int64_t m = g.m;
    const int64_t n_runs = pos[m - 1] + (fd_run_start(pkeys, m - 1) ? 1 : 0);
    GRID_STRIDE(i, m) {
        const int64_t r = pos[i] + (fd_run_start(pkeys, i) ? 1 : 0) - 1;
        const int64_t lo = run_lo[r];
        const int64_t hi = r + 1 < n_runs ? run_lo[r + 1] : m;
        const int32_t q = pcsc[i];  // the entry's CSC position
        const int32_t w = g.b_adj[q];
        const int32_t s = state[w];
        const int64_t p = g.a_off[w] + g.b_rev[q];
        fd_beg[p] = lo;
        fd_len[p] = (int32_t)(hi - lo);
        pcsc[i] = (int32_t)(fd_pos[w] - sub_off[s]);
    }
}

// For every CSR edge (u, v) with its run in u's subset: the induced wedges
// per subset (task_w) and per vertex (fd_w).  Subset sums gather in LDS when
// there are few subsets (lds_tw); per-vertex sums are segmented wave sums
// over the CSR rows.  Wave-uniform grid-stride loop.
__global__ void k_fd_slices(DevGraph g, const int32_t* __restrict__ state, int32_t S,
                            const int32_t* __restrict__ fd_pos, const int32_t* __restrict__ fd_len,
                            int64_t* task_w, int64_t* fd_w, int lds_tw) {
    extern __shared__ unsigned long long tw[];  // [S] when lds_tw
    const int lane = threadIdx.x & (kWave - 1);
    if (lds_tw) {
        for (int32_t i = threadIdx.x; i < S; i += blockDim.x) tw[i] = 0;
        __syncthreads();
    }
    UNIFORM_STRIDE(base, g.m) {
        const int64_t p = base + threadIdx.x;
        int32_t u = -1;
        int64_t x = 0;
        if (p < g.m) {
            u = g.a_row[p];
            const int32_t s = state[u];
            const int32_t len = fd_len[p];
            x = len > 1 ? len - 1 : 0;
            if (x) {
                if (lds_tw) atomicAdd(&tw[s], (unsigned long long)x);
                else atomic_add_i64(&task_w[s], x);
            }
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t y = __shfl_up(x, d, kWave);
            const int32_t uy = __shfl_up(u, d, kWave);
            if (lane >= d && uy == u) x += y;
        }
        const int32_t un = __shfl_down(u, 1, kWave);
        if (u >= 0 && (lane == kWave - 1 || un != u) && x) atomic_add_i64(&fd_w[fd_pos[u]], x);
    }
    if (lds_tw) {
        __syncthreads();
        for (int32_t i = threadIdx.x; i < S; i += blockDim.x)
            if (tw[i]) atomic_add_i64(&task_w[i], (int64_t)tw[i]);
    }
}

// Runs of the partitioned CSC (one per (row, subset) key): their start
// flags (which also give every CSR edge its run, above) and, for compaction
// in the fine-grained step (Section 4.2), every run's start position and
// subset, its length at the start, and the run count of every subset.
__global__ void k_fd_run_flags(const uint64_t* __restrict__ pkeys, int64_t m, int64_t* flag) {
    GRID_STRIDE(q, m) flag[q] = fd_run_start(pkeys, q) ? 1 : 0;
}

// pos: exclusive scan of the flags.  Runs in position order go to
// rkey/rval [0, R) (key: subset, value: start), the rest of rkey is the
// sentinel S so that a sort by subset leaves them last.
__global__ void k_fd_run_compact(const uint64_t* __restrict__ pkeys, int64_t m, int32_t S,
                                 const int64_t* __restrict__ pos, uint64_t* rkey, int32_t* rval, int64_t* sub_rcnt) {
    GRID_STRIDE(q, m) {
        rkey[q] = (uint64_t)S;
        if (fd_run_start(pkeys, q)) {
            const int32_t sub = (int32_t)(pkeys[q] % (uint64_t)S);
            const int64_t j = pos[q];
            rval[j] = (int32_t)q;
            atomic_add_i64(&sub_rcnt[sub], 1);
        }
    }
}

// Length of every run (next start - start) and the keys of the runs, once
// every run's start is in place.
__global__ void k_fd_run_len(const uint64_t* __restrict__ pkeys, int64_t m, int32_t S,
                             const int64_t* __restrict__ pos, const int32_t* __restrict__ rval, uint64_t* rkey,
                             int32_t* rlen_at) {
    const int64_t R = m > 0 ? pos[m - 1] + (fd_run_start(pkeys, m - 1) ? 1 : 0) : 0;
    GRID_STRIDE(j, R) {
        const int32_t q = rval[j];
        const int64_t next = j + 1 < R ? rval[j + 1] : m;
        rlen_at[q] = (int32_t)(next - q);
        rkey[j] = pkeys[q] % (uint64_t)S;
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

__global__ void k_fd_reset_board(FdBoard* b) {
    int32_t* w = reinterpret_cast<int32_t*>(b);
    for (int i = threadIdx.x; i < (int)(sizeof(FdBoard) / 4); i += blockDim.x) w[i] = 0;
}

// LDS of the fine-grained kernel.  The per-wave hash tables (light peeled
// vertices) and the bitmap + repeat table (heavy ones) are used in separate
// phases of a level and share storage; both are all zero between uses.
constexpr int kFdHeavyPre = 512;  // heavy vertices of a level whose rows are loaded together

struct FdLds {
    union Shared {
        struct {
            uint32_t bm[kFdBits / 32];
            unsigned long long rep[kFdRep];
        } big;
        unsigned long long wtab[kFdThreads / kWave][kFdWaveSlots];
    } u;
    int64_t sbeg[kGroup];
    int64_t pre[kGroup + 1];
    int64_t wsbeg[kFdThreads / kWave][kWave];
    int64_t wpre[kFdThreads / kWave][kWave + 1];
    int64_t red[kFdThreads / kWave];
    int32_t spill_n;
    int32_t flag;
    int32_t wave_head;   // next per-wave update of the level
    int32_t hn;          // entries of a claimed help-board chunk of pair rows
    int32_t lcnt[4];     // list lengths of a level's partition: kept, per-wave, heavy
    unsigned long long hw;  // induced wedges of a level's heavy vertices
    unsigned long long pw_all, pw_upd;  // induced wedges of a step's peeled vertices (all; with support left)
    unsigned long long racc[kFdThreads / kWave];  // HUC re-count sums, per wave
    int64_t hx_off[kFdHeavyPre];  // row offset and degree of a level's heavy vertices
    int32_t hx_deg[kFdHeavyPre];
    int32_t pn[kFdThreads / kWave + 1];  // pair-row build: entries of the row each wave (last: the workgroup) writes
};

// Next entry of the level's per-wave update list for the calling wavefront.
__device__ inline int32_t fd_next_wave_item(FdLds& L) {
    int32_t q = 0;
    if ((threadIdx.x & (kWave - 1)) == 0) q = atomicAdd(&L.wave_head, 1);
    return __shfl(q, 0, kWave);
}

// Block exclusive scan of 64-bit values (all threads take part); returns the
// thread's offset and the total.
template <int NT>
__device__ inline int64_t fd_scan_i64(FdLds& L, int64_t x, int64_t& total) {
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
    total = tot;
    __syncthreads();
    return off + inc - x;
}

template <int NT>
__device__ inline int64_t fd_min(FdLds& L, int64_t x) {
    x = wave_min_i64(x);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) L.red[wid] = x;
    __syncthreads();
    int64_t s = L.red[0];
#pragma unroll
    for (int w = 1; w < NT / kWave; ++w) s = L.red[w] < s ? L.red[w] : s;
    __syncthreads();
    return s;
}

__device__ inline void fd_wave_insert(unsigned long long* tab, uint32_t k, uint32_t mask) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & mask;
#pragma unroll 1
    for (;;) {
        unsigned long long* slot = &tab[h];
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
        h = (h + 1) & mask;
    }
}

__device__ inline void fd_rep_insert(FdLds& L, const Spill& sp, uint32_t k) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    const uint32_t h = hash32(k) & (kFdRep - 1);
#pragma unroll 1
    for (int p = 0; p < kRepProbe; ++p) {
        unsigned long long* slot = &L.u.big.rep[(h + p) & (kFdRep - 1)];
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

// Where the state of the subset being peeled lives.  Subsets of at most
// kFdLdsVerts vertices keep supports, liveness, heavy flags and the vertex
// lists in LDS for the whole task (the supports take LDS atomics, and the
// next level's minimum is tracked on the fly); larger ones keep them in HBM.
//
// sup[x] of a peeled vertex holds its tip number (the level it was peeled
// at; no update reads a peeled vertex's support), written out at the end of
// the task.  A level's peeled vertices are listed in pl: per-wave ones from
// the front, heavy ones after them.
struct FdSmall {
    int64_t sup[kFdLdsVerts];
    uint16_t lc[kFdLdsVerts], ln[kFdLdsVerts], pl[kFdLdsVerts];
    uint8_t flag[kFdLdsVerts];     // bit 0: alive, bit 1: heavy
    long long upd_min;             // least support left by this level's decrements
    int64_t red_min[kFdThreads / kWave];
};
constexpr uint8_t kFdAlive = 1, kFdHeavy = 2;
constexpr int kFdPack = 21;  // packed per-level counts: per-wave | heavy << 21 | kept << 42
static_assert(sizeof(FdLds::Shared) >= (size_t)kFdWaveKeys * (kFdThreads / kWave), "per-wave counters fit the union");

// Decrements of the subset's dead vertices are applied too: their support is
// never read again (each level reads the live list only), and skipping the
// liveness load shortens every update's chain of memory round trips.
//
// With `cx` set (a step that peels few vertices), every decrement returns the
// old support, and a vertex whose support crosses from above the level to
// at or below it is appended to cx: exactly the live vertices the next step
// at the same level must peel (a support crosses once; vertices already at
// or below the level, live or dead, never cross).
struct FdHbmState {
    int64_t* sup;
    int32_t* alive;
    const int32_t* vert;
    int32_t* cx = nullptr;    // crossing list, or nullptr
    int32_t* cxn = nullptr;   // its length (LDS)
    int64_t level = 0;
    __device__ inline bool live(int32_t) const { return true; }
    __device__ inline int32_t vtx(int32_t x) const { return vert[x]; }
    __device__ inline void dec(int32_t w, int64_t d) const {
        if (!cx) {
            atomic_add_i64(&sup[w], -d);
            return;
        }
        const int64_t old = atomic_add_i64_ret(&sup[w], -d);
        if (old > level && old - d <= level) cx[atomicAdd(cxn, 1)] = w;
    }
    static constexpr bool kMinLocal = false;
};

// HUC inside a subset (Section 4.1, last paragraph).  The support of a live
// vertex u of subset i is its support at the range start (which counts the
// butterflies with every vertex of this and later subsets) minus those it
// shares with the vertices of U_i peeled so far; a re-count walks u's wedges
// inside G_i and sums C(c(u, w), 2) over the peeled w.  As the "state" of
// the update routines: the keys they apply to are the peeled ones, and
// "decrementing" adds to the wave's (or workgroup's) accumulator.
struct FdRecountState {
    const int32_t* alive;
    const int32_t* vert;
    unsigned long long* acc;
    __device__ inline bool live(int32_t w) const { return (alive[w] & kFdAlive) == 0; }
    __device__ inline int32_t vtx(int32_t x) const { return vert[x]; }
    __device__ inline void dec(int32_t, int64_t d) const { atomicAdd(acc, (unsigned long long)d); }
};

struct FdLdsState {
    FdSmall* S;
    const int32_t* vert;  // the subset's vertices (HBM)
    __device__ inline bool live(int32_t w) const { return (S->flag[w] & kFdAlive) != 0; }
    __device__ inline int32_t vtx(int32_t x) const { return vert[x]; }
    __device__ inline void dec(int32_t w, int64_t d) const {
        const int64_t old = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&S->sup[w]),
                                               (unsigned long long)(-d));
        atomicMin(&S->upd_min, (long long)(old - d));
    }
    // the same, with the least support left folded in per wave by the caller
    static constexpr bool kMinLocal = true;
    __device__ inline int64_t dec_ret(int32_t w, int64_t d) const {
        return (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&S->sup[w]), (unsigned long long)(-d)) - d;
    }
    __device__ inline void fold_min(int64_t mn) const { atomicMin(&S->upd_min, (long long)mn); }
};

// The pair-row build as the "state" of the update routines: instead of
// decrementing w's support by C(c, 2), append (w, C(c, 2)) to the row of the
// vertex being counted; n is the row's LDS entry counter.
struct FdPairWriter {
    const int32_t* vert;
    int32_t* pw;
    int64_t* pb;
    int32_t* n;
    __device__ inline bool live(int32_t) const { return true; }
    __device__ inline int32_t vtx(int32_t x) const { return vert[x]; }
    __device__ inline void dec(int32_t w, int64_t d) const {
        const int32_t k = atomicAdd(n, 1);
        pw[k] = w;
        pb[k] = d;
    }
};

// Updates of a step from pair rows: the rows of nq peeled vertices, row q
// given by row(q, start, length).  Rows are cut into units of 64 entries;
// every wave takes units round-robin over all rows, four at a time, so that
// one long row spreads over the workgroup and short rows do not leave waves
// idle.  A unit's row is found by a ballot over the units' prefix sums of
// 64 rows at a time.  All threads call.
template <class St, class RowF>
__device__ inline void fd_pair_units(const FdBuffers& fb, int32_t nq, const RowF& row, const St& st,
                                     unsigned long long& pairs) {
    constexpr int NW = kFdThreads / kWave, R = 4;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int64_t mn = INT64_MAX;
    int32_t ub = 0;  // units of the rows before the current group of 64
    for (int32_t g0 = 0; g0 < nq; g0 += kWave) {
        const int gs = min(kWave, nq - g0);
        int64_t off = 0;
        int32_t len = 0;
        if (lane < gs) row(g0 + lane, off, len);
        const int32_t units = (len + kWave - 1) / kWave;
        const int32_t incl = wave_incl_scan_i32(units);
        const int32_t nu = __shfl(incl, kWave - 1, kWave);
        const int32_t pre = incl - units;
        // first unit of this group that falls to this wave
        const int32_t k_first = (int32_t)(((wid - ub) % NW + NW) % NW);
        for (int32_t k0 = k_first; k0 < nu; k0 += NW * R) {
            int32_t ws[R];
            int64_t bs[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int32_t k = k0 + r * NW;
                ws[r] = -1;
                bs[r] = 0;
                if (k < nu) {
                    const uint64_t le = __ballot(pre <= k);
                    const int j = 63 - __clzll((long long)le);
                    const int64_t oj = __shfl(off, j, kWave);
                    const int32_t lj = __shfl(len, j, kWave), pj = __shfl(pre, j, kWave);
                    const int32_t i = (k - pj) * kWave + lane;
                    if (i < lj) {
                        ws[r] = fb.prow_w[oj + i];
                        bs[r] = fb.prow_b[oj + i];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (ws[r] >= 0 && st.live(ws[r])) {
                    if constexpr (St::kMinLocal) {
                        const int64_t v = st.dec_ret(ws[r], bs[r]);
                        mn = v < mn ? v : mn;
                    } else {
                        st.dec(ws[r], bs[r]);
                    }
                    ++pairs;
                }
            }
        }
        ub += nu;
    }
    if constexpr (St::kMinLocal) {
        mn = wave_min_i64(mn);
        if (lane == 0 && mn != INT64_MAX) st.fold_min(mn);
    }
}

// Update of one light peeled vertex x (few wedges inside the subset) by one
// wavefront with its private hash table of `slots` entries.
template <class St, class Lds>
__device__ inline void fd_update_light(const DevGraph& g, const FdBuffers& fb, Lds& L, unsigned long long* tab,
                                       int32_t x, uint32_t slots, const St& st, unsigned long long& wedges,
                                       unsigned long long& pairs) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t mask = slots - 1;
    const int32_t ux = st.vtx(x);
    const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
    for (int64_t g0 = 0; g0 < d; g0 += kWave) {
        const int gs = (int)min<int64_t>(kWave, d - g0);
        int64_t len = 0;
        if (lane < gs) {
            const int64_t e = e0 + g0 + lane;
            L.wsbeg[wid][lane] = fb.fd_beg[e];
            len = fb.fd_len[e];
        }
        const int64_t inc = wave_incl_scan_i64<kWave>(len);
        L.wpre[wid][lane] = inc - len;
        const int64_t tot = __shfl(inc, kWave - 1, kWave);
        if (lane == 0) L.wpre[wid][kWave] = tot;
        wave_sync();
        int lo = 0;
        for (int64_t i0 = lane; i0 < tot; i0 += 4 * kWave) {
            int32_t ws[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t i = i0 + k * kWave;
                ws[k] = x;
                if (i < tot) {
                    while (lo + 1 < gs && L.wpre[wid][lo + 1] <= i) ++lo;
                    ws[k] = fb.pcsc[L.wsbeg[wid][lo] + (i - L.wpre[wid][lo])];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (ws[k] != x) fd_wave_insert(tab, (uint32_t)ws[k], mask);
        }
        if (lane == 0) wedges += (unsigned long long)(tot - gs);
        wave_sync();
    }
    for (uint32_t sl = lane; sl < slots; sl += kWave) {
        const unsigned long long v = tab[sl];
        if (v) {
            tab[sl] = 0;
            const int64_t c = (int64_t)(v & 0xffffffffull);
            const int32_t w = (int32_t)((v >> 32) - 1);
            if (c >= 2 && st.live(w)) {
                st.dec(w, choose2(c));
                ++pairs;
            }
        }
    }
    wave_sync();
}

// Counters of value >= 2 in a word of four 8-bit counters: the top bit of
// every such byte is set in the result.
__device__ inline uint32_t ge2_bytes(uint32_t v) {
    const uint32_t t = v & 0xfefefefeu;
    return (((t & 0x7f7f7f7fu) + 0x7f7f7f7fu) | t) & 0x80808080u;
}

// Update of one peeled vertex x of degree at most 255 in a subset of at most
// kFdWaveKeys vertices by one wavefront: one 8-bit LDS counter per vertex of
// the subset (c(x, w) <= d_x fits), scanned and cleared afterwards.
template <class St, class Lds>
__device__ inline void fd_update_wave_dense(const DevGraph& g, const FdBuffers& fb, Lds& L, uint32_t* cnt,
                                            int32_t x, int32_t n_i, const St& st, unsigned long long& wedges,
                                            unsigned long long& pairs) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int32_t ux = st.vtx(x);
    const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
    for (int64_t g0 = 0; g0 < d; g0 += kWave) {
        const int gs = (int)min<int64_t>(kWave, d - g0);
        int64_t len = 0;
        if (lane < gs) {
            const int64_t e = e0 + g0 + lane;
            L.wsbeg[wid][lane] = fb.fd_beg[e];
            len = fb.fd_len[e];
        }
        const int64_t inc = wave_incl_scan_i64<kWave>(len);
        L.wpre[wid][lane] = inc - len;
        const int64_t tot = __shfl(inc, kWave - 1, kWave);
        if (lane == 0) L.wpre[wid][kWave] = tot;
        wave_sync();
        int lo = 0;
        for (int64_t i0 = lane; i0 < tot; i0 += 4 * kWave) {
            int32_t ws[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t i = i0 + k * kWave;
                ws[k] = x;
                if (i < tot) {
                    while (lo + 1 < gs && L.wpre[wid][lo + 1] <= i) ++lo;
                    ws[k] = fb.pcsc[L.wsbeg[wid][lo] + (i - L.wpre[wid][lo])];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (ws[k] != x) atomicAdd(&cnt[ws[k] >> 2], 1u << ((ws[k] & 3) * 8));
        }
        if (lane == 0) wedges += (unsigned long long)(tot - gs);
        wave_sync();
    }
    const int32_t nw = (n_i + 3) >> 2;
    for (int32_t i = lane; i < nw; i += kWave) {
        const uint32_t v = cnt[i];
        if (v) {
            cnt[i] = 0;
            uint32_t m = ge2_bytes(v);
            while (m) {
                const int f = (__ffs(m) - 1) >> 3;
                m &= m - 1;
                const int32_t w = i * 4 + f;
                if (st.live(w)) {
                    st.dec(w, choose2((int64_t)((v >> (f * 8)) & 0xffu)));
                    ++pairs;
                }
            }
        }
    }
    wave_sync();
}

// Update of one heavy peeled vertex x by the whole workgroup: one LDS bit
// per key of a kFdBits-key tile, repeats in the LDS table (spilling to HBM).
template <class St>
__device__ inline void fd_update_heavy(const DevGraph& g, const FdBuffers& fb, FdLds& L, const Spill& sp,
                                       int32_t x, int64_t e0, int64_t d, int32_t n_i, const St& st,
                                       unsigned long long& wedges, unsigned long long& pairs,
                                       unsigned long long& spills) {
    constexpr int NT = kFdThreads;
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const bool multi = n_i > kFdBits;
    for (int32_t klo = 0; klo < n_i; klo += kFdBits) {
        const int32_t khi = (int32_t)min<int64_t>(n_i, (int64_t)klo + kFdBits);
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
            // exclusive scan of run lengths into L.pre
            const int64_t x64 = tid < gs ? len : 0;
            const int64_t incl = wave_incl_scan_i64<NT>(x64);
            __syncthreads();
            if (lane == kWave - 1) L.red[wid] = incl;
            __syncthreads();
            int64_t off = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int64_t v = L.red[w];
                off += w < wid ? v : 0;
                tot += v;
            }
            if (tid < gs) L.pre[tid] = off + incl - x64;
            if (tid == 0) L.pre[gs] = tot;
            __syncthreads();
            for (int64_t i = tid; i < tot; i += NT) {
                int lo = 0, hi = gs;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (L.pre[mid] <= i) lo = mid;
                    else hi = mid;
                }
                const int32_t w = fb.pcsc[L.sbeg[lo] + (i - L.pre[lo])];
                if (w != x) {
                    const uint32_t k = (uint32_t)(w - klo);
                    const uint32_t bit = 1u << (k & 31);
                    if (atomicOr(&L.u.big.bm[k >> 5], bit) & bit) fd_rep_insert(L, sp, k);
                }
            }
            if (tid == 0) wedges += (unsigned long long)(tot - (self_in ? gs : 0));
            __syncthreads();
        }
        for (int sl = tid; sl < kFdRep; sl += NT) {
            const unsigned long long v = L.u.big.rep[sl];
            if (v) {
                const int32_t w = klo + (int32_t)((v >> 32) - 1);
                if (st.live(w)) {
                    st.dec(w, choose2(1 + (int64_t)(v & 0xffffffffull)));
                    ++pairs;
                }
            }
        }
        const int32_t nsp = L.spill_n;
        if (tid == 0) spills += (unsigned long long)nsp;
        for (int32_t i = tid; i < nsp; i += NT) {
            const int32_t k = sp.list[i];
            const int32_t w = klo + k;
            if (st.live(w)) {
                st.dec(w, choose2(1 + (int64_t)sp.dense[k]));
                ++pairs;
            }
            sp.dense[k] = 0;
        }
        __syncthreads();
        const int32_t words = (khi - klo + 31) >> 5;
        for (int w = tid; w < words; w += NT) L.u.big.bm[w] = 0;
        for (int sl = tid; sl < kFdRep; sl += NT) L.u.big.rep[sl] = 0;
        if (tid == 0) L.spill_n = 0;
        __syncthreads();
    }
}

// The heavy vertices of a level, updated one after another by the whole
// workgroup.  Their row offsets and degrees are loaded first, for up to
// kFdHeavyPre of them in parallel, so that each update starts from its
// neighbour runs instead of a chain of dependent loads.  All threads call,
// after a barrier.
template <class St, class T>
__device__ inline void fd_heavy_level(const DevGraph& g, const FdBuffers& fb, FdLds& L, const Spill& sp,
                                      const T* ph, int32_t n_heavy, int32_t n_i, const St& st,
                                      unsigned long long& wedges, unsigned long long& pairs,
                                      unsigned long long& spills) {
    for (int32_t q0 = 0; q0 < n_heavy; q0 += kFdHeavyPre) {
        const int32_t nq = min(kFdHeavyPre, n_heavy - q0);
        for (int32_t q = threadIdx.x; q < nq; q += kFdThreads) {
            const int32_t ux = st.vtx((int32_t)ph[q0 + q]);
            const int64_t a = g.a_off[ux];
            L.hx_off[q] = a;
            L.hx_deg[q] = (int32_t)(g.a_off[ux + 1] - a);
        }
        __syncthreads();
        for (int32_t q = 0; q < nq; ++q)
            fd_update_heavy(g, fb, L, sp, (int32_t)ph[q0 + q], L.hx_off[q], (int64_t)L.hx_deg[q], n_i, st, wedges,
                            pairs, spills);
        __syncthreads();
    }
}

// Heavy updates taken one at a time from a help-board slot until its
// published heavy list is exhausted; the whole workgroup does each (its LDS
// bitmap and repeat table, its own spill area).  Finished entries are
// counted in hdone after their decrements are visible device-wide.  All
// threads call.
template <class St>
__device__ inline void fd_heavy_take(const DevGraph& g, const FdBuffers& fb, FdLds& L, const Spill& sp,
                                     const int32_t* ph, int32_t n_i, FdHelpSlot* hs, const St& st,
                                     unsigned long long& wedges, unsigned long long& pairs,
                                     unsigned long long& spills) {
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long wv = atomicAdd(&hs->hword, 1ull);
            const uint32_t q = (uint32_t)wv, n = (uint32_t)(wv >> 32);
            L.flag = q < n ? (int32_t)q : -1;
        }
        __syncthreads();
        const int32_t q = L.flag;
        if (q < 0) break;
        __threadfence();
        const int32_t x = ph[q];
        const int32_t ux = st.vtx(x);
        const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
        fd_update_heavy(g, fb, L, sp, x, e0, d, n_i, st, wedges, pairs, spills);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&hs->hdone, 1);
    }
    __syncthreads();
}

// Per-wave updates taken from a help-board slot until its published list is
// exhausted: one atomic on the slot word hands out `chunk` entries;
// finished entries are counted in `done` after their decrements are visible
// device-wide.
template <class St>
__device__ inline void fd_help_slot(const DevGraph& g, const FdBuffers& fb, FdLds& L, unsigned long long* tab,
                                    uint32_t* wcnt, const int32_t* pl, const int64_t* fw, int32_t n_i,
                                    FdHelpSlot* hs, int32_t chunk, const St& st, unsigned long long& wedges,
                                    unsigned long long& pairs) {
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        unsigned long long wv = 0;
        if (lane == 0) wv = atomicAdd(&hs->word, (unsigned long long)chunk);
        wv = __shfl(wv, 0, kWave);
        const uint32_t q0 = (uint32_t)wv, nl = (uint32_t)(wv >> 32);
        if (q0 >= nl) break;
        const uint32_t q1 = min(nl, q0 + (uint32_t)chunk);
        __threadfence();
        for (uint32_t q = q0; q < q1; ++q) {
            const int32_t x = pl[q];
            if (n_i <= kFdWaveKeys) fd_update_wave_dense(g, fb, L, wcnt, x, n_i, st, wedges, pairs);
            else fd_update_light(g, fb, L, tab, x, min<uint32_t>(kFdWaveSlots, wave_slots(fw[x])), st, wedges, pairs);
        }
        __threadfence();
        if (lane == 0) atomicAdd(&hs->done, (int32_t)(q1 - q0));
    }
}

// Pair-row updates taken from a help-board slot, kFdPairHelpChunk peeled
// vertices at a time by the whole workgroup, until the published list is
// exhausted; finished entries are counted in `done` after their decrements
// are visible device-wide.  All threads call.
template <class St>
__device__ inline void fd_help_pairs(const FdBuffers& fb, FdLds& L, const int32_t* pl, int64_t P0, int64_t shift,
                                     FdHelpSlot* hs, const St& st, unsigned long long& pairs) {
    static_assert(kFdPairHelpChunk <= kFdHeavyPre, "a chunk's rows are staged in hx_off / hx_deg");
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long wv = atomicAdd(&hs->word, (unsigned long long)kFdPairHelpChunk);
            const uint32_t q0 = (uint32_t)wv, n = (uint32_t)(wv >> 32);
            L.flag = q0 < n ? (int32_t)q0 : -1;
            L.hn = q0 < n ? (int32_t)min<uint32_t>(kFdPairHelpChunk, n - q0) : 0;
        }
        __syncthreads();
        const int32_t q0 = L.flag, nq = L.hn;
        if (q0 < 0) break;
        __threadfence();
        for (int32_t q = threadIdx.x; q < nq; q += kFdThreads) {
            const int32_t x = pl[q0 + q];
            L.hx_off[q] = fb.prow_off[P0 + x] + shift;
            L.hx_deg[q] = fb.prow_n[P0 + x];
        }
        __syncthreads();
        const auto row = [&](int32_t q, int64_t& off, int32_t& len) {
            off = L.hx_off[q];
            len = L.hx_deg[q];
        };
        fd_pair_units(fb, nq, row, st, pairs);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&hs->done, nq);
    }
    __syncthreads();
}

// Which update a peeled vertex j of the subset takes.  In subsets of at most
// kFdWaveKeys vertices every vertex of degree <= 255 with at most
// kFdWaveDenseMax wedges inside the subset is updated by one wavefront with
// dense 8-bit counters; in larger subsets only those with at most kFdWaveMax
// wedges are (with a hash table).  The others are heavy: the whole workgroup
// updates them one at a time.
__device__ inline bool fd_heavy(const DevGraph& g, const FdBuffers& fb, int64_t P0, int32_t n_i, int32_t j) {
    const int64_t w = fb.fd_w[P0 + j];
    if (n_i <= kFdWaveKeys) {
        const int32_t v = fb.fd_vert[P0 + j];
        return g.a_off[v + 1] - g.a_off[v] > 255 || w > kFdWaveDenseMax;
    }
    return w > kFdWaveMax;
}

// Position in an LDS-counted list for the lanes of the calling wave with
// pred; one LDS atomic per wave.  Every lane of the wave must call.
__device__ inline int32_t fd_wave_slot(bool pred, int32_t* counter) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return 0;
    const int lane = threadIdx.x & (kWave - 1);
    const int leader = __ffsll((unsigned long long)m) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(m));
    base = __shfl(base, leader, kWave);
    return base + (int32_t)__popcll(m & lanemask_lt());
}

template <int NT>
__device__ inline int64_t fd_block_sum(FdLds& L, int64_t x) {
    x = wave_sum_i64(x);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) L.red[wid] = x;
    __syncthreads();
    int64_t s = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) s += L.red[w];
    __syncthreads();
    return s;
}

// HUC re-count of every live vertex of a subset kept in HBM: support = its
// support at the range start minus the butterflies shared with the peeled
// vertices of the subset.  Light vertices one per wave, heavy ones with the
// whole workgroup; rl and rh (the step's peel lists, unused by a re-count
// step) hold the two work lists.  All threads call, after a barrier.
__device__ inline void fd_recount(const DevGraph& g, const FdBuffers& fb, FdLds& L, const Spill& sp,
                                  const int32_t* lc, int32_t n_live, int32_t* rl, int32_t* rh,
                                  const int32_t* alive, const int32_t* vert, int64_t* sup, const int64_t* fw,
                                  const int64_t* __restrict__ init, int32_t n_i, bool wave_dense,
                                  unsigned long long* tab, uint32_t* wcnt, unsigned long long& wedges,
                                  unsigned long long& pairs, unsigned long long& spills) {
    constexpr int NT = kFdThreads;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    if (tid < 4) L.lcnt[tid] = 0;
    if (tid < NT / kWave) L.racc[tid] = 0;
    if (tid == 0) L.wave_head = 0;
    __syncthreads();
    // the live vertices (the list may still hold some that were peeled)
    for (int32_t b0 = 0; b0 < n_live; b0 += NT) {
        const int32_t j = b0 + tid;
        const int32_t x = j < n_live ? lc[j] : -1;
        const int32_t f = x >= 0 ? alive[x] : 0;
        const bool lv = (f & kFdAlive) != 0;
        const bool hv = lv && (f & kFdHeavy) != 0;
        const int32_t pw = fd_wave_slot(lv && !hv, &L.lcnt[1]);
        const int32_t pq = fd_wave_slot(hv, &L.lcnt[2]);
        if (lv && !hv) rl[pw] = x;
        if (hv) rh[pq] = x;
    }
    __syncthreads();
    const int32_t n_rl = L.lcnt[1], n_rh = L.lcnt[2];
    const FdRecountState rs{alive, vert, &L.racc[wid]};
    for (int32_t q = fd_next_wave_item(L); q < n_rl; q = fd_next_wave_item(L)) {
        const int32_t x = rl[q];
        if (wave_dense) fd_update_wave_dense(g, fb, L, wcnt, x, n_i, rs, wedges, pairs);
        else fd_update_light(g, fb, L, tab, x, min<uint32_t>(kFdWaveSlots, wave_slots(fw[x])), rs, wedges, pairs);
        if (lane == 0) {
            sup[x] = init[vert[x]] - (int64_t)L.racc[wid];
            L.racc[wid] = 0;
        }
        wave_sync();
    }
    __syncthreads();
    const FdRecountState rw{alive, vert, &L.racc[0]};
    for (int32_t q = 0; q < n_rh; ++q) {
        const int32_t x = rh[q];
        const int32_t ux = vert[x];
        const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
        // ends with a barrier, so every thread's share is in racc[0]
        fd_update_heavy(g, fb, L, sp, x, e0, d, n_i, rw, wedges, pairs, spills);
        if (tid == 0) {
            sup[x] = init[vert[x]] - (int64_t)L.racc[0];
            L.racc[0] = 0;
        }
        __syncthreads();
    }
}


// DGM (Section 4.2) for a subset kept in HBM: every run of G_i keeps only
// its live members, in order (each wave compacts whole runs in place with
// ballots; every write lands at or before the entries still to be read),
// then the edges of the live vertices take their runs' new lengths.  All
// threads call.
__device__ inline void fd_compact_runs(const DevGraph& g, const FdBuffers& fb, FdLds& L, int32_t sub, int64_t P0,
                                       const int32_t* lc, int32_t n_live, const int32_t* alive,
                                       const int32_t* vert) {
    constexpr int NW = kFdThreads / kWave;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    const int64_t r0 = fb.sub_roff[sub], r1 = fb.sub_roff[sub + 1];
    for (int64_t r = r0 + wid; r < r1; r += NW) {
        const int32_t q = fb.run_q[r];
        const int32_t len = fb.rlen_at[q];
        int32_t out = 0;
        for (int32_t i0 = 0; i0 < len; i0 += kWave) {
            const int32_t i = i0 + lane;
            int32_t w = 0;
            bool keep = false;
            if (i < len) {
                w = fb.pcsc[q + i];
                keep = (alive[w] & kFdAlive) != 0;
            }
            const uint64_t km = __ballot(keep);
            wave_sync();  // every lane has read its entry before any is written
            if (keep) fb.pcsc[q + out + (int32_t)__popcll(km & lanemask_lt())] = w;
            out += (int32_t)__popcll(km);
            wave_sync();
        }
        if (lane == 0) fb.rlen_at[q] = out;
    }
    __syncthreads();
    for (int32_t j = wid; j < n_live; j += NW) {
        const int32_t x = lc[j];
        if (!(alive[x] & kFdAlive)) continue;
        const int32_t ux = vert[x];
        for (int64_t e = g.a_off[ux] + lane; e < g.a_off[ux + 1]; e += kWave) fb.fd_len[e] = fb.rlen_at[fb.fd_beg[e]];
    }
    __syncthreads();
}

// Level loop of a subset whose state lives in HBM.  With pair rows (pr)
// every peeled vertex is on the per-wave list and its row replaces the walk;
// a pair step with many peeled vertices and row entries is published on the
// help board and taken kFdPairHelpChunk rows at a time.
__device__ inline void fd_peel_hbm(const DevGraph& g, const FdBuffers& fb, const int64_t* __restrict__ init,
                                   int64_t P0, int32_t n_i, FdLds& L, unsigned long long* tab, const Spill& sp,
                                   FdHelpSlot* hs, int32_t help_chunk, int32_t help_level_min, int32_t huc_pct,
                                   int32_t sub, int32_t dgm, bool pr, int64_t shift, unsigned long long& wedges,
                                   unsigned long long& pairs,
                                   unsigned long long& levels, unsigned long long& spills,
                                   unsigned long long& huc_steps, unsigned long long& compactions) {
    constexpr int NT = kFdThreads;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    int32_t* lc = fb.lst[0] + P0;
    int32_t* ln = fb.lst[1] + P0;
    int32_t* pl = fb.lst[2] + P0;
    int32_t* ph = fb.lst[3] + P0;
    int32_t* cx = fb.lst[4] + P0;
    int64_t* sup = fb.supp_fd + P0;
    const int64_t* fw = fb.fd_w + P0;
    int32_t* alive = fb.alive + P0;
    const int32_t* vert = fb.fd_vert + P0;
    FdHbmState st{sup, alive, vert};
    const bool wave_dense = n_i <= kFdWaveKeys;
    uint32_t* wcnt = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(&L.u) + (size_t)wid * kFdWaveKeys);
    int64_t wsum = 0, esum = 0;
    for (int32_t j = tid; j < n_i; j += NT) {
        lc[j] = j;
        const int32_t v = vert[j];
        sup[j] = init[v];
        alive[j] = kFdAlive | (!pr && fd_heavy(g, fb, P0, n_i, j) ? kFdHeavy : 0);
        wsum += fw[j];
        if (dgm) esum += g.a_off[v + 1] - g.a_off[v];
    }
    // induced wedges of the live vertices: the cost of a HUC re-count
    int64_t w_live = huc_pct > 0 ? fd_block_sum<NT>(L, wsum) : 0;
    // DGM (Section 4.2): the runs of G_i are compacted each time the
    // updates since the last compaction walked as many wedges as G_i has
    // edges (the induced wedges of the peeled vertices stand for the walk)
    const int64_t m_i = dgm ? fd_block_sum<NT>(L, esum) : 0;
    int64_t walked = 0;
    __syncthreads();
    // lc: the live list (it may still hold vertices peeled by later steps of
    // a level; the next full pass drops them)
    int32_t n_live = n_i;
    int32_t n_cx = -1;  // >= 0: the next step peels the crossing list cx instead
    int64_t level = 0;
    // Full passes over the live list stride through it with kFdPassUnroll
    // entries per thread loaded before any is used, so that many of the
    // list's dependent loads (entry, then support) are in flight together;
    // partitions append through one LDS atomic per wave and list.
    constexpr int U = kFdPassUnroll;
    for (;;) {
        if (tid < 4) L.lcnt[tid] = 0;
        if (tid == 0) {
            L.wave_head = 0;
            L.hw = 0;
            L.pw_all = 0;
            L.pw_upd = 0;
        }
        if (n_cx < 0) {
            if (n_live == 0) break;
            int64_t mn = INT64_MAX;
            for (int32_t b0 = 0; b0 < n_live; b0 += NT * U) {
                int32_t xs[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t j = b0 + u * NT + tid;
                    xs[u] = j < n_live ? lc[j] : -1;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (xs[u] < 0) continue;
                    const int64_t sv = sup[xs[u]];
                    if ((alive[xs[u]] & kFdAlive) && sv < mn) mn = sv;
                }
            }
            mn = fd_min<NT>(L, mn);
            if (mn == INT64_MAX) break;  // every entry left was peeled
            level = mn > level ? mn : level;
            // peel every live vertex at or below the level; per-wave and
            // heavy ones go to separate lists, vertices without support left
            // need no update at all
            for (int32_t b0 = 0; b0 < n_live; b0 += NT * U) {
                int32_t xs[U], fl[U];
                int64_t ss[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t j = b0 + u * NT + tid;
                    xs[u] = j < n_live ? lc[j] : -1;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    ss[u] = xs[u] >= 0 ? sup[xs[u]] : 0;
                    fl[u] = xs[u] >= 0 ? alive[xs[u]] : 0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t x = xs[u];
                    const bool is_live = x >= 0 && (fl[u] & kFdAlive);
                    const bool keep = is_live && ss[u] > level;
                    const bool peel = is_live && !keep;
                    const bool heavy = peel && ss[u] > 0 && (fl[u] & kFdHeavy);
                    const bool light = peel && ss[u] > 0 && !(fl[u] & kFdHeavy);
                    const int32_t pk = fd_wave_slot(keep, &L.lcnt[0]);
                    const int32_t pw = fd_wave_slot(light, &L.lcnt[1]);
                    const int32_t pq = fd_wave_slot(heavy, &L.lcnt[2]);
                    if (keep) ln[pk] = x;
                    if (light) pl[pw] = x;
                    if (heavy) {
                        ph[pq] = x;
                        atomicAdd(&L.hw, (unsigned long long)fw[x]);
                    }
                    if (peel) {
                        alive[x] = fl[u] & ~kFdAlive;
                        fb.theta[vert[x]] = level;
                        if (huc_pct > 0 || dgm) {
                            const unsigned long long wx = (unsigned long long)fw[x];
                            atomicAdd(&L.pw_all, wx);
                            if (ss[u] > 0) atomicAdd(&L.pw_upd, wx);
                        }
                    }
                }
            }
            __syncthreads();
            int32_t* tmp = lc;
            lc = ln;
            ln = tmp;
            n_live = L.lcnt[0];
        } else {
            // the vertices the last step dropped to the level: all live
            __syncthreads();
            for (int32_t j = tid; j < n_cx; j += NT) {
                const int32_t x = cx[j];
                const int64_t sx = sup[x];
                const int32_t f = alive[x];
                alive[x] = f & ~kFdAlive;
                fb.theta[vert[x]] = level;
                if (huc_pct > 0 || dgm) {
                    const unsigned long long wx = (unsigned long long)fw[x];
                    atomicAdd(&L.pw_all, wx);
                    if (sx > 0) atomicAdd(&L.pw_upd, wx);
                }
                if (sx > 0) {
                    if (f & kFdHeavy) {
                        ph[atomicAdd(&L.lcnt[2], 1)] = x;
                        atomicAdd(&L.hw, (unsigned long long)fw[x]);
                    } else {
                        pl[atomicAdd(&L.lcnt[1], 1)] = x;
                    }
                }
            }
            __syncthreads();
        }
        const int32_t n_light = L.lcnt[1], n_heavy = L.lcnt[2];
        levels += tid == 0;
        if (huc_pct > 0) {
            // HUC: re-count the live supports instead of applying this
            // step's updates when those walk more wedges than huc_pct % of a
            // re-count of the vertices left
            w_live -= (int64_t)L.pw_all;
            const int64_t peel_w = (int64_t)L.pw_upd;
            if (peel_w > 0 && w_live > 0 && peel_w * 100 > (int64_t)huc_pct * w_live) {
                __syncthreads();
                fd_recount(g, fb, L, sp, lc, n_live, pl, ph, alive, vert, sup, fw, init, n_i, wave_dense, tab, wcnt,
                           wedges, pairs, spills);
                huc_steps += tid == 0;
                n_cx = -1;
                continue;
            }
        }
        bool publish = hs && n_light >= (pr ? kFdPairHelpMin : help_level_min);
        if (publish && pr) {
            // a pair step is shared only when its rows hold enough entries
            // to outweigh the board's fences
            int64_t e = 0;
            for (int32_t q = tid; q < n_light; q += NT) e += fb.prow_n[P0 + pl[q]];
            publish = fd_block_sum<NT>(L, e) >= kFdPairHelpEntries;
        }
        // heavy updates are shared only when there are several and enough
        // wedges to outweigh the board's fences
        const bool publish_heavy =
            !pr && hs && n_heavy >= kFdHelpHeavyMin && L.hw >= (unsigned long long)kFdHelpHeavyWedges;
        // a small step (not published, so no helper decrements) tracks the
        // vertices it drops to the level
        const bool track = !publish && !publish_heavy && n_light + n_heavy <= kFdCascadeMax;
        st.cx = track ? cx : nullptr;
        st.cxn = &L.lcnt[3];
        st.level = level;
        if (publish) {
            // publish the level's per-wave updates on the help board, take
            // entries like the helpers do, then wait for every taken entry
            // (levels with fewer updates are not worth the fences)
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                atomicExch(&hs->done, 0);
                __threadfence();
                atomicExch(&hs->word, (unsigned long long)n_light << 32);
            }
            __syncthreads();
            if (pr) fd_help_pairs(fb, L, pl, P0, shift, hs, st, pairs);
            else fd_help_slot(g, fb, L, tab, wcnt, pl, fw, n_i, hs, help_chunk, st, wedges, pairs);
            __syncthreads();
            if (tid == 0)
                while (__hip_atomic_load(&hs->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n_light)
                    __builtin_amdgcn_s_sleep(2);
            __syncthreads();
            __threadfence();
        } else if (pr) {
            // rows' starts and lengths for up to kFdHeavyPre peeled vertices
            // at a time, then their entries
            __syncthreads();
            for (int32_t c0 = 0; c0 < n_light; c0 += kFdHeavyPre) {
                const int32_t nq = min(kFdHeavyPre, n_light - c0);
                for (int32_t q = tid; q < nq; q += NT) {
                    const int32_t x = pl[c0 + q];
                    L.hx_off[q] = fb.prow_off[P0 + x] + shift;
                    L.hx_deg[q] = fb.prow_n[P0 + x];
                }
                __syncthreads();
                const auto row = [&](int32_t q, int64_t& off, int32_t& len) {
                    off = L.hx_off[q];
                    len = L.hx_deg[q];
                };
                fd_pair_units(fb, nq, row, st, pairs);
                __syncthreads();
            }
        } else {
            __syncthreads();
            for (int32_t q = fd_next_wave_item(L); q < n_light; q = fd_next_wave_item(L)) {
                const int32_t x = pl[q];
                if (wave_dense) fd_update_wave_dense(g, fb, L, wcnt, x, n_i, st, wedges, pairs);
                else fd_update_light(g, fb, L, tab, x, min<uint32_t>(kFdWaveSlots, wave_slots(fw[x])), st, wedges, pairs);
            }
        }
        __syncthreads();
        if (publish_heavy) {
            // the heavy updates go on the help board too: every workgroup
            // helping this subset takes whole heavy vertices
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                atomicExch(&hs->hdone, 0);
                __threadfence();
                atomicExch(&hs->hword, (unsigned long long)n_heavy << 32);
            }
            fd_heavy_take(g, fb, L, sp, ph, n_i, hs, st, wedges, pairs, spills);
            if (tid == 0)
                while (__hip_atomic_load(&hs->hdone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n_heavy)
                    __builtin_amdgcn_s_sleep(2);
            __syncthreads();
            __threadfence();
        } else {
            fd_heavy_level(g, fb, L, sp, ph, n_heavy, n_i, st, wedges, pairs, spills);
        }
        __syncthreads();
        n_cx = track && L.lcnt[3] > 0 ? L.lcnt[3] : -1;
        if (dgm) {
            walked += (int64_t)L.pw_upd;
            if (walked >= m_i) {
                fd_compact_runs(g, fb, L, sub, P0, lc, n_live, alive, vert);
                walked = 0;
                compactions += tid == 0;
            }
        }
        __syncthreads();
    }
}

// Level loop of a subset whose state lives in LDS.  Each level makes one
// pass over the live list (each thread a contiguous run): one block scan
// gives the offsets of the light, heavy and kept vertices and the least
// kept support.  The next level's minimum is the least of that and of the
// supports the decrements leave behind: a kept vertex that no decrement
// touched still has the support read in the pass.
//
// With pair rows (pr), the rows' starts (relative to the subset's first row)
// and lengths are kept in the LDS of the update tables, which pair updates
// do not use, and cleared at the end.
__device__ inline void fd_peel_lds(const DevGraph& g, const FdBuffers& fb, const int64_t* __restrict__ init,
                                   int64_t P0, int32_t n_i, FdLds& L, FdSmall& S, unsigned long long* tab,
                                   const Spill& sp, bool pr, int64_t shift, unsigned long long& wedges,
                                   unsigned long long& pairs,
                                   unsigned long long& levels, unsigned long long& spills) {
    constexpr int NT = kFdThreads;
    constexpr int NW = NT / kWave;
    constexpr int kSh = kFdPack;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    uint32_t* wcnt = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(&L.u) + (size_t)wid * kFdWaveKeys);
    const FdLdsState st{&S, fb.fd_vert + P0};
    static_assert(sizeof(FdLds::Shared) >= (size_t)kFdLdsVerts * 6, "pair-row starts and lengths fit the union");
    int32_t* roff = reinterpret_cast<int32_t*>(&L.u);
    uint16_t* rn = reinterpret_cast<uint16_t*>(roff + kFdLdsVerts);
    const int64_t rb0 = pr ? fb.prow_off[P0] : 0, rbase = rb0 + (pr ? shift : 0);
    int64_t mn = INT64_MAX;
    for (int32_t j = tid; j < n_i; j += NT) {
        const int32_t v = fb.fd_vert[P0 + j];
        const int64_t s0 = init[v];
        S.sup[j] = s0;
        S.flag[j] = kFdAlive | (!pr && fd_heavy(g, fb, P0, n_i, j) ? kFdHeavy : 0);
        S.lc[j] = (uint16_t)j;
        mn = s0 < mn ? s0 : mn;
        if (pr) {
            roff[j] = (int32_t)(fb.prow_off[P0 + j] - rb0);
            rn[j] = (uint16_t)fb.prow_n[P0 + j];
        }
    }
    mn = fd_min<NT>(L, mn);
    uint16_t* lc = S.lc;
    uint16_t* ln = S.ln;
    int32_t n_live = n_i;
    int64_t level = 0;
    while (n_live > 0) {
        level = mn > level ? mn : level;
        const int32_t per = (n_live + NT - 1) / NT;
        const int32_t j0 = min(n_live, tid * per), j1 = min(n_live, j0 + per);
        int64_t cnt = 0, kmin = INT64_MAX;
        for (int32_t j = j0; j < j1; ++j) {
            const int32_t x = lc[j];
            const int64_t sx = S.sup[x];
            if (sx > level) {
                cnt += 1ll << (2 * kSh);
                kmin = sx < kmin ? sx : kmin;
            } else if (sx > 0) {
                cnt += (S.flag[x] & kFdHeavy) ? (1ll << kSh) : 1ll;
            }
        }
        // block exclusive scan of the packed counts and block minimum
        const int64_t inc = wave_incl_scan_i64<NT>(cnt);
        const int64_t wmin = wave_min_i64(kmin);
        __syncthreads();
        if (lane == kWave - 1) L.red[wid] = inc;
        if (lane == 0) S.red_min[wid] = wmin;
        if (tid == 0) S.upd_min = LLONG_MAX;
        __syncthreads();
        int64_t off = 0, tot = 0, bmin = INT64_MAX;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int64_t v = L.red[w];
            off += w < wid ? v : 0;
            tot += v;
            bmin = S.red_min[w] < bmin ? S.red_min[w] : bmin;
        }
        const int64_t mask = (1ll << kSh) - 1;
        off += inc - cnt;
        int32_t ol = (int32_t)(off & mask), oh = (int32_t)((off >> kSh) & mask), ok = (int32_t)(off >> (2 * kSh));
        if (tid == 0) L.wave_head = 0;
        const int32_t n_light = (int32_t)(tot & mask), n_heavy = (int32_t)((tot >> kSh) & mask);
        const int32_t n_keep = (int32_t)(tot >> (2 * kSh));
        for (int32_t j = j0; j < j1; ++j) {
            const int32_t x = lc[j];
            const int64_t sx = S.sup[x];
            if (sx > level) {
                ln[ok++] = (uint16_t)x;
            } else {
                S.flag[x] &= (uint8_t)~kFdAlive;
                S.sup[x] = level;
                if (sx > 0) {
                    if (S.flag[x] & kFdHeavy) S.pl[n_light + oh++] = (uint16_t)x;
                    else S.pl[ol++] = (uint16_t)x;
                }
            }
        }
        __syncthreads();
        levels += tid == 0;
        if (pr) {
            // every peeled vertex is on the light list (no heavy flags)
            const auto row = [&](int32_t q, int64_t& off, int32_t& len) {
                const int32_t x = (int32_t)S.pl[q];
                off = rbase + (int64_t)roff[x];
                len = (int32_t)rn[x];
            };
            fd_pair_units(fb, n_light, row, st, pairs);
        } else {
            for (int32_t q = fd_next_wave_item(L); q < n_light; q = fd_next_wave_item(L))
                fd_update_wave_dense(g, fb, L, wcnt, (int32_t)S.pl[q], n_i, st, wedges, pairs);
            __syncthreads();
            fd_heavy_level(g, fb, L, sp, S.pl + n_light, n_heavy, n_i, st, wedges, pairs, spills);
        }
        __syncthreads();
        mn = min<int64_t>(bmin, (int64_t)S.upd_min);
        uint16_t* tmp = lc;
        lc = ln;
        ln = tmp;
        n_live = n_keep;
    }
    // tip numbers, kept in sup since each vertex was peeled
    for (int32_t j = tid; j < n_i; j += NT) fb.theta[fb.fd_vert[P0 + j]] = S.sup[j];
    if (pr) {
        // the update tables are all zero between uses
        uint32_t* z = reinterpret_cast<uint32_t*>(&L.u);
        const int32_t words = kFdLdsVerts * 6 / 4;
        for (int32_t i = tid; i < words; i += NT) z[i] = 0;
        __syncthreads();
    }
}

// One workgroup peels one subset at a time, taking subsets from the
// workload-sorted queue (dynamic allocation).  Inside a subset it runs
// bottom-up peeling level by level: the level is max(level, minimum live
// support), and every live vertex whose support is at most the level is
// peeled at that level (equal to one-at-a-time peeling, whatever the order).
// The vertices peeled at one level update the survivors concurrently: light
// ones one per wavefront with a private hash table, heavy ones one at a time
// with the whole workgroup and a key bitmap.
__global__ void __launch_bounds__(kFdThreads)
k_fd_peel(FdJobs jobs, const int64_t* __restrict__ tasks, int32_t n_tasks, FdBoard* board, SpillArena spa) {
    __shared__ FdLds L;
    __shared__ FdSmall S;
    constexpr int NT = kFdThreads;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    {
        unsigned long long* all = &L.u.wtab[0][0];
        for (int i = tid; i < (int)(sizeof(L.u) / 8); i += NT) all[i] = 0;
    }
    if (tid == 0) L.spill_n = 0;
    __syncthreads();
    const Spill sp{spa.dense + (int64_t)blockIdx.x * spa.stride, spa.list + (int64_t)blockIdx.x * spa.stride};
    unsigned long long* tab = L.u.wtab[wid];
    for (;;) {
        if (tid == 0) L.flag = atomicAdd(&board->head, 1);
        __syncthreads();
        const int32_t t = L.flag;
        __syncthreads();
        if (t >= n_tasks) break;
        // one task = one subset of one graph: tasks[t] = job << 32 | subset,
        // or, for a single graph, its own workload-ordered subset list
        const FdJob& J = tasks ? jobs.list[tasks[t] >> 32] : jobs.one;
        const FdBuffers& fb = J.fb;
        const int32_t sub = tasks ? (int32_t)(tasks[t] & 0xffffffffll) : fb.order[t];
        const int64_t P0 = fb.sub_off[sub];
        const int32_t n_i = (int32_t)(fb.sub_off[sub + 1] - P0);
        if (n_i == 0) continue;
        unsigned long long wedges = 0, pairs = 0, levels = 0, spills = 0, huc_steps = 0, compactions = 0;
        const unsigned long long t_start = jobs.trace ? wall_clock64() : 0ull;
        // pair rows, when this subset's were built
        const int64_t shift = fb.pairs_on ? fb.pshift[sub] : kNoRows;
        const bool pr = shift != kNoRows;
        if (pr && tid == 0) atomicAdd(&J.ctl->fd_pair_tasks, 1ull);
        if (n_i <= kFdLdsVerts) {
            fd_peel_lds(J.g, fb, J.init, P0, n_i, L, S, tab, sp, pr, shift, wedges, pairs, levels, spills);
        } else {
            // a large subset opens a help-board slot for its per-wave updates
            FdHelpSlot* hs = nullptr;
            if (n_i >= J.help_min) {
                if (tid == 0) {
                    const int32_t k = atomicAdd(&board->n_slots, 1);
                    L.flag = k;
                    if (k < kFdHelpSlots) {
                        FdHelpSlot& h = board->slot[k];
                        h.job = tasks ? (int32_t)(tasks[t] >> 32) : -1;
                        h.n_i = n_i;
                        h.P0 = P0;
                        h.word = 0;
                        h.done = 0;
                        h.hword = 0;
                        h.hdone = 0;
                        h.pairs = pr ? 1 : 0;
                        h.pshift = shift;
                        __threadfence();
                        atomicExch(&h.state, 1);
                    }
                }
                __syncthreads();
                if (L.flag < kFdHelpSlots) hs = &board->slot[L.flag];
                __syncthreads();
            }
            fd_peel_hbm(J.g, fb, J.init, P0, n_i, L, tab, sp, hs, J.help_chunk, J.help_level_min,
                        pr ? 0 : J.huc_pct, sub, pr ? 0 : J.dgm, pr, shift, wedges, pairs, levels, spills, huc_steps,
                        compactions);
            if (hs && tid == 0) atomicExch(&hs->state, 2);
        }
        if (jobs.trace && tid == 0 && t < jobs.trace_max) {
            unsigned long long* e = jobs.trace + 4 * (int64_t)t;
            e[0] = (unsigned long long)n_i;
            e[1] = levels;  // thread 0 counts every level
            e[2] = t_start;
            e[3] = wall_clock64();
        }
        wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
        pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
        levels = (unsigned long long)wave_sum_i64((int64_t)levels);
        spills = (unsigned long long)wave_sum_i64((int64_t)spills);
        huc_steps = (unsigned long long)wave_sum_i64((int64_t)huc_steps);
        compactions = (unsigned long long)wave_sum_i64((int64_t)compactions);
        if (lane == 0) {
            if (wedges) atomicAdd(&J.ctl->wedges_fd, wedges);
            if (pairs) atomicAdd(&J.ctl->pair_updates, pairs);
            if (levels) atomicAdd(&J.ctl->fd_levels, levels);
            if (spills) atomicAdd(&J.ctl->spills, spills);
            if (huc_steps) atomicAdd(&J.ctl->fd_huc_steps, huc_steps);
            if (compactions) atomicAdd(&J.ctl->fd_compactions, compactions);
        }
    }
    // No task left: help the large subsets still open until no slot is
    // open.  The whole workgroup works on one slot at a time (its waves share
    // the LDS counters, so they must use the same kind of update).  Owners
    // never wait for helpers, only for entries already taken, so helping is
    // optional and every wave ends.
    for (;;) {
        if (tid == 0) {
            const int32_t n_open = min(__hip_atomic_load(&board->n_slots, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                       kFdHelpSlots);
            int32_t pick = -1;  // -1: nothing open, -2: open but nothing to take now
            for (int32_t k = 0; k < n_open && pick < 0; ++k) {
                FdHelpSlot* hs = &board->slot[k];
                if (__hip_atomic_load(&hs->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1) continue;
                pick = -2;
                const unsigned long long hv = __hip_atomic_load(&hs->hword, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint32_t)hv < (uint32_t)(hv >> 32)) {
                    pick = kFdHelpSlots + k;  // heavy entries to take
                    break;
                }
                const unsigned long long wv = __hip_atomic_load(&hs->word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint32_t)wv < (uint32_t)(wv >> 32)) pick = k;
            }
            L.flag = pick;
        }
        __syncthreads();
        const int32_t k = L.flag;
        __syncthreads();
        if (k == -1) break;
        if (k >= kFdHelpSlots) {
            __threadfence();
            FdHelpSlot* hs = &board->slot[k - kFdHelpSlots];
            const FdJob& J = hs->job >= 0 ? jobs.list[hs->job] : jobs.one;
            const FdBuffers& fb = J.fb;
            const int64_t P0 = hs->P0;
            const FdHbmState st{fb.supp_fd + P0, fb.alive + P0, fb.fd_vert + P0};
            unsigned long long wedges = 0, pairs = 0, spills = 0;
            fd_heavy_take(J.g, fb, L, sp, fb.lst[3] + P0, hs->n_i, hs, st, wedges, pairs, spills);
            wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
            pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
            spills = (unsigned long long)wave_sum_i64((int64_t)spills);
            if (lane == 0) {
                if (wedges) atomicAdd(&J.ctl->wedges_fd, wedges);
                if (pairs) atomicAdd(&J.ctl->pair_updates, pairs);
                if (spills) atomicAdd(&J.ctl->spills, spills);
            }
        } else if (k >= 0) {
            __threadfence();
            FdHelpSlot* hs = &board->slot[k];
            const FdJob& J = hs->job >= 0 ? jobs.list[hs->job] : jobs.one;
            const FdBuffers& fb = J.fb;
            const int64_t P0 = hs->P0;
            const FdHbmState st{fb.supp_fd + P0, fb.alive + P0, fb.fd_vert + P0};
            uint32_t* wcnt = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(&L.u) + (size_t)wid * kFdWaveKeys);
            unsigned long long wedges = 0, pairs = 0;
            if (hs->pairs) fd_help_pairs(fb, L, fb.lst[2] + P0, P0, hs->pshift, hs, st, pairs);
            else fd_help_slot(J.g, fb, L, tab, wcnt, fb.lst[2] + P0, fb.fd_w + P0, hs->n_i, hs, J.help_chunk, st,
                              wedges, pairs);
            wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
            pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
            if (lane == 0) {
                if (wedges) atomicAdd(&J.ctl->wedges_fd, wedges);
                if (pairs) atomicAdd(&J.ctl->pair_updates, pairs);
            }
        } else {
            __builtin_amdgcn_s_sleep(64);
        }
        __syncthreads();
    }
}

// Pair rows (the fine-grained updates, precomputed).  Peeling u inside U_i
// lowers the support of every w of U_i by C(c, 2), c = |N(u) ∩ N(w)| (the
// update of Alg. 4 on G_i).  Only side A is peeled, so c never changes while
// U_i is peeled, and u's update can be listed once, before any peeling,
// with every vertex counted in parallel.  Row capacity of the vertex at
// position p: min(n_i - 1, fd_w[p] / 2), since every listed w takes at least
// two of u's induced wedges.  cap[n_a] = 0, so that an exclusive scan leaves
// the total there.
__global__ void k_fd_pair_cap(const int32_t* __restrict__ state, const int32_t* __restrict__ fd_vert,
                              const int64_t* __restrict__ sub_off, const int64_t* __restrict__ fd_w, int32_t n_a,
                              int64_t* cap) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n_a) return;
    int64_t c = 0;
    if (p < n_a) {
        const int32_t sub = state[fd_vert[p]];
        const int64_t n_i = sub_off[sub + 1] - sub_off[sub];
        c = min<int64_t>(n_i - 1, fd_w[p] / 2);
    }
    cap[p] = c;
}

// LDS of the per-wave pair-row build: per wave 8 KiB (8-bit counters of a
// subset of at most kFdPairWaveKeys vertices, or a hash table of up to
// kFdPairWaveSlots slots) and the staging of its neighbour runs.
constexpr int kFdPairThreads = 256;
constexpr int kFdPairWaves = kFdPairThreads / kWave;
constexpr int kFdPairWaveKeys = 8192;
constexpr int kFdPairWaveSlots = 1024;
constexpr int64_t kFdPairHashMax = 448;     // hash path: at most this many wedges (table at most 7/16 full)
constexpr int64_t kFdPairDenseMax = 4096;   // counter path: at most this many wedges for one wave
struct FdPairLds {
    union Shared {
        uint32_t cnt[kFdPairWaves][kFdPairWaveKeys / 4];
        unsigned long long wtab[kFdPairWaves][kFdPairWaveSlots];
    } u;
    int64_t wsbeg[kFdPairWaves][kWave];
    int64_t wpre[kFdPairWaves][kWave + 1];
    int32_t pn[kFdPairWaves];
};

// Row space in workload order (fb.order: most induced wedges first),
// greedily: a subset whose rows (contiguous in position order) still fit the
// budget gets the shift that moves them to the next free place; one that
// does not fit gets kNoRows (it walks) and the next ones are still tried.
// One workgroup of kT threads: each chunk of kT subsets' capacities is
// loaded in parallel, then placed by one thread.
__global__ void k_fd_pair_place(FdBuffers fb, int32_t S, int64_t lim) {
    __shared__ int64_t cap[kT], lo[kT];
    __shared__ int32_t sid[kT];
    int64_t used = 0;  // thread 0
    for (int32_t k0 = 0; k0 < S; k0 += kT) {
        const int32_t k = k0 + threadIdx.x;
        if (k < S) {
            const int32_t s = fb.order[k];
            const int64_t a = fb.prow_off[fb.sub_off[s]];
            sid[threadIdx.x] = s;
            lo[threadIdx.x] = a;
            cap[threadIdx.x] = fb.prow_off[fb.sub_off[s + 1]] - a;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int32_t n = min(kT, S - k0);
            for (int32_t i = 0; i < n; ++i) {
                if (used + cap[i] <= lim) {
                    fb.pshift[sid[i]] = used - lo[i];
                    used += cap[i];
                } else {
                    fb.pshift[sid[i]] = kNoRows;
                }
            }
        }
        __syncthreads();
    }
}

// Pair rows of the light vertices, every wave on its own (no workgroup
// barrier): a wave takes 64 positions at a time, strided over the whole
// range so that the hubs at the front of each subset (ranks ascend inside a
// subset) spread over many waves, classifies them in its lanes, counts each
// light vertex's wedges inside its subset (8-bit
// counters in a subset of at most kFdPairWaveKeys vertices, else a hash
// table) and writes the pairs instead of decrementing.  The other vertices
// go to the heavy list (one atomic per wave and chunk) for
// k_fd_pair_rows_heavy.  Only subsets with row space.
__global__ void __launch_bounds__(kFdPairThreads)
k_fd_pair_rows(DevGraph g, FdBuffers fb, const int32_t* __restrict__ state, int32_t* heavy, Ctl* ctl) {
    __shared__ FdPairLds L;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int32_t n_a = g.n_a;
    {
        unsigned long long* mine = L.u.wtab[wid];
        for (int i = lane; i < kFdPairWaveSlots; i += kWave) mine[i] = 0;
        if (lane == 0) L.pn[wid] = 0;
    }
    wave_sync();
    uint32_t* wcnt = L.u.cnt[wid];
    unsigned long long* tab = L.u.wtab[wid];
    unsigned long long wedges = 0, entries = 0, unused = 0;
    // chunk c holds positions c + k * n_chunks, k < 64
    const int32_t n_chunks = (int32_t)(((int64_t)n_a + kWave - 1) / kWave);
    for (;;) {
        int32_t c = 0;
        if (lane == 0) c = atomicAdd(&fb.board->pair_head, 1);
        c = __shfl(c, 0, kWave);
        if (c >= n_chunks) break;
        const int32_t p = (int32_t)min<int64_t>((int64_t)c + (int64_t)lane * n_chunks, (int64_t)n_a);
        int kind = -1;  // 0: counters, 1: hash, 2: heavy
        int64_t P0 = 0, w = 0, shift = kNoRows;
        int32_t n_i = 0;
        if (p < n_a) {
            const int32_t ux = fb.fd_vert[p];
            const int32_t sub = state[ux];
            P0 = fb.sub_off[sub];
            n_i = (int32_t)(fb.sub_off[sub + 1] - P0);
            w = fb.fd_w[p];
            shift = fb.pshift[sub];
            const int64_t d = g.a_off[ux + 1] - g.a_off[ux];
            if (shift != kNoRows) {
                if (w < 2) fb.prow_n[p] = 0;
                else if (n_i <= kFdPairWaveKeys && d <= 255 && w <= kFdPairDenseMax) kind = 0;
                else if (w <= kFdPairHashMax) kind = 1;
                else kind = 2;
            }
        }
        const uint64_t hm = __ballot(kind == 2);
        if (hm) {
            int32_t base = 0;
            if (lane == 0) base = atomicAdd(&fb.board->pair_heavy, (int32_t)__popcll(hm));
            base = __shfl(base, 0, kWave);
            if (kind == 2) heavy[base + (int32_t)__popcll(hm & lanemask_lt())] = p;
        }
        uint64_t lm = __ballot(kind == 0 || kind == 1);
        while (lm) {
            const int t = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            const int32_t pt = __shfl(p, t, kWave);
            const int64_t P0t = __shfl(P0, t, kWave), wt = __shfl(w, t, kWave);
            const int32_t n_it = __shfl(n_i, t, kWave), kt = __shfl(kind, t, kWave);
            const int64_t r0 = fb.prow_off[pt] + __shfl(shift, t, kWave);
            const FdPairWriter st{fb.fd_vert + P0t, fb.prow_w + r0, fb.prow_b + r0, &L.pn[wid]};
            const int32_t j = (int32_t)(pt - P0t);
            if (kt == 0) fd_update_wave_dense(g, fb, L, wcnt, j, n_it, st, wedges, unused);
            else fd_update_light(g, fb, L, tab, j, min<uint32_t>(kFdPairWaveSlots, wave_slots(wt)), st, wedges, unused);
            if (lane == 0) {
                const int32_t n = L.pn[wid];
                fb.prow_n[pt] = n;
                entries += (unsigned long long)n;
                L.pn[wid] = 0;
            }
            wave_sync();
        }
    }
    if (lane == 0) {
        if (wedges) atomicAdd(&ctl->wedges_fd, wedges);
        if (entries) atomicAdd(&ctl->fd_pair_entries, entries);
    }
}

// Pair rows of the heavy list: each workgroup takes one vertex at a time and
// counts it with its LDS bitmap and repeat table (fd_update_heavy).
__global__ void __launch_bounds__(kFdThreads)
k_fd_pair_rows_heavy(DevGraph g, FdBuffers fb, const int32_t* __restrict__ state, const int32_t* __restrict__ heavy,
                     Ctl* ctl, SpillArena spa) {
    __shared__ FdLds L;
    constexpr int NT = kFdThreads;
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    {
        unsigned long long* all = &L.u.wtab[0][0];
        for (int i = tid; i < (int)(sizeof(L.u) / 8); i += NT) all[i] = 0;
    }
    if (tid == 0) {
        L.spill_n = 0;
        L.pn[NW] = 0;
    }
    const int32_t n_heavy = fb.board->pair_heavy;
    if (blockIdx.x == 0 && tid == 0) ctl->fd_pair_heavy = (unsigned long long)n_heavy;
    const Spill sp{spa.dense + (int64_t)blockIdx.x * spa.stride, spa.list + (int64_t)blockIdx.x * spa.stride};
    unsigned long long wedges = 0, spills = 0, entries = 0, unused = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) L.flag = atomicAdd(&fb.board->pair_head2, 1);
        __syncthreads();
        const int32_t q = L.flag;
        if (q >= n_heavy) break;
        const int32_t p = heavy[q];
        const int32_t ux = fb.fd_vert[p];
        const int32_t sub = state[ux];
        const int64_t P0 = fb.sub_off[sub];
        const int32_t n_i = (int32_t)(fb.sub_off[sub + 1] - P0);
        const int64_t r0 = fb.prow_off[p] + fb.pshift[sub];
        const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
        const FdPairWriter st{fb.fd_vert + P0, fb.prow_w + r0, fb.prow_b + r0, &L.pn[NW]};
        fd_update_heavy(g, fb, L, sp, (int32_t)(p - P0), e0, d, n_i, st, wedges, unused, spills);
        if (tid == 0) {
            fb.prow_n[p] = L.pn[NW];
            entries += (unsigned long long)L.pn[NW];
            L.pn[NW] = 0;
        }
    }
    wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
    spills = (unsigned long long)wave_sum_i64((int64_t)spills);
    entries = (unsigned long long)wave_sum_i64((int64_t)entries);
    if (lane == 0) {
        if (wedges) atomicAdd(&ctl->wedges_fd, wedges);
        if (spills) atomicAdd(&ctl->spills, spills);
        if (entries) atomicAdd(&ctl->fd_pair_entries, entries);
    }
}

__global__ void k_scatter_i64(const int64_t* __restrict__ by_rank, const int32_t* __restrict__ orig, int32_t n,
                              int64_t* out) {
    GRID_STRIDE(r, (int64_t)n) out[orig[r]] = by_rank[r];
}

}  // namespace

// Resident workgroups of the per-wave pair-row build on the current device.
int pair_grid() {
    static std::mutex mu;
    static int cached_dev = -1, cached = 0;
    int dev = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (dev != cached_dev) {
        int cus = 0, n = 0;
        TIP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fd_pair_rows, kFdPairThreads, 0));
        cached = std::max(1, cus) * std::max(1, n);
        cached_dev = dev;
    }
    return cached;
}

int fd_occupancy() {
    int n = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fd_peel, kFdThreads, 0));
    return std::max(1, n);
}

void launch_fd_setup(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, uint64_t* tmp_keys,
                     int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp, uint64_t* keys_scratch,
                     int32_t* vals_scratch, hipStream_t s, bool runs) {
    const int32_t n_a = g.n_a;
    fill_i64(fb.task_w, 0, S, s);
    if (n_a <= 0) return;
    // vertices grouped by subset, ascending rank inside each subset
    fill_i64(fb.sub_cnt, 0, (int64_t)S + 1, s);
    {
        // a few vertices per thread, so that each workgroup's LDS counts
        // carry many of them
        const int lds_hist = S <= kFdHistMax ? 1 : 0;
        k_fd_vertex_keys<<<grid1(n_a, 256), kT, lds_hist ? sizeof(int32_t) * (size_t)S : 0, s>>>(
            pb.state, n_a, S, keys_scratch, fb.fd_vert, fb.sub_cnt, lds_hist);
    }
    TIP_HIP_TRY(hipGetLastError());
    radix_sort_pairs(keys_scratch, fb.fd_vert, tmp_keys, tmp_vals, n_a, bits_for((uint64_t)S), hist, scan_tmp, s);
    scan_exclusive_i64(fb.sub_cnt, fb.sub_off, (int64_t)S + 1, scan_tmp, s);
    k_fd_positions<<<grid1(n_a), kT, 0, s>>>(fb.fd_vert, n_a, fb.fd_pos);
    TIP_HIP_TRY(hipGetLastError());
    fill_i64(fb.fd_w, 0, n_a, s);
    if (g.m > 0) {
        k_fd_csc_keys<<<grid1(g.m), kT, 0, s>>>(g, pb.state, S, fb.pkeys, fb.pcsc);
        TIP_HIP_TRY(hipGetLastError());
        radix_sort_pairs(fb.pkeys, fb.pcsc, tmp_keys, tmp_vals, g.m,
                         bits_for((uint64_t)g.n_b * (uint64_t)S), hist, scan_tmp, s);
        {
            // runs of the sorted entries (the sort's buffers are free again:
            // keys_scratch holds the flags and their scan, tmp_keys the runs'
            // first entries), then each CSR edge's run and each entry's index
            int64_t* pos = reinterpret_cast<int64_t*>(keys_scratch);
            int64_t* run_lo = reinterpret_cast<int64_t*>(tmp_keys);
            k_fd_run_flags<<<grid1(g.m), kT, 0, s>>>(fb.pkeys, g.m, pos);
            TIP_HIP_TRY(hipGetLastError());
            scan_exclusive_i64(pos, pos, g.m, scan_tmp, s);
            k_fd_run_lo<<<grid1(g.m), kT, 0, s>>>(fb.pkeys, g.m, pos, run_lo);
            TIP_HIP_TRY(hipGetLastError());
            k_fd_run_scatter<<<grid1(g.m), kT, 0, s>>>(g, pb.state, fb.pkeys, pos, run_lo, fb.fd_pos, fb.sub_off,
                                                       fb.pcsc, fb.fd_beg, fb.fd_len);
            TIP_HIP_TRY(hipGetLastError());
        }
        const int lds_tw = S <= 4096 ? 1 : 0;
        k_fd_slices<<<grid1(g.m, 2048), kT, lds_tw ? sizeof(unsigned long long) * (size_t)S : 0, s>>>(
            g, pb.state, S, fb.fd_pos, fb.fd_len, fb.task_w, fb.fd_w, lds_tw);
        TIP_HIP_TRY(hipGetLastError());
        if (runs) {
            // the sort's buffers are free again: keys_scratch holds the flags
            // and their scan, tmp_keys the run keys
            int64_t* pos = reinterpret_cast<int64_t*>(keys_scratch);
            fill_i64(fb.sub_rcnt, 0, (int64_t)S + 2, s);
            k_fd_run_flags<<<grid1(g.m), kT, 0, s>>>(fb.pkeys, g.m, pos);
            TIP_HIP_TRY(hipGetLastError());
            scan_exclusive_i64(pos, pos, g.m, scan_tmp, s);
            k_fd_run_compact<<<grid1(g.m), kT, 0, s>>>(fb.pkeys, g.m, S, pos, tmp_keys, fb.run_q, fb.sub_rcnt);
            TIP_HIP_TRY(hipGetLastError());
            k_fd_run_len<<<grid1(g.m), kT, 0, s>>>(fb.pkeys, g.m, S, pos, fb.run_q, tmp_keys, fb.rlen_at);
            TIP_HIP_TRY(hipGetLastError());
            radix_sort_pairs(tmp_keys, fb.run_q, keys_scratch, tmp_vals, g.m, bits_for((uint64_t)S), hist, scan_tmp, s);
            scan_exclusive_i64(fb.sub_rcnt, fb.sub_roff, (int64_t)S + 2, scan_tmp, s);
        }
    }
    k_fd_order<<<1, 1024, 0, s>>>(fb.task_w, S, fb.order);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_fd_pairs(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, Ctl* ctl,
                     const SpillArena& spill, int big_grid, int64_t* scan_tmp, bool on, hipStream_t s) {
    fb.pairs_on = on && fb.pair_cap > 0 && g.n_a > 0 ? 1 : 0;
    if (!fb.pairs_on) return;
    // diagnostic: TIP_FD_PAIR_LIMIT=<entries> uses at most that many
    // entries of the budget (subsets beyond it walk), for testing the mix
    fb.pair_lim = fb.pair_cap;
    if (const char* e = std::getenv("TIP_FD_PAIR_LIMIT")) {
        const long long v = std::atoll(e);
        if (v >= 0) fb.pair_lim = std::min<int64_t>(fb.pair_cap, v);
    }
    const int32_t n_a = g.n_a;
    k_fd_pair_cap<<<grid1((int64_t)n_a + 1), kT, 0, s>>>(pb.state, fb.fd_vert, fb.sub_off, fb.fd_w, n_a, fb.prow_off);
    TIP_HIP_TRY(hipGetLastError());
    scan_exclusive_i64(fb.prow_off, fb.prow_off, (int64_t)n_a + 1, scan_tmp, s);
    k_fd_pair_place<<<1, kT, 0, s>>>(fb, S, fb.pair_lim);
    TIP_HIP_TRY(hipGetLastError());
    k_fd_reset_board<<<1, 256, 0, s>>>(fb.board);
    TIP_HIP_TRY(hipGetLastError());
    // the heavy list borrows the crossing list (written by the peeling
    // before it is read)
    int32_t* heavy = fb.lst[4];
    k_fd_pair_rows<<<std::max(1, pair_grid()), kFdPairThreads, 0, s>>>(g, fb, pb.state, heavy, ctl);
    TIP_HIP_TRY(hipGetLastError());
    k_fd_pair_rows_heavy<<<std::max(1, big_grid), kFdThreads, 0, s>>>(g, fb, pb.state, heavy, ctl, spill);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_fd(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, Ctl* ctl, const Tune& tune,
               const SpillArena& spill, int big_grid, uint64_t* tmp_keys, int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp,
               uint64_t* keys_scratch, int32_t* vals_scratch, hipStream_t s, bool trace) {
    if (g.n_a <= 0) return;
    launch_fd_setup(g, pb, fb, S, tmp_keys, tmp_vals, hist, scan_tmp, keys_scratch, vals_scratch, s,
                    tune.fd_dgm && tune.fd_huc_pct == 0);
    launch_fd_pairs(g, pb, fb, S, ctl, spill, big_grid, scan_tmp,
                    !tune.fd_walk && !tune.fd_dgm && tune.fd_huc_pct == 0, s);
    k_fd_reset_board<<<1, 256, 0, s>>>(fb.board);
    TIP_HIP_TRY(hipGetLastError());
    FdJobs jobs{};
    jobs.one = FdJob{g, fb, pb.init, ctl, tune.fd_help_min, tune.fd_help_chunk, tune.fd_help_level_min,
                     tune.fd_huc_pct, tune.fd_dgm && tune.fd_huc_pct == 0 ? 1 : 0};
    if (trace) {
        jobs.trace = fb.task_trace;
        jobs.trace_max = kFdTraceTasks;
    }
    // every resident workgroup: those without a task of their own help
    // with the large subsets
    const int grid = std::max(1, big_grid);
    k_fd_peel<<<grid, kFdThreads, 0, s>>>(jobs, nullptr, S, fb.board, spill);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_fd_batch(const FdJob* d_jobs, const int64_t* d_tasks, int32_t n_tasks, FdBoard* d_board,
                     const SpillArena& spill, int big_grid, hipStream_t s) {
    if (n_tasks <= 0) return;
    k_fd_reset_board<<<1, 256, 0, s>>>(d_board);
    TIP_HIP_TRY(hipGetLastError());
    FdJobs jobs{};
    jobs.list = d_jobs;
    const int grid = std::max(1, big_grid);
    k_fd_peel<<<grid, kFdThreads, 0, s>>>(jobs, d_tasks, n_tasks, d_board, spill);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_scatter_i64(const int64_t* by_rank, const int32_t* orig, int32_t n, int64_t* out, hipStream_t s) {
    if (n <= 0) return;
    k_scatter_i64<<<grid1(n), kT, 0, s>>>(by_rank, orig, n, out);
    TIP_HIP_TRY(hipGetLastError());
}

}  // namespace tip
