// Fine-grained decomposition (Alg. 4) and output scatter.
#include "kern_util.h"

namespace tip {
namespace {
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
// edges of the induced subgraph G_i seen from v (Alg. 4 induced subgraph),
// and the induced wedges per subset (task_w) and per vertex (fd_w).  Subset
// sums gather in LDS when there are few subsets (lds_tw); per-vertex sums are
// segmented wave sums over the CSR rows.  Wave-uniform grid-stride loop.
__global__ void k_fd_slices(DevGraph g, const int32_t* __restrict__ state, const uint64_t* __restrict__ pkeys,
                            int32_t S, const int32_t* __restrict__ fd_pos, int64_t* fd_beg, int32_t* fd_len,
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
            const int32_t v = g.a_adj[p];
            const int32_t s = state[u];
            const uint64_t k0 = (uint64_t)v * (uint64_t)S + (uint64_t)s;
            const int64_t lo = lower_bound_u64(pkeys, g.b_off[v], g.b_off[v + 1], k0);
            const int64_t hi = lower_bound_u64(pkeys, lo, g.b_off[v + 1], k0 + 1);
            fd_beg[p] = lo;
            fd_len[p] = (int32_t)(hi - lo);
            x = hi - lo > 1 ? hi - lo - 1 : 0;
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

// LDS of the fine-grained kernel.  The per-wave hash tables (light peeled
// vertices) and the bitmap + repeat table (heavy ones) are used in separate
// phases of a level and share storage; both are all zero between uses.
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
};

template <int NT>
__device__ inline int32_t fd_scan_i32(FdLds& L, int32_t x, int32_t& total) {
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

// One workgroup peels one subset at a time, taking subsets from the
// workload-sorted queue (dynamic allocation).  Inside a subset it runs
// bottom-up peeling level by level: the level is max(level, minimum live
// support), and every live vertex whose support is at most the level is
// peeled at that level (equal to one-at-a-time peeling, whatever the order).
// The vertices peeled at one level update the survivors concurrently: light
// ones one per wavefront with a private hash table, heavy ones one at a time
// with the whole workgroup and a key bitmap.
__global__ void __launch_bounds__(kFdThreads)
k_fd_peel(FdJobs jobs, const int64_t* __restrict__ tasks, int32_t n_tasks, int32_t* head, SpillArena spa) {
    __shared__ FdLds L;
    constexpr int NT = kFdThreads;
    constexpr int NW = NT / kWave;
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
        if (tid == 0) L.flag = atomicAdd(head, 1);
        __syncthreads();
        const int32_t t = L.flag;
        __syncthreads();
        if (t >= n_tasks) break;
        // one task = one subset of one graph: tasks[t] = job << 32 | subset,
        // or, for a single graph, its own workload-ordered subset list
        const FdJob& J = tasks ? jobs.list[tasks[t] >> 32] : jobs.one;
        const DevGraph& g = J.g;
        const FdBuffers& fb = J.fb;
        const int64_t* __restrict__ init = J.init;
        const int32_t sub = tasks ? (int32_t)(tasks[t] & 0xffffffffll) : fb.order[t];
        const int64_t P0 = fb.sub_off[sub];
        const int32_t n_i = (int32_t)(fb.sub_off[sub + 1] - P0);
        if (n_i == 0) continue;
        unsigned long long wedges = 0, pairs = 0, levels = 0, spills = 0;
        int32_t* lc = fb.lst[0] + P0;
        int32_t* ln = fb.lst[1] + P0;
        int32_t* pl = fb.lst[2] + P0;
        int32_t* ph = fb.lst[3] + P0;
        int64_t* sup = fb.supp_fd + P0;
        const int64_t* fw = fb.fd_w + P0;
        int32_t* alive = fb.alive + P0;
        const int32_t* vert = fb.fd_vert + P0;
        for (int32_t j = tid; j < n_i; j += NT) {
            lc[j] = j;
            sup[j] = init[vert[j]];
            alive[j] = 1;
        }
        __syncthreads();
        const bool multi = n_i > kFdBits;
        int32_t n_live = n_i;
        int64_t level = 0;
        while (n_live > 0) {
            int64_t mn = INT64_MAX;
            for (int32_t j = tid; j < n_live; j += NT) {
                const int64_t s = sup[lc[j]];
                mn = s < mn ? s : mn;
            }
            mn = fd_min<NT>(L, mn);
            level = mn > level ? mn : level;
            // peel every live vertex at or below the level; light ones (few
            // wedges inside the subset) and heavy ones go to separate lists,
            // vertices without support left need no update at all
            int32_t n_light = 0, n_heavy = 0, n_keep = 0;
            for (int32_t b0 = 0; b0 < n_live; b0 += NT) {
                const int32_t j = b0 + tid;
                int32_t x = 0;
                bool pe = false, ke = false, li = false, he = false;
                if (j < n_live) {
                    x = lc[j];
                    const int64_t sx = sup[x];
                    pe = sx <= level;
                    ke = !pe;
                    if (pe && sx > 0) {
                        he = fw[x] > kFdWaveMax;
                        li = !he;
                    }
                }
                int32_t tl, th, tk;
                const int32_t ol = fd_scan_i32<NT>(L, li ? 1 : 0, tl);
                const int32_t oh = fd_scan_i32<NT>(L, he ? 1 : 0, th);
                const int32_t ok = fd_scan_i32<NT>(L, ke ? 1 : 0, tk);
                if (pe) {
                    alive[x] = 0;
                    fb.theta[vert[x]] = level;
                }
                if (li) pl[n_light + ol] = x;
                if (he) ph[n_heavy + oh] = x;
                if (ke) ln[n_keep + ok] = x;
                n_light += tl;
                n_heavy += th;
                n_keep += tk;
            }
            __syncthreads();
            levels += tid == 0;
            // light peeled vertices: one per wave
            for (int32_t q = wid; q < n_light; q += NW) {
                const int32_t x = pl[q];
                const uint32_t slots = min<uint32_t>(kFdWaveSlots, wave_slots(fw[x]));
                const uint32_t mask = slots - 1;
                const int32_t ux = vert[x];
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
                    for (int64_t i = lane; i < tot; i += kWave) {
                        while (lo + 1 < gs && L.wpre[wid][lo + 1] <= i) ++lo;
                        const int32_t w = fb.pcsc[L.wsbeg[wid][lo] + (i - L.wpre[wid][lo])];
                        if (w != x) fd_wave_insert(tab, (uint32_t)w, mask);
                    }
                    if (lane == 0) wedges += (unsigned long long)(tot - gs);
                    wave_sync();
                }
                for (uint32_t s = lane; s < slots; s += kWave) {
                    const unsigned long long v = tab[s];
                    if (v) {
                        tab[s] = 0;
                        const int64_t c = (int64_t)(v & 0xffffffffull);
                        const int32_t w = (int32_t)((v >> 32) - 1);
                        if (c >= 2 && alive[w]) {
                            atomic_add_i64(&sup[w], -choose2(c));
                            ++pairs;
                        }
                    }
                }
                wave_sync();
            }
            __syncthreads();
            // heavy peeled vertices: one at a time with the whole workgroup
            for (int32_t q = 0; q < n_heavy; ++q) {
                const int32_t x = ph[q];
                const int32_t ux = vert[x];
                const int64_t e0 = g.a_off[ux], d = g.a_off[ux + 1] - e0;
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
                        int32_t tot32;
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
                        (void)tot32;
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
                    for (int s = tid; s < kFdRep; s += NT) {
                        const unsigned long long v = L.u.big.rep[s];
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
                    const int32_t words = (khi - klo + 31) >> 5;
                    for (int w = tid; w < words; w += NT) L.u.big.bm[w] = 0;
                    for (int s = tid; s < kFdRep; s += NT) L.u.big.rep[s] = 0;
                    if (tid == 0) L.spill_n = 0;
                    __syncthreads();
                }
            }
            int32_t* tmp = lc;
            lc = ln;
            ln = tmp;
            n_live = n_keep;
        }
        wedges = (unsigned long long)wave_sum_i64((int64_t)wedges);
        pairs = (unsigned long long)wave_sum_i64((int64_t)pairs);
        levels = (unsigned long long)wave_sum_i64((int64_t)levels);
        spills = (unsigned long long)wave_sum_i64((int64_t)spills);
        if (lane == 0) {
            if (wedges) atomicAdd(&J.ctl->wedges_fd, wedges);
            if (pairs) atomicAdd(&J.ctl->pair_updates, pairs);
            if (levels) atomicAdd(&J.ctl->fd_levels, levels);
            if (spills) atomicAdd(&J.ctl->spills, spills);
        }
    }
}

__global__ void k_scatter_i64(const int64_t* __restrict__ by_rank, const int32_t* __restrict__ orig, int32_t n,
                              int64_t* out) {
    GRID_STRIDE(r, (int64_t)n) out[orig[r]] = by_rank[r];
}

}  // namespace

int fd_occupancy() {
    int n = 0;
    TIP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fd_peel, kFdThreads, 0));
    return std::max(1, n);
}

void launch_fd_setup(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, uint64_t* tmp_keys,
                     int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp, uint64_t* keys_scratch,
                     int32_t* vals_scratch, hipStream_t s) {
    const int32_t n_a = g.n_a;
    fill_i64(fb.task_w, 0, S, s);
    if (n_a <= 0) return;
    // vertices grouped by subset, ascending rank inside each subset
    fill_i64(fb.sub_cnt, 0, (int64_t)S + 1, s);
    k_fd_vertex_keys<<<grid1(n_a), kT, 0, s>>>(pb.state, n_a, keys_scratch, fb.fd_vert, fb.sub_cnt);
    TIP_HIP_TRY(hipGetLastError());
    radix_sort_pairs(keys_scratch, fb.fd_vert, tmp_keys, tmp_vals, n_a, bits_for((uint64_t)S), hist, scan_tmp, s);
    scan_exclusive_i64(fb.sub_cnt, fb.sub_off, (int64_t)S + 1, scan_tmp, s);
    k_fd_positions<<<grid1(n_a), kT, 0, s>>>(fb.fd_vert, n_a, fb.fd_pos);
    TIP_HIP_TRY(hipGetLastError());
    fill_i64(fb.fd_w, 0, n_a, s);
    if (g.m > 0) {
        k_fd_csc_keys<<<grid1(g.m), kT, 0, s>>>(g, pb.state, fb.fd_pos, fb.sub_off, S, fb.pkeys, fb.pcsc);
        TIP_HIP_TRY(hipGetLastError());
        radix_sort_pairs(fb.pkeys, fb.pcsc, tmp_keys, tmp_vals, g.m,
                         bits_for((uint64_t)g.n_b * (uint64_t)S), hist, scan_tmp, s);
        const int lds_tw = S <= 4096 ? 1 : 0;
        k_fd_slices<<<grid1(g.m, 2048), kT, lds_tw ? sizeof(unsigned long long) * (size_t)S : 0, s>>>(
            g, pb.state, fb.pkeys, S, fb.fd_pos, fb.fd_beg, fb.fd_len, fb.task_w, fb.fd_w, lds_tw);
        TIP_HIP_TRY(hipGetLastError());
    }
    k_fd_order<<<1, 1024, 0, s>>>(fb.task_w, S, fb.order);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_fd(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, Ctl* ctl, const SpillArena& spill,
               int big_grid, uint64_t* tmp_keys, int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp,
               uint64_t* keys_scratch, int32_t* vals_scratch, hipStream_t s) {
    if (g.n_a <= 0) return;
    launch_fd_setup(g, pb, fb, S, tmp_keys, tmp_vals, hist, scan_tmp, keys_scratch, vals_scratch, s);
    k_fd_reset_head<<<1, 1, 0, s>>>(ctl);
    TIP_HIP_TRY(hipGetLastError());
    FdJobs jobs{};
    jobs.one = FdJob{g, fb, pb.init, ctl};
    const int grid = std::max(1, std::min<int>(S, big_grid));
    k_fd_peel<<<grid, kFdThreads, 0, s>>>(jobs, nullptr, S, &ctl->fd_head, spill);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_fd_batch(const FdJob* d_jobs, const int64_t* d_tasks, int32_t n_tasks, int32_t* d_head,
                     const SpillArena& spill, int big_grid, hipStream_t s) {
    if (n_tasks <= 0) return;
    fill_i32(d_head, 0, 1, s);
    FdJobs jobs{};
    jobs.list = d_jobs;
    const int grid = std::max(1, std::min<int>(n_tasks, big_grid));
    k_fd_peel<<<grid, kFdThreads, 0, s>>>(jobs, d_tasks, n_tasks, d_head, spill);
    TIP_HIP_TRY(hipGetLastError());
}

void launch_scatter_i64(const int64_t* by_rank, const int32_t* orig, int32_t n, int64_t* out, hipStream_t s) {
    if (n <= 0) return;
    k_scatter_i64<<<grid1(n), kT, 0, s>>>(by_rank, orig, n, out);
    TIP_HIP_TRY(hipGetLastError());
}

}  // namespace tip
