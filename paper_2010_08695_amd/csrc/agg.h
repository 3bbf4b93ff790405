// Device-side wedge aggregation shared by the counting, peeling and
// fine-grained kernels.
//
// For one vertex x, the wedges (x, y, z) are the entries z of the neighbour
// lists N_y, y in N_x.  The number of wedges that end at z is c(x, z), and the
// butterflies x shares with z are C(c(x, z), 2) (Alg. 2, update).  Almost all
// z are reached once (c = 1, no butterfly), so the workgroup path keeps one
// bit per key in LDS and only keys reached again go to a small LDS hash table
// of repeat counts; keys that do not fit there within a bounded probe go to a
// dense per-workgroup count array in HBM.  A key is always found in exactly
// one of the two places: slots only fill, so a key's probe sequence that is
// full once stays full.
//
// The wave path (few wedges) keeps every key in a per-wave LDS hash table.
#pragma once

#include "tip_common.h"

namespace tip {

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
}

// Appends `val` to list[*counter ...] for every lane with pred; one atomic
// per wave.  Must be reached by all lanes of the wave.
__device__ inline void wave_append(bool pred, int32_t val, int32_t* list, int32_t* counter) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
    base = __shfl(base, leader, kWave);
    if (pred) list[base + __popcll(mask & lanemask_lt())] = val;
}

__device__ inline int64_t wave_sum_i64(int64_t x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

__device__ inline int64_t wave_min_i64(int64_t x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        int64_t y = __shfl_xor(x, d, kWave);
        x = y < x ? y : x;
    }
    return x;
}

template <int NT>
__device__ inline int64_t wave_incl_scan_i64(int64_t x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline int32_t wave_incl_scan_i32(int32_t x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Lower bound of `key` in the sorted range adj[lo, hi).
__device__ inline int64_t lower_bound_i32(const int32_t* __restrict__ adj, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (adj[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Workgroup path
// ---------------------------------------------------------------------------
struct BigLds {
    uint32_t bm[kBmWords];
    unsigned long long rep[kRepSlots];
    int64_t sbeg[kGroup];
    int64_t pre[kGroup + 1];
    int64_t acc[kGroup];
    int64_t red[kBigThreads / kWave];
    int32_t spill_n;
    int32_t flag;
    int64_t bcast;
};

struct Spill {
    int32_t* dense;  // [kBmBits]
    int32_t* list;   // [kBmBits]
};

__device__ inline void rep_insert(BigLds& L, const Spill& sp, uint32_t k) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & (kRepSlots - 1);
#pragma unroll 1
    for (int p = 0; p < kRepProbe; ++p) {
        unsigned long long* slot = &L.rep[(h + p) & (kRepSlots - 1)];
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

// c(x, z) for a tile-relative key that has been marked: 1 + repeats.
__device__ inline int32_t rep_lookup(const BigLds& L, const Spill& sp, bool spilled, uint32_t k) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & (kRepSlots - 1);
    bool full = true;
#pragma unroll 1
    for (int p = 0; p < kRepProbe; ++p) {
        const unsigned long long cur = L.rep[(h + p) & (kRepSlots - 1)];
        if (cur == 0) {
            full = false;
            break;
        }
        if ((cur & 0xffffffff00000000ull) == tag) return 1 + (int32_t)(cur & 0xffffffffull);
    }
    if (full && spilled) return 1 + sp.dense[k];
    return 1;
}

__device__ inline void bm_mark(BigLds& L, const Spill& sp, uint32_t k) {
    const uint32_t bit = 1u << (k & 31);
    const uint32_t old = atomicOr(&L.bm[k >> 5], bit);
    if (old & bit) rep_insert(L, sp, k);
}

// Block reduction (all threads get the sum).
template <int NT>
__device__ inline int64_t block_sum_i64(BigLds& L, int64_t x) {
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

template <int NT>
__device__ inline int64_t block_min_i64(BigLds& L, int64_t x) {
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

// Exclusive scan of per-slice lengths held by threads j < gs into L.pre
// (L.pre[gs] = total).  Returns the total.
template <int NT>
__device__ inline int64_t block_scan_lengths(BigLds& L, int gs, int64_t len) {
    static_assert(kGroup <= NT, "one slice per thread");
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wid = tid / kWave;
    const int64_t x = tid < gs ? len : 0;
    const int64_t inc = wave_incl_scan_i64<NT>(x);
    __syncthreads();
    if (lane == kWave - 1) L.red[wid] = inc;
    __syncthreads();
    int64_t off = 0;
    int64_t tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        const int64_t v = L.red[w];
        off += w < wid ? v : 0;
        tot += v;
    }
    if (tid < gs) L.pre[tid] = off + inc - x;
    if (tid == 0) L.pre[gs] = tot;
    __syncthreads();
    return tot;
}

// Index j of the slice holding flattened wedge i: the largest j with pre[j] <= i.
__device__ inline int find_slice(const BigLds& L, int gs, int64_t i) {
    int lo = 0, hi = gs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int NT>
__device__ inline void bm_clear(BigLds& L, int64_t nkeys) {
    const int64_t words = (nkeys + 31) >> 5;
    for (int64_t w = threadIdx.x; w < words; w += NT) L.bm[w] = 0;
    for (int s = threadIdx.x; s < kRepSlots; s += NT) L.rep[s] = 0;
}

// ---------------------------------------------------------------------------
// Wave path: per-wave hash table of (key + 1) << 32 | count.
// ---------------------------------------------------------------------------
struct WaveLds {
    unsigned long long tab[kSmallSlots];
    int64_t sbeg[kWave];
    int64_t pre[kWave + 1];
    int64_t acc[kWave];
};

// Slots used for a vertex with `wedges` wedges: a power of two >= 2 * wedges
// (at least one per lane), so the table stays at most half full.
__device__ inline uint32_t wave_slots(int64_t wedges) {
    uint32_t s = kWave;
    while (s < kSmallSlots && (int64_t)s < 2 * wedges) s <<= 1;
    return s;
}

__device__ inline void wave_insert(WaveLds& W, uint32_t k, uint32_t mask = kSmallSlots - 1) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & mask;
#pragma unroll 1
    for (;;) {
        unsigned long long* slot = &W.tab[h];
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

__device__ inline int32_t wave_lookup(const WaveLds& W, uint32_t k, uint32_t mask = kSmallSlots - 1) {
    const unsigned long long tag = (unsigned long long)(k + 1) << 32;
    uint32_t h = hash32(k) & mask;
#pragma unroll 1
    for (uint32_t p = 0; p <= mask; ++p) {
        const unsigned long long cur = W.tab[h];
        if (cur == 0) return 0;
        if ((cur & 0xffffffff00000000ull) == tag) return (int32_t)(cur & 0xffffffffull);
        h = (h + 1) & mask;
    }
    return 0;
}

// Wave exclusive scan of lane lengths into W.pre (W.pre[64] = total).
__device__ inline int64_t wave_scan_lengths(WaveLds& W, int64_t len) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t inc = wave_incl_scan_i64<kWave>(len);
    W.pre[lane] = inc - len;
    const int64_t tot = __shfl(inc, kWave - 1, kWave);
    if (lane == 0) W.pre[kWave] = tot;
    wave_sync();
    return tot;
}

__device__ inline int wave_find_slice(const WaveLds& W, int gs, int64_t i) {
    int lo = 0, hi = gs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (W.pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace tip
