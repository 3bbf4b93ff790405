// Device-side canonicalisation of a bipartite COO edge list.
//
// Steps (Alg. 1, first two steps, plus duplicate merging):
//   1. check ids, 2. sort (a, b) keys and drop duplicates, 3. degrees,
//   4. per-side ranks by (degree descending, id ascending), 5. CSR A->B and
//   CSC B->A over ranks with every list sorted ascending, 6. for every edge
//   the position of its row vertex inside the neighbour's list, 7. the
//   joint-priority cut of every list used by the counting kernels.
#include "tip_ingest.h"

namespace tip {
namespace {

constexpr int kT = 256;

inline unsigned grid1(int64_t n) {
    int64_t g = (n + kT - 1) / kT;
    if (g < 1) g = 1;
    if (g > 262144) g = 262144;
    return (unsigned)g;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_validate(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t m,
                           int32_t n_a, int32_t n_b, int32_t* err) {
    GRID_STRIDE(i, m) {
        int32_t x = a[i], y = b[i];
        if (x < 0 || x >= n_a || y < 0 || y >= n_b) atomicOr(err, 1);
    }
}

__global__ void k_pair_keys(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t m,
                            int32_t n_b, uint64_t* keys, int32_t* vals) {
    GRID_STRIDE(i, m) {
        keys[i] = (uint64_t)a[i] * (uint64_t)n_b + (uint64_t)b[i];
        vals[i] = 0;
    }
}

__global__ void k_unique_flags(const uint64_t* __restrict__ keys, int64_t m, int64_t* flags) {
    GRID_STRIDE(i, m) { flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0; }
}

// Scatter the first key of each run; `pos` is the exclusive scan of flags.
__global__ void k_unique_compact(const uint64_t* __restrict__ keys, const int64_t* __restrict__ pos,
                                 int64_t m, int32_t n_b, int32_t* ea, int32_t* eb, int64_t* m_out) {
    GRID_STRIDE(i, m) {
        const bool first = (i == 0 || keys[i] != keys[i - 1]);
        if (first) {
            const int64_t p = pos[i];
            ea[p] = (int32_t)(keys[i] / (uint64_t)n_b);
            eb[p] = (int32_t)(keys[i] % (uint64_t)n_b);
        }
        if (i == m - 1) *m_out = pos[i] + (first ? 1 : 0);
    }
}

// ea is sorted, so side A's degrees are counted per run of equal ids inside
// each wave (one atomic per run piece); side B's ids are in no order.  The
// loop's trip count is uniform across each wave.
__global__ void k_degrees(const int32_t* __restrict__ ea, const int32_t* __restrict__ eb, const int64_t* m_p,
                          int32_t* deg_a, int32_t* deg_b) {
    const int64_t m = *m_p;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        int32_t a = -1, x = 0;
        if (i < m) {
            a = ea[i];
            x = 1;
            atomicAdd(&deg_b[eb[i]], 1);
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t y = __shfl_up(x, d, 64);
            const int32_t ay = __shfl_up(a, d, 64);
            if (lane >= d && ay == a) x += y;
        }
        const int32_t an = __shfl_down(a, 1, 64);
        if (a >= 0 && (lane == 63 || an != a)) atomicAdd(&deg_a[a], x);
    }
}

// key = (n_other - degree) << 32 | id: ascending key order is degree
// descending, ties by ascending id.
__global__ void k_rank_keys(const int32_t* __restrict__ deg, int32_t n, int32_t n_other, uint64_t* keys,
                            int32_t* vals) {
    GRID_STRIDE(i, (int64_t)n) {
        keys[i] = ((uint64_t)(uint32_t)(n_other - deg[i]) << 32) | (uint64_t)(uint32_t)i;
        vals[i] = (int32_t)i;
    }
}

// orig[r] = id of rank r (the sorted values); rank[id] = r; degr[r] = degree.
__global__ void k_rank_finish(const int32_t* __restrict__ sorted_ids, int32_t n, const int32_t* __restrict__ deg,
                              int32_t* orig, int32_t* rank, int32_t* degr, int64_t* degr64) {
    GRID_STRIDE(r, (int64_t)n) {
        const int32_t id = sorted_ids[r];
        orig[r] = id;
        rank[id] = (int32_t)r;
        degr[r] = deg[id];
        degr64[r] = deg[id];
    }
}

__global__ void k_relabel_keys(const int32_t* __restrict__ ea, const int32_t* __restrict__ eb, const int64_t* m_p,
                               const int32_t* __restrict__ rank_a, const int32_t* __restrict__ rank_b,
                               int32_t n_b, uint64_t* keys, int32_t* vals) {
    const int64_t m = *m_p;
    GRID_STRIDE(i, m) {
        keys[i] = (uint64_t)rank_a[ea[i]] * (uint64_t)n_b + (uint64_t)rank_b[eb[i]];
        vals[i] = 0;
    }
}

// After the CSR sort: a_adj[p] = B rank; build the CSC keys with the CSR
// position as the value.
__global__ void k_csr_fill(const uint64_t* __restrict__ keys, const int64_t* m_p, int32_t n_a, int32_t n_b,
                           int32_t* a_adj, int32_t* a_row, uint64_t* ckeys, int32_t* cvals) {
    const int64_t m = *m_p;
    GRID_STRIDE(p, m) {
        const uint64_t k = keys[p];
        const uint64_t ra = k / (uint64_t)n_b, rb = k % (uint64_t)n_b;
        a_adj[p] = (int32_t)rb;
        a_row[p] = (int32_t)ra;
        ckeys[p] = rb * (uint64_t)n_a + ra;
        cvals[p] = (int32_t)p;
    }
}

__global__ void k_csc_fill(const uint64_t* __restrict__ ckeys, const int32_t* __restrict__ cvals,
                           const int64_t* m_p, int32_t n_a, const int64_t* __restrict__ a_off,
                           const int64_t* __restrict__ b_off, int32_t* b_adj, int32_t* b_row, int32_t* a_rev,
                           int32_t* b_rev) {
    const int64_t m = *m_p;
    GRID_STRIDE(q, m) {
        const uint64_t k = ckeys[q];
        const int64_t rb = (int64_t)(k / (uint64_t)n_a), ra = (int64_t)(k % (uint64_t)n_a);
        const int64_t p = cvals[q];
        b_adj[q] = (int32_t)ra;
        b_row[q] = (int32_t)rb;
        a_rev[p] = (int32_t)(q - b_off[rb]);
        b_rev[q] = (int32_t)(p - a_off[ra]);
    }
}

// Joint priority order over U and V: degree descending, then original U
// before original V (ties cannot occur across a side with equal ids since
// the sides differ).  cut[x] = number of leading entries of N_x (sorted by
// the other side's rank, i.e. degree descending) that precede x.
__global__ void k_cut(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int32_t n,
                      const int32_t* __restrict__ deg_self, const int32_t* __restrict__ deg_other,
                      int32_t other_is_u, int32_t* cut) {
    GRID_STRIDE(x, (int64_t)n) {
        const int32_t d = deg_self[x];
        int64_t lo = off[x], hi = off[x + 1];
        const int64_t base = lo;
        // first entry y that does not precede x
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            const int32_t dy = deg_other[adj[mid]];
            const bool before = dy > d || (dy == d && other_is_u);
            if (before) lo = mid + 1;
            else hi = mid;
        }
        cut[x] = (int32_t)(lo - base);
    }
}

int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

}  // namespace

void ingest_alloc(Arena& ar, int32_t n_a, int32_t n_b, int64_t m, IngestBuffers& ib) {
    const int64_t n_max = std::max<int64_t>({(int64_t)n_a, (int64_t)n_b, m, 1});
    ib.keys = ar.take<uint64_t>(n_max);
    ib.keys2 = ar.take<uint64_t>(n_max);
    ib.vals = ar.take<int32_t>(n_max);
    ib.vals2 = ar.take<int32_t>(n_max);
    ib.flags = ar.take<int64_t>(n_max);
    ib.hist = ar.take<int64_t>(radix_hist_elems(n_max));
    ib.scan_tmp = ar.take<int64_t>(std::max(scan_tmp_elems(radix_hist_elems(n_max)),
                                            scan_tmp_elems(n_max + 1)) + 1);
    ib.ea = ar.take<int32_t>(std::max<int64_t>(m, 1));
    ib.eb = ar.take<int32_t>(std::max<int64_t>(m, 1));
    ib.deg_a = ar.take<int32_t>(std::max<int32_t>(n_a, 1));
    ib.deg_b = ar.take<int32_t>(std::max<int32_t>(n_b, 1));
    ib.rank_a = ar.take<int32_t>(std::max<int32_t>(n_a, 1));
    ib.rank_b = ar.take<int32_t>(std::max<int32_t>(n_b, 1));
    ib.m_dev = ar.take<int64_t>(4);
    ib.err = ar.take<int32_t>(4);
}

void graph_alloc(Arena& ar, int32_t n_a, int32_t n_b, int64_t m, DevGraph& g, GraphAux& aux) {
    g.n_a = n_a;
    g.n_b = n_b;
    const int64_t mm = std::max<int64_t>(m, 1);
    g.a_off = ar.take<int64_t>((int64_t)n_a + 1);
    g.b_off = ar.take<int64_t>((int64_t)n_b + 1);
    g.a_adj = ar.take<int32_t>(mm);
    g.b_adj = ar.take<int32_t>(mm);
    g.a_rev = ar.take<int32_t>(mm);
    g.b_rev = ar.take<int32_t>(mm);
    g.a_row = ar.take<int32_t>(mm);
    g.b_row = ar.take<int32_t>(mm);
    g.a_cut = ar.take<int32_t>(std::max<int32_t>(n_a, 1));
    g.b_cut = ar.take<int32_t>(std::max<int32_t>(n_b, 1));
    g.a_orig = ar.take<int32_t>(std::max<int32_t>(n_a, 1));
    g.b_orig = ar.take<int32_t>(std::max<int32_t>(n_b, 1));
    aux.deg_a = ar.take<int32_t>(std::max<int32_t>(n_a, 1));
    aux.deg_b = ar.take<int32_t>(std::max<int32_t>(n_b, 1));
    aux.deg_a64 = ar.take<int64_t>((int64_t)n_a + 1);
    aux.deg_b64 = ar.take<int64_t>((int64_t)n_b + 1);
}

// Builds the canonical graph from device COO arrays (a = decomposed side).
// Returns false if an id is out of range (nothing else is meaningful then).
bool ingest(const int32_t* d_a, const int32_t* d_b, int32_t n_a, int32_t n_b, int64_t m, bool a_is_u,
            IngestBuffers& ib, DevGraph& g, GraphAux& aux, hipStream_t s) {
    g.n_a = n_a;
    g.n_b = n_b;
    TIP_HIP_TRY(hipMemsetAsync(ib.err, 0, sizeof(int32_t), s));
    TIP_HIP_TRY(hipMemsetAsync(ib.m_dev, 0, sizeof(int64_t), s));
    if (m > 0) {
        k_validate<<<grid1(m), kT, 0, s>>>(d_a, d_b, m, n_a, n_b, ib.err);
        TIP_HIP_TRY(hipGetLastError());
        int32_t err = 0;
        TIP_HIP_TRY(hipMemcpyAsync(&err, ib.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        if (err) return false;

        // 2. duplicate merging
        k_pair_keys<<<grid1(m), kT, 0, s>>>(d_a, d_b, m, n_b, ib.keys, ib.vals);
        TIP_HIP_TRY(hipGetLastError());
        const int pair_bits = bits_for((uint64_t)n_a * (uint64_t)n_b);
        radix_sort_pairs(ib.keys, ib.vals, ib.keys2, ib.vals2, m, pair_bits, ib.hist, ib.scan_tmp, s);
        k_unique_flags<<<grid1(m), kT, 0, s>>>(ib.keys, m, ib.flags);
        TIP_HIP_TRY(hipGetLastError());
        scan_exclusive_i64(ib.flags, ib.flags, m, ib.scan_tmp, s);
        k_unique_compact<<<grid1(m), kT, 0, s>>>(ib.keys, ib.flags, m, n_b, ib.ea, ib.eb, ib.m_dev);
        TIP_HIP_TRY(hipGetLastError());
    }
    int64_t mu = 0;
    TIP_HIP_TRY(hipMemcpyAsync(&mu, ib.m_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TIP_HIP_TRY(hipStreamSynchronize(s));
    g.m = mu;

    // 3. degrees
    fill_i32(ib.deg_a, 0, n_a, s);
    fill_i32(ib.deg_b, 0, n_b, s);
    if (mu > 0) {
        k_degrees<<<grid1(mu), kT, 0, s>>>(ib.ea, ib.eb, ib.m_dev, ib.deg_a, ib.deg_b);
        TIP_HIP_TRY(hipGetLastError());
    }
    // 4. ranks per side
    auto rank_side = [&](const int32_t* deg, int32_t n, int32_t n_other, int32_t* orig, int32_t* rank,
                         int32_t* degr, int64_t* degr64) {
        if (n <= 0) return;
        k_rank_keys<<<grid1(n), kT, 0, s>>>(deg, n, n_other, ib.keys, ib.vals);
        TIP_HIP_TRY(hipGetLastError());
        const int rbits = 32 + bits_for((uint64_t)n_other);
        radix_sort_pairs(ib.keys, ib.vals, ib.keys2, ib.vals2, n, rbits, ib.hist, ib.scan_tmp, s);
        k_rank_finish<<<grid1(n), kT, 0, s>>>(ib.vals, n, deg, orig, rank, degr, degr64);
        TIP_HIP_TRY(hipGetLastError());
    };
    rank_side(ib.deg_a, n_a, n_b, g.a_orig, ib.rank_a, aux.deg_a, aux.deg_a64);
    rank_side(ib.deg_b, n_b, n_a, g.b_orig, ib.rank_b, aux.deg_b, aux.deg_b64);

    // 5. offsets from rank-ordered degrees
    fill_i64(aux.deg_a64 + n_a, 0, 1, s);
    fill_i64(aux.deg_b64 + n_b, 0, 1, s);
    scan_exclusive_i64(aux.deg_a64, g.a_off, (int64_t)n_a + 1, ib.scan_tmp, s);
    scan_exclusive_i64(aux.deg_b64, g.b_off, (int64_t)n_b + 1, ib.scan_tmp, s);

    if (mu > 0) {
        // CSR A -> B
        k_relabel_keys<<<grid1(mu), kT, 0, s>>>(ib.ea, ib.eb, ib.m_dev, ib.rank_a, ib.rank_b, n_b, ib.keys,
                                                 ib.vals);
        TIP_HIP_TRY(hipGetLastError());
        const int pair_bits = bits_for((uint64_t)n_a * (uint64_t)n_b);
        radix_sort_pairs(ib.keys, ib.vals, ib.keys2, ib.vals2, mu, pair_bits, ib.hist, ib.scan_tmp, s);
        // CSC B -> A, carrying CSR positions
        k_csr_fill<<<grid1(mu), kT, 0, s>>>(ib.keys, ib.m_dev, n_a, n_b, g.a_adj, g.a_row, ib.keys2, ib.vals2);
        TIP_HIP_TRY(hipGetLastError());
        radix_sort_pairs(ib.keys2, ib.vals2, ib.keys, ib.vals, mu, pair_bits, ib.hist, ib.scan_tmp, s);
        k_csc_fill<<<grid1(mu), kT, 0, s>>>(ib.keys2, ib.vals2, ib.m_dev, n_a, g.a_off, g.b_off, g.b_adj,
                                             g.b_row, g.a_rev, g.b_rev);
        TIP_HIP_TRY(hipGetLastError());
    }
    // 7. joint-priority cuts (original U before original V on equal degree)
    if (n_a > 0) {
        k_cut<<<grid1(n_a), kT, 0, s>>>(g.a_off, g.a_adj, n_a, aux.deg_a, aux.deg_b, a_is_u ? 0 : 1, g.a_cut);
        TIP_HIP_TRY(hipGetLastError());
    }
    if (n_b > 0) {
        k_cut<<<grid1(n_b), kT, 0, s>>>(g.b_off, g.b_adj, n_b, aux.deg_b, aux.deg_a, a_is_u ? 1 : 0, g.b_cut);
        TIP_HIP_TRY(hipGetLastError());
    }
    return true;
}

}  // namespace tip
