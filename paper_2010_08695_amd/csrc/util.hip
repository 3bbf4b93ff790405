// Device-wide building blocks: exclusive scan, stable LSD radix sort, fills.
#include "tip_common.h"

namespace tip {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

__device__ inline int64_t wave_incl_scan(int64_t x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and stores the block total in `total` (same value in every thread).
template <int NT>
__device__ int64_t block_excl_scan(int64_t x, int64_t& total) {
    constexpr int NW = NT / kWave;
    __shared__ int64_t wsum[NW];
    __shared__ int64_t wtot;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int64_t inc = wave_incl_scan(x);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        const int64_t v = lane < NW ? wsum[lane] : 0;
        const int64_t vi = wave_incl_scan(v);
        if (lane < NW) wsum[lane] = vi - v;
        if (lane == NW - 1) wtot = vi;
    }
    __syncthreads();
    const int64_t res = wsum[wid] + inc - x;
    total = wtot;
    __syncthreads();
    return res;
}

__global__ void __launch_bounds__(kScanThreads)
scan_tile_sums(const int64_t* __restrict__ in, int64_t* __restrict__ sums, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    int64_t tot;
    block_excl_scan<kScanThreads>(s, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads)
scan_tile_apply(const int64_t* in, int64_t* out, const int64_t* __restrict__ offs, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_excl_scan<kScanThreads>(s, tot);
    ex += offs ? offs[blockIdx.x] : 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = ex;
        ex += v[i];
    }
}

__global__ void __launch_bounds__(kSortThreads)
radix_hist_kernel(const uint64_t* __restrict__ keys, int64_t n, int shift, int64_t* __restrict__ hist,
                  int64_t nblocks) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int i = 0; i < kSortItems; ++i) {
        int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                     uint64_t* __restrict__ okeys, int32_t* __restrict__ ovals, int64_t n, int shift,
                     const int64_t* __restrict__ hist, int64_t nblocks) {
    __shared__ int64_t base[256];
    __shared__ int32_t running[256];
    __shared__ int32_t wcnt[kSortThreads / kWave][256];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    base[tid] = hist[(int64_t)tid * nblocks + blockIdx.x];
    running[tid] = 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
#pragma unroll
        for (int w = 0; w < kSortThreads / kWave; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t idx = tile + (int64_t)it * kSortThreads + tid;
        const bool valid = idx < n;
        uint64_t key = 0;
        int32_t val = 0;
        int digit = 0;
        if (valid) {
            key = keys[idx];
            val = vals[idx];
            digit = (int)((key >> shift) & 255);
        }
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1;
            const uint64_t bb = __ballot(valid && bit);
            match &= bit ? bb : ~bb;
        }
        const int rank = __popcll(match & lt_mask);
        if (valid && rank == 0) wcnt[wid][digit] = __popcll(match);
        __syncthreads();
        {
            int32_t r = running[tid];
#pragma unroll
            for (int w = 0; w < kSortThreads / kWave; ++w) {
                int32_t c = wcnt[w][tid];
                wcnt[w][tid] = r;
                r += c;
            }
            running[tid] = r;
        }
        __syncthreads();
        if (valid) {
            const int64_t dst = base[digit] + wcnt[wid][digit] + rank;
            okeys[dst] = key;
            ovals[dst] = val;
        }
        __syncthreads();
    }
}

__global__ void fill_i64_kernel(int64_t* p, int64_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void iota_i32_kernel(int32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

int grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

size_t scan_tmp_elems(int64_t n) {
    if (n <= kScanTile) return 0;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)nb + scan_tmp_elems(nb);
}

void scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        scan_tile_apply<<<1, kScanThreads, 0, s>>>(in, out, nullptr, n);
        TIP_HIP_TRY(hipGetLastError());
        return;
    }
    int64_t* sums = tmp;
    scan_tile_sums<<<(unsigned)nb, kScanThreads, 0, s>>>(in, sums, n);
    TIP_HIP_TRY(hipGetLastError());
    scan_exclusive_i64(sums, sums, nb, tmp + nb, s);
    scan_tile_apply<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, sums, n);
    TIP_HIP_TRY(hipGetLastError());
}

size_t radix_hist_elems(int64_t n) {
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb < 1) nb = 1;
    return (size_t)(256 * nb);
}

void radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* tmp_keys, int32_t* tmp_vals,
                      int64_t n, int bits, int64_t* hist, int64_t* scan_tmp, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    uint64_t* ka = keys;
    int32_t* va = vals;
    uint64_t* kb = tmp_keys;
    int32_t* vb = tmp_vals;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_hist_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(ka, n, shift, hist, nb);
        TIP_HIP_TRY(hipGetLastError());
        scan_exclusive_i64(hist, hist, 256 * nb, scan_tmp, s);
        radix_scatter_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(ka, va, kb, vb, n, shift, hist, nb);
        TIP_HIP_TRY(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
        ++passes;
    }
    if (passes & 1) {
        TIP_HIP_TRY(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        TIP_HIP_TRY(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
}

void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    fill_i64_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    TIP_HIP_TRY(hipGetLastError());
}
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    fill_i32_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    TIP_HIP_TRY(hipGetLastError());
}
void iota_i32(int32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    iota_i32_kernel<<<grid_for(n, 256), 256, 0, s>>>(p, n);
    TIP_HIP_TRY(hipGetLastError());
}

}  // namespace tip
