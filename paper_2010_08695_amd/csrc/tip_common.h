// Internal declarations shared by the libtip translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <string>

namespace tip {

// ---------------------------------------------------------------------------
// Tunables.  The bitmap covers BM_BITS keys per tile (one bit per same-side
// vertex); the repeat table keeps keys seen at least twice.
// ---------------------------------------------------------------------------
constexpr int kWave = 64;
constexpr int kBigThreads = 1024;          // threads of the workgroup-per-vertex kernels
constexpr int kBmBits = 1 << 20;           // keys per bitmap tile (128 KiB of LDS)
constexpr int kBmWords = kBmBits / 32;
constexpr int kRepSlots = 2048;            // LDS repeat-table slots (16 KiB)
constexpr int kRepProbe = 16;              // bounded probing before spilling to HBM
constexpr int kGroup = 512;                // neighbour slices staged per pass
constexpr int kSmallThreads = 256;         // threads of the wave-per-vertex kernels
constexpr int kSmallSlots = 1024;          // per-wave hash slots (8 KiB)
constexpr int64_t kSmallMaxWedges = 448;   // wave path handles <= this many wedges

// Coarse-grained update kernels (see peel.hip).
constexpr int kBmThreads = 1024;           // threads of the bitmap-path workgroup (one per CU)
constexpr int kBmTile = 1 << 19;           // keys per bitmap-path tile (64 KiB of bits)
constexpr int kBmRep = 8192;               // bitmap-path repeat slots (64 KiB)
constexpr int kBmRuns = 1024;              // neighbour runs staged per pass by the bitmap path
constexpr int kUnit = 128;                 // consecutive list entries per traversal unit
constexpr int kDenseThreads = 512;         // threads of the dense (vertex, key range) kernel
constexpr int kDenseLdsBytes = 65536;      // counter bytes per dense workgroup (two per CU)
// Update bins: wave path, bitmap path, and the dense path per counter width
// (2, 4, 8, 16, 32 bits) split into light and heavy vertices; a heavy vertex
// is cut into kHeavySplit times more (smaller) work items.
constexpr int kDenseKinds = 5;
constexpr int kBins = 2 + 2 * kDenseKinds;
constexpr int kBinWave = 0, kBinBitmap = 1;
constexpr int kDefaultDenseDiv = 1024;     // dense needs w[u] > n * bits / div (tip_opts.tune[0])
constexpr int64_t kDefaultBitmapMax = 2048;   // bitmap path up to this many wedges (tip_opts.tune[1])
constexpr int kApplyBatch = 4;             // (key, c) pairs a lane gathers before applying them
constexpr int64_t kItemWedges = 16384;     // a dense item of a light vertex has at most about this many wedges
constexpr int kHeavySplit = 8;
constexpr int kDensePasses = 4;            // key-range passes of one light dense work item
constexpr int64_t kDense16Stage = 4;       // 16-bit dense: wedges >= this * degree * key-range passes
constexpr int64_t kBmHubWedges = 16384;    // ... or more wedges than one bitmap workgroup takes without spilling
// CD lists are compacted at a range start once the entries of vertices
// assigned since the last compaction reach this share (per mille) of the
// entries left (tip_opts.tune[2]).
constexpr int64_t kDefaultCompactPermille = 125;

// Counter width (bits) of the dense kernel for a vertex of degree d: c(u, w)
// <= d_u must fit; 0 = too wide for the dense kernel.
__host__ __device__ inline int dense_bits(int64_t d) {
    return d <= 3 ? 2 : d <= 15 ? 4 : d <= 255 ? 8 : d <= 65535 ? 16 : d <= INT32_MAX ? 32 : 0;
}
__host__ __device__ inline int dense_kind(int bits) {
    return bits == 2 ? 0 : bits == 4 ? 1 : bits == 8 ? 2 : bits == 16 ? 3 : 4;
}
__host__ __device__ inline int dense_bin_of_kind(int kind, bool heavy) { return 2 + 2 * kind + (heavy ? 1 : 0); }
__host__ __device__ inline int dense_bin(int bits, bool heavy) { return dense_bin_of_kind(dense_kind(bits), heavy); }

// Granularity (keys) of the per-list tile-bound table for a side of n keys:
// 16K keys, or coarser so that there are at most 512 tiles; but 32K keys (one
// tile of 16-bit dense counters fills a dense workgroup's LDS) while that
// keeps at most 2048 tiles, so that sides of up to 64M keys keep the 16-bit
// dense path.
inline int32_t dense_tile_keys(int64_t n) {
    int64_t t = 16384;
    while (t * 512 < n && !(t == 32768 && t * 2048 >= n)) t <<= 1;
    return (int32_t)t;
}

// Table tiles covered by one light dense work item of a given counter width:
// the keys whose counters fill kDenseLdsBytes, at least one tile, at most all.
inline int32_t dense_item_tiles(int bits, int32_t tk, int32_t ntt) {
    const int64_t k = (int64_t)kDenseLdsBytes * 8 / bits;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(ntt, k / tk));
}

constexpr int32_t kLive = -1;              // subset id of a vertex not yet assigned

// 64-bit hash-table slot: (key + 1) << 32 | count; 0 = empty.
__host__ __device__ inline uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__host__ __device__ inline int64_t choose2(int64_t c) { return c * (c - 1) / 2; }

// Device view of a canonical graph.  "A" is the side being decomposed (or the
// first side when counting), "B" the other.  Vertex ids on each side are
// local ranks by (degree descending, original id ascending); every list is
// sorted ascending.
struct DevGraph {
    int32_t n_a = 0, n_b = 0;
    int64_t m = 0;
    int64_t* a_off = nullptr;   // [n_a+1]
    int32_t* a_adj = nullptr;   // [m]  B ranks
    int64_t* b_off = nullptr;   // [n_b+1]
    int32_t* b_adj = nullptr;   // [m]  A ranks
    int32_t* a_cut = nullptr;   // [n_a] leading entries of N_x with higher joint priority than x
    int32_t* b_cut = nullptr;   // [n_b]
    int32_t* a_rev = nullptr;   // [m]  position of the row vertex inside its neighbour's list
    int32_t* b_rev = nullptr;   // [m]
    int32_t* a_orig = nullptr;  // [n_a] rank -> original id
    int32_t* b_orig = nullptr;  // [n_b]
    int32_t* a_row = nullptr;   // [m]  row (A rank) of each CSR position
    int32_t* b_row = nullptr;   // [m]  row (B rank) of each CSC position
};

// Per-workgroup spill buffers (HBM) for repeat keys that do not fit in LDS.
// Workgroup b uses dense/list + b * stride; stride >= the largest tile of
// keys any kernel uses on this graph.  `dense` is all zero between uses.
struct SpillArena {
    int32_t* dense = nullptr;    // [slots * stride] repeat counts
    int32_t* list = nullptr;     // [slots * stride] spilled keys
    int64_t stride = 0;
    int32_t slots = 0;           // number of workgroup slots (= resident workgroups)
};

// Error reporting (thread-local message behind tip_last_error).
void set_error(const std::string& msg);
const char* last_error();

#define TIP_HIP_TRY(expr)                                                        \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            throw ::tip::HipFailure(std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                        \
    } while (0)

struct HipFailure {
    std::string msg;
    explicit HipFailure(std::string m) : msg(std::move(m)) {}
};
struct AllocFailure {
    std::string msg;
    explicit AllocFailure(std::string m) : msg(std::move(m)) {}
};
struct InvalidArg {
    std::string msg;
    explicit InvalidArg(std::string m) : msg(std::move(m)) {}
};

// ---------------------------------------------------------------------------
// Launch wrappers implemented in the kernel translation units.
// ---------------------------------------------------------------------------

// util.hip
void scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
// Ping-pongs between the two buffers; on return the sorted data is in
// (keys, vals).  tmp_keys/tmp_vals hold n entries; hist holds radix_hist_elems(n).
void radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* tmp_keys, int32_t* tmp_vals,
                      int64_t n, int bits, int64_t* hist, int64_t* scan_tmp, hipStream_t s);
size_t radix_hist_elems(int64_t n);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void iota_i32(int32_t* p, int64_t n, hipStream_t s);

}  // namespace tip
