// Internal: small device/host helpers shared by the kernel translation units.
#pragma once

#include "agg.h"
#include "tip_kernels.h"

namespace tip {

constexpr int kT = 256;

inline unsigned grid1(int64_t n, int64_t cap = 262144) {
    int64_t g = (n + kT - 1) / kT;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

inline int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
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

}  // namespace tip
