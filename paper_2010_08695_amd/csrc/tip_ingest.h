// Internal: device workspace arena and the graph-ingest entry points.
#pragma once

#include <algorithm>

#include "tip_common.h"

namespace tip {

// Bump allocator over one device buffer.  With base == nullptr it only sums
// sizes (used to size workspaces before allocating them).
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t off = 0;

    template <class T>
    T* take(int64_t n) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (size_t)std::max<int64_t>(n, 0);
        if (base && off > cap) throw AllocFailure("workspace too small");
        return p;
    }
};

struct IngestBuffers {
    uint64_t* keys = nullptr;
    uint64_t* keys2 = nullptr;
    int32_t* vals = nullptr;
    int32_t* vals2 = nullptr;
    int64_t* flags = nullptr;
    int64_t* hist = nullptr;
    int64_t* scan_tmp = nullptr;
    int32_t* ea = nullptr;
    int32_t* eb = nullptr;
    int32_t* deg_a = nullptr;  // by original id
    int32_t* deg_b = nullptr;
    int32_t* rank_a = nullptr;  // original id -> rank
    int32_t* rank_b = nullptr;
    int64_t* m_dev = nullptr;
    int32_t* err = nullptr;
};

struct GraphAux {
    int32_t* deg_a = nullptr;    // by rank
    int32_t* deg_b = nullptr;
    int64_t* deg_a64 = nullptr;  // [n_a+1] by rank (scan input)
    int64_t* deg_b64 = nullptr;
};

void ingest_alloc(Arena& ar, int32_t n_a, int32_t n_b, int64_t m, IngestBuffers& ib);
void graph_alloc(Arena& ar, int32_t n_a, int32_t n_b, int64_t m, DevGraph& g, GraphAux& aux);
bool ingest(const int32_t* d_a, const int32_t* d_b, int32_t n_a, int32_t n_b, int64_t m, bool a_is_u,
            IngestBuffers& ib, DevGraph& g, GraphAux& aux, hipStream_t s);

}  // namespace tip
