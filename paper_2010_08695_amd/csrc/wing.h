// Internal: edge peeling (wing decomposition) and k-tip extraction.
#pragma once

#include "tip_ingest.h"
#include "tip_kernels.h"
#include "../../include/tip.h"

namespace tip {

// Device control block of one edge-peeling or k-tip call.
struct WingCtl {
    int32_t n_live;
    int32_t n_front;
    int32_t n_next;
    int32_t pad;
    unsigned long long min_supp;  // least live support at a level start
    long long level;
    unsigned long long head;
    unsigned long long wedges_count, wedges_peel, decrements, rounds, levels;
};

struct WingWork {
    IngestBuffers ib;
    DevGraph g;
    GraphAux aux;
    int32_t* eid_b = nullptr;     // [m] edge id of every CSC position
    int64_t* wu = nullptr;        // [n_u] sum over N_u of (d_v - 1)
    int64_t* wv = nullptr;        // [n_v]
    // edge peeling
    int64_t* supp = nullptr;      // [m] raw supports (the per-edge counts first)
    int64_t* psi = nullptr;       // [m] wing numbers by edge id
    int32_t* state = nullptr;     // [m]
    int32_t* live[2] = {nullptr, nullptr};
    int32_t* front[2] = {nullptr, nullptr};
    int64_t* out = nullptr;       // [m] results in input order
    // k-tips
    int64_t* theta_orig = nullptr, *theta_rank = nullptr;
    int32_t* parent = nullptr, *min_id = nullptr, *comp = nullptr;
    WingCtl* ctl = nullptr;
    SpillArena spill;             // per-workgroup direct-address arrays
};

// Workgroups the edge kernels keep resident.
int wing_slots();
// Carves (or, with a null arena base, sizes) the buffers of one call on a
// graph with U as side A; ktip = true for k-tip extraction of side U or V
// (then n_u, n_v are given as (side, other side)).
void wing_plan(Arena& ar, int32_t n_u, int32_t n_v, int64_t m, int slots, bool ktip, WingWork& w);
// Per-edge butterfly counts (decompose = false) or wing numbers of every
// input edge into d_out [m].
tip_status wing_run(WingWork& w, const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                    bool decompose, int64_t* d_out, tip_stats* st, hipStream_t s);
// k-tips of `side` given its tip numbers (host, by original id): d_comp[x] =
// smallest id of x's k-tip, -1 when theta_x < k.
tip_status ktip_run(WingWork& w, const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                    int32_t side, const int64_t* theta_host, int64_t k, int32_t* d_comp, hipStream_t s);

}  // namespace tip
