// Internal: control block and launch wrappers of the decomposition kernels.
#pragma once

#include "agg.h"
#include "fd_tune.h"

namespace tip {

// Counters that many waves add to in every launch are spread over
// kSpread sub-slots (chosen by block index) so their atomics do not
// serialise on one address; the host sums the slots.
constexpr int kSpread = 64;
enum SpreadCounter {
    kScWedgesCd = 0, kScPairs, kScSkipped, kScSpills, kScBigWedges, kScBigPairs, kScBigEdges, kScWRange,
    kScDeadEdges, kScWRem, kScCount
};

// Device-resident control block of one decomposition.
struct Ctl {
    int32_t n_live;         // live-list length (after the last compaction)
    int32_t n_live_next;    // compaction output counter
    int32_t n_front[kBins]; // current frontier sizes per update kernel
    int32_t n_next[kBins];  // next frontier sizes
    int32_t n_items[2];     // counting work items [wave bin, workgroup bin]
    int32_t pad0;
    int32_t sel_found;      // 0 once no support value reaches the target
    int32_t pad[4];
    long long w_range;      // wedge proxy summed over the current subset
    unsigned long long sel_prefix;
    long long sel_cum;
    long long sel_tgt;
    long long hi;
    unsigned long long wedges_count;
    unsigned long long wedges_cd;
    unsigned long long wedges_fd;
    unsigned long long pair_updates;
    unsigned long long spills;
    unsigned long long skipped;
    unsigned long long fd_levels;
    unsigned long long big_wedges;   // workgroup peeling kernel only
    unsigned long long big_edges;
    unsigned long long big_pairs;
    unsigned long long head[kBins];  // next work item of each update kernel in the current round
    unsigned long long dead_edges;   // list entries of vertices assigned since the last compaction
    long long cd_m;                  // entries left in the CD lists
    int32_t key_hi;                  // every live vertex of side A has a rank below this
    int32_t pad2;
    unsigned long long spread[kSpread][kScCount];
    unsigned long long spread_max[kSpread];  // largest live support at a range start, per workgroup group
    // Range state read by the round kernels, so that a sequence of rounds
    // can be launched (or replayed from a graph) without host arguments.
    long long range_hi;      // upper bound of the current range
    int32_t range_label;     // subset id of the current range
    int32_t range_live;      // which live list holds the range's live vertices
    int32_t range_n_live;    // its length
    int32_t front_buf;       // which frontier buffer is current
    unsigned long long rounds_done;  // rounds with a non-empty activeSet
    // HUC (Section 4.1): huc_now asks this round to re-count instead of
    // peeling; decided from the wedge proxy its activeSet added to the range
    int32_t huc_now;
    int32_t huc_n_a;              // vertices of side A
    long long huc_pct;            // re-count when peel work > huc_pct % of re-count work; 0 = never
    unsigned long long huc_w_prev;  // range wedge proxy at the previous decision
    unsigned long long huc_rounds;  // rounds that re-counted
    unsigned long long fd_huc_steps;  // fine-grained steps that re-counted
    unsigned long long cd_compactions, fd_compactions;
    unsigned long long fd_pair_entries;  // entries written to the fine-grained pair rows
    unsigned long long fd_pair_tasks;    // subsets peeled from pair rows
    unsigned long long fd_pair_heavy;    // rows built by the workgroup-per-vertex kernel
};

__device__ inline void spread_add(Ctl* ctl, int c, unsigned long long v) {
    atomicAdd(&ctl->spread[blockIdx.x & (kSpread - 1)][c], v);
}

inline unsigned long long spread_sum(const Ctl& c, int k) {
    unsigned long long s = 0;
    for (int i = 0; i < kSpread; ++i) s += c.spread[i][k];
    return s;
}

struct CountBuffers {
    int64_t* bfly_a;     // [n_a]
    int64_t* bfly_b;     // [n_b]
    int64_t* work;       // [n_a + n_b]
    int32_t* items_small;
    int32_t* items_big;
};

// findHi's radix select: digit width and histogram bins.
constexpr int kSelBits = 11;
constexpr int kSelBins = 1 << kSelBits;

struct PeelBuffers {
    int64_t* supp;       // [n_a] raw supports (= bfly_a)
    int64_t* wprox;      // [n_a] wedges of u in the original graph
    int32_t* state;      // [n_a] kLive or subset id
    int64_t* init;       // [n_a] support at the start of u's range
    int32_t* live[2];    // [n_a] live lists (ping-pong)
    int32_t* front[2][kBins];  // [buffer][bin] frontier lists
    int64_t* sel_hist;   // [kSelBins]
    uint8_t* bin;        // [n_a] update kernel of each vertex
    int32_t* tb;         // [n_b * (ntt + 1)] tile bounds of every CD list
    int32_t tk;          // keys per tile (dense_tile_keys(n_a))
    int32_t ntt;         // number of tiles of side A
    // The lists N_v the coarse-grained update traverses: a copy of the CSC
    // from which peeled vertices are periodically removed (DGM); the CSC
    // itself stays whole for the fine-grained step.
    int64_t* cd_off;     // [n_b + 1]
    int32_t* cd_adj;     // [m]
    int32_t* cd_row;     // [m]
    int64_t* cd_tmp_off; // [n_b + 1] compaction scratch
    int64_t* wlive;      // [n_a] wedges of u over the CD lists (selects u's update kernel)
};

// Scratch borrowed from the ingest buffers (idle during the coarse-grained
// step) by the list compaction.
struct CompactScratch {
    int64_t* flag;       // [m]
    int64_t* pos;        // [m]
    int64_t* scan_tmp;
    int32_t* adj;        // [m]
    int32_t* row;        // [m]
};

// Help board of one fine-grained launch.  A workgroup peeling a large subset
// opens a slot and publishes, level by level, its list of per-wave updates;
// workgroups whose task queue has run dry take entries from open slots.  All
// zero before the launch.
struct FdHelpSlot {
    unsigned long long word;  // (published entries << 32) | next entry to take
    int32_t done;             // entries of the published level finished
    int32_t hdone;            // heavy entries of the published level finished
    unsigned long long hword; // heavy updates: (published << 32) | next to take
    int32_t state;            // 0 unused, 1 open, 2 closed
    int32_t pairs;            // published entries are pair rows, taken kFdPairHelpChunk at a time
    int64_t pshift;           // the subset's row shift (pair rows)
    int32_t job;              // index in the job list, -1 for the single job
    int32_t n_i;              // subset size
    int64_t P0;               // subset start (position)
};
constexpr int kFdHelpSlots = 64;
struct FdBoard {
    int32_t head;     // task queue head
    int32_t pair_head;  // next vertex position of the pair-row build
    int32_t pair_heavy; // vertices on the pair-row build's heavy list
    int32_t pair_head2; // next entry of that list
    int32_t n_slots;  // slots handed out
    FdHelpSlot slot[kFdHelpSlots];
};

struct FdBuffers {
    int32_t* fd_vert;    // [n_a] vertices grouped by subset, ascending rank inside
    int32_t* fd_pos;     // [n_a]
    int64_t* sub_off;    // [S + 1]
    int64_t* sub_cnt;    // [S + 1]
    uint64_t* pkeys;     // [m] partitioned CSC keys (row * S + subset)
    int32_t* pcsc;       // [m] local ids
    int64_t* fd_beg;     // [m] per CSR edge: slice begin in pcsc
    int32_t* fd_len;     // [m]
    int64_t* task_w;     // [S]
    int32_t* order;      // [S]
    int64_t* supp_fd;    // [n_a] by subset position
    int64_t* fd_w;       // [n_a] wedges of each vertex inside its subset's subgraph, by position
    int32_t* alive;      // [n_a] by subset position
    int32_t* lst[5];     // [n_a] live / next-live / light-peel / heavy-peel / crossing lists by subset position
    // runs of the partitioned CSC grouped by subset (built with TIP_FLAG_FD_DGM)
    int32_t* run_q;      // [m] start position of each run, runs of subset s at [sub_roff[s], sub_roff[s + 1])
    int32_t* rlen_at;    // [m] current length of the run starting at a position
    int64_t* sub_roff;   // [S + 2]
    int64_t* sub_rcnt;   // [S + 2]
    int64_t* theta;      // [n_a] by rank
    FdBoard* board;      // task queue and help board of the launch
    unsigned long long* task_trace;  // [4 * kFdTraceTasks] per-task timing (diagnostic)
    // Pair rows: row p (the vertex at subset position p) holds every w of
    // its subset with c(u, w) >= 2, as w's index inside the subset and
    // C(c, 2).  Row space goes to the subsets in workload order, each that
    // still fits the budget; row p starts at prow_off[p] + pshift[s] for its
    // subset s, and a subset without rows has pshift kNoRows.
    int64_t* prow_off;   // [n_a + 1] exclusive scan of the row capacities in position order
    int64_t* pshift;     // [S]
    int32_t* prow_n;     // [n_a] entries of each row
    int32_t* prow_w;     // [pair_cap]
    int64_t* prow_b;     // [pair_cap]
    int64_t pair_cap;    // entries allocated
    int64_t pair_lim;    // entries this run may use (<= pair_cap)
    int32_t pairs_on;    // set per run
};

// Update-kernel selection thresholds (tip_opts.tune[0], tune[1]).
struct Tune {
    int64_t dense_div = kDefaultDenseDiv;
    int64_t bitmap_max = kDefaultBitmapMax;
    int64_t compact_permille = kDefaultCompactPermille;  // 0: never compact
    int64_t huc_pct = 0;  // tip_opts.tune[3]
    // fine-grained help board (tip_opts.tune[4..6])
    int32_t fd_help_chunk = kFdHelpChunk;
    int32_t fd_help_level_min = kFdHelpLevelMin;
    int32_t fd_help_min = kFdHelpMin;
    int32_t fd_huc_pct = 0;  // tip_opts.tune[7]
    bool fd_dgm = false;     // TIP_FLAG_FD_DGM
    bool dgm_paper = false;  // TIP_FLAG_DGM_PAPER
    bool fd_walk = false;    // TIP_FLAG_FD_WALK
};

// Pair-row entries a workspace holds for a graph of m edges (0: every
// fine-grained update walks its wedges).
inline int64_t fd_pair_entries(int64_t m, const Tune& t) {
    if (t.fd_walk || t.fd_dgm || t.fd_huc_pct > 0) return 0;
    return std::min(kFdPairsMax, kFdPairsPerEdge * std::max<int64_t>(m, 1));
}

// counting
void launch_count(const DevGraph& g, CountBuffers& cb, Ctl* ctl, const SpillArena& spill, int big_grid,
                  hipStream_t s);
// CD
void launch_peel_setup(const DevGraph& g, const int32_t* deg_b_rank, PeelBuffers& pb, const Tune& tune, Ctl* ctl,
                       hipStream_t s);
void launch_range_start(PeelBuffers& pb, int cur_live, int32_t n_live, Ctl* ctl, hipStream_t s);
// Removes every vertex that is no longer live from the CD lists (DGM),
// rebuilds their tile bounds and re-selects the update kernel of every live
// vertex from its wedges over the compacted lists.  cd_m: entries before;
// the count after is left in ctl->cd_m.  Range bounds keep using the
// original wedge proxy, so the partition does not depend on compaction.
void launch_compact(const DevGraph& g, PeelBuffers& pb, const CompactScratch& cs, int64_t cd_m, const Tune& tune,
                    Ctl* ctl, hipStream_t s);
void launch_select(PeelBuffers& pb, int cur_live, int32_t n_live, uint64_t max_supp, int64_t tgt, Ctl* ctl,
                   hipStream_t s);
// Sets the range state and builds the range's first activeSet.
// hi < 0 takes the bound from the select launched just before.
void launch_range_begin(const DevGraph& g, PeelBuffers& pb, int cur_live, int32_t n_live, int64_t hi,
                        uint64_t max_supp, int32_t label, Ctl* ctl, hipStream_t s, bool huc);
// One coarse-grained round, driven entirely by the control block: update
// kernels over the current activeSet, then the next activeSet and the buffer
// swap.  Fixed grids, no host synchronisation, so it can be graph-captured.
// ev_big: optional pair of events recorded around the dense update kernel,
// the one timed by TIP_FLAG_TIME_KERNELS (not while capturing).
// n_cur: the frontier sizes per bin when the host knows them (kernels
// without work are then skipped), or nullptr (graph capture: every kernel
// is launched and checks its own work).
// HUC re-count of the live side-A supports, when the control block asks for it.
void launch_recount(const DevGraph& g, CountBuffers& cb, const int32_t* state, Ctl* ctl, const SpillArena& spill,
                    int big_grid, hipStream_t s);
// One coarse-grained round; cb != nullptr adds the HUC re-count launches.
void launch_round(const DevGraph& g, PeelBuffers& pb, Ctl* ctl, const SpillArena& spill, int big_grid,
                  hipStream_t s, hipEvent_t* ev_big, const int32_t* n_cur, CountBuffers* cb);
void launch_assign_live(PeelBuffers& pb, int cur_live, int32_t n_live, int32_t label, hipStream_t s);
// One graph's part of a fine-grained launch.
struct FdJob {
    DevGraph g;
    FdBuffers fb;
    const int64_t* init;  // [n_a] support at the start of each vertex's range
    Ctl* ctl;             // receives the job's work counters
    int32_t help_min;        // subsets of at least this many vertices open a help-board slot
    int32_t help_chunk;      // per-wave updates taken at once from a slot
    int32_t help_level_min;  // levels with fewer per-wave updates are not published
    int32_t huc_pct;         // HUC in subsets kept in HBM (0 = never)
    int32_t dgm;             // compaction of the runs of subsets kept in HBM
};

// The jobs of one launch: a device array, or (list == nullptr) one job
// passed by value.
struct FdJobs {
    const FdJob* list;
    FdJob one;
    // diagnostic: per task t < trace_max, (subset size, levels, start, end)
    // in wall-clock ticks; null when not asked for
    unsigned long long* trace;
    int32_t trace_max;
};

// FD
// Subset grouping, partitioned CSC and workload order of one graph (up to,
// not including, the peeling launch); fb.task_w holds the induced wedges.
void launch_fd_setup(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, uint64_t* tmp_keys,
                     int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp, uint64_t* keys_scratch,
                     int32_t* vals_scratch, hipStream_t s, bool runs);
// Pair rows of the subsets that fit fb.pair_lim, taken in workload order
// (after launch_fd_setup); off (fb.pairs_on = 0) when `on` is false.
void launch_fd_pairs(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, Ctl* ctl,
                     const SpillArena& spill, int big_grid, int64_t* scan_tmp, bool on, hipStream_t s);
// Persistent peeling of the subsets of many graphs in one launch: tasks[t] =
// job << 32 | subset, in the order they are to be taken; *head is the queue
// head (reset here).
void launch_fd_batch(const FdJob* d_jobs, const int64_t* d_tasks, int32_t n_tasks, FdBoard* d_board,
                     const SpillArena& spill, int big_grid, hipStream_t s);
void launch_fd(const DevGraph& g, PeelBuffers& pb, FdBuffers& fb, int32_t S, Ctl* ctl, const Tune& tune,
               const SpillArena& spill,
               int big_grid, uint64_t* tmp_keys, int32_t* tmp_vals, int64_t* hist, int64_t* scan_tmp,
               uint64_t* keys_scratch, int32_t* vals_scratch, hipStream_t s, bool trace = false);
// output
void launch_scatter_i64(const int64_t* by_rank, const int32_t* orig, int32_t n, int64_t* out, hipStream_t s);

// resident workgroups per CU of the workgroup kernels of each unit
int count_occupancy();
int peel_occupancy();
int fd_occupancy();

}  // namespace tip
