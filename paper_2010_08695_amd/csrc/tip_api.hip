// C ABI of libtip (include/tip.h): argument checks, workspace planning and the
// host-side orchestration of counting, coarse-grained and fine-grained
// decomposition.  All arithmetic runs in the HIP kernels; the host only
// sequences launches and reads a small control block between CD rounds.
#include <cmath>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/tip.h"
#include "tip_ingest.h"
#include "tip_kernels.h"
#include "wing.h"

// Scratch of tip_decompose_noalloc: one copy per device, held until the
// process ends.  Host code never uses this name as an address (on the host it
// is only a stand-in for the symbol); it takes the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
constexpr size_t kNoAllocScratchBytes = size_t(512) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace tip {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

namespace {

constexpr int kDefaultP = 150;
constexpr int kMaxP = 65535;

struct Work {
    IngestBuffers ib;
    DevGraph g;
    GraphAux aux;
    CountBuffers cb;
    PeelBuffers pb;
    FdBuffers fb;
    Ctl* ctl = nullptr;
    SpillArena spill;
    int64_t* total = nullptr;
    // set by tip_decompose_noalloc: no HIP graph, no events, no pinned host
    // memory (every coarse-grained round is launched from the host)
    bool no_alloc = false;
};

int resident_workgroups() {
    static std::mutex mu;
    static int cached_dev = -1, cached = 0;
    int dev = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (dev != cached_dev) {
        int cus = 0;
        TIP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cached = std::max(1, cus) * std::min(count_occupancy(), std::min(peel_occupancy(), fd_occupancy()));
        cached_dev = dev;
    }
    return cached;
}

// Allocates every buffer of one decomposition from the arena (or, with a
// null arena base, only sums the sizes); `pairs`: pair-row entries of the
// fine-grained step (fd_pair_entries).
void plan(Arena& ar, int32_t n_a, int32_t n_b, int64_t m, int32_t P, int slots, int64_t pairs, Work& w) {
    const int32_t S = P + 1;
    const int64_t na = std::max<int32_t>(n_a, 1), nb = std::max<int32_t>(n_b, 1), mm = std::max<int64_t>(m, 1);
    ingest_alloc(ar, n_a, n_b, m, w.ib);
    graph_alloc(ar, n_a, n_b, m, w.g, w.aux);
    w.cb.bfly_a = ar.take<int64_t>(na);
    w.cb.bfly_b = ar.take<int64_t>(nb);
    w.cb.work = ar.take<int64_t>(na + nb);
    w.cb.items_small = ar.take<int32_t>(na + nb);
    w.cb.items_big = ar.take<int32_t>(na + nb);
    w.pb.supp = w.cb.bfly_a;
    w.pb.wprox = ar.take<int64_t>(na);
    w.pb.state = ar.take<int32_t>(na);
    w.pb.init = ar.take<int64_t>(na);
    for (int i = 0; i < 2; ++i) w.pb.live[i] = ar.take<int32_t>(na);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < kBins; ++j) w.pb.front[i][j] = ar.take<int32_t>(na);
    w.pb.sel_hist = ar.take<int64_t>(kSelBins);
    w.pb.bin = ar.take<uint8_t>(na);
    w.pb.tk = dense_tile_keys(na);
    // the bitmap path walks whole table tiles of at most kBmTile keys
    if (w.pb.tk > kBmTile) throw InvalidArg("a side with more than 2^28 vertices is not supported");
    w.pb.ntt = (int32_t)((na + w.pb.tk - 1) / w.pb.tk);
    w.pb.tb = ar.take<int32_t>(nb * (w.pb.ntt + 1));
    w.pb.cd_off = ar.take<int64_t>(nb + 1);
    w.pb.cd_adj = ar.take<int32_t>(mm);
    w.pb.cd_row = ar.take<int32_t>(mm);
    w.pb.cd_tmp_off = ar.take<int64_t>(nb + 1);
    w.pb.wlive = ar.take<int64_t>(na);
    w.fb.fd_vert = ar.take<int32_t>(na);
    w.fb.fd_pos = ar.take<int32_t>(na);
    w.fb.sub_off = ar.take<int64_t>(S + 1);
    w.fb.sub_cnt = ar.take<int64_t>(S + 1);
    w.fb.pkeys = ar.take<uint64_t>(mm);
    w.fb.pcsc = ar.take<int32_t>(mm);
    w.fb.fd_beg = ar.take<int64_t>(mm);
    w.fb.fd_len = ar.take<int32_t>(mm);
    w.fb.task_w = ar.take<int64_t>(S);
    w.fb.order = ar.take<int32_t>(S);
    w.fb.supp_fd = ar.take<int64_t>(na);
    w.fb.fd_w = ar.take<int64_t>(na);
    w.fb.alive = ar.take<int32_t>(na);
    for (int i = 0; i < 5; ++i) w.fb.lst[i] = ar.take<int32_t>(na);
    w.fb.run_q = ar.take<int32_t>(mm);
    w.fb.rlen_at = ar.take<int32_t>(mm);
    w.fb.sub_roff = ar.take<int64_t>(S + 2);
    w.fb.sub_rcnt = ar.take<int64_t>(S + 2);
    w.fb.theta = ar.take<int64_t>(na);
    w.fb.board = ar.take<FdBoard>(1);
    w.fb.task_trace = ar.take<unsigned long long>(4 * kFdTraceTasks);
    w.fb.pair_cap = pairs;
    w.fb.pair_lim = 0;
    w.fb.pairs_on = 0;
    w.fb.prow_off = pairs > 0 ? ar.take<int64_t>(na + 1) : nullptr;
    w.fb.pshift = pairs > 0 ? ar.take<int64_t>(S) : nullptr;
    w.fb.prow_n = pairs > 0 ? ar.take<int32_t>(na) : nullptr;
    w.fb.prow_w = pairs > 0 ? ar.take<int32_t>(pairs) : nullptr;
    w.fb.prow_b = pairs > 0 ? ar.take<int64_t>(pairs) : nullptr;
    w.ctl = ar.take<Ctl>(1);
    w.total = ar.take<int64_t>(2);
    const int64_t keys = std::max<int64_t>(std::max(na, nb), 1);
    w.spill.stride = std::min<int64_t>(kBmBits, (keys + 63) & ~int64_t(63));
    w.spill.slots = slots;
    w.spill.dense = ar.take<int32_t>(w.spill.stride * slots);
    w.spill.list = ar.take<int32_t>(w.spill.stride * slots);
}

// Pinned host mirror of the control block, one per host thread.
struct PinnedCtl {
    Ctl* h = nullptr;
    ~PinnedCtl() {
        if (h) (void)hipHostFree(h);
    }
};

// pinned = false: a plain host mirror, for calls that must not allocate
Ctl* host_ctl(bool pinned) {
    thread_local Ctl plain;
    if (!pinned) return &plain;
    thread_local PinnedCtl pc;
    if (!pc.h) {
        void* p = nullptr;
        TIP_HIP_TRY(hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault));
        pc.h = static_cast<Ctl*>(p);
    }
    return pc.h;
}

const Ctl& read_ctl(const Work& w, hipStream_t s) {
    Ctl* h = host_ctl(!w.no_alloc);
    TIP_HIP_TRY(hipMemcpyAsync(h, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    TIP_HIP_TRY(hipStreamSynchronize(s));
    return *h;
}

// K coarse-grained rounds captured once into a HIP graph and replayed; the
// rounds take all their state from the device control block, and rounds
// past the end of a range do nothing, so the host reads one flag per replay
// instead of one per round.
constexpr int kRoundsPerGraph = 3;

struct RoundGraph {
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    void build(const DevGraph& g, PeelBuffers& pb, Ctl* ctl, const SpillArena& spill, int big_grid,
               CountBuffers* cb) {
        TIP_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        TIP_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < kRoundsPerGraph; ++k) launch_round(g, pb, ctl, spill, big_grid, cs, nullptr, nullptr, cb);
        TIP_HIP_TRY(hipStreamEndCapture(cs, &graph));
        TIP_HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    ~RoundGraph() {
        if (cs) {
            hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(cs, &st) == hipSuccess && st == hipStreamCaptureStatusActive) {
                hipGraph_t partial = nullptr;
                if (hipStreamEndCapture(cs, &partial) == hipSuccess && partial) (void)hipGraphDestroy(partial);
            }
            (void)hipGetLastError();
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

// Phase events; not created (records do nothing, times read 0) for calls
// that must not allocate.
struct Events {
    hipEvent_t e[6] = {};
    explicit Events(bool create = true) {
        if (create)
            for (auto& x : e) TIP_HIP_TRY(hipEventCreate(&x));
    }
    ~Events() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
    void rec(int i, hipStream_t s) {
        if (e[i]) TIP_HIP_TRY(hipEventRecord(e[i], s));
    }
    double ms(int a, int b) const {
        float t = 0;
        if (!e[a] || !e[b] || hipEventElapsedTime(&t, e[a], e[b]) != hipSuccess) return 0.0;
        return t;
    }
};

__global__ void k_sum_i64(const int64_t* a, int32_t n, int64_t* out) {
    __shared__ unsigned long long r[1024];
    unsigned long long s = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += (unsigned long long)a[i];
    r[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += r[i];
        out[0] = (int64_t)t;
    }
}

struct RunOut {
    int64_t* theta = nullptr;      // device, by original id
    int64_t* bfly_a = nullptr;     // device, by original id (count mode)
    int64_t* bfly_b = nullptr;
    int32_t* subset = nullptr;     // device, by original id (optional)
    int64_t* init = nullptr;       // device, by original id (optional)
    std::vector<int64_t>* bounds = nullptr;
    int32_t* n_subsets = nullptr;
};

__global__ void k_scatter_i32(const int32_t* by_rank, const int32_t* orig, int32_t n, int32_t* out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        out[orig[r]] = by_rank[r];
}

// Ingest + count (+ CD + FD when decomposing).  Returns TIP_OK or an error
// status (EINVAL for out-of-range ids found on the device).
// State carried from the first part of a run (ingest, count, CD, FD set-up
// or all of FD) to the second (outputs and statistics).
struct RunState {
    explicit RunState(bool events = true) : ev(events), kev(events) {}
    Events ev;
    Events kev;  // [0], [1]: around the dense update kernel of one round
    double peel_ms = 0.0;
    int64_t peel_launches = 0;
    int32_t S = 0;
    std::vector<int64_t> bounds;
    unsigned long long cd_walked_at = 0;  // coarse-grained wedges walked at the last compaction
    int64_t cd_compactions = 0;
};

// fd_inline = false stops after the set-up of FD (Alg. 4): the caller then
// peels the subsets, possibly together with other graphs', and calls
// run_back.
tip_status run_front(Work& w, const int32_t* d_a, const int32_t* d_b, int32_t n_a, int32_t n_b, int64_t m,
                     bool a_is_u, int32_t P, int32_t flags, const Tune& tune, bool decompose, bool fd_inline,
                     RunState& rs, hipStream_t s) {
    Events& ev = rs.ev;
    Events& kev = rs.kev;
    const bool time_kernels = (flags & TIP_FLAG_TIME_KERNELS) != 0;
    // diagnostic: with kernel timing on, TIP_TRACE_ROUNDS=1 prints every
    // coarse-grained round's frontier sizes and update time to stderr
    static const bool trace_rounds = [] {
        const char* e = std::getenv("TIP_TRACE_ROUNDS");
        return e && e[0] == '1';
    }();
    double& peel_ms = rs.peel_ms;
    int64_t& peel_launches = rs.peel_launches;
    // rounds run eagerly (one launch sequence per round, host-timed) when
    // kernels are timed or graphs are disabled, else from a replayed graph
    const bool eager = time_kernels || (flags & TIP_FLAG_NO_GRAPH) != 0 || w.no_alloc;
    std::unique_ptr<RoundGraph> rg;
    ev.rec(0, s);
    TIP_HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(Ctl), s));
    if (!ingest(d_a, d_b, n_a, n_b, m, a_is_u, w.ib, w.g, w.aux, s)) {
        set_error("an edge endpoint id is out of range");
        return TIP_EINVAL;
    }
    // No count can overflow: with c(x, w) <= d_x, the butterflies of x are at
    // most (d_x - 1) / 2 * sum_{y in N_x} (d_y - 1), so either side's counts
    // sum to at most 1/2 * sum over edges (x, y) of (d_x - 1)(d_y - 1) <
    // m^2 / 2 < 2^61 for m < 2^31 (the largest m the boundary accepts).
    ev.rec(1, s);
    const DevGraph& g = w.g;
    const int big_grid = w.spill.slots;

    // Per-vertex butterfly counting (Alg. 1).
    launch_count(g, w.cb, w.ctl, w.spill, big_grid, s);
    ev.rec(2, s);

    int32_t& S = rs.S;
    if (!decompose) {
        ev.rec(3, s);
        ev.rec(4, s);
    } else {
        // Coarse-grained decomposition (Alg. 3).
        PeelBuffers& pb = w.pb;
        // HUC re-count launches join the rounds only when asked for
        CountBuffers* huc_cb = tune.huc_pct > 0 ? &w.cb : nullptr;
        launch_peel_setup(g, w.aux.deg_b, pb, tune, w.ctl, s);
        const CompactScratch cscr{w.ib.flags, reinterpret_cast<int64_t*>(w.ib.keys), w.ib.scan_tmp, w.ib.ea, w.ib.eb};
        fill_i32(pb.state, kLive, n_a, s);
        iota_i32(pb.live[0], n_a, s);
        int cur_live = 0;
        int32_t n_live = n_a;
        double scale = 1.0;
        std::vector<int64_t>& bounds = rs.bounds;
        bounds.assign(1, 0);
        int32_t label = 0;
        for (; label < P && n_live > 0; ++label) {
            launch_range_start(pb, cur_live, n_live, w.ctl, s);
            const Ctl& c0 = read_ctl(w, s);
            n_live = c0.n_live_next;
            cur_live ^= 1;
            if (n_live == 0) break;
            // DGM: drop the vertices of finished ranges from the CD lists once
            // they hold enough of the remaining entries
            const unsigned long long dead = spread_sum(c0, kScDeadEdges);
            const unsigned long long walked = spread_sum(c0, kScWedgesCd);
            bool compact = false;
            if (tune.dgm_paper)  // Section 4.2: after as many wedges as entries left
                compact = tune.compact_permille > 0 && dead > 0 && walked - rs.cd_walked_at >= (unsigned long long)c0.cd_m;
            else
                compact = tune.compact_permille > 0 && dead > 0 &&
                          (double)dead * 1000.0 >= (double)c0.cd_m * (double)tune.compact_permille;
            if (compact) {
                launch_compact(g, pb, cscr, c0.cd_m, tune, w.ctl, s);
                rs.cd_walked_at = walked;
                ++rs.cd_compactions;
            }
            uint64_t max_supp = 0;
            for (int i = 0; i < kSpread; ++i) max_supp = std::max<uint64_t>(max_supp, c0.spread_max[i]);
            const long long w_rem = (long long)spread_sum(c0, kScWRem);
            // adaptive target: remaining wedges over remaining subsets,
            // scaled by how far the previous subset overshot its target
            double tgt_d = std::ceil(scale * (double)w_rem / (double)(P - label));
            int64_t tgt = tgt_d < 1.0 ? 1 : (int64_t)tgt_d;
            // the range's upper bound stays on the device (k_set_range takes
            // the select's result); the host learns it at the next read
            int64_t hi = -1;
            if (max_supp == 0) hi = 1;
            else launch_select(pb, cur_live, n_live, max_supp, tgt, w.ctl, s);
            launch_range_begin(g, pb, cur_live, n_live, hi, max_supp, label, w.ctl, s, huc_cb != nullptr);
            // replayed rounds go out before the frontier is read: rounds past
            // the end of a range do nothing, so a read per replay suffices
            for (;;) {
                if (!eager) {
                    if (!rg) {
                        rg.reset(new RoundGraph);
                        rg->build(g, pb, w.ctl, w.spill, big_grid, huc_cb);
                    }
                    TIP_HIP_TRY(hipGraphLaunch(rg->exec, s));
                }
                const Ctl& c2 = read_ctl(w, s);
                int32_t n_cur[kBins];
                int64_t n_tot = 0;
                for (int b = 0; b < kBins; ++b) n_tot += (n_cur[b] = c2.n_front[b]);
                if (n_tot == 0) break;
                if (!eager) continue;
                int32_t nb = 0;  // vertices for the timed (dense) update kernel
                for (int b = dense_bin_of_kind(0, false); b < kBins; ++b) nb += n_cur[b];
                launch_round(g, pb, w.ctl, w.spill, big_grid, s, time_kernels && nb > 0 ? kev.e : nullptr, n_cur,
                             huc_cb);
                if (nb > 0) {
                    ++peel_launches;
                    if (time_kernels) {
                        TIP_HIP_TRY(hipEventSynchronize(kev.e[1]));
                        const double ms = kev.ms(0, 1);
                        peel_ms += ms;
                        if (trace_rounds) {
                            std::string bins;
                            for (int b = 0; b < kBins; ++b) bins += (b ? "," : "") + std::to_string(n_cur[b]);
                            std::fprintf(stderr, "tip-round range=%d bins=%s ms=%.4f\n", label, bins.c_str(), ms);
                        }
                    }
                }
            }
            // the loop ends on a read with nothing launched after it
            const Ctl& c3 = *host_ctl(!w.no_alloc);
            bounds.push_back((int64_t)c3.range_hi);
            const long long w_range = (long long)spread_sum(c3, kScWRange);
            if (w_range > 0) scale = std::min(1.0, (double)tgt / (double)w_range);
        }
        // Vertices left after P ranges form one more subset.
        launch_range_start(pb, cur_live, n_live, w.ctl, s);
        const Ctl& c4 = read_ctl(w, s);
        n_live = c4.n_live_next;
        cur_live ^= 1;
        if (n_live > 0) {
            launch_assign_live(pb, cur_live, n_live, label, s);
            bounds.push_back(INT64_MAX);
            S = label + 1;
        } else {
            S = label;
        }
        ev.rec(3, s);
        // Fine-grained decomposition (Alg. 4).
        if (fd_inline) {
            // diagnostic: with kernel timing on, TIP_TRACE_FD=1 prints every
            // fine-grained task's size, levels and start and end times
            static const bool trace_fd = [] {
                const char* e = std::getenv("TIP_TRACE_FD");
                return e && e[0] == '1';
            }();
            const bool tr = trace_fd && time_kernels && S > 0;
            if (S > 0)
                launch_fd(g, pb, w.fb, S, w.ctl, tune, w.spill, big_grid, w.ib.keys2, w.ib.vals2, w.ib.hist,
                          w.ib.scan_tmp, w.ib.keys, w.ib.vals, s, tr);
            ev.rec(4, s);
            if (tr) {
                const int32_t n = std::min<int32_t>(S, kFdTraceTasks);
                std::vector<unsigned long long> h(4 * (size_t)n);
                TIP_HIP_TRY(hipMemcpyAsync(h.data(), w.fb.task_trace, h.size() * sizeof(unsigned long long),
                                           hipMemcpyDeviceToHost, s));
                TIP_HIP_TRY(hipStreamSynchronize(s));
                unsigned long long t0 = ~0ull;
                for (int32_t t = 0; t < n; ++t)
                    if (h[4 * t] > 0) t0 = std::min(t0, h[4 * t + 2]);
                // the wall clock counts at 100 MHz
                for (int32_t t = 0; t < n; ++t)
                    if (h[4 * t] > 0)
                        std::fprintf(stderr, "tip-fd-task task=%d n=%llu levels=%llu start_us=%.1f end_us=%.1f\n", t,
                                     h[4 * t], h[4 * t + 1], (double)(h[4 * t + 2] - t0) / 100.0,
                                     (double)(h[4 * t + 3] - t0) / 100.0);
                if (w.fb.pairs_on) {
                    int64_t cap_total = 0;
                    unsigned long long entries = 0;
                    TIP_HIP_TRY(hipMemcpyAsync(&cap_total, w.fb.prow_off + n_a, sizeof(int64_t), hipMemcpyDeviceToHost, s));
                    TIP_HIP_TRY(hipMemcpyAsync(&entries, &w.ctl->fd_pair_entries, sizeof(entries),
                                               hipMemcpyDeviceToHost, s));
                    unsigned long long n_heavy = 0;
                    TIP_HIP_TRY(hipMemcpyAsync(&n_heavy, &w.ctl->fd_pair_heavy, sizeof(n_heavy),
                                               hipMemcpyDeviceToHost, s));
                    TIP_HIP_TRY(hipStreamSynchronize(s));
                    std::fprintf(stderr, "tip-fd-pairs capacity=%lld budget=%lld entries=%llu heavy=%llu\n",
                                 (long long)cap_total, (long long)w.fb.pair_lim, entries, n_heavy);
                }
            }
        } else {
            launch_fd_setup(g, pb, w.fb, S, w.ib.keys2, w.ib.vals2, w.ib.hist, w.ib.scan_tmp, w.ib.keys, w.ib.vals, s,
                            tune.fd_dgm && tune.fd_huc_pct == 0);
            if (S > 0)
                launch_fd_pairs(g, pb, w.fb, S, w.ctl, w.spill, big_grid, w.ib.scan_tmp,
                                !tune.fd_walk && !tune.fd_dgm && tune.fd_huc_pct == 0, s);
        }
    }
    return TIP_OK;
}

// Outputs and statistics of a run whose FD has completed on stream s.
void run_back(Work& w, int32_t n_a, int32_t n_b, bool decompose, RunOut& out, RunState& rs, tip_stats* st,
              hipStream_t s) {
    Events& ev = rs.ev;
    const DevGraph& g = w.g;
    PeelBuffers& pb = w.pb;
    const int32_t S = rs.S;
    if (!decompose) {
        if (out.bfly_a) launch_scatter_i64(w.cb.bfly_a, g.a_orig, n_a, out.bfly_a, s);
        if (out.bfly_b) launch_scatter_i64(w.cb.bfly_b, g.b_orig, n_b, out.bfly_b, s);
    } else {
        launch_scatter_i64(w.fb.theta, g.a_orig, n_a, out.theta, s);
        if (out.subset && n_a > 0) {
            k_scatter_i32<<<(n_a + 255) / 256, 256, 0, s>>>(pb.state, g.a_orig, n_a, out.subset);
            TIP_HIP_TRY(hipGetLastError());
        }
        if (out.init) launch_scatter_i64(pb.init, g.a_orig, n_a, out.init, s);
        if (out.bounds) *out.bounds = rs.bounds;
        if (out.n_subsets) *out.n_subsets = S;
    }
    ev.rec(5, s);
    const Ctl& cf = read_ctl(w, s);
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->wedges_count = (int64_t)cf.wedges_count;
        st->wedges_cd = (int64_t)spread_sum(cf, kScWedgesCd);
        st->wedges_fd = (int64_t)cf.wedges_fd;
        st->pair_updates = (int64_t)(cf.pair_updates + spread_sum(cf, kScPairs));
        st->rounds = (int64_t)cf.rounds_done;
        st->huc_rounds = (int64_t)cf.huc_rounds;
        st->fd_huc_steps = (int64_t)cf.fd_huc_steps;
        st->compactions = rs.cd_compactions + (int64_t)(cf.fd_compactions << 32);
        st->fd_pair_entries = (int64_t)cf.fd_pair_entries;
        st->fd_pair_subsets = (int64_t)cf.fd_pair_tasks;
        st->subsets = S;
        st->fd_levels = (int64_t)cf.fd_levels;
        st->spills = (int64_t)(cf.spills + spread_sum(cf, kScSpills));
        st->skipped = (int64_t)spread_sum(cf, kScSkipped);
        st->m_unique = g.m;
        st->peel_launches = rs.peel_launches;
        st->peel_wedges = (int64_t)spread_sum(cf, kScBigWedges);
        st->peel_edges = (int64_t)spread_sum(cf, kScBigEdges);
        st->peel_pairs = (int64_t)spread_sum(cf, kScBigPairs);
        st->peel_ms = rs.peel_ms;
        st->t_ingest_ms = ev.ms(0, 1);
        st->t_count_ms = ev.ms(1, 2);
        st->t_cd_ms = ev.ms(2, 3);
        st->t_fd_ms = ev.ms(3, 4);
        st->t_total_ms = ev.ms(0, 5);
    }
}

tip_status run(Work& w, const int32_t* d_a, const int32_t* d_b, int32_t n_a, int32_t n_b, int64_t m, bool a_is_u,
               int32_t P, int32_t flags, const Tune& tune, bool decompose, RunOut& out, tip_stats* st,
               hipStream_t s) {
    RunState rs(!w.no_alloc);
    const tip_status rc = run_front(w, d_a, d_b, n_a, n_b, m, a_is_u, P, flags, tune, decompose, true, rs, s);
    if (rc != TIP_OK) return rc;
    run_back(w, n_a, n_b, decompose, out, rs, st, s);
    return TIP_OK;
}

struct DeviceBuffer {
    void* p = nullptr;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t bytes) {
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw AllocFailure("hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
};

struct StreamHolder {
    hipStream_t s = nullptr;
    StreamHolder() { TIP_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
    ~StreamHolder() {
        if (s) (void)hipStreamDestroy(s);
    }
};

void check_edges(const tip_edges* g) {
    if (!g) throw InvalidArg("graph is NULL");
    if (g->n_u < 0 || g->n_v < 0) throw InvalidArg("negative vertex count");
    if (g->m < 0) throw InvalidArg("negative edge count");
    if (g->m > INT32_MAX) throw InvalidArg("more than 2^31-1 edges");
    if (g->m > 0 && (!g->eu || !g->ev)) throw InvalidArg("edge arrays are NULL");
    for (int64_t i = 0; i < g->m; ++i) {
        if ((uint32_t)g->eu[i] >= (uint32_t)g->n_u || (uint32_t)g->ev[i] >= (uint32_t)g->n_v)
            throw InvalidArg("edge " + std::to_string(i) + " has an endpoint id out of range");
    }
}

constexpr int32_t kKnownFlags = TIP_FLAG_TIME_KERNELS | TIP_FLAG_NO_GRAPH | TIP_FLAG_BATCH_PLAIN | TIP_FLAG_NO_COMPACT |
                                TIP_FLAG_OPTS_PER_GRAPH | TIP_FLAG_BATCH_STREAMS | TIP_FLAG_FD_DGM |
                                TIP_FLAG_DGM_PAPER | TIP_FLAG_FD_WALK;

int32_t check_opts(const tip_opts* opt, bool batch = false) {
    if (!opt) return kDefaultP;
    if (opt->P < 0 || opt->P > kMaxP) throw InvalidArg("P must be in [0, 65535]");
    if (opt->flags & ~kKnownFlags) throw InvalidArg("unknown flag bits");
    if (!batch && (opt->flags & TIP_FLAG_OPTS_PER_GRAPH))
        throw InvalidArg("TIP_FLAG_OPTS_PER_GRAPH is for tip_decompose_batch only");
    for (int i = 0; i < 8; ++i)
        if (opt->tune[i] < 0) throw InvalidArg("tune[0..7] must be >= 0");
    if (opt->tune[4] > (1 << 20)) throw InvalidArg("tune[4] must be at most 2^20");
    return opt->P == 0 ? kDefaultP : opt->P;
}

Tune tune_of(const tip_opts* opt) {
    Tune t;
    if (opt && opt->tune[0] > 0) t.dense_div = opt->tune[0];
    if (opt && opt->tune[1] > 0) t.bitmap_max = opt->tune[1];
    if (opt && opt->tune[2] > 0) t.compact_permille = opt->tune[2];
    if (opt) t.huc_pct = opt->tune[3];
    if (opt && opt->tune[4] > 0) t.fd_help_chunk = opt->tune[4];
    if (opt && opt->tune[5] > 0) t.fd_help_level_min = opt->tune[5];
    if (opt && opt->tune[6] > 0) t.fd_help_min = opt->tune[6];
    if (opt) t.fd_huc_pct = opt->tune[7];
    if (opt && (opt->flags & TIP_FLAG_NO_COMPACT)) t.compact_permille = 0;
    if (opt) t.fd_dgm = (opt->flags & TIP_FLAG_FD_DGM) != 0;
    if (opt) t.dgm_paper = (opt->flags & TIP_FLAG_DGM_PAPER) != 0;
    if (opt) t.fd_walk = (opt->flags & TIP_FLAG_FD_WALK) != 0;
    return t;
}

template <class F>
tip_status guard(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const InvalidArg& e) {
        set_error(e.msg);
        return TIP_EINVAL;
    } catch (const AllocFailure& e) {
        set_error(e.msg);
        return TIP_ENOMEM;
    } catch (const HipFailure& e) {
        set_error(e.msg);
        return TIP_EDEVICE;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return TIP_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return TIP_EDEVICE;
    }
}

// Host-pointer decomposition of one graph (side already validated).
tip_status decompose_host(const tip_edges* g, int32_t side, int64_t* theta, int32_t P, int32_t flags,
                          const Tune& tune, tip_stats* st, int32_t* subset, int64_t* init, int64_t* bounds,
                          int32_t* n_subsets) {
    const bool a_is_u = side == TIP_SIDE_U;
    const int32_t n_a = a_is_u ? g->n_u : g->n_v;
    const int32_t n_b = a_is_u ? g->n_v : g->n_u;
    const int64_t m = g->m;
    StreamHolder sh;
    Work w;
    const int slots = resident_workgroups();
    Arena sizer;
    plan(sizer, n_a, n_b, m, P, slots, fd_pair_entries(m, tune), w);
    const size_t extra = sizeof(int32_t) * (2 * (size_t)std::max<int64_t>(m, 1)) +
                         (sizeof(int64_t) * 2 + sizeof(int32_t)) * (size_t)std::max<int32_t>(n_a, 1) + 4096;
    DeviceBuffer buf;
    buf.alloc(sizer.off + extra);
    Arena ar{static_cast<char*>(buf.p), sizer.off + extra, 0};
    plan(ar, n_a, n_b, m, P, slots, fd_pair_entries(m, tune), w);
    int32_t* d_a = ar.take<int32_t>(std::max<int64_t>(m, 1));
    int32_t* d_b = ar.take<int32_t>(std::max<int64_t>(m, 1));
    int64_t* d_theta = ar.take<int64_t>(std::max<int32_t>(n_a, 1));
    int64_t* d_init = ar.take<int64_t>(std::max<int32_t>(n_a, 1));
    int32_t* d_sub = ar.take<int32_t>(std::max<int32_t>(n_a, 1));
    const hipStream_t s = sh.s;
    TIP_HIP_TRY(hipMemsetAsync(w.spill.dense, 0, sizeof(int32_t) * w.spill.stride * w.spill.slots, s));
    if (m > 0) {
        TIP_HIP_TRY(hipMemcpyAsync(d_a, a_is_u ? g->eu : g->ev, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        TIP_HIP_TRY(hipMemcpyAsync(d_b, a_is_u ? g->ev : g->eu, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
    }
    RunOut out;
    out.theta = d_theta;
    out.subset = subset ? d_sub : nullptr;
    out.init = init ? d_init : nullptr;
    std::vector<int64_t> bvec;
    out.bounds = &bvec;
    int32_t ns = 0;
    out.n_subsets = &ns;
    const tip_status rc = run(w, d_a, d_b, n_a, n_b, m, a_is_u, P, flags, tune, true, out, st, s);
    if (rc != TIP_OK) return rc;
    if (n_a > 0) {
        TIP_HIP_TRY(hipMemcpyAsync(theta, d_theta, sizeof(int64_t) * n_a, hipMemcpyDeviceToHost, s));
        if (subset) TIP_HIP_TRY(hipMemcpyAsync(subset, d_sub, sizeof(int32_t) * n_a, hipMemcpyDeviceToHost, s));
        if (init) TIP_HIP_TRY(hipMemcpyAsync(init, d_init, sizeof(int64_t) * n_a, hipMemcpyDeviceToHost, s));
    }
    TIP_HIP_TRY(hipStreamSynchronize(s));
    if (bounds) {
        for (size_t i = 0; i < bvec.size(); ++i) bounds[i] = bvec[i];
    }
    if (n_subsets) *n_subsets = ns;
    return TIP_OK;
}

// ---------------------------------------------------------------------------
// Batch: every graph's ingest, counting and CD run concurrently on worker
// streams (the GPU overlaps the kernels of different graphs); then the FD
// subsets of all graphs are peeled in ONE persistent launch that takes tasks
// from a single queue ordered by induced wedges across the whole batch
// (workload-aware scheduling of Alg. 4 over all graphs).
// ---------------------------------------------------------------------------
constexpr int kBatchWorkers = 8;

struct BatchItem {
    int32_t n_a = 0, n_b = 0;
    int64_t m = 0;
    bool a_is_u = true;
    int32_t P = kDefaultP;
    Tune tune;
    Work w;
    DeviceBuffer buf;
    RunState rs;
    int64_t* d_theta = nullptr;
    tip_status rc = TIP_OK;
    std::string err;
};

// Graph k runs with Ps[k] ranges and tunes[k].
tip_status decompose_batched(int32_t n, const tip_edges* gs, const int32_t* sides, int64_t* const* thetas,
                             const std::vector<int32_t>& Ps, int32_t flags, const std::vector<Tune>& tunes,
                             tip_stats* st) {
    if (n == 0) return TIP_OK;
    int dev = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    const int slots = resident_workgroups();
    std::vector<std::unique_ptr<BatchItem>> items(n);
    std::vector<int32_t> order(n);
    for (int32_t k = 0; k < n; ++k) order[k] = k;
    // largest graphs first, so the tail of the concurrent phase is short
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return gs[a].m > gs[b].m; });
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        hipStream_t s = nullptr;
        try {
            TIP_HIP_TRY(hipSetDevice(dev));
            TIP_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        } catch (const HipFailure&) {
            return;  // the items this worker would have taken are picked up by others
        }
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= n) break;
            const int32_t k = order[i];
            std::unique_ptr<BatchItem> it(new BatchItem);
            BatchItem& b = *it;
            try {
                const tip_edges* g = &gs[k];
                b.P = Ps[k];
                b.tune = tunes[k];
                const int32_t P = b.P;
                b.a_is_u = sides[k] == TIP_SIDE_U;
                b.n_a = b.a_is_u ? g->n_u : g->n_v;
                b.n_b = b.a_is_u ? g->n_v : g->n_u;
                b.m = g->m;
                Arena sizer;
                plan(sizer, b.n_a, b.n_b, b.m, P, slots, fd_pair_entries(b.m, b.tune), b.w);
                const size_t extra = sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(b.m, 1) +
                                     sizeof(int64_t) * (size_t)std::max<int32_t>(b.n_a, 1) + 4096;
                b.buf.alloc(sizer.off + extra);
                Arena ar{static_cast<char*>(b.buf.p), sizer.off + extra, 0};
                plan(ar, b.n_a, b.n_b, b.m, P, slots, fd_pair_entries(b.m, b.tune), b.w);
                int32_t* d_a = ar.take<int32_t>(std::max<int64_t>(b.m, 1));
                int32_t* d_b = ar.take<int32_t>(std::max<int64_t>(b.m, 1));
                b.d_theta = ar.take<int64_t>(std::max<int32_t>(b.n_a, 1));
                TIP_HIP_TRY(hipMemsetAsync(b.w.spill.dense, 0, sizeof(int32_t) * b.w.spill.stride * b.w.spill.slots, s));
                if (b.m > 0) {
                    TIP_HIP_TRY(hipMemcpyAsync(d_a, b.a_is_u ? g->eu : g->ev, sizeof(int32_t) * b.m,
                                               hipMemcpyHostToDevice, s));
                    TIP_HIP_TRY(hipMemcpyAsync(d_b, b.a_is_u ? g->ev : g->eu, sizeof(int32_t) * b.m,
                                               hipMemcpyHostToDevice, s));
                }
                b.rc = run_front(b.w, d_a, d_b, b.n_a, b.n_b, b.m, b.a_is_u, P, flags, b.tune, true, false, b.rs, s);
                if (b.rc != TIP_OK) b.err = last_error();
                TIP_HIP_TRY(hipStreamSynchronize(s));
            } catch (const AllocFailure& e) {
                b.rc = TIP_ENOMEM;
                b.err = e.msg;
            } catch (const HipFailure& e) {
                b.rc = TIP_EDEVICE;
                b.err = e.msg;
            } catch (const std::bad_alloc&) {
                b.rc = TIP_ENOMEM;
                b.err = "host allocation failed";
            } catch (...) {
                b.rc = TIP_EDEVICE;
                b.err = "unexpected internal error";
            }
            items[k] = std::move(it);
        }
        (void)hipStreamDestroy(s);
    };
    {
        std::vector<std::thread> pool;
        const int nw = std::min<int>(n, kBatchWorkers);
        for (int t = 0; t < nw; ++t) pool.emplace_back(worker);
        for (auto& t : pool) t.join();
    }
    for (int32_t k = 0; k < n; ++k) {
        if (!items[k]) {
            set_error("batch worker could not start");
            return TIP_EDEVICE;
        }
        if (items[k]->rc != TIP_OK) {
            set_error("graph " + std::to_string(k) + ": " + items[k]->err);
            return items[k]->rc;
        }
    }
    // one task list over all graphs, heaviest induced subgraph first
    StreamHolder sh;
    const hipStream_t s = sh.s;
    std::vector<FdJob> jobs;
    std::vector<std::pair<int64_t, int64_t>> tasks;  // (weight, job << 32 | subset)
    std::vector<int64_t> tw;
    int64_t stride = 64;
    for (int32_t k = 0; k < n; ++k) {
        BatchItem& b = *items[k];
        if (b.rs.S <= 0 || b.n_a <= 0) continue;
        tw.resize(b.rs.S);
        TIP_HIP_TRY(hipMemcpyAsync(tw.data(), b.w.fb.task_w, sizeof(int64_t) * b.rs.S, hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        const int64_t j = (int64_t)jobs.size();
        jobs.push_back(FdJob{b.w.g, b.w.fb, b.w.pb.init, b.w.ctl, b.tune.fd_help_min, b.tune.fd_help_chunk,
                             b.tune.fd_help_level_min, b.tune.fd_huc_pct,
                             b.tune.fd_dgm && b.tune.fd_huc_pct == 0 ? 1 : 0});
        for (int32_t i = 0; i < b.rs.S; ++i) tasks.emplace_back(tw[i], (j << 32) | i);
        stride = std::max(stride, b.w.spill.stride);
    }
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
                         return a.first > b.first;
                     });
    DeviceBuffer fdbuf;
    if (!tasks.empty()) {
        // five sub-allocations, each aligned by the arena
        const size_t bytes = sizeof(FdJob) * jobs.size() + sizeof(int64_t) * tasks.size() + sizeof(FdBoard) +
                             2 * sizeof(int32_t) * (size_t)stride * slots + 4096;
        fdbuf.alloc(bytes);
        Arena ar{static_cast<char*>(fdbuf.p), bytes, 0};
        FdJob* d_jobs = ar.take<FdJob>(jobs.size());
        int64_t* d_tasks = ar.take<int64_t>(tasks.size());
        FdBoard* d_board = ar.take<FdBoard>(1);
        SpillArena spill;
        spill.stride = stride;
        spill.slots = slots;
        spill.dense = ar.take<int32_t>(stride * slots);
        spill.list = ar.take<int32_t>(stride * slots);
        std::vector<int64_t> tv(tasks.size());
        for (size_t i = 0; i < tasks.size(); ++i) tv[i] = tasks[i].second;
        TIP_HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(FdJob) * jobs.size(), hipMemcpyHostToDevice, s));
        TIP_HIP_TRY(hipMemcpyAsync(d_tasks, tv.data(), sizeof(int64_t) * tv.size(), hipMemcpyHostToDevice, s));
        TIP_HIP_TRY(hipMemsetAsync(spill.dense, 0, sizeof(int32_t) * stride * slots, s));
        launch_fd_batch(d_jobs, d_tasks, (int32_t)tasks.size(), d_board, spill, slots, s);
    }
    for (int32_t k = 0; k < n; ++k) items[k]->rs.ev.rec(4, s);
    for (int32_t k = 0; k < n; ++k) {
        BatchItem& b = *items[k];
        RunOut out;
        out.theta = b.d_theta;
        run_back(b.w, b.n_a, b.n_b, true, out, b.rs, st ? &st[k] : nullptr, s);
        if (b.n_a > 0)
            TIP_HIP_TRY(hipMemcpyAsync(thetas[k], b.d_theta, sizeof(int64_t) * b.n_a, hipMemcpyDeviceToHost, s));
    }
    TIP_HIP_TRY(hipStreamSynchronize(s));
    return TIP_OK;
}

// ---------------------------------------------------------------------------
// Batch as one graph: the graphs (each with its decomposed side as side A)
// are laid side by side as one disjoint union -- graph k's A ids shifted by
// the A vertices of the graphs before it, its B ids likewise -- and the
// union is decomposed once.  No butterfly joins two graphs, so every
// vertex's count, its f over any set and its tip number are those of its own
// graph (tip numbers of a disjoint union are those of the parts); one
// ingest, one count, one coarse-grained round loop over the whole batch's
// activeSets (one device control block) and one fine-grained launch over
// every graph's subsets.
// ---------------------------------------------------------------------------

__global__ void k_add_offset(int32_t* a, int64_t n, int32_t off) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] += off;
}

// false (nothing done) when the union exceeds the id or edge limits
bool decompose_union(int32_t n, const tip_edges* gs, const int32_t* sides, int64_t* const* thetas, int32_t P,
                     int32_t flags, const Tune& tune, tip_stats* st, tip_status& rc) {
    int64_t na = 0, nb = 0, m = 0;
    for (int32_t k = 0; k < n; ++k) {
        const bool u = sides[k] == TIP_SIDE_U;
        na += u ? gs[k].n_u : gs[k].n_v;
        nb += u ? gs[k].n_v : gs[k].n_u;
        m += gs[k].m;
    }
    if (na > INT32_MAX || nb > INT32_MAX || m > INT32_MAX) return false;
    const int32_t n_a = (int32_t)na, n_b = (int32_t)nb;
    StreamHolder sh;
    const hipStream_t s = sh.s;
    Work w;
    const int slots = resident_workgroups();
    Arena sizer;
    plan(sizer, n_a, n_b, m, P, slots, fd_pair_entries(m, tune), w);
    const size_t extra = sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(m, 1) +
                         sizeof(int64_t) * (size_t)std::max<int32_t>(n_a, 1) + 4096;
    DeviceBuffer buf;
    buf.alloc(sizer.off + extra);
    Arena ar{static_cast<char*>(buf.p), sizer.off + extra, 0};
    plan(ar, n_a, n_b, m, P, slots, fd_pair_entries(m, tune), w);
    int32_t* d_a = ar.take<int32_t>(std::max<int64_t>(m, 1));
    int32_t* d_b = ar.take<int32_t>(std::max<int64_t>(m, 1));
    int64_t* d_theta = ar.take<int64_t>(std::max<int32_t>(n_a, 1));
    TIP_HIP_TRY(hipMemsetAsync(w.spill.dense, 0, sizeof(int32_t) * w.spill.stride * w.spill.slots, s));
    std::vector<int32_t> off_a(n + 1, 0);
    int64_t moff = 0;
    int32_t ob = 0;
    for (int32_t k = 0; k < n; ++k) {
        const tip_edges& g = gs[k];
        const bool u = sides[k] == TIP_SIDE_U;
        const int32_t ka = u ? g.n_u : g.n_v, kb = u ? g.n_v : g.n_u;
        if (g.m > 0) {
            TIP_HIP_TRY(hipMemcpyAsync(d_a + moff, u ? g.eu : g.ev, sizeof(int32_t) * g.m, hipMemcpyHostToDevice, s));
            TIP_HIP_TRY(hipMemcpyAsync(d_b + moff, u ? g.ev : g.eu, sizeof(int32_t) * g.m, hipMemcpyHostToDevice, s));
            const unsigned grid = (unsigned)std::min<int64_t>(4096, (g.m + 255) / 256);
            if (off_a[k]) k_add_offset<<<grid, 256, 0, s>>>(d_a + moff, g.m, off_a[k]);
            if (ob) k_add_offset<<<grid, 256, 0, s>>>(d_b + moff, g.m, ob);
            TIP_HIP_TRY(hipGetLastError());
        }
        moff += g.m;
        off_a[k + 1] = off_a[k] + ka;
        ob += kb;
    }
    RunOut out;
    out.theta = d_theta;
    tip_stats tot;
    rc = run(w, d_a, d_b, n_a, n_b, m, true, P, flags, tune, true, out, st ? &tot : nullptr, s);
    if (rc != TIP_OK) return true;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t ka = off_a[k + 1] - off_a[k];
        if (ka > 0)
            TIP_HIP_TRY(hipMemcpyAsync(thetas[k], d_theta + off_a[k], sizeof(int64_t) * ka, hipMemcpyDeviceToHost, s));
    }
    TIP_HIP_TRY(hipStreamSynchronize(s));
    if (st) {
        // one decomposition: its totals go to graph 0, the other entries are 0
        for (int32_t k = 0; k < n; ++k) std::memset(&st[k], 0, sizeof(tip_stats));
        if (n > 0) st[0] = tot;
    }
    return true;
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
constexpr int kMaxDevices = 64;

void* noalloc_scratch() {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = 0;
    TIP_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw InvalidArg("device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        TIP_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipFailure("hipGetSymbolAddress returned no address for the scratch array");
        ptr[dev] = p;
    }
    return ptr[dev];
}

}  // namespace
}  // namespace tip

using namespace tip;

extern "C" {

const char* tip_last_error(void) { return tip::last_error(); }

int32_t tip_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

tip_status tip_count_butterflies(const tip_edges* g, int64_t* bfly_u, int64_t* bfly_v, int64_t* total) {
    return guard([&]() -> tip_status {
        check_edges(g);
        const int32_t n_a = g->n_u, n_b = g->n_v;
        const int64_t m = g->m;
        StreamHolder sh;
        Work w;
        const int slots = resident_workgroups();
        Arena sizer;
        plan(sizer, n_a, n_b, m, 1, slots, 0, w);
        const size_t extra = sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(m, 1) +
                             sizeof(int64_t) * ((size_t)std::max(n_a, 1) + std::max(n_b, 1)) + 4096;
        DeviceBuffer buf;
        buf.alloc(sizer.off + extra);
        Arena ar{static_cast<char*>(buf.p), sizer.off + extra, 0};
        plan(ar, n_a, n_b, m, 1, slots, 0, w);
        int32_t* d_a = ar.take<int32_t>(std::max<int64_t>(m, 1));
        int32_t* d_b = ar.take<int32_t>(std::max<int64_t>(m, 1));
        int64_t* d_bu = ar.take<int64_t>(std::max(n_a, 1));
        int64_t* d_bv = ar.take<int64_t>(std::max(n_b, 1));
        const hipStream_t s = sh.s;
        TIP_HIP_TRY(hipMemsetAsync(w.spill.dense, 0, sizeof(int32_t) * w.spill.stride * w.spill.slots, s));
        if (m > 0) {
            TIP_HIP_TRY(hipMemcpyAsync(d_a, g->eu, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
            TIP_HIP_TRY(hipMemcpyAsync(d_b, g->ev, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        }
        RunOut out;
        out.bfly_a = d_bu;
        out.bfly_b = d_bv;
        const tip_status rc = run(w, d_a, d_b, n_a, n_b, m, true, 1, 0, Tune{}, false, out, nullptr, s);
        if (rc != TIP_OK) return rc;
        if (total) {
            k_sum_i64<<<1, 1024, 0, s>>>(w.cb.bfly_a, n_a, w.total);
            TIP_HIP_TRY(hipGetLastError());
        }
        int64_t tot2 = 0;
        if (bfly_u && n_a > 0)
            TIP_HIP_TRY(hipMemcpyAsync(bfly_u, d_bu, sizeof(int64_t) * n_a, hipMemcpyDeviceToHost, s));
        if (bfly_v && n_b > 0)
            TIP_HIP_TRY(hipMemcpyAsync(bfly_v, d_bv, sizeof(int64_t) * n_b, hipMemcpyDeviceToHost, s));
        if (total) TIP_HIP_TRY(hipMemcpyAsync(&tot2, w.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        if (total) *total = tot2 / 2;
        return TIP_OK;
    });
}

tip_status tip_decompose_ex(const tip_edges* g, int32_t side, int64_t* theta, const tip_opts* opt, tip_stats* st,
                            int32_t* subset, int64_t* init_support, int64_t* bounds, int32_t* n_subsets) {
    return guard([&]() -> tip_status {
        check_edges(g);
        if (side != TIP_SIDE_U && side != TIP_SIDE_V) throw InvalidArg("side must be 0 (U) or 1 (V)");
        const int32_t P = check_opts(opt);
        const int32_t n_side = side == TIP_SIDE_U ? g->n_u : g->n_v;
        if (n_side > 0 && !theta) throw InvalidArg("theta is NULL");
        return decompose_host(g, side, theta, P, opt ? opt->flags : 0, tune_of(opt), st, subset,
                              init_support, bounds, n_subsets);
    });
}

tip_status tip_decompose(const tip_edges* g, int32_t side, int64_t* theta, const tip_opts* opt, tip_stats* st) {
    return tip_decompose_ex(g, side, theta, opt, st, nullptr, nullptr, nullptr, nullptr);
}

tip_status tip_decompose_batch(int32_t n, const tip_edges* gs, const int32_t* sides, int64_t* const* thetas,
                               const tip_opts* opt, tip_stats* st) {
    return guard([&]() -> tip_status {
        if (n < 0) throw InvalidArg("negative batch size");
        if (n > 0 && (!gs || !sides || !thetas)) throw InvalidArg("batch arrays are NULL");
        const int32_t flags = opt ? opt->flags : 0;
        const bool per_graph = (flags & TIP_FLAG_OPTS_PER_GRAPH) != 0;
        // options of graph k: opt[k] with TIP_FLAG_OPTS_PER_GRAPH, else *opt
        std::vector<int32_t> Ps(std::max(n, 0));
        std::vector<Tune> tunes(std::max(n, 0));
        for (int32_t k = 0; k < n; ++k) {
            const tip_opts* ok = per_graph ? &opt[k] : opt;
            if (per_graph && ok->flags != flags) throw InvalidArg("per-graph options must carry the same flags");
            Ps[k] = check_opts(ok, true);
            tunes[k] = tune_of(ok);
        }
        if (!per_graph) check_opts(opt, true);
        for (int32_t k = 0; k < n; ++k) {
            check_edges(&gs[k]);
            if (sides[k] != TIP_SIDE_U && sides[k] != TIP_SIDE_V) throw InvalidArg("side must be 0 or 1");
            const int32_t n_side = sides[k] == TIP_SIDE_U ? gs[k].n_u : gs[k].n_v;
            if (n_side > 0 && !thetas[k]) throw InvalidArg("theta is NULL");
        }
        const int32_t run_flags = flags & ~(TIP_FLAG_OPTS_PER_GRAPH | TIP_FLAG_BATCH_STREAMS);
        if (!(flags & (TIP_FLAG_BATCH_PLAIN | TIP_FLAG_BATCH_STREAMS)) && !per_graph && n > 0) {
            tip_status rc = TIP_OK;
            if (decompose_union(n, gs, sides, thetas, Ps[0], run_flags, tunes[0], st, rc)) return rc;
        }
        if (!(flags & TIP_FLAG_BATCH_PLAIN)) return decompose_batched(n, gs, sides, thetas, Ps, run_flags, tunes, st);
        // the plain form: one full decomposition after another
        for (int32_t k = 0; k < n; ++k) {
            const tip_status rc = decompose_host(&gs[k], sides[k], thetas[k], Ps[k], run_flags, tunes[k],
                                                 st ? &st[k] : nullptr, nullptr, nullptr, nullptr, nullptr);
            if (rc != TIP_OK) return rc;
        }
        return TIP_OK;
    });
}

tip_status tip_decompose_noalloc(const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                                 int32_t side, int64_t* d_theta, void* stream, const tip_opts* opt, tip_stats* st) {
    return guard([&]() -> tip_status {
        if (n_u < 0 || n_v < 0 || m < 0 || m > INT32_MAX) throw InvalidArg("bad graph size");
        if (m > 0 && (!d_eu || !d_ev)) throw InvalidArg("edge arrays are NULL");
        if (side != TIP_SIDE_U && side != TIP_SIDE_V) throw InvalidArg("side must be 0 or 1");
        const int32_t P = check_opts(opt);
        const int32_t flags = opt ? opt->flags : 0;
        if (flags & TIP_FLAG_TIME_KERNELS) throw InvalidArg("TIP_FLAG_TIME_KERNELS needs events, which this call does not create");
        const bool a_is_u = side == TIP_SIDE_U;
        const int32_t n_a = a_is_u ? n_u : n_v, n_b = a_is_u ? n_v : n_u;
        if (n_a > 0 && !d_theta) throw InvalidArg("theta is NULL");
        Work w;
        w.no_alloc = true;
        Arena sizer;
        const int slots = resident_workgroups();
        plan(sizer, n_a, n_b, m, P, slots, 0, w);
        if (sizer.off > kNoAllocScratchBytes)
            throw AllocFailure("graph needs " + std::to_string(sizer.off) + " bytes of scratch; tip_decompose_noalloc "
                               "holds " + std::to_string(kNoAllocScratchBytes) + " (use tip_decompose_async)");
        Arena ar{static_cast<char*>(noalloc_scratch()), kNoAllocScratchBytes, 0};
        plan(ar, n_a, n_b, m, P, slots, 0, w);
        const hipStream_t s = static_cast<hipStream_t>(stream);
        // the scratch keeps the previous call's contents: the repeat-count
        // spill area must start at zero (everything else is written before
        // it is read, as with a fresh workspace)
        fill_i32(w.spill.dense, 0, w.spill.stride * w.spill.slots, s);
        RunOut out;
        out.theta = d_theta;
        return run(w, a_is_u ? d_eu : d_ev, a_is_u ? d_ev : d_eu, n_a, n_b, m, a_is_u, P, flags, tune_of(opt), true,
                   out, st, s);
    });
}

// Host-pointer calls on the edge-peeling path: ingest, then wing_run or
// ktip_run, results copied back in input order.
struct EdgeCall {
    StreamHolder sh;
    WingWork w;
    DeviceBuffer buf;
    int32_t* d_eu = nullptr;
    int32_t* d_ev = nullptr;
    int64_t* d_scalar = nullptr;
    int32_t* d_comp = nullptr;

    EdgeCall(const tip_edges* g, bool ktip, int32_t side) {
        const int64_t m = g->m;
        const int32_t n_a = ktip && side == TIP_SIDE_V ? g->n_v : g->n_u;
        const int32_t n_b = ktip && side == TIP_SIDE_V ? g->n_u : g->n_v;
        const int slots = wing_slots();
        Arena sizer;
        wing_plan(sizer, n_a, n_b, m, slots, ktip, w);
        const size_t extra = sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(m, 1) +
                             sizeof(int32_t) * (size_t)std::max(n_a, 1) + 4096;
        buf.alloc(sizer.off + extra);
        Arena ar{static_cast<char*>(buf.p), sizer.off + extra, 0};
        wing_plan(ar, n_a, n_b, m, slots, ktip, w);
        d_eu = ar.take<int32_t>(std::max<int64_t>(m, 1));
        d_ev = ar.take<int32_t>(std::max<int64_t>(m, 1));
        d_scalar = ar.take<int64_t>(1);
        d_comp = ar.take<int32_t>(std::max(n_a, 1));
        if (m > 0) {
            TIP_HIP_TRY(hipMemcpyAsync(d_eu, g->eu, sizeof(int32_t) * m, hipMemcpyHostToDevice, sh.s));
            TIP_HIP_TRY(hipMemcpyAsync(d_ev, g->ev, sizeof(int32_t) * m, hipMemcpyHostToDevice, sh.s));
        }
    }
};

tip_status tip_count_edge_butterflies(const tip_edges* g, int64_t* bfly_e, int64_t* total) {
    return guard([&]() -> tip_status {
        check_edges(g);
        if (g->m > 0 && !bfly_e && !total) throw InvalidArg("bfly_e and total are both NULL");
        EdgeCall c(g, false, TIP_SIDE_U);
        const hipStream_t s = c.sh.s;
        const int64_t m = g->m;
        const tip_status rc = wing_run(c.w, c.d_eu, c.d_ev, g->n_u, g->n_v, m, false, c.w.out, nullptr, s);
        if (rc != TIP_OK) return rc;
        int64_t sum = 0;
        if (total && c.w.g.m > 0) {
            k_sum_i64<<<1, 1024, 0, s>>>(c.w.supp, (int32_t)c.w.g.m, c.d_scalar);
            TIP_HIP_TRY(hipGetLastError());
            TIP_HIP_TRY(hipMemcpyAsync(&sum, c.d_scalar, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        }
        if (m > 0 && bfly_e)
            TIP_HIP_TRY(hipMemcpyAsync(bfly_e, c.w.out, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        if (total) *total = sum / 4;  // every butterfly has four edges
        return TIP_OK;
    });
}

tip_status tip_wing_decompose(const tip_edges* g, int64_t* psi, const tip_opts* opt, tip_stats* st) {
    return guard([&]() -> tip_status {
        check_edges(g);
        if (g->m > 0 && !psi) throw InvalidArg("psi is NULL");
        if (opt && (opt->P != 0 || opt->flags != 0 || std::any_of(opt->tune, opt->tune + 8, [](int32_t t) { return t != 0; })))
            throw InvalidArg("tip_wing_decompose takes no options yet: opt must be NULL or all zero");
        EdgeCall c(g, false, TIP_SIDE_U);
        const hipStream_t s = c.sh.s;
        const int64_t m = g->m;
        const tip_status rc = wing_run(c.w, c.d_eu, c.d_ev, g->n_u, g->n_v, m, true, c.w.out, st, s);
        if (rc != TIP_OK) return rc;
        if (m > 0) TIP_HIP_TRY(hipMemcpyAsync(psi, c.w.out, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        return TIP_OK;
    });
}

tip_status tip_ktips(const tip_edges* g, int32_t side, const int64_t* theta, int64_t k, int32_t* comp) {
    return guard([&]() -> tip_status {
        check_edges(g);
        if (side != TIP_SIDE_U && side != TIP_SIDE_V) throw InvalidArg("side must be 0 (U) or 1 (V)");
        const int32_t n_side = side == TIP_SIDE_U ? g->n_u : g->n_v;
        if (n_side > 0 && (!theta || !comp)) throw InvalidArg("theta or comp is NULL");
        for (int32_t x = 0; x < n_side; ++x)
            if (theta[x] < 0) throw InvalidArg("tip numbers are never negative");
        EdgeCall c(g, true, side);
        const hipStream_t s = c.sh.s;
        const tip_status rc = ktip_run(c.w, c.d_eu, c.d_ev, g->n_u, g->n_v, g->m, side, theta, k, c.d_comp, s);
        if (rc != TIP_OK) return rc;
        if (n_side > 0) TIP_HIP_TRY(hipMemcpyAsync(comp, c.d_comp, sizeof(int32_t) * n_side, hipMemcpyDeviceToHost, s));
        TIP_HIP_TRY(hipStreamSynchronize(s));
        return TIP_OK;
    });
}

tip_status tip_workspace_size(int32_t n_u, int32_t n_v, int64_t m, int32_t side, const tip_opts* opt,
                              size_t* bytes) {
    return guard([&]() -> tip_status {
        if (!bytes) throw InvalidArg("bytes is NULL");
        if (n_u < 0 || n_v < 0 || m < 0 || m > INT32_MAX) throw InvalidArg("bad graph size");
        if (side != TIP_SIDE_U && side != TIP_SIDE_V) throw InvalidArg("side must be 0 or 1");
        const int32_t P = check_opts(opt);
        const int32_t n_a = side == TIP_SIDE_U ? n_u : n_v, n_b = side == TIP_SIDE_U ? n_v : n_u;
        Work w;
        Arena sizer;
        plan(sizer, n_a, n_b, m, P, resident_workgroups(), fd_pair_entries(m, tune_of(opt)), w);
        *bytes = sizer.off + 256;
        return TIP_OK;
    });
}

tip_status tip_decompose_async(const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                               int32_t side, int64_t* d_theta, void* d_workspace, size_t ws_bytes, void* stream,
                               const tip_opts* opt, tip_stats* st) {
    return guard([&]() -> tip_status {
        if (n_u < 0 || n_v < 0 || m < 0 || m > INT32_MAX) throw InvalidArg("bad graph size");
        if (m > 0 && (!d_eu || !d_ev)) throw InvalidArg("edge arrays are NULL");
        if (side != TIP_SIDE_U && side != TIP_SIDE_V) throw InvalidArg("side must be 0 or 1");
        const int32_t P = check_opts(opt);
        const bool a_is_u = side == TIP_SIDE_U;
        const int32_t n_a = a_is_u ? n_u : n_v, n_b = a_is_u ? n_v : n_u;
        if (n_a > 0 && !d_theta) throw InvalidArg("theta is NULL");
        if (!d_workspace) throw InvalidArg("workspace is NULL");
        Work w;
        Arena sizer;
        const int slots = resident_workgroups();
        plan(sizer, n_a, n_b, m, P, slots, fd_pair_entries(m, tune_of(opt)), w);
        if (ws_bytes < sizer.off) throw AllocFailure("workspace smaller than tip_workspace_size");
        Arena ar{static_cast<char*>(d_workspace), ws_bytes, 0};
        plan(ar, n_a, n_b, m, P, slots, fd_pair_entries(m, tune_of(opt)), w);
        const hipStream_t s = static_cast<hipStream_t>(stream);
        TIP_HIP_TRY(hipMemsetAsync(w.spill.dense, 0, sizeof(int32_t) * w.spill.stride * w.spill.slots, s));
        RunOut out;
        out.theta = d_theta;
        return run(w, a_is_u ? d_eu : d_ev, a_is_u ? d_ev : d_eu, n_a, n_b, m, a_is_u, P, opt ? opt->flags : 0,
                   tune_of(opt), true, out, st, s);
    });
}

}  // extern "C"
