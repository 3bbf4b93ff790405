/*
 * tip.h -- C ABI of libtip: butterfly counting and tip decomposition of
 * bipartite graphs on an AMD Instinct MI355X (gfx950).
 *
 * Method: Lakhotia, Kannan, Prasanna, De Rose, "RECEIPT: REfine CoarsE-grained
 * IndePendent Tasks for Parallel Tip decomposition of Bipartite Graphs"
 * (arXiv 2010.08695).
 *
 * Conventions shared by every call
 *   - A graph is given as a COO edge list: edge i joins U vertex eu[i] and V
 *     vertex ev[i]; ids are 0-based, eu[i] < n_u, ev[i] < n_v.  Duplicate
 *     edges are merged (the method is defined on simple graphs).  Isolated
 *     vertices are allowed and get count 0 and tip number 0.
 *   - All counts and tip numbers are exact signed 64-bit integers.
 *   - The caller owns every buffer.  Host-pointer calls copy their inputs to
 *     the device, allocate and free their own device memory and return after
 *     the results are in the caller's host buffers.
 *   - Every call returns a tip_status.  Nothing throws across the ABI.  On an
 *     error the output buffers are unspecified and tip_last_error() describes
 *     the failure.  Argument errors (TIP_EINVAL) are detected on the host
 *     before any device work and leave the outputs untouched.
 *   - Calls may be made concurrently from several host threads; each call
 *     uses its own device memory and stream.
 */
#ifndef TIP_H
#define TIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tip_status;
enum {
    TIP_OK = 0,
    TIP_EINVAL = -1,    /* NULL required pointer, id out of range, bad side, negative or too large size */
    TIP_ENOMEM = -2,    /* device or host allocation failed, or the workspace is too small */
    TIP_EDEVICE = -3,   /* a HIP runtime error; tip_last_error() holds the HIP message */
    TIP_EOVERFLOW = -4, /* reserved: no call returns it.  With m <= 2^31 - 1 no count can
                           overflow: the counts of either side sum to at most
                           1/2 * sum over edges (x, y) of (d_x - 1)(d_y - 1) < m^2 / 2 < 2^61
                           (c(x, w) <= d_x bounds every shared-butterfly term C(c, 2)) */
    TIP_EBUSY = -5      /* reserved */
};

/* The vertex side to decompose.  The paper decomposes one side at a time
 * (Background section); deciding V is deciding U of the transposed graph. */
typedef enum { TIP_SIDE_U = 0, TIP_SIDE_V = 1 } tip_side;

/* Host COO edge list.  m <= 2^31 - 1. */
typedef struct {
    int32_t n_u, n_v;
    int64_t m;
    const int32_t* eu; /* [m] U ids */
    const int32_t* ev; /* [m] V ids */
} tip_edges;

/* TIP_FLAG_TIME_KERNELS: time every launch of the coarse-grained dense
 * update kernel (k_peel_dense: (vertex, key range) work items with LDS
 * counters; the single kernel with the most device time on power-law
 * graphs) with HIP events on the call's stream and report it in
 * tip_stats.peel_*.  Rounds are then launched from the host. */
#define TIP_FLAG_TIME_KERNELS 1

/* TIP_FLAG_NO_GRAPH: launch every coarse-grained round from the host
 * instead of replaying a HIP graph of several rounds (same results; for
 * testing and comparison).  TIP_FLAG_TIME_KERNELS implies it. */
#define TIP_FLAG_NO_GRAPH 2

/* TIP_FLAG_BATCH_PLAIN: tip_decompose_batch runs one full decomposition
 * after another (the plain per-graph launch sequence) instead of the batched
 * form; same results, for comparison. */
#define TIP_FLAG_BATCH_PLAIN 4

/* TIP_FLAG_NO_COMPACT: never remove peeled vertices from the adjacency
 * lists the coarse-grained update traverses (Dynamic Graph Maintenance
 * section; on by default).  Same results, more wedges traversed. */
#define TIP_FLAG_NO_COMPACT 8

/* TIP_FLAG_OPTS_PER_GRAPH (tip_decompose_batch only): `opt` points to n
 * tip_opts, one per graph, instead of one for all; graph k runs with
 * opt[k].P and opt[k].tune (for example each graph's autotuned values).
 * Every opt[k].flags must be equal and carry this bit. */
#define TIP_FLAG_OPTS_PER_GRAPH 16

/* TIP_FLAG_BATCH_STREAMS: tip_decompose_batch runs the graphs' counting and
 * coarse-grained steps concurrently on several host threads and streams,
 * then one fine-grained launch over all graphs' subsets (the batched form
 * used with TIP_FLAG_OPTS_PER_GRAPH, or when the batch's disjoint union
 * would exceed 2^31 - 1 ids or edges); same results. */
#define TIP_FLAG_BATCH_STREAMS 32

/* TIP_FLAG_FD_DGM: Dynamic Graph Maintenance (Section 4.2) in the
 * fine-grained step too: a subset kept in HBM removes its peeled vertices
 * from the neighbour runs of its induced subgraph G_i each time the updates
 * since the last compaction walked as many wedges as G_i has edges (the
 * section's trigger).  Not combined with tune[7] (a HUC re-count there
 * needs the peeled vertices).  Same results, fewer wedges traversed. */
#define TIP_FLAG_FD_DGM 64

/* TIP_FLAG_DGM_PAPER: the coarse-grained step compacts its lists at a range
 * start once the wedges traversed since the last compaction reach the
 * entries left (Section 4.2's trigger), instead of tune[2]'s share of
 * entries held by peeled vertices.  Same results. */
#define TIP_FLAG_DGM_PAPER 128

/* TIP_FLAG_FD_WALK: every update of the fine-grained step walks the peeled
 * vertex's wedges inside G_i (Alg. 4 as written) instead of reading its
 * pair row.  By default, before peeling, each vertex u of a subset U_i gets
 * the list of every w in U_i with c = |N(u) ∩ N(w)| >= 2 and C(c, 2): the
 * update of u in Alg. 4, which does not change while U_i is peeled because
 * the other side is never peeled.  The rows of a subset are built only if
 * they fit the workspace's pair budget (16 entries of 12 bytes per edge, at
 * most 2^31 entries; tip_workspace_size includes it);
 * other subsets, and every subset under TIP_FLAG_FD_DGM or tune[7], walk.
 * Same results. */
#define TIP_FLAG_FD_WALK 256

/* Options.  Zero-initialised means defaults. */
typedef struct {
    int32_t P;       /* number of tip-number ranges of the coarse-grained step
                        (Alg. 3); 0 = 150, the value the paper's experiments
                        settle on; at most 65535 */
    int32_t flags;   /* TIP_FLAG_* bits; other bits must be 0 */
    int32_t tune[8]; /* update-kernel selection of the coarse-grained step;
                        a vertex of degree d with w wedges in its 2-hop
                        neighbourhood is updated by the dense key-range
                        kernel when w > tune[1] and w > k * bits(d) /
                        tune[0] (bits(d) = 2, 4, 8, 16, 32 for d <= 3, 15,
                        255, 65535, above; k = ids below the largest live
                        one), and one
                        list tile of such counters fits the LDS, else by a
                        per-vertex kernel;
                        tune[0]: 0 = 1024; tune[1]: 0 = 2048;
                        tune[2]: compaction of the traversed lists at a
                        range start once the entries of vertices peeled
                        since the last compaction reach tune[2] per mille of
                        the entries left (0 = 125);
                        tune[3]: HUC (Section 4.1): a coarse-grained round
                        whose peel work (wedge proxy of its activeSet) exceeds
                        tune[3] percent of the re-count work (counting wedges
                        scaled by the live share of the side) re-counts the
                        live vertices' supports instead of applying the
                        round's decrements; 0 = never (the default; on the
                        GPU a re-count costs about nine times a peel per
                        wedge), 100 = the rule of the paper; the results do
                        not change;
                        tune[4..6]: the fine-grained step's help board
                        (Alg. 4 subsets large enough let idle workgroups
                        take their per-wave updates): tune[4] updates taken
                        per claim (0 = 16, at most 2^20), tune[5] fewest
                        updates of a level worth publishing (0 = 256),
                        tune[6] smallest subset that opens a slot (0 =
                        4096); the results do not change;
                        tune[7]: HUC in the fine-grained step (Section 4.1,
                        last paragraph): a step of a subset kept in HBM
                        whose peeled vertices' induced wedges exceed
                        tune[7] percent of the live vertices' re-counts
                        the live supports instead (support at the range
                        start minus the butterflies shared with the
                        subset's peeled vertices); 0 = never (the
                        default); the results do not change;
                        tune[0..7] >= 0 */
} tip_opts;

/* Work and time accounting of one decomposition (NULL = not wanted). */
typedef struct {
    int64_t wedges_count; /* wedges traversed by per-vertex counting (Alg. 1) */
    int64_t wedges_cd;    /* wedges traversed by coarse-grained peeling (Alg. 3) */
    int64_t wedges_fd;    /* wedges traversed by fine-grained peeling (Alg. 4) */
    int64_t pair_updates; /* support decrements issued: (peeled, other) pairs with c >= 2; a pair
                             whose other vertex is already peeled may be counted, its support is
                             never read again */
    int64_t rounds;       /* coarse-grained peeling iterations (synchronisation rounds) */
    int64_t subsets;      /* vertex subsets created (P, plus 1 if vertices were left over) */
    int64_t fd_levels;    /* peeling levels run by the fine-grained step */
    int64_t spills;       /* repeat keys that did not fit in LDS (kept in HBM) */
    int64_t skipped;      /* peeled vertices with no butterfly left (no update needed) */
    int64_t m_unique;     /* edges after duplicate merging */
    /* the coarse-grained dense update kernel alone (k_peel_dense) */
    int64_t peel_launches; /* launches */
    int64_t peel_wedges;   /* wedges it traversed */
    int64_t peel_edges;    /* first-hop edges (u, v) it read */
    int64_t peel_pairs;    /* support decrements it applied */
    double peel_ms;        /* summed launch time (TIP_FLAG_TIME_KERNELS), else 0 */
    double t_ingest_ms, t_count_ms, t_cd_ms, t_fd_ms, t_total_ms; /* device time per phase */
    int64_t huc_rounds;    /* coarse-grained rounds that re-counted instead of peeling (tune[3]) */
    int64_t fd_huc_steps;  /* fine-grained steps that re-counted instead of peeling (tune[7]) */
    int64_t compactions;   /* list compactions: coarse-grained (low 32 bits) + fine-grained << 32 */
    int64_t fd_pair_entries; /* entries of the fine-grained pair rows built (TIP_FLAG_FD_WALK) */
    int64_t fd_pair_subsets; /* subsets peeled from pair rows; the others walked their wedges */
} tip_stats;

/* Per-vertex butterfly counts of both sides (Alg. 1, Section 2.1) and the
 * total number of butterflies.  bfly_u [n_u], bfly_v [n_v] and total may each
 * be NULL.  Sum of bfly_u = sum of bfly_v = 2 * total. */
tip_status tip_count_butterflies(const tip_edges* g, int64_t* bfly_u, int64_t* bfly_v, int64_t* total);

/* Tip numbers of every vertex of `side` (Def. 1; RECEIPT: Alg. 3 then Alg. 4).
 * theta has n_u (side U) or n_v (side V) entries.  opt and st may be NULL. */
tip_status tip_decompose(const tip_edges* g, int32_t side, int64_t* theta, const tip_opts* opt, tip_stats* st);

/* tip_decompose plus the coarse-grained state (Alg. 3 outputs), for checking:
 *   subset       [n_side]  index i of the range R_i = [bounds[i], bounds[i+1])
 *                          holding the vertex's tip number, or NULL
 *   init_support [n_side]  support of the vertex when its subset's range
 *                          began (the support-initialisation vector), or NULL
 *   bounds       [P + 2]   range bounds; bounds[0] = 0, the last used bound of
 *                          a left-over subset is INT64_MAX, or NULL
 *   n_subsets              number of subsets created, or NULL */
tip_status tip_decompose_ex(const tip_edges* g, int32_t side, int64_t* theta, const tip_opts* opt,
                            tip_stats* st, int32_t* subset, int64_t* init_support, int64_t* bounds,
                            int32_t* n_subsets);

/* Decomposes n independent graphs: graph k's side sides[k] into thetas[k].
 * Batched form (default): the graphs, each with its decomposed side first,
 * are laid side by side as one disjoint union (no butterfly joins two of
 * them, so each part keeps its own tip numbers) and the union is decomposed
 * once: one ingest, one count, one coarse-grained round loop whose rounds
 * take every graph's activeSet, and one fine-grained launch over every
 * graph's subsets.  st may be NULL or point to n entries; in this form
 * st[0] receives the totals of the whole batch and the other entries are
 * zero.  With TIP_FLAG_OPTS_PER_GRAPH, TIP_FLAG_BATCH_STREAMS, or a union
 * beyond 2^31 - 1 ids or edges, the graphs run concurrently on host threads
 * and streams instead, with one fine-grained launch over all graphs'
 * subsets ordered by induced wedges, and st[k] holds graph k's figures.
 * TIP_FLAG_BATCH_PLAIN runs one full decomposition after another.  Results
 * are identical in every form. */
tip_status tip_decompose_batch(int32_t n, const tip_edges* gs, const int32_t* sides, int64_t* const* thetas,
                               const tip_opts* opt, tip_stats* st);

/* Device-memory bytes tip_decompose_async needs for a graph of this size
 * (m counted before duplicate merging). */
tip_status tip_workspace_size(int32_t n_u, int32_t n_v, int64_t m, int32_t side, const tip_opts* opt,
                              size_t* bytes);

/* Device-resident variant for callers that keep graphs on the GPU.
 *   d_eu, d_ev  device COO arrays [m]
 *   d_theta     device output [n_u or n_v]
 *   d_workspace device buffer of ws_bytes >= tip_workspace_size(...)
 *   stream      a hipStream_t (NULL = the default stream)
 * Uses no device memory besides the workspace and the outputs and issues all
 * work on `stream`.  The call returns once the decomposition is complete (the
 * coarse-grained step reads a few control words back between peeling rounds).
 * Id range errors are detected on the device and reported as TIP_EINVAL. */
tip_status tip_decompose_async(const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                               int32_t side, int64_t* d_theta, void* d_workspace, size_t ws_bytes, void* stream,
                               const tip_opts* opt, tip_stats* st);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): tip_decompose_async without a workspace
 * argument.  The scratch holds no pair rows, so the fine-grained step walks
 * every update's wedges (as with TIP_FLAG_FD_WALK; same results).  The
 * library's scratch is a static device array of 512 MiB per
 * device, created when the library's device code is loaded and held until
 * the process ends; the call itself allocates nothing (no device, pinned or
 * library memory, no HIP graph, no events).
 *   d_eu, d_ev  device COO arrays [m]; d_theta device output [n_u or n_v]
 *   stream      a hipStream_t (NULL = the default stream); all work is issued
 *               on it and the call returns once the decomposition is done
 *               (the coarse-grained step reads a few control words back
 *               between rounds, so the call cannot be captured in a graph)
 *   opt, st     as for tip_decompose_async; TIP_FLAG_TIME_KERNELS is
 *               rejected and the t_*_ms times of st read 0
 * Graphs whose tip_workspace_size with TIP_FLAG_FD_WALK exceeds 512 MiB are
 * refused with TIP_ENOMEM before any device work.  Every call on one device shares that
 * device's scratch and leaves its contents behind: calls that overlap on one
 * device (from several host threads or streams) race and must be
 * serialised by the caller. */
tip_status tip_decompose_noalloc(const int32_t* d_eu, const int32_t* d_ev, int32_t n_u, int32_t n_v, int64_t m,
                                 int32_t side, int64_t* d_theta, void* stream, const tip_opts* opt, tip_stats* st);

/* Butterflies containing each edge: bfly_e[i] for input edge i (duplicates of
 * one edge get the same value), and the total number of butterflies (every
 * butterfly has four edges).  The edge analogue of the per-vertex counts of
 * Section 2.1: for e = (u, v) it is the sum over u' != u adjacent to v of
 * |N_u intersect N_u'| - 1.  bfly_e [m] or total may be NULL (not both when
 * m > 0). */
tip_status tip_count_edge_butterflies(const tip_edges* g, int64_t* bfly_e, int64_t* total);

/* Wing numbers (edge peeling, the extension of the method to edges named in
 * the Extensions section): psi[i] for input edge i is the largest k such that the edge
 * lies in a k-wing, a subgraph in which every edge is in at least k
 * butterflies.  Computed by level-synchronous bottom-up edge peeling: each
 * round removes every live edge whose support is at most the current level,
 * and a butterfly with several edges removed in the same round is taken out
 * of the surviving edges' supports once, by its removed edge of smallest id.
 * opt must be NULL or all zero.  st (NULL ok): wedges_count = wedges walked
 * by the per-edge count, wedges_cd = (x', y'') pairs walked by peeling,
 * pair_updates = support decrements, rounds = peeling rounds, fd_levels =
 * distinct levels, m_unique; other fields 0. */
tip_status tip_wing_decompose(const tip_edges* g, int64_t* psi, const tip_opts* opt, tip_stats* st);

/* k-tips (Def. 1) of `side`: comp[x] = the smallest vertex id of the k-tip
 * holding x, or -1 when theta[x] < k.  theta [n_side] holds the side's tip
 * numbers (from tip_decompose); the k-tips are the butterfly-connected
 * components of {x : theta[x] >= k}, two vertices being connected when they
 * share at least two neighbours.  k may be any value (k <= 0 takes every
 * vertex; a vertex in no butterfly is then a k-tip of its own). */
tip_status tip_ktips(const tip_edges* g, int32_t side, const int64_t* theta, int64_t k, int32_t* comp);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next tip_* call on this thread. */
const char* tip_last_error(void);

/* Number of HIP devices visible to the library (0 if none). */
int32_t tip_device_count(void);

#ifdef __cplusplus
}
#endif

#endif /* TIP_H */
