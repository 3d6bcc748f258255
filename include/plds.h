/*
 * plds.h -- C ABI of the MI355X (gfx950) batch-dynamic approximate k-core
 * library: the parallel level data structure (PLDS) of Liu, Shi, Yu,
 * Dhulipala and Shun, "Parallel Batch-Dynamic Algorithms for k-Core
 * Decomposition and Related Graph Problems" (SPAA'22, arXiv 2106.03824).
 *
 * The structure keeps, for an undirected graph on vertices 0..n-1 that changes
 * by batches of edge insertions and deletions (problem statement,
 * Preliminaries: batch-dynamic setting), a level for every vertex such that
 * Invariants 1 and 2 hold (Section "Detailed PLDS Algorithm"), and from it a
 * (2+3/lambda)(1+delta)-approximate coreness estimate (Def. coreness
 * estimate, Lemma decomp-bound).
 *
 * Conventions for every function:
 *   - return value: PLDS_OK (0) or a negative PLDS_E* code; nothing throws.
 *   - "device pointer": memory the caller allocated on the GPU of the handle
 *     (hipMalloc or a torch CUDA tensor).  The caller owns it and keeps it
 *     alive until the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is ordered on it.  Batch calls (insert/delete/update/load_state)
 *     return only after their work on `stream` is complete; plds_coreness,
 *     plds_levels and plds_degrees only enqueue work.  Batch calls block
 *     because the host drives the level loops: it issues prebuilt graphs of
 *     level steps and reads the small control block back between them to
 *     learn whether a sweep has ended (a few host round trips per call; the
 *     count is in plds_stats_t.host_syncs).  The HIP graphs of this
 *     toolchain have no conditional nodes, and a persistent kernel with grid
 *     barriers (sweep mode 0) measures slower, so a call cannot end its own
 *     loop on the device.  Device errors are latched in the control block and
 *     returned by the call that meets them.
 *   - a handle is not thread-safe; distinct handles are independent.
 *   - vertex ids are int32 in [0, n); n <= 2^31 - 1.
 */
#ifndef PLDS_H
#define PLDS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLDS_OK 0
#define PLDS_EINVAL -1 /* bad argument: n < 1, delta <= 0, lambda <= 0, NULL, count < 0 */
#define PLDS_ERANGE -2 /* a vertex id outside [0, n); the batch is rejected, state unchanged */
#define PLDS_ENOMEM -3 /* device or host allocation failed; state unchanged            */
#define PLDS_EHIP -4   /* a HIP runtime call failed; the handle should be destroyed     */
#define PLDS_ESTATE -5 /* an internal consistency check failed (see plds_check)          */

typedef struct plds plds_t;

typedef struct {
    int64_t n;          /* number of vertices                                         */
    int64_t m;          /* current number of undirected edges                         */
    int32_t t;          /* least t >= 0 with (1+delta)^t >= n                          */
    int32_t L;          /* levels per group (default 4t, at least 1)                  */
    int32_t G;          /* number of groups, t+1                                      */
    int32_t K;          /* number of levels, G*L                                      */
    double delta, lambda;
    int64_t slab_slots; /* adjacency slots allocated (pool capacity, int32 each)     */
    int64_t slab_used;  /* slots handed out (live slabs plus abandoned ones)          */
    int32_t ngraphs;    /* graphs held by the handle (1 unless made by plds_create_multi) */
    int32_t reserved32;
} plds_info_t;

typedef struct {
    int64_t applied_ins;   /* unique new edges inserted by the last batch call          */
    int64_t applied_del;   /* unique present edges deleted by the last batch call       */
    int64_t sweeps_ins;    /* levels at which some vertex moved up                      */
    int64_t sweeps_del;    /* levels to which some vertex moved down                    */
    int64_t moves_up;      /* one-level up-moves                                         */
    int64_t moves_down;    /* down-moves (each vertex at most once per batch)            */
    int64_t dl_calcs;      /* desire-level computations                                  */
    int64_t slots_scanned; /* adjacency slots read by the level sweeps                   */
    int64_t top_level;     /* highest level reached during the call                      */
    int64_t viol_ins0;     /* Invariant-1 violators right after the insertions           */
    int64_t viol_del0;     /* Invariant-2 violators right after the deletions            */
    int64_t host_syncs;    /* host round trips made by the call                          */
    int64_t alg_bytes_up;  /* algorithmic bytes of the up-moves: 8 per up-neighbour read,
                              8 per counter update of a neighbour one level up, 4 per
                              level write (the paper's U[v] scan model)                 */
    int64_t timed_launches;/* launches of the kernel selected by plds_set_timing         */
    double timed_ms;       /* their summed duration in ms, from HIP events on `stream`   */
    int64_t alg_bytes_peel;/* algorithmic bytes of the static peeling's relax kernel, summed
                              over plds_static_kcore calls: 8 per adjacency slot (id and
                              bucket; 2m per call), 8 per count update of an alive
                              neighbour of a peeled vertex                              */
    int64_t alg_bytes_up_loop; /* the part of alg_bytes_up moved by the single-block loop of
                              small insertion steps (the rest by the insertion scan
                              kernel)                                                   */
    int64_t ins_steps;     /* level steps of the insertion sweeps (a multi-level step counts once) */
    int64_t ins_loop_steps;/* of those, the steps run by the single-block loop           */
    int64_t ins_loop_launches; /* launches of that loop that found a sweep running       */
} plds_stats_t;

/* Create an empty structure on the current HIP device: all n vertices at
 * level 0, no edges.  delta > 0 and lambda > 0 are the constants of
 * Invariants 1-2.  Groups g_0..g_t with t = ceil(log_{1+delta} n), each of
 * 4t levels (Section "Detailed PLDS Algorithm"). */
int plds_create(int64_t n, double delta, double lambda, plds_t **out);

/* As plds_create; levels_per_group > 0 overrides 4t (e.g. 3 for the paper's
 * worked examples), PLDS_LPG_OPT selects the experiments' PLDSOpt variant
 * (ceil(log_{1+delta} n / 50) levels per group, that is ceil(t / 50): fewer
 * levels, a looser approximation); edge_capacity_hint (>= 0) pre-sizes the
 * adjacency pool. */
#define PLDS_LPG_OPT (-1)
int plds_create_ex(int64_t n, double delta, double lambda, int32_t levels_per_group, int64_t edge_capacity_hint,
                   plds_t **out);

/* Options of plds_create_opts (zero-initialise, then set what differs):
 *   levels_per_group, edge_capacity_hint: as plds_create_ex;
 *   up_coeff: 0 for the Invariant-1 coefficient 2 + 3/lambda of the
 *     analysis, or a value >= 1 that replaces it (the experiments'
 *     heuristic parameters use 1.1; the approximation guarantee then no
 *     longer holds).  Any value >= 1 keeps floor(c x) >= ceil(x) - 1, which
 *     the desire-level search relies on; smaller values are PLDS_EINVAL;
 *   up_jump: 0 for Algorithm 2 (violators move up one level per sweep);
 *     1 for the procedure of the PLDS implementation details: at each level
 *     holding Invariant-1 violators (lowest first) every violator takes its
 *     desire-level (Def. desire-level: the closest level where both
 *     invariants hold, here the first level above it where Invariant 1
 *     holds), computed from the levels before any of them moves, and all of
 *     them move there together.  Each such level counts as one sweep
 *     (sweeps_ins) and each mover as one move (moves_up).  Deletions follow
 *     Algorithm 3 either way. */
typedef struct {
    int32_t levels_per_group;
    int32_t up_jump;
    int64_t edge_capacity_hint;
    double up_coeff;
    int64_t reserved[4];
} plds_options_t;

int plds_create_opts(int64_t n, double delta, double lambda, const plds_options_t *opts, plds_t **out);

int plds_destroy(plds_t *h);

/* Batched form: one handle holding `ngraphs` independent graphs, graph g
 * with n[g] vertices (host array), all with the same delta and lambda.  Each
 * graph keeps its own levels per group (4t_g from its own n[g], or
 * levels_per_group when > 0, or ceil(t_g / 50) for PLDS_LPG_OPT) and its own
 * thresholds, exactly as a handle
 * made by plds_create_ex(n[g], ...) would, so every graph goes through the
 * same states as it would alone: no edge joins two graphs, and whether a
 * vertex moves at a level depends only on its own neighbours and its own
 * graph's thresholds (Algorithms 2 and 3 move, level by level, exactly the
 * violators of that level).  The
 * graphs occupy consecutive vertex ranges of one vertex space of
 * sum(n[g]) <= 2^31 - 1 vertices; plds_graph_info gives each range's first
 * vertex.  Every level step of a batch serves all graphs at once.
 * plds_levels, plds_degrees, plds_coreness and plds_dump_state/
 * plds_load_state work on the whole vertex space (global ids);
 * plds_thresholds returns graph 0's tables; plds_stats counts all graphs. */
int plds_create_multi(int32_t ngraphs, const int64_t *n, double delta, double lambda, int32_t levels_per_group,
                      int64_t edge_capacity_hint, plds_t **out);

/* One batch for every graph of a multi-graph handle, applied as Update(B)
 * of Algorithm 1 to each graph (insertions and their sweep for all graphs,
 * then deletions and theirs).  ins[g] / del[g]: device int32 [count][2]
 * edge lists of graph g in its own ids [0, n[g]); ins, n_ins, del, n_del are
 * host arrays of ngraphs entries (an array may be NULL: no such lists).
 * Batch semantics per graph as plds_update; an id outside its own graph's
 * range rejects the whole call with PLDS_ERANGE before anything changes. */
int plds_update_multi(plds_t *h, const int32_t *const *ins, const int64_t *n_ins, const int32_t *const *del,
                      const int64_t *n_del, void *stream);

/* Applied updates per graph of the last plds_update_multi call: host
 * arrays ins[ngraphs] and del[ngraphs] receive the unique new edges
 * inserted into and the present edges deleted from each graph (for a plain
 * handle, the last call's totals).  Waits for the work on `stream`. */
int plds_graph_applied(plds_t *h, int64_t *ins, int64_t *del, void *stream);

/* Empty graph g of a multi-graph handle and give it n_new vertices, 1 <=
 * n_new <= the n it was created with (its capacity): all its edges are
 * removed and its vertices sit at level 0; its levels per group and
 * thresholds become those of a handle of n_new vertices (same delta,
 * lambda, levels-per-group rule and coefficient), so from here on it goes
 * through the states of a fresh plds_create_ex(n_new, ...) handle.  Ids of
 * its later batches must lie in [0, n_new).  The other graphs are untouched.
 * A serving loop reuses a graph slot for a newly admitted graph this way.
 * Returns after the work on `stream` is complete. */
int plds_reset_graph(plds_t *h, int32_t g, int64_t n_new, void *stream);

/* Graph g of a handle: *vertex_base receives its first global vertex id,
 * *out its n, t, L, G, K (m, delta, lambda and the slab figures are those
 * of the whole handle).  Either pointer may be NULL. */
int plds_graph_info(const plds_t *h, int32_t g, int64_t *vertex_base, plds_info_t *out);

/* Update(B) of Algorithm 1 with B = (ins, del): all insertions are applied
 * and rebalanced (RebalanceInsertions, Algorithm 2), then all deletions
 * (RebalanceDeletions, Algorithm 3, desire-levels per Def. desire-level).
 * ins / del: device pointers to int32 [count][2] edge lists (u, v); either
 * may be NULL with count 0.  Preprocessing (framework section): pairs are
 * undirected, self-loops are ignored, duplicates collapse, inserting a
 * present edge or deleting an absent one has no effect.  Deletions are
 * checked against the graph after the insertions, so a pair in both lists
 * ends absent.  Any id outside [0, n) in either list rejects the whole call
 * with PLDS_ERANGE before anything changes. */
int plds_update(plds_t *h, const int32_t *ins, int64_t n_ins, const int32_t *del, int64_t n_del, void *stream);
int plds_batch_insert(plds_t *h, const int32_t *edges, int64_t count, void *stream);
int plds_batch_delete(plds_t *h, const int32_t *edges, int64_t count, void *stream);

/* Coreness estimate (Def. coreness estimate): (1+delta)^max(floor((l+1)/L)-1,0)
 * for a vertex at level l with at least one edge, 0.0 for an isolated one.
 * vertices: device int32 [count], or NULL for all n (count ignored).
 * out: device float64 [count] (or [n]).  The power is read from a table built
 * on the host by repeated double multiplication (see plds_thresholds).  An id
 * outside [0, n) yields -1.0 and latches PLDS_ERANGE for plds_sync. */
int plds_coreness(plds_t *h, const int32_t *vertices, int64_t count, double *out, void *stream);

/* Low out-degree orientation (orientation section, Algorithm 5): an edge
 * points from the endpoint at the lower level to the one at the higher
 * level; on equal levels the edge {u, v} with u < v points u -> v (the rule
 * of Algorithm 5's flip conditions; the section's prose states the other tie
 * order).  Every vertex's out-degree is then at most its up-degree, hence
 * within the cap of its group (Invariant 1).
 *
 * plds_orient: (tail, head) of each of `count` pairs of the device int32
 * [count][2] list `edges` under the current levels, into device int32
 * [count][2] `out` (any pair of vertices, present in the graph or not).  An
 * id outside [0, n) yields (-1, -1) and latches PLDS_ERANGE for plds_sync.
 * Only enqueues work. */
int plds_orient(plds_t *h, const int32_t *edges, int64_t count, int32_t *out, void *stream);

/* Orientation tracking (Algorithm 5's outputs F and J).  While switched on
 * (on != 0; allocates n int32 of device memory on first use), every update
 * call keeps the levels it started from and its applied updates; the two
 * calls below then report on the last update call (PLDS_EINVAL if tracking
 * was off during it, if it failed, or after plds_load_state).  A call
 * without updates reports empty sets. */
int plds_track_orientation(plds_t *h, int32_t on);

/* F: the edges present both before and after the last update call whose
 * orientation changed, each as oriented before the call (tail, head), in no
 * particular order, into device int32 [cap][2] `out`.  *count receives the
 * number of such edges (only the first `cap` are written).  Found from the
 * edges of the vertices whose level the call changed (Algorithm 5's searched
 * edges).  Returns after the work on `stream` is complete. */
int plds_flips(plds_t *h, int32_t *out, int64_t cap, int64_t *count, void *stream);

/* J: the last update call's applied insertions oriented under the levels
 * after the call, and its applied deletions under the levels before it, as
 * (tail, head) into device int32 [ins_cap][2] / [del_cap][2]; *n_ins and
 * *n_del receive the full counts (only the first caps are written; the order
 * is the call's internal one).  Only enqueues work. */
int plds_oriented_updates(plds_t *h, int32_t *ins_out, int64_t ins_cap, int64_t *n_ins, int32_t *del_out,
                          int64_t del_cap, int64_t *n_del, void *stream);

/* Densest-subgraph value (densest-subgraph corollary): the largest coreness
 * estimate over the vertices of graph `graph` (0 for a plain handle; a graph
 * of a multi-graph handle otherwise), 0.0 for a graph without edges.  With
 * degeneracy d, the densest subgraph's density lies in [d/2, d], so this is a
 * constant-factor approximation of it.  Written to host *out; returns after
 * the work on `stream` is complete. */
int plds_densest_value(plds_t *h, int32_t graph, double *out, void *stream);

/* Static approximate k-core of the handle's current graph (static section,
 * Algorithm 6): bucketed peeling with bucket base 1+eps (eps > 0), the
 * (2+eps')-approximation with (2+eps)(1+eps) = 2+eps'.  Read as follows
 * (the section's prose, listing and worked example disagree; this reading
 * reproduces the worked example): a vertex with count C >= 1 sits in bucket
 * ceil(log_{1+eps} C) (C starts at the degree); a threshold t is the
 * smallest bucket; its peels take the smallest bucket in turn while it is
 * within (2+eps)(1+eps)^t, at most ceil(log_{1+2/eps} n) peels per
 * threshold; a peel lowers each alive neighbour's C by its peeled
 * neighbours, to no less than ceil((1+eps)^(t-1)), and re-buckets it to no
 * less than t; a vertex peeled from bucket b gets the estimate (1+eps)^b;
 * vertices without edges get 0.  est_out: device float64 [n].  Leaves the
 * handle's levels unchanged.  Plain handles only (PLDS_EINVAL for a
 * multi-graph handle, or for eps so small that the powers of 1+eps below n
 * exceed 4096 buckets).  Returns after the work on `stream` is complete. */
int plds_static_kcore(plds_t *h, double eps, double *est_out, void *stream);

/* plds_static_kcore for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result as plds_static_kcore, but its scratch arrays
 * (the peeling counts, buckets and round counters of every vertex, and the
 * bucket table) live in one array of about 24 MiB per device, defined by the
 * library and held until the process ends, instead of memory allocated on
 * the handle's first call; the call makes no device or host allocation.
 * Handles of at most PLDS_NOALLOC_MAX_N vertices (PLDS_EINVAL beyond).
 * Every call on a device shares that device's array and leaves its last
 * contents there (the call clears what must start at zero): calls that
 * overlap on one device, on any streams or handles, race and must not be
 * issued.  PLDS_EHIP if the array's device address could not be looked up
 * when the handle was created.  Returns after the work on `stream` is
 * complete. */
#define PLDS_NOALLOC_MAX_N (1 << 21)
int plds_static_kcore_noalloc(plds_t *h, double eps, double *est_out, void *stream);

/* Vertex updates (section on vertex insertions and deletions).
 *
 * plds_delete_vertices: every edge incident to one of the `count` vertices of
 * the device int32 list `vertices` is deleted as one batch of edge deletions
 * (Algorithm 3); the vertices stay, without edges, at level 0.  Listing a
 * vertex twice, or both ends of an edge, deletes the edge once.  An id
 * outside [0, n) rejects the call with PLDS_ERANGE before anything changes.
 * Statistics as plds_update.  Returns after the work on `stream` is
 * complete.
 *
 * plds_rebuild: a new plain handle (*out, owned by the caller) with new_n
 * vertices, the same delta, lambda and levels-per-group rule, holding the
 * graph of `h`, rebuilt from scratch by one batch of insertions of all its
 * edges (Algorithm 2).  Without `relabel`, new_n >= n and ids are kept (new
 * vertices join at level 0: vertex insertion past n).  With `relabel`
 * (device int32 [n]: the new id of each vertex, or -1 to drop it with its
 * edges), ids are renumbered; a new id outside [0, new_n) fails with
 * PLDS_ERANGE.  The level structure follows new_n (4 ceil(log_{1+delta}
 * new_n) levels per group by default).  `h` is unchanged.  Plain handles
 * only.  Returns after the work on `stream` is complete. */
int plds_delete_vertices(plds_t *h, const int32_t *vertices, int64_t count, void *stream);
int plds_rebuild(plds_t *h, int64_t new_n, const int32_t *relabel, plds_t **out, void *stream);

/* Current level of every vertex: device int32 [n]. */
int plds_levels(plds_t *h, int32_t *out, void *stream);
/* Current degree of every vertex: device int32 [n]. */
int plds_degrees(plds_t *h, int32_t *out, void *stream);

int plds_info(const plds_t *h, plds_info_t *out);

/* Host copies of the per-group tables (G entries each, any may be NULL):
 * up_max[g] = floor((2+3/lambda)(1+delta)^g)  -- Invariant 1 holds iff up <= it;
 * dn_min[g] = ceil((1+delta)^g)               -- Invariant 2 holds iff up* >= it;
 * pow_tab[g] = (1+delta)^g formed by g repeated double multiplications. */
int plds_thresholds(const plds_t *h, int32_t *up_max, int32_t *dn_min, double *pow_tab);

/* Statistics of the last batch call. */
int plds_stats(const plds_t *h, plds_stats_t *out);

/* Per-step record of the last batch call, up to 4K rows of 4 int64 each,
 * copied to host memory `out` [cap][4]; *rows receives the number written by
 * the call.  Insertion step: (l, level the movers left, movers, work items
 * of its scan + 2^48 * kind), the movers landing at l+1; kind 0 = movers
 * scan their slabs, 1 = climbing step, 2 = exit step (no move; l+1 = the
 * level left).  Deletion step: (-1-l, pending vertices, movers,
 * cumulative slots scanned + 2^48 if the step ran in the grid kernels
 * rather than the single-block loop), the movers landing at l. */
int plds_step_log(plds_t *h, int64_t *out, int64_t cap, int64_t *rows);

/* How the level loops run.  Insertions: 0 = the whole loop in one
 * cooperative launch with grid barriers between its parts (when the device
 * supports it, else as 2); 1 (default) = one kernel per part, with climbing
 * steps (a large group of movers climbing level after level is kept flagged,
 * and only the vertices it leaves behind and the residents of the next two
 * levels scan their slabs); 2 = one kernel per part, every step scanning its
 * movers' slabs; 3 = as 1, with climbing steps for groups of any size (not
 * only large ones), which exercises them on small graphs.  In modes 1 and 3
 * the insertion steps with at most 2^11 movers and 2^13 slab slots of
 * movers run back to back in one single-block kernel, larger ones (and
 * climbing steps) by the per-part kernels.  Deletions: the
 * steps run in one single-block kernel, a step with more than 2^11 pending
 * vertices or 2^12 slab slots of movers by the grid kernels; in mode 2 every
 * step (with any slab slots) goes to the grid kernels.  Results are
 * identical.  Mode 4 tests the bounded waits of mode 0: the grid barrier's
 * abort flag is raised before the cooperative launch, every block leaves at
 * its first barrier, and the insertion call returns PLDS_ESTATE (the handle
 * is then unusable).  A barrier wait that gives up in mode 0 ends the same
 * way. */
int plds_set_sweep_mode(plds_t *h, int32_t mode);

/* Launch schedule of the level loops.  Every field chooses how many
 * workgroups (blocks) a kernel of the sweeps gets, or how the steps are
 * grouped into prebuilt HIP graphs; none changes what is computed, so levels,
 * coreness and statistics other than timings are identical under every
 * schedule.  0 in a field selects the default.
 *   scan_blocks      blocks of the insertion scan, 64..2048 (default: the
 *                    blocks the device holds at once, at most 5 per CU);
 *   graph_steps      insertion step slots per prebuilt step graph, even,
 *                    2..64 (default 16; a slot is the step kernels' pair,
 *                    preceded by the single-block loop when it runs the
 *                    small steps); slots issued past a sweep's end return at
 *                    once but still cost their launch;
 *   dl_blocks        blocks of the desire-level kernels of deletions and
 *                    of upward jumps, 64..4096 (default 1024);
 *   del_scan_blocks  blocks of the deletion scan and of the jump scan,
 *                    64..8192 (default 2048).
 * reserved must be zero.  Out-of-range values: PLDS_EINVAL, nothing
 * changed.  The setting belongs to the handle (plds_rebuild carries it over)
 * and takes effect at the next update call; it is what a schedule search
 * (an autotuner timing candidate schedules on a workload) sets. */
typedef struct {
    int32_t scan_blocks;
    int32_t graph_steps;
    int32_t dl_blocks;
    int32_t del_scan_blocks;
    int32_t reserved[4];
} plds_launch_t;
int plds_set_launch(plds_t *h, const plds_launch_t *cfg);
/* The schedule in force, defaults resolved (no field is 0). */
int plds_get_launch(const plds_t *h, plds_launch_t *out);

/* Failure injection, for tests of error handling: after `after` more device
 * allocations by the library on the calling thread, the next one fails (the
 * call that makes it returns PLDS_ENOMEM), then allocations succeed again;
 * after < 0 switches it off.  An allocation that fails before a batch
 * changes anything leaves the state unchanged; one that fails while a batch
 * is being applied leaves the handle unusable (later calls: PLDS_ESTATE). */
int plds_inject_alloc_failure(int64_t after);

/* Time one kernel (0 = off, 1 = insertion scan (which also finishes the
 * movers), 2 = deletion scan, 3 = desire-level, 4 = insertion step
 * preparation, 5 = the edge scan of plds_flips, 6 = the cooperative
 * insertion sweep, 7 = the relax kernel of plds_static_kcore, 8 = the
 * application of a deletion list, 9 = the single-block deletion loop,
 * 10 = the edge scan of a round of jumps of a handle made with up_jump,
 * 11 = the single-block loop of small insertion steps).  Each launch of
 * that kernel carries a HIP event pair that the
 * runtime stamps at the dispatch's own start and end (hipExtLaunchKernel);
 * the cooperative sweep has events recorded around it on the stream.
 * While kind 1 or 4 is timed, insertion steps are launched one by one
 * instead of from the prebuilt step graph.  Every launch counts, including
 * those of steps after the sweep has finished (steps are issued in runs;
 * such launches return at once).  Results appear in plds_stats
 * (timed_launches, timed_ms). */
int plds_set_timing(plds_t *h, int32_t kernel);

/* Checkpoint.  plds_dump_state writes the edge list (u < v, unordered) to the
 * device buffer edges [cap][2] and the levels to device int32 [n]; *m_out
 * receives m (PLDS_EINVAL and nothing written if cap < m).  plds_load_state
 * replaces the whole state by the given edges (device int32 [m][2]) and
 * levels (device int32 [n], each in [0, K)); it returns plds_check() of the
 * loaded state. */
int plds_dump_state(plds_t *h, int32_t *edges, int64_t cap, int64_t *m_out, int32_t *levels, void *stream);
int plds_load_state(plds_t *h, const int32_t *edges, int64_t m, const int32_t *levels, void *stream);

/* Full on-device check: up/up* counters equal recounted degrees, Invariants
 * 1 and 2 hold at every vertex, isolated vertices sit at level 0, levels lie
 * in [0, K), slab contents match degrees.  PLDS_OK or PLDS_ESTATE. */
int plds_check(plds_t *h, void *stream);

/* Wait for all work of the handle on `stream`; returns and clears a latched
 * asynchronous error (PLDS_ERANGE from plds_coreness). */
int plds_sync(plds_t *h, void *stream);

const char *plds_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
