// plds.hip -- MI355X (gfx950) implementation of the parallel level data
// structure (PLDS) for batch-dynamic (2+eps)-approximate k-core decomposition
// (Liu, Shi, Yu, Dhulipala, Shun, SPAA'22).  C ABI in include/plds.h.
//
// Device state (all in HBM, int32 unless noted):
//   level[n], deg[n], up[n], ups[n]    level, degree, up-degree, up*-degree
//   off[n] (int64), cap[n], fill[n]    per-vertex open-addressing hash slab in
//                                      one pool: slots pool[off .. off+cap),
//                                      -1 empty, -2 tombstone, else neighbour id
//   stay[n], cnt2[n], addc[n], dl[n], rcstamp[n]   per-batch scratch
// The level loops (Algorithms 2 and 3) run as short kernels ordered on one
// stream; the host enqueues a run of steps and reads a small control block
// back between runs.  Each step reads its level from the control block, so
// the host never needs the level to enqueue it.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <new>
#include <mutex>
#include <vector>

#include "../../include/plds.h"

namespace {

constexpr int32_t kEmpty = -1;
constexpr int32_t kTomb = -2;
constexpr uint64_t kEmpty64 = ~0ull;
constexpr int kBlock = 256;          // threads per block of the sweep kernels
constexpr int kWave = 64;            // CDNA wavefront
constexpr int32_t kChunk = 256;      // slab slots per work item of a sweep
constexpr int32_t kMinCap = 8;       // smallest slab, slots
constexpr int kSweepGrid = 2048;     // blocks of the sweep kernels (most blocks of the insertion scan)
// Insertion scan blocks per compute unit.  The scan fits 7 (about 20 KB of
// LDS each); on the RMAT-20 stream 4 to 6 per unit measured best (1,024 to
// 1,536 blocks within 1% of each other), 7 about 12% slower, 2,048 (more
// than one resident round) 14% slower.
constexpr int kScanPerCU = 5;
constexpr int kDlGrid = 1024;        // blocks of the desire-level kernel
constexpr int kGraphStepsDef = 16;   // insertion steps per prebuilt step graph (default)
constexpr int32_t kInsLoopMovers = 2048;   // most movers of an insertion step run by the single-block loop
constexpr int32_t kInsLoopSlots = 8192;    // most slab slots of its movers
constexpr int kListGrid = 256;       // blocks of the per-mover list kernels
constexpr int kApplyGrid = 1024;     // most blocks of the batch-application kernels
constexpr int32_t kInf = INT32_MAX;
// During an insertion step its movers carry a bit in level[] that depends on
// the step's parity (set by the step's preparation, cleared by the next
// one), so one gather of a neighbour's level also tells whether it moves.
constexpr int32_t kMover0 = 1 << 30;   // mover of an insertion step of parity 0
constexpr int32_t kMover1 = 1 << 29;   // mover of an insertion step of parity 1
// Member of a climbing group (see climb_decide): its level field is stale,
// the group's level is the step's.
constexpr int32_t kClimb = 1 << 28;
// Member of a climbing group that stops at the end of the current step (set
// by the scan that finds it; other scans of the step still see it climb).
constexpr int32_t kStop = 1 << 27;
constexpr int32_t kLevelMask = (1 << 27) - 1;
constexpr int kCw = 64;                // slots per work item of a climbing step
constexpr int32_t kClimbMin = 8192;    // smallest group that climbs
// step modes
constexpr int32_t kPull = 0, kClimbStep = 1, kExit = 2;

// error bits latched on device
constexpr int32_t kErrRange = 1;     // id out of range
constexpr int32_t kErrFull = 2;      // slab insert found no free slot
constexpr int32_t kErrLevel = 4;     // a level left [0, K)
constexpr int32_t kErrOrder = 8;     // a desire-level not above the processed level
constexpr int32_t kErrPool = 16;     // pool exhausted
constexpr int32_t kErrHang = 32;     // a grid barrier wait gave up

// State of one insertion step: the movers sit at level `phys` (the vertices
// of that level that violate Invariant 1: its sorted candidates and its
// marked vertices, kept in cascade list `cur`) and land at level l+1.
// Normally phys == l; phys < l is a multi-level step (see ins_decide).
// `fresh` marks the first step of a sweep (chosen by the seeding, not by a
// decision).
struct InsStep {
    int32_t l, phys, jump, cur, done, fresh, mode;
};

struct Ctl {
    int32_t l;            // level of the current step
    int32_t done;         // loop finished
    int32_t cur;          // ping-pong index of the cascade / pending lists
    int32_t n_mv;         // movers of the current step
    int32_t casc_n[2];    // cascade list sizes
    int32_t p_n[2];       // pending list sizes (deletion)
    int32_t n_chunks;     // work items of the current step
    int32_t n_cls[4];     // movers per slab-size class (deletion work lists unused)
    int32_t n_cls2[2][4]; // insertion: movers per slab-size class, by step parity
    int32_t n_chunks2[2]; // insertion: large-slab work items, by step parity
    int32_t n_log;        // rows written to the step log in the current call
    int32_t n_steps;      // insertion steps of the current sweep
    int32_t nmvb[2];      // flagged movers of the last insertion step of parity 0 / 1 (mover lists)
    int32_t nmove[2];     // vertices moved by the last step of parity 0 / 1 (climbers of a climbing step)
    int32_t n_cl;         // entries of the climber list
    int32_t n_cl_snap;    // entries of the climber list before the current preparation
    int32_t n_exit;       // members an exit step appends after the joiners (folded into casc_n by its scan)
    int32_t n_sl[2];      // stoppers landed by the last step of parity 0 / 1
    int32_t n_cw[2];      // work items of the climbing step of parity 0 / 1
    int32_t step_dec[2];  // up-decrements of climbers by the climbing step of parity 0 / 1
    int64_t sum_up;       // sum of up over the climbing group
    InsStep st[2];        // insertion step state by step parity
    int32_t pend_phys, pend_l1, pend_n;   // occupancy change of the last step, applied one kernel later
    int32_t n_rc;         // desire-level recomputations of the current step
    int32_t nm;           // running minimum of pending desire-levels
    int32_t blocks_done;  // last-block election
    int32_t err;          // latched error bits
    int32_t n_valid;      // valid unique edges of the batch being applied
    int32_t n_touch;      // distinct endpoints of those edges
    int32_t n_grow;       // slabs to regrow
    int32_t n_pieces;     // work items of the large regrown slabs
    int32_t n_fl[4];      // moved vertices of the flip scan by slab class
    int64_t n_flip;       // flipped edges found
    uint64_t dv_bits;     // largest coreness estimate of a graph (bits of a non-negative double)
    // static approximate k-core (Algorithm 6)
    int32_t sk_t, sk_bp, sk_peels, sk_round, sk_done, sk_nT;
    int32_t sk_ncl[4];    // the round's peeled vertices by slab class
    int64_t sk_alive;
    int64_t sk_relaxed;   // count decrements of alive neighbours (sum of r over the rounds)
    // vertex deletion: incident edges counted, then gathered
    int64_t vd_deg, vd_n;
    int32_t vd_ncl[4];    // the listed vertices by slab class
    int32_t viol_del0;    // the deletion sweep's first candidates (Invariant-2 violators)
    int32_t n_cand;       // initial candidates
    int32_t step_id;      // deletion step counter (stamps)
    int32_t del_big;      // the current deletion step is run by the grid kernels (too large for one block)
    int32_t n_big;        // violators with large slabs, listed for the block pass of the desire-levels
    int32_t big_steps;    // deletion steps of the current sweep run by the grid kernels
    int32_t phys;         // level the movers of the current insertion step sit at
    int32_t jump;         // 1 if they land at l+1 from below l (a multi-level step)
    int64_t grow_req;     // slots requested by regrowth
    int64_t pool_top;     // next free pool slot
    int64_t sweeps, moves, scanned, dl_calcs, top, m_out;
    int64_t alg_U, alg_up1;   // up-neighbours read, neighbours one level up (insertion scans)
    // the single-block insertion loop (k_ins_loop)
    int32_t ins_p;        // parity of the next insertion step (of the step left to the step kernels when ins_big)
    int32_t ins_big;      // that step is run by the step kernels (k_ins_prep, k_ins_scan)
    int32_t ins_trips;    // launches of the loop that found the sweep running
    int64_t lp_scanned, lp_U, lp_up1, lp_moves;   // the loop's share of the scan statistics and moves
    int32_t lp_steps;     // steps run by the loop
    int32_t n_small;      // pull steps of the step kernels with at most kInsLoopMovers movers
    int32_t n_climbable;  // steps decided with at least kClimbMin movers (a climbing group could form)
};

// Everything a kernel needs, passed by value.
struct Dev {
    int32_t n, L, G, K;               // L, G, K: the largest over the graphs of the handle
    int32_t *up_max, *dn_min;         // per graph g: [G_g+1] from gtab[g] (entry G_g = INT_MAX)
    double *pow_tab;                  // per graph g: [G_g+1] from gtab[g]
    // A handle holds ng independent graphs on disjoint vertex ranges (ng = 1
    // for a plain handle).  Each graph has its own levels per group and
    // thresholds; every level step serves all graphs at once.
    int32_t ng;
    int32_t *gid;                     // [n] graph of each vertex (ng > 1)
    int32_t *gL, *gK, *gtab;          // [ng] levels per group, levels, table offset
    int32_t *Ls;                      // [nLs] the distinct levels-per-group values
    unsigned long long *gapp;         // [2][ng] applied insertions / deletions per graph of the last call (ng > 1)
    int32_t nLs;
    int32_t *level, *deg, *up, *ups, *cap, *fill;
    int64_t *off;
    int32_t *pool;
    int64_t pool_cap;
    int32_t *stay, *cnt2, *addc, *dl, *rcstamp;
    Ctl *ctl;
    // batch scratch
    uint64_t *hset;
    uint64_t hmask;
    int32_t *valid;                   // [batch][2]
    int32_t *touch;                   // [n]
    int32_t *grow, *newcap;           // [n]
    int64_t *oldoff;                  // [n]
    int32_t *oldcap;                  // [n]
    // level loop scratch
    int32_t *cand, *sorted;           // [n]
    int32_t *lvl_cnt, *lvl_start, *next_nz;   // [K+1]
    int32_t *occ;                     // [K+1] number of vertices at each level
    int32_t *lvl_fill;                // [K+1] scatter cursors
    int32_t *casc0, *casc1;           // [n]
    int32_t *mv;                      // [n] movers (deletion; insertion steps of parity 0)
    int32_t *mv1;                     // [n] movers of insertion steps of parity 1
    int64_t *sp;                      // [n] packed (stay << 32 | work items left) of insertion movers
    int32_t *cls[4];                  // [n] movers with slabs of <= 8, 16, 32, 64 slots
    int64_t *steplog;                 // [4K][4] per-step record of the last call
    int64_t *part;                    // [kSweepGrid][3] per-block statistics of a scan
    int64_t *chunks;                  // [chunk_cap]
    int64_t chunk_cap;
    int32_t *p0, *p1;                 // [n]
    int32_t *rc;                      // [n]
    // climbing steps
    int32_t climb_ok;                 // climbing steps allowed in this sweep (per-part kernels)
    int32_t ins_loop;                 // small insertion steps run by the single-block loop (per-part kernels)
    int32_t climb_min;                // smallest group that enters a climbing step
    int32_t loop_slots;               // most slab slots of a deletion step run by the single-block loop
    int32_t *lvb_start;               // [K+2] vertices with edges, bucketed by level at the sweep start
    int32_t *lvb_fill;                // [K+2]
    int32_t *lvb;                     // [n]
    int32_t *cl;                      // [n] climber list (members that stopped are skipped by flag)
    int32_t *sl0, *sl1;               // [n] vertices that stopped, by step parity
    int64_t *cw;                      // [cw_cap] climbing-step work items (vertex, role, 64-slot piece)
    int64_t cw_cap;
    // orientation tracking (allocated when switched on)
    int32_t *prevlvl;                 // [n] levels at the start of the last update call
    int2 *lvp;                        // [n] (prevlvl, level) side by side, for the flip scan's gathers
};

// Levels per group and table offset of the graph that holds vertex v.
struct GP {
    int32_t L, tab;
};
__device__ __forceinline__ GP gp(const Dev &d, int32_t v) {
    if (d.ng == 1) return GP{d.L, 0};
    int32_t g = d.gid[v];
    return GP{d.gL[g], d.gtab[g]};
}
// Invariant 1 cap and Invariant 2 floor of a vertex of graph p at level lvl
__device__ __forceinline__ int32_t up_cap(const Dev &d, GP p, int32_t lvl) { return d.up_max[p.tab + lvl / p.L]; }
// Whether level x is the first level of a group in some graph of the handle.
__device__ __forceinline__ bool group_start(const Dev &d, int32_t x) {
    if (d.ng == 1) return x % d.L == 0;
    bool hit = false;   // no early exit: the loads of the list are independent
    for (int i = 0; i < d.nLs; i++) hit |= x % d.Ls[i] == 0;
    return hit;
}
// The first level above x that starts a group in some graph of the handle.
__device__ __forceinline__ int32_t next_group_start(const Dev &d, int32_t x) {
    if (d.ng == 1) return (x / d.L + 1) * d.L;
    int32_t b = INT32_MAX;
    for (int i = 0; i < d.nLs; i++) b = min(b, (x / d.Ls[i] + 1) * d.Ls[i]);
    return b;
}
__device__ __forceinline__ int32_t dn_floor(const Dev &d, GP p, int32_t lvl) {
    return d.dn_min[p.tab + (lvl - 1) / p.L];
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // integer finaliser (low-bias 32-bit mixer)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
// home slot of `key` in a slab of `cap` slots (multiply-high range map)
__device__ __forceinline__ uint32_t home(int32_t key, int32_t cap) {
    return (uint32_t)(((uint64_t)mix32((uint32_t)key) * (uint32_t)cap) >> 32);
}

__device__ __forceinline__ int32_t wave_sum(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ void latch(Ctl *c, int32_t bits) { atomicOr(&c->err, bits); }

// append x to list[0..cap) through counter *n; an overflow is latched
__device__ __forceinline__ void push(int32_t *list, int32_t *n, int32_t cap, int32_t x, Ctl *c) {
    int32_t k = atomicAdd(n, 1);
    if (k < cap) list[k] = x;
    else latch(c, kErrLevel);
}

// Wavefront-aggregated append: every active lane calls it; lanes with `pred`
// append x, with one atomic per wavefront.
__device__ __forceinline__ void wpush(int32_t *list, int32_t *n, int32_t cap, bool pred, int32_t x, Ctl *c) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(n, __popcll(mask));
    base = __shfl(base, leader, kWave);
    if (pred) {
        int32_t k = base + __popcll(mask & ((1ull << lane) - 1));
        if (k < cap) list[k] = x;
        else latch(c, kErrLevel);
    }
}

// Every active lane calls it; lanes with key >= 0 add one to arr[key].  Lanes
// that share a key are served by one atomic; each gets a distinct slot
// (the counter value before its own increment), -1 for key < 0.
__device__ __forceinline__ int32_t wadd_key(int32_t *arr, int32_t key) {
    int lane = __lane_id();
    int32_t res = -1;
    uint64_t todo = __ballot(key >= 0);
    while (todo) {
        int leader = __ffsll((unsigned long long)todo) - 1;
        int32_t k = __shfl(key, leader, kWave);
        uint64_t same = __ballot(key == k) & todo;
        int32_t base = 0;
        if (lane == leader) base = atomicAdd(&arr[k], __popcll(same));
        base = __shfl(base, leader, kWave);
        if ((same >> lane) & 1) res = base + __popcll(same & ((1ull << lane) - 1));
        todo &= ~same;
    }
    return res;
}

// Every active lane calls it; lanes with key >= 0 add `delta` to arr[key],
// with one atomic per distinct key of the wavefront.
__device__ __forceinline__ void wave_add_key(int32_t *arr, int32_t key, int32_t delta) {
    uint64_t todo = __ballot(key >= 0);
    const int lane = __lane_id();
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t k = __shfl(key, leader, kWave);
        const uint64_t same = __ballot(key == k) & todo;
        if (lane == leader) atomicAdd(&arr[k], delta * __popcll(same));
        todo &= ~same;
    }
}

// exclusive prefix sum over the wavefront; *total receives the sum
__device__ __forceinline__ int32_t wave_excl(int32_t x, int32_t *total) {
    int lane = __lane_id();
    int32_t v = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t y = __shfl_up(v, o, kWave);
        if (lane >= o) v += y;
    }
    *total = __shfl(v, kWave - 1, kWave);
    return v - x;
}

// Block-wide exclusive prefix sum (every thread of the block calls it);
// *total receives the block sum.  sh: LDS of at least kBlock/kWave+1 ints.
__device__ __forceinline__ int32_t block_excl(int32_t x, int32_t *total, int32_t *sh) {
    int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nwv = blockDim.x / kWave;
    int32_t wt = 0;
    int32_t off = wave_excl(x, &wt);
    if (lane == 0) sh[wv] = wt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int i = 0; i < nwv; i++) {
            int32_t t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[nwv] = acc;
    }
    __syncthreads();
    int32_t r = sh[wv] + off;
    *total = sh[nwv];
    __syncthreads();
    return r;
}

// Block-wide append to N lists at once (every thread calls it): the thread
// adds cnt[k] entries to list k and pos[k] receives the list position of its
// first one.  The N counters are bumped by N lanes of the first wavefront in
// one instruction, so a block pays one atomic round trip for all lists
// instead of one per list.  sh: LDS of at least N*(kBlock/kWave+2) ints.
template <int N>
__device__ __forceinline__ void block_append(const int32_t (&cnt)[N], int32_t *const (&ctr)[N], int32_t (&pos)[N],
                                             int32_t *sh) {
    constexpr int S = kBlock / kWave + 2;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nwv = blockDim.x / kWave;
    int32_t off[N];
#pragma unroll
    for (int k = 0; k < N; k++) {
        int32_t t = 0;
        off[k] = wave_excl(cnt[k], &t);
        if (lane == 0) sh[k * S + wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        const int k = threadIdx.x;
        int32_t *mine = nullptr;
#pragma unroll
        for (int j = 0; j < N; j++)
            if (k == j) mine = ctr[j];
        int32_t acc = 0;
        for (int i = 0; i < nwv; i++) {
            int32_t t = sh[k * S + i];
            sh[k * S + i] = acc;
            acc += t;
        }
        sh[k * S + nwv] = acc > 0 ? atomicAdd(mine, acc) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) pos[k] = sh[k * S + nwv] + sh[k * S + wv] + off[k];
    __syncthreads();
}

// Store x at list position at (pred only); positions at or beyond cap latch an error.
__device__ __forceinline__ void put(int32_t *list, int32_t at, int32_t cap, bool pred, int32_t x, Ctl *c) {
    if (!pred) return;
    if (at < cap) list[at] = x;
    else latch(c, kErrLevel);
}

// Block-staged append.  Lanes add entries to a queue in LDS (one LDS atomic
// per wavefront); the block moves the queue to the global list with a single
// atomic on the list's counter, when fewer than `room` free entries are left
// or at the end (room = the queue's capacity).  Same-address atomics on a
// global counter are serialised by the memory system, so a hot loop that
// appends from many wavefronts pays one per block and flush instead of one
// per wavefront.  Loops that flush are block-uniform.
template <class T, int CAP>
struct StageT {
    int32_t n, base;
    T buf[CAP];
};

template <class T, int CAP>
__device__ __forceinline__ void st_init(StageT<T, CAP> &q) {
    if (threadIdx.x == 0) q.n = 0;
    __syncthreads();
}

// every active lane calls it; lanes with `pred` stage x (the caller keeps
// the number staged since the last flush within CAP)
template <class T, int CAP>
__device__ __forceinline__ void st_push(StageT<T, CAP> &q, bool pred, T x) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&q.n, __popcll(mask));
    base = __shfl(base, leader, kWave);
    if (pred) q.buf[base + __popcll(mask & ((1ull << lane) - 1))] = x;
}

// every thread of the block calls it; wr(i, x) stores entry x at list
// position i (positions at or beyond `cap` are dropped and latch an error)
template <class T, int CAP, class Wr>
__device__ void st_flush(StageT<T, CAP> &q, int32_t room, int32_t *counter, int32_t cap, Ctl *c, Wr wr) {
    __syncthreads();
    int32_t k = q.n;
    __syncthreads();
    if (k == 0 || k + room <= CAP) return;
    if (threadIdx.x == 0) q.base = atomicAdd(counter, k);
    __syncthreads();
    int32_t b = q.base;
    if (b + k > cap && threadIdx.x == 0) latch(c, kErrLevel);
    for (int i = threadIdx.x; i < k; i += blockDim.x)
        if (b + i < cap) wr(b + i, q.buf[i]);
    __syncthreads();
    if (threadIdx.x == 0) q.n = 0;
    __syncthreads();
}

constexpr int kStage = 4096;
using Stage = StageT<int32_t, kStage>;

__device__ __forceinline__ void stage_init(Stage &q) { st_init(q); }
__device__ __forceinline__ void stage_push(Stage &q, bool pred, int32_t x) { st_push(q, pred, x); }
__device__ __forceinline__ void stage_flush(Stage &q, int32_t room, int32_t *list, int32_t *n, int32_t cap, Ctl *c) {
    st_flush(q, room, n, cap, c, [=](int32_t i, int32_t x) { list[i] = x; });
}

// Final flush of two staged queues (every thread of the block calls it):
// both counters are bumped by two lanes of one instruction, so the two
// round trips overlap.
template <class QA, class QB, class WA, class WB>
__device__ void st_flush_both(QA &qa, int32_t *ca, int32_t capa, WA wa, QB &qb, int32_t *cb, int32_t capb, WB wb,
                              Ctl *c) {
    __syncthreads();
    const int32_t ka = qa.n, kb = qb.n;
    if (ka == 0 && kb == 0) return;   // block-uniform
    if (threadIdx.x < 2) {
        const bool b = threadIdx.x == 1;
        const int32_t k = b ? kb : ka;
        const int32_t base = k ? atomicAdd(b ? cb : ca, k) : 0;
        if (b) qb.base = base;
        else qa.base = base;
    }
    __syncthreads();
    const int32_t ba = qa.base, bb = qb.base;
    if (threadIdx.x == 0 && ((ka && ba + ka > capa) || (kb && bb + kb > capb))) latch(c, kErrLevel);
    for (int i = threadIdx.x; i < ka; i += blockDim.x)
        if (ba + i < capa) wa(ba + i, qa.buf[i]);
    for (int i = threadIdx.x; i < kb; i += blockDim.x)
        if (bb + i < capb) wb(bb + i, qb.buf[i]);
    __syncthreads();
    if (threadIdx.x == 0) qa.n = qb.n = 0;
    __syncthreads();
}

// Per-level histograms in LDS are used when the handle has at most this many
// levels (the dynamic LDS of one block, beside a Stage).
constexpr int kHistMax = 11264;

// ----------------------------------------------------------------- slabs
__device__ bool slab_has(const int32_t *s, int32_t cap, int32_t key) {
    if (cap == 0) return false;
    uint32_t i = home(key, cap);
    for (int32_t p = 0; p < cap; p++) {
        int32_t x = s[i];
        if (x == key) return true;
        if (x == kEmpty) return false;
        if (++i == (uint32_t)cap) i = 0;
    }
    return false;
}

// key is known absent; space is guaranteed by the growth plan.  The
// slab's fill count grows by the endpoint's new edges after the batch
// (k_ins_seed); a put that reuses a tombstone takes its slot back from it.
__device__ bool slab_put(int32_t *s, int32_t cap, int32_t key, int32_t *fill) {
    if (cap == 0) return false;
    uint32_t i = home(key, cap);
    for (int32_t p = 0; p < cap; p++) {
        int32_t x = s[i];
        if (x == kEmpty || x == kTomb) {
            int32_t prev = atomicCAS(&s[i], x, key);
            if (prev == x) {
                if (x == kTomb && fill) atomicSub(fill, 1);
                return true;
            }
        }
        if (++i == (uint32_t)cap) i = 0;
    }
    return false;
}

__device__ bool slab_del(int32_t *s, int32_t cap, int32_t key) {
    if (cap == 0) return false;
    uint32_t i = home(key, cap);
    for (int32_t p = 0; p < cap; p++) {
        int32_t x = s[i];
        if (x == key) {
            s[i] = kTomb;
            return true;
        }
        if (x == kEmpty) return false;
        if (++i == (uint32_t)cap) i = 0;
    }
    return false;
}

// ------------------------------------------------------- preprocessing
__global__ void k_range_check(const int32_t *e, int64_t cnt, int32_t n, Ctl *ctl) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * cnt; i += stride) {
        int32_t x = e[i];
        if (x < 0 || x >= n) latch(ctl, kErrRange);
    }
}

// Batch preprocessing (framework section): canonical (min,max) pair, no
// self-loop, first copy only (hash set), then keep it iff its presence in the
// graph equals want_present (insertions: absent, deletions: present).  A
// kept edge counts one new (or removed) slot at each endpoint (addc); the
// first count lists the endpoint (touch).
__global__ void k_dedupe(Dev d, const int32_t *e, int64_t cnt, int want_present) {
    __shared__ StageT<int64_t, 2048> q;
    __shared__ Stage qt;
    st_init(q);
    stage_init(qt);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t *valid = (int64_t *)d.valid;   // pair (u, v) as one little-endian int64
    auto wr = [=](int32_t k, int64_t x) { valid[k] = x; };
    for (int64_t ib = blockIdx.x * (int64_t)blockDim.x; ib < cnt; ib += stride) {
        int64_t i = ib + threadIdx.x;
        bool keep = false;
        int32_t u = 0, v = 0;
        if (i < cnt) {
            int32_t a = e[2 * i], b = e[2 * i + 1];
            u = min(a, b);
            v = max(a, b);
            // ids out of range are left out (the call is then rejected
            // before anything is applied)
            if (a != b && u >= 0 && v < d.n) {
                uint64_t key = ((uint64_t)(uint32_t)u << 32) | (uint32_t)v;
                uint64_t j = mix64(key) & d.hmask;
                bool fresh = false;
                for (uint64_t p = 0; p <= d.hmask; p++) {
                    uint64_t x = d.hset[j];
                    if (x == key) break;
                    if (x == kEmpty64) {
                        uint64_t prev = atomicCAS((unsigned long long *)&d.hset[j], (unsigned long long)kEmpty64,
                                                  (unsigned long long)key);
                        if (prev == kEmpty64) {
                            fresh = true;
                            break;
                        }
                        if (prev == key) break;
                    }
                    j = (j + 1) & d.hmask;
                }
                if (fresh) {
                    // probe the smaller slab of the two endpoints
                    int32_t s = d.cap[u] <= d.cap[v] ? u : v, t = s == u ? v : u;
                    bool present = slab_has(d.pool + d.off[s], d.cap[s], t);
                    keep = (int)present == want_present;
                }
            }
        }
        const bool first_u = keep && atomicAdd(&d.addc[u], 1) == 0;
        const bool first_v = keep && atomicAdd(&d.addc[v], 1) == 0;
        st_push(q, keep, (int64_t)(((uint64_t)(uint32_t)v << 32) | (uint32_t)u));
        stage_push(qt, first_u, u);
        stage_push(qt, first_v, v);
        st_flush(q, (int32_t)blockDim.x, &d.ctl->n_valid, INT32_MAX, d.ctl, wr);
        stage_flush(qt, 2 * (int32_t)blockDim.x, d.touch, &d.ctl->n_touch, d.n, d.ctl);
    }
    st_flush(q, 2048, &d.ctl->n_valid, INT32_MAX, d.ctl, wr);
    stage_flush(qt, kStage, d.touch, &d.ctl->n_touch, d.n, d.ctl);
}

// slabs that would exceed 80% occupancy are regrown to 60% of the new size
__global__ void k_plan_growth(Dev d) {
    __shared__ StageT<int64_t, 2048> q;
    __shared__ int64_t red[kBlock / kWave];
    st_init(q);
    int32_t nt = d.ctl->n_touch;
    int stride = gridDim.x * blockDim.x;
    int64_t req = 0;
    auto wr = [=](int32_t k, int64_t e) {
        d.grow[k] = (int32_t)(e & 0xffffffff);
        d.newcap[k] = (int32_t)(e >> 32);
    };
    for (int ib = blockIdx.x * blockDim.x; ib < nt; ib += stride) {
        int i = ib + threadIdx.x;
        bool grow = false;
        int32_t x = -1, ncap = 0;
        if (i < nt) {
            x = d.touch[i];
            int64_t k = d.addc[x], c = d.cap[x];
            if ((d.fill[x] + k) * 5 > c * 4) {
                int64_t live = d.deg[x] + k;
                int64_t nc = (live * 5 + 2) / 3;
                nc = ((std::max<int64_t>(nc, kMinCap) + 7) / 8) * 8;
                if (nc > INT32_MAX / 2) {
                    latch(d.ctl, kErrPool);
                    nc = 8;
                }
                grow = true;
                ncap = (int32_t)nc;
                req += nc;
            }
        }
        st_push(q, grow, (int64_t)(((uint64_t)(uint32_t)ncap << 32) | (uint32_t)x));
        st_flush(q, (int32_t)blockDim.x, &d.ctl->n_grow, d.n, d.ctl, wr);
    }
    st_flush(q, 2048, &d.ctl->n_grow, d.n, d.ctl, wr);
    req = wave_sum64(req);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = req;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < (int)blockDim.x / kWave; i++) t += red[i];
        if (t) atomicAdd((unsigned long long *)&d.ctl->grow_req, (unsigned long long)t);
    }
}

// Allocate the new slabs from the pool, one atomic per wavefront.  All slabs
// of one batch are carved from one contiguous region that the host has
// already filled with empty slots.
constexpr int kGrowLds = 2048;     // slots of a new slab built in LDS (per wavefront)
constexpr int kGrowPiece = 1024;   // old slots per work item of a larger regrown slab

__global__ void k_grow_alloc(Dev d) {
    int32_t ng = d.ctl->n_grow;
    int gid = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x % kWave;
    int stride = gridDim.x * blockDim.x;
    for (int g0 = gid - lane; g0 < ng; g0 += stride) {   // wave-uniform
        int g = g0 + lane;
        const bool in = g < ng;
        int32_t nc = in ? d.newcap[g] : 0;
        int32_t total = 0;
        int32_t off = wave_excl(nc, &total);
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd((unsigned long long *)&d.ctl->pool_top, (unsigned long long)total);
        base = __shfl(base, 0, kWave);
        int32_t npc = 0;   // work items of a new slab too large for LDS: pieces of its old slab
        if (in) {
            int32_t x = d.grow[g];
            int32_t oc = d.cap[x];
            d.oldoff[g] = d.off[x];
            d.oldcap[g] = oc;
            if (base + off + nc > d.pool_cap) {
                latch(d.ctl, kErrPool);
                d.newcap[g] = 0;
            } else {
                d.off[x] = base + off;
                d.cap[x] = nc;
                d.fill[x] = 0;
                if (nc > kGrowLds) npc = (oc + kGrowPiece - 1) / kGrowPiece;
            }
        }
        int32_t ptot = 0;
        int32_t poff = wave_excl(npc, &ptot);
        int32_t pbase = 0;
        if (lane == 0 && ptot) pbase = atomicAdd(&d.ctl->n_pieces, ptot);
        pbase = __shfl(pbase, 0, kWave);
        if ((int64_t)pbase + ptot > d.chunk_cap) {
            if (lane == 0 && ptot) latch(d.ctl, kErrPool);
        } else {
            for (int32_t k = 0; k < npc; k++) d.chunks[pbase + poff + k] = ((int64_t)g << 32) | (uint32_t)k;
        }
    }
}

// Move the live entries of each regrown slab into its new slab.  The new
// slab starts empty and only its movers write it, so every entry lands on an
// empty slot and its fill is the number of entries moved.  A new slab of at
// most kGrowLds slots is built in LDS (CAS on LDS, then one coalesced write
// of the whole slab; fill stored once); any linear-probing placement is a
// valid slab, since the new slab has no tombstones.  A wavefront takes four
// regrown slabs per pass: when all four new slabs fit in a quarter of its
// table, lane groups of 16 build them side by side, else the whole
// wavefront builds them one after another.  The tables are per wavefront,
// so the phases are ordered by wavefront-local fences.  Larger slabs are
// filled in place, kGrowPiece old slots per wavefront (fill added once per
// piece), so that a hub's slab is spread over many wavefronts.

__device__ __forceinline__ bool lds_put(int32_t *t, int32_t cap, int32_t key) {
    uint32_t i = home(key, cap);
    for (int32_t p = 0; p < cap; p++) {
        if (atomicCAS(&t[i], kEmpty, key) == kEmpty) return true;
        if (++i == (uint32_t)cap) i = 0;
    }
    return false;
}

// the new slab (nc slots at ns) of vertex x from its old slab (oc slots at
// os), in table t, by the lanes l, l + nl, ... of a group of nl lanes;
// returns the entries this lane moved
__device__ __forceinline__ int32_t grow_build(Dev &d, int32_t *t, const int32_t *os, int32_t oc, int32_t *ns, int32_t nc,
                                              int l, int nl) {
    for (int i = l; i < nc; i += nl) t[i] = kEmpty;
    __threadfence_block();
    int32_t moved = 0;
    for (int i = l; i < oc; i += nl) {
        const int32_t w = os[i];
        if (w >= 0) {
            if (lds_put(t, nc, w)) moved++;
            else latch(d.ctl, kErrFull);
        }
    }
    __threadfence_block();
    for (int i = l; i < nc; i += nl) ns[i] = t[i];
    __threadfence_block();   // the table is reused next
    return moved;
}

constexpr int kGrowSub = 4;                       // regrown slabs per wavefront pass
constexpr int kGrowSubLanes = kWave / kGrowSub;   // lanes per slab when they fit side by side
constexpr int kGrowSubCap = kGrowLds / kGrowSub;  // slots of each side-by-side table

__global__ void __launch_bounds__(kBlock) k_grow_move(Dev d) {
    __shared__ int32_t tab[kBlock / kWave][kGrowLds];
    const int32_t ng = d.ctl->n_grow;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    int32_t *t = tab[wv];
    const int sub = lane / kGrowSubLanes, sl = lane % kGrowSubLanes;
    for (int gb = wid * kGrowSub; gb < ng; gb += nw * kGrowSub) {   // wave-uniform
        const int g = gb + sub;
        const bool has = g < ng && d.newcap[g] != 0;
        const int32_t x = has ? d.grow[g] : -1;
        const int32_t nc = has ? d.cap[x] : 0, oc = has ? d.oldcap[g] : 0;
        const int64_t oo = has ? d.oldoff[g] : 0, no = has ? d.off[x] : 0;
        if (__all(nc <= kGrowSubCap)) {
            int32_t moved = grow_build(d, t + sub * kGrowSubCap, d.pool + oo, oc, d.pool + no, nc, sl, kGrowSubLanes);
            for (int o = kGrowSubLanes / 2; o > 0; o >>= 1) moved += __shfl_xor(moved, o, kWave);
            if (has && sl == 0) d.fill[x] = moved;
        } else {
            for (int k = 0; k < kGrowSub; k++) {
                const int src = k * kGrowSubLanes;
                const int32_t xk = __shfl(x, src, kWave), nck = __shfl(nc, src, kWave), ock = __shfl(oc, src, kWave);
                const int64_t ook = __shfl(oo, src, kWave), nok = __shfl(no, src, kWave);
                if (xk < 0 || nck > kGrowLds) continue;   // wave-uniform; larger slabs go in pieces
                const int32_t moved = wave_sum(grow_build(d, t, d.pool + ook, ock, d.pool + nok, nck, lane, kWave));
                if (lane == 0) d.fill[xk] = moved;
            }
        }
    }
    // the larger slabs, a piece per wavefront
    const int32_t np = (int32_t)min((int64_t)d.ctl->n_pieces, d.chunk_cap);
    for (int i = wid; i < np; i += nw) {
        const int64_t desc = d.chunks[i];
        const int32_t g = (int32_t)(desc >> 32), k = (int32_t)(desc & 0xffffffff);
        const int32_t x = d.grow[g], oc = d.oldcap[g], nc = d.cap[x];
        const int32_t *os = d.pool + d.oldoff[g];
        int32_t *ns = d.pool + d.off[x];
        const int32_t lo = k * kGrowPiece, hi = min(lo + kGrowPiece, oc);
        int32_t moved = 0;
        for (int32_t e = lo + lane; e < hi; e += kWave) {
            const int32_t w = os[e];
            if (w >= 0) {
                if (slab_put(ns, nc, w, nullptr)) moved++;
                else latch(d.ctl, kErrFull);
            }
        }
        moved = wave_sum(moved);
        if (lane == 0 && moved) atomicAdd(&d.fill[x], moved);
    }
}

// Insert both directed copies; up/up* counters follow the current levels:
// up(a) counts b iff level(b) >= level(a), up*(a) iff level(b) >= level(a)-1.
__global__ void k_apply_ins(Dev d) {
    int32_t nv = d.ctl->n_valid;
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        int32_t a = d.valid[2 * i], b = d.valid[2 * i + 1];
        if (!slab_put(d.pool + d.off[a], d.cap[a], b, &d.fill[a])) latch(d.ctl, kErrFull);
        if (!slab_put(d.pool + d.off[b], d.cap[b], a, &d.fill[b])) latch(d.ctl, kErrFull);
        int32_t la = d.level[a], lb = d.level[b];
        // deg grows by the endpoint counts in k_ins_seed
        if (lb >= la) atomicAdd(&d.up[a], 1);
        if (lb >= la - 1) atomicAdd(&d.ups[a], 1);
        if (la >= lb) atomicAdd(&d.up[b], 1);
        if (la >= lb - 1) atomicAdd(&d.ups[b], 1);
    }
}

// Remove both directed copies (tombstones) and the counter contributions.
__global__ void k_apply_del(Dev d) {
    int32_t nv = d.ctl->n_valid;
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        int32_t a = d.valid[2 * i], b = d.valid[2 * i + 1];
        if (!slab_del(d.pool + d.off[a], d.cap[a], b)) latch(d.ctl, kErrFull);
        if (!slab_del(d.pool + d.off[b], d.cap[b], a)) latch(d.ctl, kErrFull);
        int32_t la = d.level[a], lb = d.level[b];
        // deg drops by the endpoint counts in k_del_cand (a hub would serialise here)
        if (lb >= la) atomicSub(&d.up[a], 1);
        if (lb >= la - 1) atomicSub(&d.ups[a], 1);
        if (la >= lb) atomicSub(&d.up[b], 1);
        if (la >= lb - 1) atomicSub(&d.ups[b], 1);
    }
}

// --------------------------------------------------- insertion sweep
// Initial candidates of Algorithm 2: endpoints of inserted edges that
// violate Invariant 1, bucketed by level.
__global__ void k_ins_seed(Dev d) {
    extern __shared__ int32_t hist[];   // [K] when K <= kHistMax
    __shared__ Stage q;
    const bool lds = d.K <= kHistMax;
    stage_init(q);
    if (lds) {
        for (int i = threadIdx.x; i < d.K; i += blockDim.x) hist[i] = 0;
        __syncthreads();
    }
    int32_t nt = d.ctl->n_touch;
    int stride = gridDim.x * blockDim.x;
    for (int ib = blockIdx.x * blockDim.x; ib < nt; ib += stride) {
        int i = ib + threadIdx.x;
        int32_t x = -1, key = -1;
        if (i < nt) {
            x = d.touch[i];
            const int32_t k = d.addc[x];   // the endpoint's new edges (counted by k_dedupe)
            d.deg[x] += k;
            d.fill[x] += k;
            d.addc[x] = 0;
            int32_t lx = d.level[x];
            if (d.up[x] > up_cap(d, gp(d, x), lx)) key = lx;
        }
        stage_push(q, key >= 0, x);
        stage_flush(q, blockDim.x, d.cand, &d.ctl->n_cand, d.n, d.ctl);
        if (lds) {
            if (key >= 0) atomicAdd(&hist[key], 1);
        } else {
            wadd_key(d.lvl_cnt, key);
        }
    }
    stage_flush(q, kStage, d.cand, &d.ctl->n_cand, d.n, d.ctl);
    if (lds) {   // the flush above ended with a barrier
        for (int i = threadIdx.x; i < d.K; i += blockDim.x)
            if (hist[i]) atomicAdd(&d.lvl_cnt[i], hist[i]);
    }
}

// One block of 1024 threads: exclusive scan of the per-level candidate
// counts (bucket starts and scatter cursors) and, for every level, the next
// level at or above it that has candidates.
__global__ void k_level_scan(Dev d) {
    __shared__ int32_t part[1024], first[1024];
    int K = d.K, tid = threadIdx.x, nt = blockDim.x;
    int per = (K + nt - 1) / nt, lo = min(K, tid * per), hi = min(K, lo + per);
    int32_t sum = 0, f = K;
    for (int i = lo; i < hi; i++) {
        int32_t x = d.lvl_cnt[i];
        sum += x;
        if (x > 0 && f == K) f = i;
    }
    part[tid] = sum;
    first[tid] = f;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {          // inclusive prefix sums, suffix minima
        int32_t a = tid >= o ? part[tid - o] : 0;
        int32_t b = tid + o < nt ? first[tid + o] : K;
        __syncthreads();
        part[tid] += a;
        first[tid] = min(first[tid], b);
        __syncthreads();
    }
    int32_t acc = part[tid] - sum;
    int32_t nz = tid + 1 < nt ? first[tid + 1] : K;
    for (int i = lo; i < hi; i++) {
        d.lvl_start[i] = acc;
        d.lvl_fill[i] = acc;
        acc += d.lvl_cnt[i];
    }
    for (int i = hi - 1; i >= lo; i--) {
        if (d.lvl_cnt[i] > 0) nz = i;
        d.next_nz[i] = nz;
    }
    if (tid == nt - 1) {
        d.lvl_start[K] = part[nt - 1];
        d.next_nz[K] = K;
    }
    if (tid == 0) {
        int32_t z = first[0];
        d.ctl->l = z;
        d.ctl->phys = z;
        d.ctl->jump = 0;
        d.ctl->done = z >= K;
        d.ctl->cur = 0;
        d.ctl->st[1] = InsStep{z, z, 0, 0, z >= K, 1, kPull};
        d.ctl->pend_n = 0;
        d.ctl->nmvb[0] = d.ctl->nmvb[1] = 0;
        d.ctl->nmove[0] = d.ctl->nmove[1] = 0;
        d.ctl->n_sl[0] = d.ctl->n_sl[1] = 0;
        d.ctl->n_cw[0] = d.ctl->n_cw[1] = 0;
        d.ctl->step_dec[0] = d.ctl->step_dec[1] = 0;
        d.ctl->n_cl = 0;
        d.ctl->n_exit = 0;
        d.ctl->n_steps = 0;
        d.ctl->sum_up = 0;
        for (int q = 0; q < 2; q++) {
            d.ctl->n_chunks2[q] = 0;
            d.ctl->n_cls2[q][0] = d.ctl->n_cls2[q][1] = d.ctl->n_cls2[q][2] = d.ctl->n_cls2[q][3] = 0;
        }
        d.ctl->casc_n[0] = d.ctl->casc_n[1] = 0;
        d.ctl->n_chunks = 0;
        d.ctl->n_cls[0] = d.ctl->n_cls[1] = d.ctl->n_cls[2] = d.ctl->n_cls[3] = 0;
        d.ctl->blocks_done = 0;
        d.ctl->ins_p = 0;
        d.ctl->ins_big = 0;
        d.ctl->ins_trips = 0;
        d.ctl->lp_scanned = d.ctl->lp_U = d.ctl->lp_up1 = d.ctl->lp_moves = 0;
        d.ctl->lp_steps = 0;
        d.ctl->n_small = 0;
        d.ctl->n_climbable = 0;
    }
}

// Candidates into their level buckets.  With a histogram in LDS: each block
// counts its candidates per level, takes one range per level from the
// global cursors, and places its candidates in it.
__global__ void k_level_scatter(Dev d) {
    extern __shared__ int32_t hist[];   // [K] when K <= kHistMax
    int32_t nc = d.ctl->n_cand;
    int stride = gridDim.x * blockDim.x;
    if (d.K > kHistMax) {
        int gid = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x % kWave;
        for (int i0 = gid - lane; i0 < nc; i0 += stride) {
            int i = i0 + lane;
            int32_t x = i < nc ? d.cand[i] : -1;
            int32_t pos = wadd_key(d.lvl_fill, x >= 0 ? d.level[x] : -1);
            if (x >= 0) d.sorted[pos] = x;
        }
        return;
    }
    for (int i = threadIdx.x; i < d.K; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) atomicAdd(&hist[d.level[d.cand[i]]], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < d.K; b += blockDim.x) {
        int32_t c = hist[b];
        if (c) hist[b] = atomicAdd(&d.lvl_fill[b], c);
    }
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        int32_t x = d.cand[i];
        d.sorted[atomicAdd(&hist[d.level[x]], 1)] = x;
    }
}

// Work items of a step: kChunk-slot pieces of the movers' slabs, appended
// with one atomic per wavefront.  All lanes of the wave call it; lanes with
// v < 0 add nothing.
__device__ __forceinline__ void add_chunks_w(Dev &d, int32_t v) {
    int32_t nch = v >= 0 ? (d.cap[v] + kChunk - 1) / kChunk : 0;
    int32_t total = 0;
    int32_t off = wave_excl(nch, &total);
    if (total == 0) return;
    int lane = __lane_id();
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&d.ctl->n_chunks, total);
    base = __shfl(base, 0, kWave);
    if (base + total > d.chunk_cap) {
        if (lane == 0) latch(d.ctl, kErrPool);
        return;
    }
    for (int32_t k = 0; k < nch; k++) d.chunks[base + off + k] = ((int64_t)v << 32) | (uint32_t)k;
}


// Step of Algorithm 2, part 1 (step parity p): take the previous step's
// flag off its movers, gather this step's movers, flag them with the
// parity-p bit in level[], give each mover whose slab is cut into chunks its
// packed (stay, chunks left) counter, and sort the movers into work lists by
// slab size.  All level[] writes are plain stores: a previous mover that
// moves again was already given the parity-p bit by the scan that finished
// it, so the clearing and the flagging write the same value to it.  When
// `st.done`, only clears.  Returns false (on every block alike) if the step
// is out of range.
// The previous step's movers: the thread's first share, read before the
// step is decided (the reads do not depend on the decision) so that they
// overlap the decision's reads; written by ins_clear_flags.
struct PrevFlags {
    int32_t np, u, raw;
};
__device__ __forceinline__ PrevFlags prev_flags_load(const Dev &d, int p, int bid) {
    PrevFlags f;
    f.np = d.ctl->nmvb[p ^ 1];
    const int32_t *prev = p ? d.mv : d.mv1;
    const int i = bid * blockDim.x + threadIdx.x;
    f.u = i < f.np ? prev[i] : -1;
    f.raw = f.u >= 0 ? d.level[f.u] : 0;
    return f;
}

__device__ void ins_clear_flags(Dev &d, int p, int bid, int nblk, int32_t F, const PrevFlags &f) {
    // the previous step's movers: a mover that still violates carries this
    // step's parity bit (it moves again), which becomes F, the flag this
    // step gives its movers.  The gathering of this kernel writes the same
    // value, before or after; a value it wrote first (with F) must come out
    // unchanged, so F survives when it is kClimb.  The value written depends
    // only on what the previous scan left, so reading it early is the same.
    int32_t Mp = p ? kMover1 : kMover0;
    if (f.u >= 0) d.level[f.u] = (f.raw & (kLevelMask | kClimb)) | ((f.raw & Mp) ? F : 0);
    int stride = nblk * blockDim.x;
    const int32_t *prev = p ? d.mv : d.mv1;
    for (int i = bid * blockDim.x + threadIdx.x + stride; i < f.np; i += stride) {
        int32_t u = prev[i];
        int32_t raw = d.level[u];
        d.level[u] = (raw & (kLevelMask | kClimb)) | ((raw & Mp) ? F : 0);
    }
}

// mv: {first sorted position, sorted movers, cascaded movers} of the step
// when the caller has them, else nullptr.
__device__ bool ins_prep_phase(Dev &d, const InsStep &st, int p, int bid, int nblk, int32_t *sh, const PrevFlags &pf,
                               const int32_t *mvk) {
    int32_t Mp = p ? kMover1 : kMover0;
    int stride = nblk * blockDim.x;
    ins_clear_flags(d, p, bid, nblk, Mp, pf);
    if (st.done) return true;
    int32_t l = st.l, phys = st.phys, cur = st.cur;
    if (phys < 0 || phys > l || l + 1 >= d.K) {
        if (bid == 0 && threadIdx.x == 0) latch(d.ctl, kErrLevel);
        return false;
    }
    int32_t a0, nA, nB;
    if (mvk) {
        a0 = mvk[0];
        nA = mvk[1];
        nB = mvk[2];
    } else {
        a0 = d.lvl_start[phys];
        nA = d.lvl_start[phys + 1] - a0;
        nB = d.ctl->casc_n[cur];
    }
    const int32_t *casc = cur ? d.casc1 : d.casc0;
    if (nA + nB > d.n) {
        if (bid == 0 && threadIdx.x == 0) latch(d.ctl, kErrLevel);
        return false;
    }
    int32_t *mv = p ? d.mv1 : d.mv;
    int32_t *ncls = d.ctl->n_cls2[p];
    int32_t *const ctr[5] = {&ncls[0], &ncls[1], &ncls[2], &ncls[3], &d.ctl->n_chunks2[p]};
    for (int i0 = bid * blockDim.x; i0 < nA + nB; i0 += stride) {
        int i = i0 + threadIdx.x;
        int32_t v = -1, cl = -1, nch = 0;
        if (i < nA + nB) {
            v = i < nA ? d.sorted[a0 + i] : casc[i - nA];
            mv[i] = v;
            d.level[v] = phys | Mp;
            int32_t cap = d.cap[v];
            cl = cap <= 8 ? 0 : cap <= 16 ? 1 : cap <= 32 ? 2 : cap <= 64 ? 3 : 4;
            if (cl == 4) {
                nch = (cap + kChunk - 1) / kChunk;
                d.sp[v] = nch;
            }
        }
        const int32_t cnt[5] = {cl == 0, cl == 1, cl == 2, cl == 3, nch};
        int32_t pos[5];
        block_append(cnt, ctr, pos, sh);
#pragma unroll
        for (int k = 0; k < 4; k++) put(d.cls[k], pos[k], d.n, cl == k, v, d.ctl);
        if (cl == 4) {
            if (pos[4] + nch > d.chunk_cap) latch(d.ctl, kErrPool);
            else
                for (int32_t k = 0; k < nch; k++) d.chunks[pos[4] + k] = ((int64_t)v << 32) | (uint32_t)k;
        }
    }
    if (bid == 0 && threadIdx.x == 0) d.ctl->nmvb[p] = d.ctl->nmove[p] = nA + nB;
    return true;
}

// Part 2: every mover v scans its slab.  A neighbour flagged as a mover of
// this step stays in v's up-set and is neither counted nor updated; a
// neighbour w at level l stays behind (counted in v's `stay`); w at l+1 gains
// v as up-neighbour (and, in a multi-level step, as up*-neighbour) and is
// marked if that makes it exceed the cap of level l+1; w at l+2 gains v as
// up*-neighbour.  Work items: movers with slabs of at most 8/16/32/64 slots
// are served by lane groups of that width (8/4/2/1 movers per wavefront);
// larger slabs are cut into kChunk-slot pieces, a wavefront each.  The work
// item that completes a mover's slab finishes it (a lone item at once, a
// chunked slab through one atomic on its packed counter): level l+1, up*(v)
// = old up(v), up(v) = old up(v) - stay; a mover still above the cap of l+1
// stays marked and also gets the next step's flag, since it moves again.
// The flag of this step stays on, so other scans never touch its counters.
// Per-block statistics go to d.part[3*bid..] (stored, or added when accum).
// The two LDS queues of a scan (its cascade or joiner appends, its
// stoppers), declared once by the kernel and shared by the pull and the
// climbing phases (a launch runs one of them), which keeps the scan's LDS
// at about 20 KB per block: 7 blocks per compute unit.
struct ScanQ {
    Stage a;
    StageT<int32_t, 1024> b;
};

__device__ void ins_scan_phase(Dev &d, const InsStep &st, int p, int bid, int nblk, bool accum, ScanQ &sq) {
    int32_t l = st.l, nxt = st.cur ^ 1, jump = st.jump;
    int32_t Mp = p ? kMover1 : kMover0, Mn = p ? kMover0 : kMover1;
    int32_t *casc = nxt ? d.casc1 : d.casc0;
    const int32_t ub1_all = d.ng == 1 ? d.up_max[(l + 1) / d.L] : 0;
    int lane = threadIdx.x % kWave, wpb = blockDim.x / kWave;
    int nw = nblk * wpb;
    const int32_t *ncls = d.ctl->n_cls2[p];
    int32_t n0 = ncls[0], n1c = ncls[1], n2 = ncls[2], n3 = ncls[3];
    int32_t i0 = (n0 + 7) / 8, i1 = (n1c + 3) / 4, i2 = (n2 + 1) / 2, i3 = n3;
    int32_t i4 = (int32_t)min((int64_t)d.ctl->n_chunks2[p], d.chunk_cap);
    int32_t total = i0 + i1 + i2 + i3 + i4;
    if (bid * (int)(blockDim.x / kWave) >= total) return;   // no work item for this block (block-uniform)
    int32_t scanned = 0, nU = 0, n1 = 0;
    // pushes of one round: per wavefront up to kChunk neighbours plus 8 movers
    const int32_t room = wpb * (kChunk + kWave / 8);
    Stage &q_casc = sq.a;
    StageT<int32_t, 1024> &q_stop = sq.b;   // movers that stop at l+1 (residents of the next step)
    int32_t *slist = p ? d.sl1 : d.sl0;
    stage_init(q_casc);
    st_init(q_stop);
    auto wr_stop = [=](int32_t k, int32_t x) { slist[k] = x; };
    // rounds are block-uniform (every wavefront of the block runs the same
    // number), so the staged pushes can be flushed between rounds
    for (int tb = bid * wpb; tb < total; tb += nw) {
        int32_t t = tb + threadIdx.x / kWave;
        int cl = 0;
        int32_t tl = t < total ? t : INT32_MAX;
        if (tl < i0) cl = 0;
        else if ((tl -= i0) < i1) cl = 1;
        else if ((tl -= i1) < i2) cl = 2;
        else if ((tl -= i2) < i3) cl = 3;
        else {
            tl -= i3;
            cl = 4;
        }
        if (t >= total) cl = 0;
        int W = cl == 4 ? kWave : (8 << cl);
        int grp = lane / W, q = lane % W;
        // up(v) is read with the slab's size: no other scan of the step
        // touches a mover's counters (they see its flag)
        int32_t v = -1, lo = 0, hi = 0, upv = 0;
        if (t >= total) {
            // no work item for this wavefront in the last round
        } else if (cl < 4) {
            int32_t ncl = cl == 0 ? n0 : cl == 1 ? n1c : cl == 2 ? n2 : n3;
            int32_t j = tl * (kWave / W) + grp;
            if (j < ncl) {
                v = d.cls[cl][j];
                hi = d.cap[v];
                if (q == 0) upv = d.up[v];
            }
        } else {
            int64_t desc = d.chunks[tl];
            v = (int32_t)(desc >> 32);
            lo = (int32_t)(desc & 0xffffffff) * kChunk;
            hi = min(lo + kChunk, d.cap[v]);
            if (q == 0) upv = d.up[v];
        }
        const int32_t *s = v >= 0 ? d.pool + d.off[v] : d.pool;
        // the cap of level l+1 in v's graph (neighbours share v's graph)
        const int32_t ub1 = d.ng == 1 ? ub1_all : (v >= 0 ? up_cap(d, gp(d, v), l + 1) : 0);
        int32_t stay = 0;
        int iters = cl == 4 ? kChunk / kWave : 1;
        for (int it = 0; it < iters; it++) {
            int32_t e = lo + it * W + q;
            int32_t w = v >= 0 && e < hi ? s[e] : -1;
            int32_t raw = w >= 0 ? d.level[w] : -1;
            bool comover = w >= 0 && (raw & Mp);
            int32_t lw = (w < 0 || comover) ? -1 : (raw & kLevelMask);
            bool cross = false;
            nU += comover || lw >= l;
            if (lw == l) {
                stay++;
            } else if (lw == l + 1) {
                n1++;
                int32_t old = atomicAdd(&d.up[w], 1);
                cross = old == ub1;
                if (jump) atomicAdd(&d.ups[w], 1);
            } else if (lw == l + 2) {
                atomicAdd(&d.ups[w], 1);
            }
            stage_push(q_casc, cross, w);
        }
        if (v >= 0) scanned += (q == 0) ? hi - lo : 0;
        for (int o = W / 2; o > 0; o >>= 1) stay += __shfl_xor(stay, o, kWave);
        bool viol = false, stop = false;
        if (q == 0 && v >= 0) {
            bool last = true;
            int32_t total_stay = stay;
            if (cl == 4) {
                unsigned long long delta = ((unsigned long long)(uint32_t)stay << 32) - 1ull;
                unsigned long long old = atomicAdd((unsigned long long *)&d.sp[v], delta);
                last = (old & 0xffffffffull) == 1;
                total_stay += (int32_t)(old >> 32);
            }
            if (last) {
                int32_t u = upv;
                d.ups[v] = u;
                u -= total_stay;
                d.up[v] = u;
                viol = u > ub1;
                stop = !viol && d.climb_ok;
                d.level[v] = (l + 1) | Mp | (viol ? Mn : 0);
            }
        }
        stage_push(q_casc, viol, v);
        st_push(q_stop, stop, v);
        stage_flush(q_casc, room, casc, &d.ctl->casc_n[nxt], d.n, d.ctl);
        st_flush(q_stop, wpb * (kWave / 8), &d.ctl->n_sl[p], d.n, d.ctl, wr_stop);
    }
    st_flush_both(q_casc, &d.ctl->casc_n[nxt], d.n, [=](int32_t k, int32_t x) { casc[k] = x; }, q_stop,
                  &d.ctl->n_sl[p], d.n, wr_stop, d.ctl);
    __shared__ int32_t red[3][kBlock / kWave];
    nU = wave_sum(nU);
    n1 = wave_sum(n1);
    scanned = wave_sum(scanned);
    if (lane == 0) {
        red[0][threadIdx.x / kWave] = scanned;
        red[1][threadIdx.x / kWave] = nU;
        red[2][threadIdx.x / kWave] = n1;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int64_t t = 0;
        for (int i = 0; i < kBlock / kWave; i++) t += red[threadIdx.x][i];
        if (accum) d.part[3 * bid + threadIdx.x] += t;
        else d.part[3 * bid + threadIdx.x] = t;
    }
    __syncthreads();
}


// ---- climbing groups.  In long insertion sweeps a large set of vertices
// often climbs level after level through levels that hold few other
// vertices; every step would rescan all their slabs.  A climbing step
// instead keeps the group flagged (kClimb; their level fields go stale) and
// lets the other vertices do the work, which gives the same counters:
//   * a vertex that stays at the step's level l (a resident of l, or a
//     member that stopped there) takes one from up(v) of every climbing
//     neighbour v (v moves to l+1 and leaves it behind); the decrement that
//     takes up(v) to the cap of level l+1 marks v as stopping there;
//   * a resident w of level l+1 gains one up-neighbour per climbing
//     neighbour and joins the group if that lifts it over its cap;
//   * a resident of level l+2 gains one up*-neighbour per climbing neighbour.
// Climbers never gain up-neighbours (everything they count stays at or
// above them) and keep violating the same cap inside a group, so the group
// is exactly Algorithm 2's mover set of every level it passes.  A member
// that stops has up(v) right; its up*(v) no longer changes in the sweep (the
// levels below the sweep's frontier stay as they are) and is counted afresh
// from its slab after the sweep (k_ups_recount).  Residents come from buckets of every vertex with edges by its
// level at the start of the sweep: the sweep has not reached those levels.
// With no resident at or just above the group's level, nothing can change
// until the next occupied level, and the group skips there in one step.
// Before the group would cross a group boundary (the cap changes), or when
// it gets small against the levels' residents, an exit step puts the
// members back on their level as ordinary movers of the next step.

// Work item of a climbing step: (vertex, role, kCw-slot piece)
__device__ __forceinline__ int64_t cw_item(int32_t v, int32_t role, int32_t piece) {
    return ((int64_t)v << 32) | ((int64_t)role << 30) | (int64_t)piece;
}
constexpr int32_t kRoleStay = 0, kRoleUp1 = 2, kRoleUp2 = 3;

// Append the kCw-slot pieces of vertex v (v < 0: none) with `role`, one
// atomic per block.  Every thread of the block calls it.
__device__ __forceinline__ void add_cw_b(Dev &d, int32_t v, int32_t role, int32_t *counter, int32_t *sh) {
    int32_t cap = v >= 0 ? d.cap[v] : 0;
    int32_t np = (cap + kCw - 1) / kCw;
    int32_t total = 0;
    int32_t off = block_excl(np, &total, sh);
    if (total == 0) return;
    if (threadIdx.x == 0) sh[kBlock / kWave + 1] = atomicAdd(counter, total);
    __syncthreads();
    int32_t base = sh[kBlock / kWave + 1];
    __syncthreads();
    if (base + total > d.cw_cap) {
        if (threadIdx.x == 0) latch(d.ctl, kErrPool);
        return;
    }
    for (int32_t k = 0; k < np; k++) d.cw[base + off + k] = cw_item(v, role, k);
}

// Block-wide sum of an int64 (every thread calls it; valid in every thread).
__device__ __forceinline__ int64_t block_sum64(int64_t x, int64_t *red) {
    x = wave_sum64(x);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = x;
    __syncthreads();
    int64_t t = 0;
    for (int i = 0; i < (int)blockDim.x / kWave; i++) t += red[i];
    __syncthreads();
    return t;
}

// After climbing step `prv`: the group's size, and whether it climbs on
// (possibly skipping empty levels) or exits.  Every thread of a block calls it.
__device__ InsStep climb_decide(Dev &d, const InsStep &prv, int p, int32_t *sh1, int32_t *nc_out) {
    Ctl *c = d.ctl;
    InsStep nx;
    nx.jump = 0;
    nx.done = 0;
    nx.fresh = 0;
    int32_t x1 = prv.l + 1;   // the group's level after the step
    int32_t ns = d.lvl_start[x1 + 1] - d.lvl_start[x1];
    // occupancies are read with the counts (clamped indices; used only when
    // the group can go on), so the reads overlap
    const int32_t o0 = d.occ[min(x1, d.K)], o1 = d.occ[min(x1 + 1, d.K)], o2 = d.occ[min(x1 + 2, d.K)];
    int32_t nC = c->nmove[p ^ 1] - c->n_sl[p ^ 1] + c->casc_n[prv.cur ^ 1] + ns;
    bool top = x1 + 2 > d.K;
    bool go = nC > 0 && !top;
    int32_t stay = 0, r1 = 0, r2 = 0;
    if (go) {
        // occupancy after the step (its own move is applied one kernel later)
        stay = o0 + c->nmove[p ^ 1] - nC;
        r1 = o1;
        r2 = o2;
        go = (int64_t)(stay + r1 + r2) * 2 <= nC;
    }
    __syncthreads();
    if (!go) {
        *nc_out = 0;
        nx.mode = kExit;
        nx.l = x1 - 1;
        nx.phys = x1;
        nx.cur = prv.cur;   // it consumes nothing and adds the members to the joiners' list
        return nx;
    }
    *nc_out = nC;
    nx.mode = kClimbStep;
    nx.cur = prv.cur ^ 1;
    nx.phys = nx.l = x1;
    if (stay == 0 && r1 == 0) {
        int32_t b = min(next_group_start(d, x1), d.K);   // first level of the next group (of any graph)
        if (threadIdx.x == 0) sh1[0] = b;
        __syncthreads();
        for (int32_t z = x1 + 2 + threadIdx.x; z < b; z += blockDim.x)
            if (d.occ[z] > 0) atomicMin(&sh1[0], z);
        __syncthreads();
        int32_t xl = sh1[0] - 2;   // the first occupied level is xl+2 (or the group ends at xl+2)
        __syncthreads();
        if (xl > x1) {
            nx.l = xl;
            nx.jump = 1;
        }
    }
    return nx;
}

// Part 1 of a climbing step (parity p) at level st.l, the group at st.phys:
// stopped members of the previous climbing step back to a plain level
// (listed for the recount of up* after the sweep), joiners (the cascade list and the level's sorted
// candidates) into the group, then the step's work items: the vertices that
// stay at l (when the group moves from its own level), the residents of l+1
// and l+2.
__device__ void climb_prep_phase(Dev &d, const InsStep &prv, const InsStep &st, int p, int bid, int nblk,
                                 int32_t *sh, const PrevFlags &pf) {
    __shared__ int64_t red[kBlock / kWave];
    Ctl *c = d.ctl;
    ins_clear_flags(d, p, bid, nblk, kClimb, pf);
    const int stride = nblk * blockDim.x;
    const int32_t x = st.phys, l = st.l;
    const bool after_climb = prv.mode == kClimbStep;
    const bool landed_here = !prv.fresh && prv.l + 1 == x;   // the previous step's stoppers sit at x
    const int32_t *slp = p ? d.sl0 : d.sl1;
    const int32_t nsl = landed_here ? c->n_sl[p ^ 1] : 0;
    const int32_t *casc = st.cur ? d.casc1 : d.casc0;
    const int32_t nj = c->casc_n[st.cur];
    const int32_t a0 = d.lvl_start[x], ns = d.lvl_start[x + 1] - a0;
    // Landing on the first level of a group raises the cap: the members
    // whose up is within the new cap stop there without any decrement (in
    // a multi-graph handle, the members of the graphs whose group starts there).
    const bool boundary = l == x && group_start(d, x + 1);
    // the new cap for member v, or -1 if x+1 does not start a group of its graph
    auto cap_new = [&](int32_t v) -> int32_t {
        const GP g = gp(d, v);
        return (x + 1) % g.L == 0 ? up_cap(d, g, x + 1) : -1;
    };
    int32_t *sln = p ? d.sl1 : d.sl0;
    const int32_t ncl0 = boundary ? c->n_cl_snap : 0;   // members of earlier steps
    int64_t dsum = 0;
    // fix-ups: stopped members, joiners; at a boundary, members that stop
    for (int i0 = bid * blockDim.x; i0 < nsl + nj + ns + ncl0; i0 += stride) {
        int i = i0 + threadIdx.x;
        int32_t v = -1, stopn = -1;
        int32_t rcv = -1;
        if (i < nsl) {
            if (after_climb) {
                int32_t u = slp[i];
                dsum -= d.up[u];
                d.level[u] = x;
                rcv = u;
            }
        } else if (i < nsl + nj + ns) {
            v = i < nsl + nj ? casc[i - nsl] : d.sorted[a0 + i - nsl - nj];
            int32_t uv = d.up[v];
            bool st_now = boundary && uv <= cap_new(v);
            d.level[v] = x | kClimb | (st_now ? kStop : 0);
            dsum += uv;
            if (st_now) stopn = v;
        } else if (i < nsl + nj + ns + ncl0) {
            int32_t u = d.cl[i - nsl - nj - ns];
            int32_t raw = d.level[u];
            // stopped members of the previous step are being fixed right
            // now: they read as kStop or as a plain level, both skipped
            if ((raw & kClimb) && !(raw & kStop) && d.up[u] <= cap_new(u)) {
                d.level[u] = raw | kStop;
                stopn = u;
            }
        }
        const int32_t cnt[3] = {v >= 0, stopn >= 0, rcv >= 0};
        int32_t *const ctr[3] = {&c->n_cl, &c->n_sl[p], &c->n_rc};
        int32_t pos[3];
        block_append(cnt, ctr, pos, sh);
        put(d.cl, pos[0], d.n, v >= 0, v, c);
        put(sln, pos[1], d.n, stopn >= 0, stopn, c);
        put(d.rc, pos[2], d.n, rcv >= 0, rcv, c);
    }
    dsum = block_sum64(dsum, red);
    if (threadIdx.x == 0 && dsum) atomicAdd((unsigned long long *)&c->sum_up, (unsigned long long)dsum);
    // work items
    const int32_t *bk = d.lvb;
    int32_t s0 = 0, s1 = 0, r1a = 0, r1b = 0, r2a = 0, r2b = 0;
    if (l == x) {
        s0 = d.lvb_start[x];
        s1 = d.lvb_start[x + 1];
    }
    r1a = d.lvb_start[min(l + 1, d.K)];
    r1b = d.lvb_start[min(l + 2, d.K)];
    r2a = r1b;
    r2b = d.lvb_start[min(l + 3, d.K)];
    const int32_t nst = s1 - s0, nss = l == x ? nsl : 0, n1 = r1b - r1a, n2 = r2b - r2a;
    const int32_t tot = nst + nss + n1 + n2;
    for (int i0 = bid * blockDim.x; i0 < tot; i0 += stride) {
        int i = i0 + threadIdx.x;
        int32_t v = -1, role = 0;
        if (i < nst) {
            int32_t u = bk[s0 + i];
            int32_t raw = d.level[u];
            // a resident of x that stays (not climbing, within the cap); joiners
            // being flagged right now are over the cap
            if (!(raw & kClimb) && (raw & kLevelMask) == x && d.up[u] <= up_cap(d, gp(d, u), x)) v = u;
            role = kRoleStay;
        } else if (i < nst + nss) {
            v = slp[i - nst];
            role = kRoleStay;
        } else if (i < nst + nss + n1) {
            v = bk[r1a + i - nst - nss];
            role = kRoleUp1;
        } else if (i < tot) {
            v = bk[r2a + i - nst - nss - n1];
            role = kRoleUp2;
        }
        add_cw_b(d, v, role, &c->n_cw[p], sh);
    }
}

// Part 1 of an exit step (the group at st.phys): stopped members of the last
// climbing step back to a plain level (up* recounted after the sweep), and
// every member still climbing back on its level, appended to the joiners'
// list so that the next step moves them as ordinary movers.  The appends go
// behind the list's current end through their own counter (n_exit): the
// list's size is an input of every block's step decision in this kernel and
// must not change while blocks still read it.  The step's scan adds n_exit
// to the size.
__device__ void exit_prep_phase(Dev &d, const InsStep &prv, const InsStep &st, int p, int bid, int nblk,
                                int32_t *sh) {
    Ctl *c = d.ctl;
    const int stride = nblk * blockDim.x;
    const int32_t x = st.phys;
    const int32_t *slp = p ? d.sl0 : d.sl1;
    const int32_t nsl = c->n_sl[p ^ 1];
    const int32_t base = c->casc_n[st.cur ^ 1];
    int32_t *join = ((st.cur ^ 1) ? d.casc1 : d.casc0) + base;
    const int32_t ncl = c->n_cl;
    for (int i0 = bid * blockDim.x; i0 < nsl + ncl; i0 += stride) {
        int i = i0 + threadIdx.x;
        int32_t v = -1, w = -1;
        if (i < nsl) {
            v = slp[i];
            d.level[v] = x;
        } else if (i < nsl + ncl) {
            int32_t u = d.cl[i - nsl];
            int32_t raw = d.level[u];
            // still climbing (members that stopped carry kStop until their
            // fix-up in this same kernel writes their plain level)
            if ((raw & kClimb) && !(raw & kStop)) {
                d.level[u] = x;
                w = u;
            }
        }
        const int32_t cnt[2] = {w >= 0, v >= 0};
        int32_t *const ctr[2] = {&c->n_exit, &c->n_rc};
        int32_t pos[2];
        block_append(cnt, ctr, pos, sh);
        put(join, pos[0], d.n - base, w >= 0, w, c);
        put(d.rc, pos[1], d.n, v >= 0, v, c);
    }
    (void)prv;
}

// Part 2 of a climbing step: the work items of part 1, a wavefront each
// (kCw slots).  Exit steps have none.
__device__ void climb_scan_phase(Dev &d, const InsStep &st, int p, int bid, int nblk, ScanQ &sq) {
    Stage &q_join = sq.a;
    StageT<int32_t, 1024> &q_stop = sq.b;
    __shared__ int64_t red[kBlock / kWave];
    Ctl *c = d.ctl;
    const bool climb = st.mode == kClimbStep;
    const int32_t l = st.l;
    int32_t *join = (st.cur ^ 1) ? d.casc1 : d.casc0;
    int32_t *slist = p ? d.sl1 : d.sl0;
    auto wr_stop = [=](int32_t k, int32_t x) { slist[k] = x; };
    const int32_t cap1_all = d.ng == 1 ? up_cap(d, gp(d, 0), l + 1) : 0;   // the cap of level l+1 (plain handle)
    const int lane = threadIdx.x % kWave, wpb = blockDim.x / kWave;
    const int nw = nblk * wpb;
    const int32_t total = (int32_t)min((int64_t)c->n_cw[p], d.cw_cap);
    if (bid * wpb >= total && !(bid == 0 && climb)) return;   // no item for this block (block-uniform)
    stage_init(q_join);
    st_init(q_stop);
    int64_t scanned = 0, m1 = 0, dec = 0;
    for (int tb = bid * wpb; tb < total; tb += nw) {
        int32_t t = tb + threadIdx.x / kWave;
        int32_t v = -1, role = 0, lo = 0, hi = 0;
        if (t < total) {
            int64_t desc = d.cw[t];
            v = (int32_t)(desc >> 32);
            role = (int32_t)((desc >> 30) & 3);
            lo = (int32_t)(desc & ((1 << 30) - 1)) * kCw;
            hi = min(lo + kCw, d.cap[v]);
        }
        int32_t e = lo + lane;
        int32_t w = v >= 0 && e < hi ? d.pool[d.off[v] + e] : -1;
        int32_t raw = w >= 0 ? d.level[w] : 0;
        bool clim = w >= 0 && (raw & kClimb);
        bool stop = false;
        if (climb && role == kRoleStay && clim) {
            int32_t old = atomicSub(&d.up[w], 1);
            stop = old == (d.ng == 1 ? cap1_all : up_cap(d, gp(d, w), l + 1)) + 1;
            if (stop) d.level[w] = raw | kStop;   // the only write to w's level in this step
            dec++;
        }
        st_push(q_stop, stop, w);
        int32_t cnt = role >= kRoleUp1 ? clim : 0;
        cnt = wave_sum(cnt);
        bool jn = false;
        if (lane == 0 && v >= 0) {
            scanned += hi - lo;
            if (role == kRoleUp1) {
                if (cnt) {
                    const int32_t cap1 = d.ng == 1 ? cap1_all : up_cap(d, gp(d, v), l + 1);
                    int32_t old = atomicAdd(&d.up[v], cnt);
                    jn = old <= cap1 && old + cnt > cap1;
                    m1 += cnt;
                }
            } else if (role == kRoleUp2) {
                if (cnt) atomicAdd(&d.ups[v], cnt);
            }
        }
        stage_push(q_join, jn, v);
        stage_flush(q_join, wpb, join, &c->casc_n[st.cur ^ 1], d.n, c);
        st_flush(q_stop, wpb * kWave, &c->n_sl[p], d.n, c, wr_stop);
    }
    st_flush_both(q_join, &c->casc_n[st.cur ^ 1], d.n, [=](int32_t k, int32_t x) { join[k] = x; }, q_stop,
                  &c->n_sl[p], d.n, wr_stop, c);
    // statistics: slots read, the group's up-neighbours (the U[v] reads of
    // its moves), neighbours of level l+1 gained; decrements of the group's up
    dec = block_sum64(dec, red);
    if (threadIdx.x == 0 && dec) atomicAdd(&c->step_dec[p], (int32_t)dec);
    scanned = block_sum64(scanned, red);
    m1 = block_sum64(m1, red);
    if (threadIdx.x == 0) {
        int64_t u = (bid == 0 && climb) ? c->sum_up * (int64_t)(st.l + 1 - st.phys) : 0;
        d.part[3 * bid] += scanned;
        d.part[3 * bid + 1] += u;
        d.part[3 * bid + 2] += m1;
    }
}

// Part 4: the next step after step `st` (every thread of a block calls it and
// gets the same answer).  The next movers sit at level z0: the marked
// vertices at l+1, else the next level with sorted candidates.  If they are
// every vertex of z0 and the levels above z0 are empty up to level y (at most
// the first level of the next group), they climb in lockstep: at each of
// those levels their up-degree counts the same set (themselves and the
// vertices at or above y) against the same cap, and no other vertex is at or
// next to those levels.  The next step then moves them from z0 to y in one
// go, its level set to y-1; the skipped sweeps and moves are counted by the
// caller.  occ[] is read without this step's own update (applied later by
// the caller): occ[z0] after the step is occ[z0] + (z0 == l+1 ? movers : 0).
__device__ InsStep ins_decide(Dev &d, const InsStep &st, int32_t nmv, int32_t cn, int32_t *sh1,
                              int32_t *movers_out, int32_t *occz_out, int32_t *a0_out = nullptr) {
    InsStep nx;
    nx.cur = st.cur ^ 1;
    nx.jump = 0;
    nx.done = 0;
    nx.fresh = 0;
    nx.mode = kPull;
    *movers_out = *occz_out = 0;
    int32_t l = st.l;
    // level l+1's entries are read whatever z0 turns out to be (it usually
    // is l+1), together with next_nz, so the reads overlap
    const int32_t l1 = min(l + 1, d.K), l2 = min(l + 2, d.K);
    const int32_t nz = d.next_nz[l1], s1 = d.lvl_start[l1], s2 = d.lvl_start[l2], o1 = d.occ[l1];
    int32_t z0 = cn > 0 ? l + 1 : (l + 1 < d.K ? nz : d.K);
    if (z0 >= d.K - 1) {       // nothing left (no vertex of the top group can violate Invariant 1)
        if (z0 == d.K - 1 && threadIdx.x == 0) latch(d.ctl, kErrLevel);
        nx.done = 1;
        nx.l = nx.phys = d.K;
        return nx;
    }
    const bool near = z0 == l + 1;
    const int32_t a0 = near ? s1 : d.lvl_start[z0];
    int32_t ns = (near ? s2 : d.lvl_start[z0 + 1]) - a0;
    int32_t movers = (near ? cn : 0) + ns;
    int32_t occz = (near ? o1 : d.occ[z0]) + (near ? nmv : 0);
    *movers_out = movers;
    *occz_out = occz;
    if (a0_out) *a0_out = a0;
    bool all = occz == movers;
    __syncthreads();
    if (threadIdx.x == 0) sh1[0] = INT32_MAX;
    if (threadIdx.x == 1) sh1[1] = min((z0 / d.L + 1) * d.L, d.K - 1);   // first level of the next group
    __syncthreads();
    if (d.ng > 1)   // several graphs: the first group boundary above z0 of any of them
        for (int i = threadIdx.x; i < d.nLs; i += blockDim.x) atomicMin(&sh1[1], (z0 / d.Ls[i] + 1) * d.Ls[i]);
    __syncthreads();
    int32_t limit = sh1[1];
    if (all && z0 + 2 <= limit)
        for (int32_t z = z0 + 1 + threadIdx.x; z < limit; z += blockDim.x)
            if (d.occ[z] > 0) atomicMin(&sh1[0], z);
    __syncthreads();
    int32_t y = min(sh1[0], limit);
    __syncthreads();
    if (all && y >= z0 + 2) {
        nx.l = y - 1;
        nx.phys = z0;
        nx.jump = 1;
    } else {
        nx.l = z0;
        nx.phys = z0;
    }
    return nx;
}

// Sum of the scans' per-block statistics over nparts blocks (all threads of
// one block call it; the result is valid in thread 0).
__device__ void sum_parts(Dev &d, int nparts, int64_t out[3]) {
    __shared__ int64_t ps[3][kBlock];
    int64_t a = 0, b = 0, e = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += d.part[3 * i];
        b += d.part[3 * i + 1];
        e += d.part[3 * i + 2];
    }
    ps[0][threadIdx.x] = a;
    ps[1][threadIdx.x] = b;
    ps[2][threadIdx.x] = e;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int k = 0; k < 3; k++) ps[k][threadIdx.x] += ps[k][threadIdx.x + o];
        __syncthreads();
    }
    for (int k = 0; k < 3; k++) out[k] = ps[k][0];
    __syncthreads();
}

// Bookkeeping of a finished step (one thread): counts, step log, and the
// reset of the cascade list the step consumed.  items: the step's work items
// (the scan statistics are summed per block and totalled after the sweep).
__device__ void ins_account(Dev &d, const InsStep &st, int32_t nmv, int64_t items) {
    Ctl *c = d.ctl;
    int64_t steps = st.l + 1 - st.phys;
    c->n_steps++;
    c->sweeps += steps;
    c->moves += (int64_t)nmv * steps;
    c->top = max(c->top, (int64_t)(st.l + 1));
    if (c->n_log < 4 * d.K) {
        int64_t *row = d.steplog + 4 * c->n_log++;
        row[0] = st.l;
        row[1] = st.phys;
        row[2] = nmv;
        row[3] = items | ((int64_t)st.mode << 48);
    }
    c->casc_n[st.cur] = 0;
}

// Work items of the last step of parity q (its slab-size lists and chunks).
__device__ __forceinline__ int64_t ins_items(const Ctl *c, int q) {
    const int32_t *k = c->n_cls2[q];
    return (k[0] + 7) / 8 + (k[1] + 3) / 4 + (k[2] + 1) / 2 + k[3] + c->n_chunks2[q];
}

// up* of the members that stopped in climbing steps: #neighbours at level
// >= level(v) - 1, counted from the slab after the sweep (a wavefront per
// vertex).
__global__ void k_ups_recount(Dev d) {
    int32_t cnt = d.ctl->n_rc;
    int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    int nw = gridDim.x * blockDim.x / kWave;
    for (int i = wid; i < cnt; i += nw) {
        int32_t v = d.rc[i];
        int32_t lv = d.level[v], cap = d.cap[v];
        const int32_t *s = d.pool + d.off[v];
        int32_t k = 0;
        for (int32_t e = lane; e < cap; e += kWave) {
            int32_t w = s[e];
            k += w >= 0 && d.level[w] >= lv - 1;
        }
        k = wave_sum(k);
        if (lane == 0) d.ups[v] = k;
    }
}

// Totals of the scans' per-block statistics, accumulated over a sweep (one block).
__global__ void k_ins_totals(Dev d, int nparts) {
    int64_t sums[3];
    sum_parts(d, nparts, sums);
    if (threadIdx.x == 0) {
        d.ctl->scanned = sums[0] + d.ctl->lp_scanned;
        d.ctl->alg_U = sums[1] + d.ctl->lp_U;
        d.ctl->alg_up1 = sums[2] + d.ctl->lp_up1;
    }
}

__device__ __forceinline__ void ins_store(Ctl *c, const InsStep &nx) {
    c->l = nx.l;
    c->phys = nx.phys;
    c->jump = nx.jump;
    c->cur = nx.cur;
    c->done = nx.done;
}

__device__ __forceinline__ InsStep ins_load(const Ctl *c) {
    return InsStep{c->l, c->phys, c->jump, c->cur, c->done, 0, kPull};
}

// ---- one kernel per part.  A step of parity p is two kernels: decide+prep
// and scan.  Kernels of parity p read the step state st[p]; decide+prep
// computes it from st[p^1] (the previous step, or the seeding's first step)
// in every block alike and block 1 stores it, so no block reads a slot
// that is written during the same kernel.  That block also does the
// previous step's bookkeeping and resets the work-list counters of parity
// p^1; the step's occupancy change is applied by the next kernel (the
// scan), when no block reads occ any more.
__global__ void k_ins_prep(Dev d, int p) {
    __shared__ int32_t sh[5 * (kBlock / kWave + 2)];
    __shared__ int32_t sh1[2];
    Ctl *c = d.ctl;
    if (d.ins_loop) {   // only the steps the single-block loop leaves, with their own parity
        if (!c->ins_big) return;
        p = c->ins_p;
    }
    // the bookkeeping is done by block 1, which starts as early as block 0
    // but has movers to gather only in large steps, so that its reads do not
    // delay the gathering of small steps
    const bool writer = blockIdx.x == min(1, (int)gridDim.x - 1) && threadIdx.x == 0;
    const PrevFlags pf = prev_flags_load(d, p, blockIdx.x);
    InsStep prv = c->st[p ^ 1];
    if (prv.done) {
        if (writer) c->st[p] = prv;
        return;
    }
    InsStep cur;
    int32_t nmove = 0, movers = 0, occz = 0;
    int32_t mvk[3] = {0, 0, 0};   // the pull step's first sorted position, sorted and cascaded movers
    bool have_mvk = false;
    if (prv.fresh) {
        cur = prv;
        cur.fresh = 0;
        if (!cur.done) {
            movers = d.lvl_start[cur.phys + 1] - d.lvl_start[cur.phys];
            occz = d.occ[cur.phys];
        }
    } else if (prv.mode == kClimbStep) {
        cur = climb_decide(d, prv, p, sh1, &nmove);
    } else {
        const int32_t cn = c->casc_n[prv.cur ^ 1];
        cur = ins_decide(d, prv, c->nmove[p ^ 1], cn, sh1, &movers, &occz, &mvk[0]);
        mvk[1] = movers - cn;
        mvk[2] = cn;
        have_mvk = true;
    }
    // (not right after an exit step: the members that stopped in its last
    // climbing step are residents of its level that no list holds)
    // (the group-boundary test last: in a multi-graph handle it reads the list of levels per group)
    if (prv.mode == kPull && d.climb_ok && !cur.done && !cur.jump && cur.l == cur.phys && cur.l + 2 <= d.K &&
        movers >= d.climb_min && !group_start(d, cur.l + 1)) {
        // enter a climbing step if the level's other vertices and the two
        // levels above hold few vertices next to the movers
        int32_t work = occz - movers + d.occ[cur.l + 1] + d.occ[cur.l + 2];
        if ((int64_t)work * 2 <= movers) {
            cur.mode = kClimbStep;
            nmove = movers;
        }
    }
    if (writer) {
        if (!prv.fresh) {
            int32_t nm = c->nmove[p ^ 1];
            ins_account(d, prv, nm, prv.mode == kPull ? ins_items(c, p ^ 1) : c->n_cw[p ^ 1]);
            c->pend_phys = prv.phys;
            c->pend_l1 = prv.l + 1;
            c->pend_n = nm;
            if (prv.mode == kClimbStep)
                atomicAdd((unsigned long long *)&c->sum_up, (unsigned long long)(-(int64_t)c->step_dec[p ^ 1]));
        }
        c->st[p] = cur;
        ins_store(c, cur);
        c->n_chunks2[p ^ 1] = 0;
        c->n_cls2[p ^ 1][0] = c->n_cls2[p ^ 1][1] = c->n_cls2[p ^ 1][2] = c->n_cls2[p ^ 1][3] = 0;
        c->n_cw[p ^ 1] = 0;
        c->step_dec[p] = 0;
        if (cur.mode == kPull && !cur.done && movers <= kInsLoopMovers) c->n_small++;
        if (!cur.done && movers >= kClimbMin) c->n_climbable++;
        if (cur.mode != kPull) {
            c->nmvb[p] = 0;
            c->nmove[p] = nmove;
        }
    }
    if (cur.mode == kClimbStep) climb_prep_phase(d, prv, cur, p, blockIdx.x, gridDim.x, sh, pf);
    else if (cur.mode == kExit) exit_prep_phase(d, prv, cur, p, blockIdx.x, gridDim.x, sh);
    else ins_prep_phase(d, cur, p, blockIdx.x, gridDim.x, sh, pf, have_mvk ? mvk : nullptr);
}

__global__ void k_ins_scan(Dev d, int p) {
    Ctl *c = d.ctl;
    if (d.ins_loop) {
        if (!c->ins_big) return;
        p = c->ins_p;
    }
    // bookkeeping: atomics whose result is not waited for, so block 0 goes
    // on with its work items at once
    const bool keeper = blockIdx.x == 0 && threadIdx.x == 0;
    if (keeper) {
        const int32_t pn = c->pend_n;
        if (pn) {
            atomicSub(&d.occ[c->pend_phys], pn);
            atomicAdd(&d.occ[c->pend_l1], pn);
            c->pend_n = 0;
        }
    }
    InsStep st = c->st[p];
    if (st.done) return;
    if (keeper) {
        // the next step's stoppers list (the preparation of this step read
        // the previous one's); the climber list is not appended to here
        c->n_sl[p ^ 1] = 0;
        if (st.mode == kExit) {   // the group is gone; its members are joiners now
            atomicAdd(&c->casc_n[st.cur ^ 1], c->n_exit);
            c->n_exit = 0;
            c->n_cl = 0;
            c->sum_up = 0;
        }
        c->n_cl_snap = c->n_cl;
    }
    __shared__ ScanQ sq;
    if (st.mode == kPull) ins_scan_phase(d, st, p, blockIdx.x, gridDim.x, true, sq);
    else climb_scan_phase(d, st, p, blockIdx.x, gridDim.x, sq);
}

// Vertices with edges, bucketed by level at the start of an insertion sweep
// (counting sort with a histogram in LDS per block; K <= kHistMax).
__global__ void k_bucket_count(Dev d) {
    extern __shared__ int32_t hist[];
    for (int i = threadIdx.x; i < d.K; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n; v += stride)
        if (d.deg[v] > 0) atomicAdd(&hist[d.level[v]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < d.K; i += blockDim.x)
        if (hist[i]) atomicAdd(&d.lvb_fill[i], hist[i]);
}

// One block of 1024: the counts in lvb_fill to bucket starts (lvb_start,
// K+2 entries) and scatter cursors (lvb_fill).
__global__ void k_bucket_scan(Dev d) {
    __shared__ int32_t part[1024];
    int K = d.K, tid = threadIdx.x, nt = blockDim.x;
    int per = (K + nt - 1) / nt, lo = min(K, tid * per), hi = min(K, lo + per);
    int32_t sum = 0;
    for (int i = lo; i < hi; i++) sum += d.lvb_fill[i];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        int32_t a = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += a;
        __syncthreads();
    }
    int32_t acc = part[tid] - sum;
    for (int i = lo; i < hi; i++) {
        int32_t cnt = d.lvb_fill[i];
        d.lvb_start[i] = acc;
        d.lvb_fill[i] = acc;
        acc += cnt;
    }
    if (tid == nt - 1) d.lvb_start[K] = d.lvb_start[K + 1] = part[nt - 1];
}

__global__ void k_bucket_scatter(Dev d) {
    extern __shared__ int32_t hist[];
    for (int i = threadIdx.x; i < d.K; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n; v += stride)
        if (d.deg[v] > 0) atomicAdd(&hist[d.level[v]], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < d.K; b += blockDim.x) {
        int32_t cnt = hist[b];
        if (cnt) hist[b] = atomicAdd(&d.lvb_fill[b], cnt);
    }
    __syncthreads();
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n; v += stride)
        if (d.deg[v] > 0) d.lvb[atomicAdd(&hist[d.level[v]], 1)] = v;
}

// ---- the whole level loop in one cooperative launch
struct Bar {
    unsigned count, gen;
    int abort;
};

constexpr long kSpinLimit = 1L << 22;

// Grid-wide barrier for a cooperative launch (all blocks co-resident).
// Agent-scope fences make every block's writes visible to all XCDs.  A wait
// gives up after kSpinLimit polls, raises `abort`, and every block then
// leaves the loop at its next barrier.  Returns false once aborted.
__device__ bool grid_sync(Bar *b, unsigned nblk) {
    __shared__ int ab;
    __syncthreads();
    if (threadIdx.x == 0) {
        int aborted = 0;
        unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned arrived = atomicAdd(&b->count, 1u);
        if (arrived == nblk - 1) {
            __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&b->gen, 1u);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    aborted = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    atomicExch(&b->abort, 1);
                    aborted = 1;
                    break;
                }
            }
        }
        __threadfence();
        ab = aborted || __hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return !ab;
}

// Every step is prep | scan with a grid barrier after each part; the
// decision for the next step is taken by every block on its own (same inputs,
// same answer) at the start of the next iteration.  Block 0 does the
// bookkeeping, applies each step's occupancy change one phase later (when no
// block reads occ) and resets the work-list counters of the other parity.
__global__ void __launch_bounds__(kBlock) k_ins_sweep(Dev d, Bar *bar) {
    __shared__ int32_t sh[5 * (kBlock / kWave + 2)];
    __shared__ int32_t sh1[2];
    __shared__ ScanQ sq;
    const int bid = blockIdx.x, nblk = gridDim.x;
    const bool writer = bid == 0 && threadIdx.x == 0;
    Ctl *c = d.ctl;
    InsStep st = ins_load(c);
    InsStep prev{};
    int32_t prev_nmv = 0;
    int p = 0;
    bool have_prev = false, occ_pending = false;
    while (true) {
        if (have_prev) {
            int32_t cn = c->casc_n[prev.cur ^ 1], mv_unused, oc_unused;
            st = ins_decide(d, prev, prev_nmv, cn, sh1, &mv_unused, &oc_unused);
            if (writer) {
                ins_account(d, prev, prev_nmv, ins_items(c, p ^ 1));
                ins_store(c, st);
                c->n_chunks2[p ^ 1] = 0;
                c->n_cls2[p ^ 1][0] = c->n_cls2[p ^ 1][1] = c->n_cls2[p ^ 1][2] = c->n_cls2[p ^ 1][3] = 0;
            }
            occ_pending = true;
        }
        if (!ins_prep_phase(d, st, p, bid, nblk, sh, prev_flags_load(d, p, bid), nullptr)) {
            if (writer) c->done = 1;
            break;
        }
        if (st.done) break;
        if (!grid_sync(bar, nblk)) break;
        if (writer && occ_pending) {
            d.occ[prev.phys] -= prev_nmv;
            d.occ[prev.l + 1] += prev_nmv;
            occ_pending = false;
        }
        ins_scan_phase(d, st, p, bid, nblk, true, sq);
        if (!grid_sync(bar, nblk)) break;
        prev_nmv = c->nmvb[p];
        prev = st;
        have_prev = true;
        p ^= 1;
    }
    if (writer && occ_pending) {
        d.occ[prev.phys] -= prev_nmv;
        d.occ[prev.l + 1] += prev_nmv;
    }
    (void)grid_sync(bar, nblk);   // the statistics are totalled by the caller
    if (writer && __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        latch(c, kErrHang);
        c->done = 1;
    }
}

// ------------------------------------------------------ deletion sweep
// Desire-level (Def. desire-level) of an Invariant-2 violator w at level lw:
// the largest l' in [1, lw-1] with cnt(l'-1) >= dn_min[gn(l'-1)], where
// cnt(j) = #neighbours at level >= j; 0 if there is none.  Such an l' also
// satisfies Invariant 1 (the count one level up is below dn_min <= up_max).
//
// cnt(j) never grows with j and dn_min[gn(j)] never shrinks, so the test
// cnt(j) >= dn_min[gn(j)] holds on a prefix of [0, lw-2]: the answer is one
// more than the last j of that prefix, found by binary search.  It holds at
// j = 0 whenever w has a neighbour (dn_min[0] = 1), and fails above the
// highest neighbour level.  Each probe counts the neighbours at level >= j,
// so the work is O(deg(w) log lw), independent of how many levels lie below
// w.  Neighbour levels are clamped to lw-1 (a probe never exceeds lw-2).

constexpr int kDlRegs = 8;                       // slab slots per lane kept in registers
constexpr int32_t kDlWaveCap = kDlRegs * kWave;  // slabs of up to 512 slots take one wavefront

// Both searches below find the last j of a window [lo, hi] where the count
// cnt(j) of w's neighbours at level >= j reaches a per-group threshold:
// dn_min (the desire-level of a deletion) or up_max + 1 (the first level
// above an insertion violator where Invariant 1 holds is one more).  The
// test holds on a prefix of the window (cnt never grows with j, the
// thresholds never shrink); the result is lo - 1 if it fails at lo.
// Neighbour levels are clamped to `clamp` (>= hi).
struct Srch {
    int32_t lo, hi, clamp, up;   // up = 0: dn_min[g], 1: up_max[g] + 1
};
__device__ __forceinline__ int32_t srch_thr(const Dev &d, GP p, const Srch &q, int32_t j) {
    return q.up ? min(d.up_max[p.tab + j / p.L], INT32_MAX - 1) + 1 : d.dn_min[p.tab + j / p.L];
}

// One wavefront (every lane calls it; w is wave-uniform, cap = d.cap[w] <= kDlWaveCap).
__device__ int32_t wave_srch(const Dev &d, int32_t w, int32_t cap, const Srch &q) {
    const int lane = threadIdx.x % kWave;
    const GP p = gp(d, w);
    const int32_t *s = d.pool + d.off[w];
    const int nr = (cap + kWave - 1) / kWave;
    int32_t x[kDlRegs], y[kDlRegs];
#pragma unroll
    for (int r = 0; r < kDlRegs; r++) {
        const int32_t e = r * kWave + lane;
        x[r] = (r < nr && e < cap) ? s[e] : -1;
    }
    int32_t ymax = -1;
#pragma unroll
    for (int r = 0; r < kDlRegs; r++) {
        y[r] = x[r] >= 0 ? min(d.level[x[r]], q.clamp) : -1;
        ymax = max(ymax, y[r]);
    }
    ymax = wave_max(ymax);
    int32_t lo = q.lo - 1, hi = min(q.hi, ymax);   // answer in [lo, hi]; lo = "fails at q.lo"
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        int32_t c = 0;
#pragma unroll
        for (int r = 0; r < kDlRegs; r++)
            if (r < nr) c += __popcll(__ballot(y[r] >= mid));
        if (c >= srch_thr(d, p, q, mid)) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Desire-level of an Invariant-2 violator at level lw (largest l' in
// [1, lw-1] with cnt(l'-1) >= dn_min[gn(l'-1)], else 0).
__device__ __forceinline__ int32_t wave_dl(const Dev &d, int32_t w, int32_t lw, int32_t cap) {
    return wave_srch(d, w, cap, Srch{0, lw - 2, max(lw - 1, 0), 0}) + 1;
}

// One global atomic per block for a running minimum, maximum or sum that
// every thread contributes to (every thread of the block calls it; block-
// uniform control flow).  Same-address device atomics serialise, so a
// contribution per lane or per wavefront would queue thousands of them.
__device__ __forceinline__ void block_min_to(int32_t x, int32_t *dst) {
    __shared__ int32_t acc;
    if (threadIdx.x == 0) acc = kInf;
    __syncthreads();
    x = -wave_max(-x);
    if (threadIdx.x % kWave == 0 && x < kInf) atomicMin(&acc, x);
    __syncthreads();
    if (threadIdx.x == 0 && acc < kInf) atomicMin(dst, acc);
}
__device__ __forceinline__ void block_add64_to(int64_t x, unsigned long long *dst) {
    __shared__ unsigned long long acc;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    x = wave_sum64(x);
    if (threadIdx.x % kWave == 0 && x) atomicAdd(&acc, (unsigned long long)x);
    __syncthreads();
    if (threadIdx.x == 0 && acc) atomicAdd(dst, acc);
}

// Block-wide sums and maxima (every thread calls them; red holds one int per
// wavefront of the block).
__device__ __forceinline__ int32_t block_sum32(int32_t x, int32_t *red) {
    x = wave_sum(x);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = x;
    __syncthreads();
    int32_t t = 0;
    for (int i = 0; i < (int)blockDim.x / kWave; i++) t += red[i];
    __syncthreads();
    return t;
}
__device__ __forceinline__ int32_t block_max32(int32_t x, int32_t *red) {
    x = wave_max(x);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = x;
    __syncthreads();
    int32_t t = INT32_MIN;
    for (int i = 0; i < (int)blockDim.x / kWave; i++) t = max(t, red[i]);
    __syncthreads();
    return t;
}

// The whole block, for a slab of any size (block-uniform call): a
// segmented histogram of the neighbour levels in LDS.  A pass counts the
// neighbours whose (clamped) level falls in a window of values [a, a+span),
// in at most kDlBins bins of width W; suffix sums of the bins plus the
// neighbours above the window give cnt() at every bin start, and the last
// bin start where the test holds brackets the answer within W levels.  The
// next pass refines that bin, until W = 1: one pass while lw <= nbins, two
// up to nbins^2 levels.  hist: LDS [nbins]; sh: LDS of at least
// blockDim/kWave + 2 ints.
constexpr int32_t kDlBins = 2048;   // bins of the single-block deletion loop

__device__ int32_t block_srch(const Dev &d, int32_t w, const Srch &q, int32_t *hist, int32_t nbins, int32_t *sh) {
    const int tid = threadIdx.x, nt = blockDim.x, nwv = blockDim.x / kWave;
    if (q.hi < q.lo) return q.lo - 1;   // block-uniform
    const GP p = gp(d, w);
    const int32_t cap = d.cap[w];
    const int32_t *s = d.pool + d.off[w];
    int32_t *sh_base = sh + nwv + 1;
    // the first kDlRegs slots of each thread stay in registers (clamped
    // levels) across the passes; the loads of a batch are issued together
    int32_t y0[kDlRegs];
    {
        int32_t x[kDlRegs];
#pragma unroll
        for (int r = 0; r < kDlRegs; r++) {
            const int32_t e = r * nt + tid;
            x[r] = e < cap ? s[e] : -1;
        }
#pragma unroll
        for (int r = 0; r < kDlRegs; r++) y0[r] = x[r] >= 0 ? min(d.level[x[r]], q.clamp) : -1;
    }
    // window of values [a, a+span): below q.lo nothing matters, above the
    // clamp nothing exists
    int32_t a = q.lo, span = q.clamp + 1 - q.lo, base = 0;
    for (;;) {   // block-uniform
        const int32_t nb = min(span, nbins);
        const int32_t W = (span + nb - 1) / nb;
        for (int i = tid; i < nb; i += nt) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kDlRegs; r++) {
            const int32_t y = y0[r] - a;
            if (y0[r] >= 0 && y >= 0 && y < span) atomicAdd(&hist[y / W], 1);
        }
        for (int32_t e0 = kDlRegs * nt; e0 < cap; e0 += kDlRegs * nt) {
            int32_t x[kDlRegs];
#pragma unroll
            for (int r = 0; r < kDlRegs; r++) {
                const int32_t e = e0 + r * nt + tid;
                x[r] = e < cap ? s[e] : -1;
            }
#pragma unroll
            for (int r = 0; r < kDlRegs; r++) {
                if (x[r] < 0) continue;
                const int32_t y = min(d.level[x[r]], q.clamp) - a;
                if (y >= 0 && y < span) atomicAdd(&hist[y / W], 1);
            }
        }
        __syncthreads();
        // thread t owns the bins of segment nt-1-t, so that the exclusive
        // prefix over threads counts the bins above its segment
        const int32_t per = (nb + nt - 1) / nt;
        const int32_t b0 = (nt - 1 - tid) * per, b1 = min(nb, b0 + per);
        int32_t mine = 0;
        for (int32_t b = b0; b < b1; b++) mine += hist[b];
        int32_t tot;
        int32_t cnt = block_excl(mine, &tot, sh) + base;
        int32_t best = -1, above_best = 0;
        for (int32_t b = b1 - 1; b >= b0; b--) {
            const int32_t hb = hist[b];
            cnt += hb;   // cnt(a + b*W)
            const int32_t j = a + b * W;
            if (j <= q.hi && cnt >= srch_thr(d, p, q, j)) {
                best = b;
                above_best = cnt - hb;
                break;
            }
        }
        const int32_t bmax = block_max32(best, sh);
        if (bmax < 0) return q.lo - 1;   // the test fails at q.lo (only possible in the first pass)
        if (best == bmax) *sh_base = above_best;
        __syncthreads();
        base = *sh_base;
        a += bmax * W;
        __syncthreads();
        if (W == 1) return a;
        span = W;
    }
}

__device__ __forceinline__ int32_t block_dl(const Dev &d, int32_t w, int32_t lw, int32_t *hist, int32_t nbins,
                                            int32_t *sh) {
    return block_srch(d, w, Srch{0, lw - 2, max(lw - 1, 0), 0}, hist, nbins, sh) + 1;
}

__device__ __forceinline__ bool del_viol(const Dev &d, int32_t w, int32_t lw) {
    return lw > 0 && d.ups[w] < dn_floor(d, gp(d, w), lw);
}
// A load that reads the device-coherent value (bypassing the compute unit's
// L1): for counters that atomics of the same kernel have changed.
__device__ __forceinline__ int32_t ld_dev(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool del_viol_dev(const Dev &d, int32_t w, int32_t lw) {
    return lw > 0 && ld_dev(&d.ups[w]) < dn_floor(d, gp(d, w), lw);
}

// mode 0: seed from the endpoints of deleted edges (list = touch, pending
// list = cur).  mode 1: recompute for the vertices listed in rc during a
// step (pending list = next); the last block then closes the step.
// The batch's touched endpoints that violate Invariant 2 (Algorithm 3's
// first candidates), a thread each, into the recompute list; on the way each
// endpoint's degree drops by its count of deleted edges, and the count is
// cleared.  Usually a handful of the
// touched endpoints violate, so the desire-level kernel (a block per vertex)
// only sees those.
__global__ void k_del_cand(Dev d) {
    __shared__ Stage q;
    stage_init(q);
    const int32_t nt = d.ctl->n_touch;
    const int stride = gridDim.x * blockDim.x;
    for (int ib = blockIdx.x * blockDim.x; ib < nt; ib += stride) {
        const int i = ib + threadIdx.x;
        bool viol = false;
        int32_t w = -1;
        if (i < nt) {
            w = d.touch[i];
            d.deg[w] -= d.addc[w];   // the endpoint's deleted edges (counted by k_dedupe)
            d.addc[w] = 0;
            const int32_t lw = d.level[w];
            viol = lw > 0 && d.ups[w] < dn_floor(d, gp(d, w), lw);
        }
        stage_push(q, viol, w);
        stage_flush(q, blockDim.x, d.rc, &d.ctl->n_rc, d.n, d.ctl);
    }
    stage_flush(q, kStage, d.rc, &d.ctl->n_rc, d.n, d.ctl);
}

// Desire-levels of the vertices of the recompute list that violate
// Invariant 2 (mode 0: the batch's candidates listed by k_del_cand; mode 1:
// the neighbours a step's moves left violating, when the step was too large
// for the single-block loop).  A wavefront per vertex whose slab fits its
// registers; then, in a second pass, a block per larger slab.
__device__ __forceinline__ bool dl_record(const Dev &d, Ctl *c, int32_t w, int32_t lw, int32_t dv, int32_t l) {
    if (dv <= l || dv >= lw) latch(c, kErrOrder);
    const bool fresh = d.dl[w] < 0;   // not pending yet
    d.dl[w] = dv;
    return fresh;
}

// A wavefront per listed vertex: violators whose slab fits the wavefront's
// registers get their desire-level; larger ones are listed (the idle
// cascade list casc1, counter n_big) for k_dl_big.  The iterations are
// block-uniform so that new pending vertices are staged in LDS and appended
// with one atomic per block, and the running minimum of the desire-levels
// takes one atomic per block.
__global__ void __launch_bounds__(kBlock) k_dl(Dev d, int mode) {
    __shared__ Stage q;
    Ctl *c = d.ctl;
    if (mode == 1 && (c->done || !c->del_big)) return;
    stage_init(q);
    const int32_t cur = c->cur, tgt = mode == 0 ? cur : (cur ^ 1);
    int32_t *plist = tgt ? d.p1 : d.p0;
    const int32_t l = mode == 0 ? -1 : c->l;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    constexpr int nwb = kBlock / kWave;
    const int32_t cnt = c->n_rc;
    int32_t best = kInf;
    int64_t ncalc = 0;
    for (int base = blockIdx.x * nwb; base < cnt; base += gridDim.x * nwb) {   // block-uniform
        const int i = base + wid;
        bool fresh = false;
        int32_t w = -1;
        if (i < cnt) {   // wave-uniform
            w = d.rc[i];
            const int32_t lw = d.level[w];
            if (del_viol(d, w, lw)) {
                const int32_t cap = d.cap[w];
                if (cap > kDlWaveCap) {
                    if (lane == 0) push(d.casc1, &c->n_big, d.n, w, c);
                } else {
                    const int32_t dv = wave_dl(d, w, lw, cap);
                    if (lane == 0) {
                        ncalc++;
                        fresh = dl_record(d, c, w, lw, dv, l);
                        best = min(best, dv);
                    }
                }
            }
        }
        stage_push(q, fresh, w);
        stage_flush(q, blockDim.x, plist, &c->p_n[tgt], d.n, c);
    }
    stage_flush(q, kStage, plist, &c->p_n[tgt], d.n, c);
    block_min_to(best, &c->nm);
    block_add64_to(ncalc, (unsigned long long *)&c->dl_calcs);
}

// A block of kBigBlock threads per listed violator with a large slab; its
// histogram has one bin per level (min(K, kHistMax) bins of dynamic LDS), so
// one pass over the slab usually suffices.
constexpr int kBigBlock = 1024;
constexpr int kBigGrid = 512;      // deletions: many hub violators per step in some streams
constexpr int kJmpBigGrid = 128;   // jumps: few large-slab movers per round
__global__ void __launch_bounds__(kBigBlock) k_dl_big(Dev d, int mode, int32_t nbins) {
    extern __shared__ int32_t hist[];
    __shared__ int32_t red[kBigBlock / kWave + 2];
    Ctl *c = d.ctl;
    if (mode == 1 && (c->done || !c->del_big)) return;
    const int32_t cur = c->cur, tgt = mode == 0 ? cur : (cur ^ 1);
    int32_t *plist = tgt ? d.p1 : d.p0;
    const int32_t l = mode == 0 ? -1 : c->l;
    const int32_t cnt = c->n_big;
    int32_t ncalc = 0, best = kInf;
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {   // block-uniform
        const int32_t w = d.casc1[i];
        const int32_t lw = d.level[w];
        const int32_t dv = block_dl(d, w, lw, hist, nbins, red);
        if (threadIdx.x == 0) {
            ncalc++;
            if (dl_record(d, c, w, lw, dv, l)) push(plist, &c->p_n[tgt], d.n, w, c);
            best = min(best, dv);
        }
    }
    block_min_to(best, &c->nm);
    if (threadIdx.x == 0 && ncalc) atomicAdd((unsigned long long *)&c->dl_calcs, (unsigned long long)ncalc);
}

// One thread: close a deletion step (mode 1) or the seeding (mode 0), and
// set the next level to the smallest pending desire-level.
__global__ void k_del_next(Dev d, int mode) {
    Ctl *c = d.ctl;
    if (mode == 1 && (c->done || !c->del_big)) return;
    if (mode == 1) {
        int32_t cur = c->cur;
        c->del_big = 0;   // the next step goes back to the single-block loop
        c->big_steps += 1;
        if (c->n_log < 4 * d.K) {
            int64_t *row = d.steplog + 4 * c->n_log++;
            row[0] = -1 - c->l;
            row[1] = c->p_n[cur];
            row[2] = c->n_mv;
            row[3] = c->scanned | (1LL << 48);   // run by the grid kernels
        }
        c->sweeps += 1;
        c->moves += c->n_mv;
        c->p_n[cur] = 0;
        c->cur = cur ^ 1;
        c->n_mv = 0;
        c->n_chunks = 0;
        c->n_rc = 0;
        c->step_id += 1;
    }
    c->n_big = 0;
    if (mode == 0) {
        c->n_rc = 0;   // the candidates' list has been read
        c->viol_del0 = c->p_n[c->cur];
    }
    int32_t nm = c->nm;
    c->nm = kInf;
    if (nm == kInf) c->done = 1;
    else c->l = nm;
}

// Step of Algorithm 3 at level l, part 1: the movers are the pending
// vertices whose desire-level is l; the rest stay pending.
__global__ void k_del_select(Dev d) {
    Ctl *c = d.ctl;
    if (c->done || !c->del_big) return;
    int32_t l = c->l, cur = c->cur, nxt = cur ^ 1, np = c->p_n[cur];
    const int32_t *P = cur ? d.p1 : d.p0;
    int32_t *Q = nxt ? d.p1 : d.p0;
    int gid = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x % kWave;
    int stride = gridDim.x * blockDim.x;
    int32_t best = kInf;
    for (int i0 = gid - lane; i0 < np; i0 += stride) {
        int i = i0 + lane;
        int32_t v = -1, dv = -1;
        if (i < np) {
            v = P[i];
            dv = d.dl[v];
            if (dv != l) {
                if (dv < l) latch(c, kErrOrder);
                best = min(best, dv);
            }
        }
        bool mover = i < np && dv == l;
        wpush(d.mv, &c->n_mv, d.n, mover, v, c);
        wpush(Q, &c->p_n[nxt], d.n, i < np && dv != l, v, c);
        add_chunks_w(d, mover ? v : -1);
    }
    block_min_to(best, &c->nm);
}

// Part 2: every mover v (previous level pv) scans its slab.  A neighbour w
// with dl(w) = l moves too.  Any other w loses v from its up-degree if
// l < level(w) <= pv and from its up*-degree if l+1 < level(w) <= pv+1; a w
// that starts violating Invariant 2, or that is already pending, gets its
// desire-level recomputed after the step.  v's own degrees at level l are
// counted on the way.
// Whether a pending vertex's desire-level dw (-1: not pending) can change
// when a neighbour moves down from level pv to l in a deletion step.  The
// desire-level is the largest l' whose count of neighbours at level >= l'-1
// reaches the floor; the move lowers the counts at the levels in (l, pv]
// alone, and counts only fall during the pass, so dw can change only when
// dw-1 is among those levels.  Otherwise the stored value stays exact and
// no recomputation is needed.
__device__ __forceinline__ bool pending_changes(int32_t dw, int32_t l, int32_t pv) {
    return dw >= 0 && dw - 1 > l && dw - 1 <= pv;
}

__global__ void k_del_scan(Dev d) {
    Ctl *c = d.ctl;
    if (c->done || !c->del_big) return;
    int32_t l = c->l, nch = c->n_chunks, sid = c->step_id;
    int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    int nw = gridDim.x * blockDim.x / kWave;
    int32_t scanned = 0;
    for (int ci = wid; ci < nch; ci += nw) {
        int64_t desc = d.chunks[ci];
        int32_t v = (int32_t)(desc >> 32), k = (int32_t)(desc & 0xffffffff);
        int32_t cap = d.cap[v], pv = d.level[v];
        const int32_t *s = d.pool + d.off[v];
        int32_t lo = k * kChunk, hi = min(lo + kChunk, cap);
        int32_t cu = 0, cus = 0;
        for (int32_t e0 = lo; e0 < hi; e0 += kWave) {
            int32_t e = e0 + lane;
            int32_t w = e < hi ? s[e] : -1;
            bool fresh = false;
            if (w >= 0) {
                int32_t dw = d.dl[w];
                if (dw == l) {
                    cu++;
                    cus++;
                } else {
                    int32_t lw = d.level[w];
                    cu += lw >= l;
                    cus += lw >= l - 1;
                    bool again = pending_changes(dw, l, pv);
                    if (lw > l && lw <= pv) atomicSub(&d.up[w], 1);
                    if (lw > l + 1 && lw <= pv + 1) {
                        int32_t old = atomicSub(&d.ups[w], 1);
                        if (old == dn_floor(d, gp(d, w), lw)) again = true;
                    }
                    fresh = again && atomicExch(&d.rcstamp[w], sid) != sid;
                }
            }
            wpush(d.rc, &c->n_rc, d.n, fresh, w, c);
        }
        scanned += hi - lo;
        cu = wave_sum(cu);
        cus = wave_sum(cus);
        if (lane == 0) {
            if (cu) atomicAdd(&d.stay[v], cu);
            if (cus) atomicAdd(&d.cnt2[v], cus);
        }
    }
    if (lane == 0 && scanned) atomicAdd((unsigned long long *)&c->scanned, (unsigned long long)scanned);
}

// Part 3: movers take level l with their recounted degrees and leave the
// pending set.
__global__ void k_del_fin(Dev d) {
    Ctl *c = d.ctl;
    if (c->done || !c->del_big) return;
    int32_t l = c->l, nmv = c->n_mv;
    int stride = gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&d.occ[l], nmv);   // every mover lands at level l
    const int lane = threadIdx.x % kWave;
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < nmv; i0 += stride) {
        const int i = i0 + lane;
        const int32_t v = i < nmv ? d.mv[i] : -1;
        wave_add_key(d.occ, v >= 0 ? d.level[v] : -1, -1);
        if (v < 0) continue;
        d.level[v] = l;
        d.up[v] = d.stay[v];
        d.ups[v] = d.cnt2[v];
        d.stay[v] = 0;
        d.cnt2[v] = 0;
        d.dl[v] = -1;
    }
}

// The deletion level loop of Algorithm 3 in one block, for steps that are
// small (the usual case: a batch of deletions moves few vertices down, over
// few levels, and each step of the grid kernels above would cost a chain of
// five launches).  Each step is the same as select / scan / fin / k_dl /
// k_del_next: the pending vertices whose desire-level is l move to l
// together; their neighbours' up and up* counters drop; the neighbours left
// violating Invariant 2 (and pending ones that lost a neighbour) get their
// desire-levels recomputed; the next level is the smallest pending
// desire-level.  A step whose pending list or movers' slabs exceed the
// limits below is handed to the grid kernels (del_big), which run that one
// step and hand the loop back.  Every step moves to a strictly higher level
// (Lemma smaller-level), so at most K steps run; a desire-level that breaks
// this latches kErrOrder and ends the loop.
constexpr int kLoopBlock = 1024;
constexpr int32_t kLoopPending = 2048;   // most pending vertices of a step run here
constexpr int32_t kLoopSlots = 4096;     // most slab slots of a step's movers run here (d.loop_slots;
                                         // 0 in sweep mode 2, which sends every step to the grid kernels)

__global__ void __launch_bounds__(kLoopBlock) k_del_loop(Dev d) {
    __shared__ int32_t red[kLoopBlock / kWave + 2];
    __shared__ int32_t hist[kDlBins];
    __shared__ int64_t red64[kLoopBlock / kWave];
    __shared__ int32_t s_stop, s_l, s_cur, s_np, s_nmv, s_nq, s_nm, s_nrc, s_nbig, s_nsmall, s_calc, s_sid;
    __shared__ unsigned long long s_scanned;
    Ctl *c = d.ctl;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    constexpr int nw = kLoopBlock / kWave;
    if (tid == 0) {
        s_stop = c->done || c->del_big || (ld_dev(&c->err) & kErrOrder);
        s_l = c->l;
        s_cur = c->cur;
        s_np = c->p_n[c->cur];
    }
    __syncthreads();
    for (int32_t steps = 0; !s_stop; steps++) {
        const int32_t l = s_l, cur = s_cur, np = s_np;
        const int32_t *P = cur ? d.p1 : d.p0;
        int32_t *Q = cur ? d.p0 : d.p1;
        // size of the step
        int32_t nm = 0;
        int64_t slots = 0;
        if (np <= kLoopPending)
            for (int i = tid; i < np; i += kLoopBlock) {
                const int32_t v = P[i];
                if (d.dl[v] == l) {
                    nm++;
                    slots += d.cap[v];
                }
            }
        nm = block_sum32(nm, red);
        slots = block_sum64(slots, red64);
        if (np > kLoopPending || slots > d.loop_slots || steps > d.K) {
            if (tid == 0) {
                if (steps > d.K) latch(c, kErrOrder);   // cannot happen with exact desire-levels
                else c->del_big = 1;
            }
            break;   // block-uniform
        }
        if (tid == 0) {
            s_nmv = 0;
            s_nq = c->p_n[cur ^ 1];
            s_nm = kInf;
            s_nrc = 0;
            s_nbig = 0;
            s_nsmall = 0;
            s_calc = 0;
            s_scanned = 0;
            s_sid = c->step_id;
        }
        __syncthreads();
        // select: movers to d.mv, the rest stay pending in Q
        for (int i = tid; i < np; i += kLoopBlock) {
            const int32_t v = P[i], dv = d.dl[v];
            if (dv == l) {
                d.mv[atomicAdd(&s_nmv, 1)] = v;
            } else {
                if (dv < l) latch(c, kErrOrder);
                atomicMin(&s_nm, dv);
                Q[atomicAdd(&s_nq, 1)] = v;
            }
        }
        __syncthreads();
        // scan: a wavefront per mover
        const int32_t nmv = s_nmv, sid = s_sid;
        for (int mi = wid; mi < nmv; mi += nw) {
            const int32_t v = d.mv[mi];
            const int32_t cap = d.cap[v], pv = d.level[v];
            const int32_t *sl = d.pool + d.off[v];
            int32_t cu = 0, cus = 0;
            for (int32_t e0 = 0; e0 < cap; e0 += kWave) {
                const int32_t e = e0 + lane;
                const int32_t w = e < cap ? sl[e] : -1;
                bool fresh = false;
                if (w >= 0) {
                    const int32_t dw = d.dl[w];
                    if (dw == l) {
                        cu++;
                        cus++;
                    } else {
                        const int32_t lw = d.level[w];
                        cu += lw >= l;
                        cus += lw >= l - 1;
                        bool again = pending_changes(dw, l, pv);
                        if (lw > l && lw <= pv) atomicSub(&d.up[w], 1);
                        if (lw > l + 1 && lw <= pv + 1) {
                            const int32_t old = atomicSub(&d.ups[w], 1);
                            if (old == dn_floor(d, gp(d, w), lw)) again = true;
                        }
                        fresh = again && atomicExch(&d.rcstamp[w], sid) != sid;
                    }
                }
                const uint64_t mask = __ballot(fresh);
                if (mask) {
                    int32_t base = 0;
                    const int leader = __ffsll((unsigned long long)mask) - 1;
                    if (lane == leader) base = atomicAdd(&s_nrc, __popcll(mask));
                    base = __shfl(base, leader, kWave);
                    if (fresh) d.rc[base + __popcll(mask & ((1ull << lane) - 1))] = w;
                }
            }
            cu = wave_sum(cu);
            cus = wave_sum(cus);
            if (lane == 0) {
                d.stay[v] = cu;
                d.cnt2[v] = cus;
                atomicAdd(&s_scanned, (unsigned long long)cap);
            }
        }
        __syncthreads();
        // fin: the movers take level l with their recounted degrees
        for (int i = tid; i < nmv; i += kLoopBlock) {
            const int32_t v = d.mv[i];
            atomicSub(&d.occ[d.level[v]], 1);
            atomicAdd(&d.occ[l], 1);
            d.level[v] = l;
            d.up[v] = d.stay[v];
            d.ups[v] = d.cnt2[v];
            d.stay[v] = 0;
            d.cnt2[v] = 0;
            d.dl[v] = -1;
        }
        __syncthreads();
        // desire-levels of the recompute list: its violators are listed, a
        // thread per entry, into the idle cascade lists (slabs that fit a
        // wavefront's registers from the front of casc0, larger ones into
        // casc1); then a wavefront per small slab and the whole block per
        // larger one
        const int32_t nrc = s_nrc;
        for (int i = tid; i < nrc; i += kLoopBlock) {
            const int32_t w = d.rc[i];
            const int32_t lw = d.level[w];
            if (!del_viol_dev(d, w, lw)) continue;
            if (d.cap[w] > kDlWaveCap) d.casc1[atomicAdd(&s_nbig, 1)] = w;
            else d.casc0[atomicAdd(&s_nsmall, 1)] = w;
        }
        __syncthreads();
        const int32_t nsmall = s_nsmall;
        for (int i = wid; i < nsmall; i += nw) {
            const int32_t w = d.casc0[i];
            const int32_t lw = d.level[w];
            const int32_t dv = wave_dl(d, w, lw, d.cap[w]);
            if (lane == 0) {
                atomicAdd(&s_calc, 1);
                if (dv <= l || dv >= lw) latch(c, kErrOrder);
                if (d.dl[w] < 0) Q[atomicAdd(&s_nq, 1)] = w;
                d.dl[w] = dv;
                atomicMin(&s_nm, dv);
            }
        }
        __syncthreads();
        const int32_t nbig = s_nbig;
        for (int i = 0; i < nbig; i++) {   // block-uniform
            const int32_t w = d.casc1[i];
            const int32_t lw = d.level[w];
            const int32_t dv = block_dl(d, w, lw, hist, kDlBins, red);
            if (tid == 0) {
                s_calc++;
                if (dv <= l || dv >= lw) latch(c, kErrOrder);
                if (d.dl[w] < 0) Q[s_nq++] = w;
                d.dl[w] = dv;
                s_nm = min(s_nm, dv);
            }
        }
        __syncthreads();
        // close the step (as k_del_next)
        if (tid == 0) {
            if (c->n_log < 4 * d.K) {
                int64_t *row = d.steplog + 4 * c->n_log++;
                row[0] = -1 - l;
                row[1] = np;
                row[2] = nmv;
                row[3] = c->scanned + (int64_t)s_scanned;
            }
            c->scanned += (int64_t)s_scanned;
            c->dl_calcs += s_calc;
            c->sweeps += 1;
            c->moves += nmv;
            c->p_n[cur] = 0;
            c->p_n[cur ^ 1] = s_nq;
            c->cur = cur ^ 1;
            c->n_mv = 0;
            c->n_chunks = 0;
            c->n_rc = 0;
            c->step_id += 1;
            const int32_t nxt = s_nm;
            if (nxt == kInf) c->done = 1;
            else c->l = nxt;
            s_l = nxt;
            s_cur = cur ^ 1;
            s_np = s_nq;
            s_stop = c->done || (ld_dev(&c->err) & kErrOrder);
        }
        __syncthreads();
    }
}

// ---- small insertion steps in one block.  Most steps of an insertion sweep
// move a handful of vertices with small slabs; as two grid-wide kernels
// (k_ins_prep, k_ins_scan) such a step costs mostly launch gaps and the
// latency of its dependent memory accesses.  k_ins_loop runs such steps back
// to back in one workgroup.  Each step is decided, prepared and scanned as
// those two kernels do it, with the same lists, flags, counters and
// bookkeeping (the movers' slabs are cut into slots spread over the block's
// threads), so that either side can take over after any step.  The loop
// stops before a step with more than kInsLoopMovers movers or kInsLoopSlots
// slab slots, a climbing or exit step (or the step after one), or when the
// sweep is done.  A step it leaves is run by the step kernels launched after
// it (they return at once otherwise): ins_big is set and ins_p holds the
// step's parity; the next launch of the loop takes over after that step.
// The previous step's occupancy change is applied after the next step is
// decided, where the step kernels apply it, so a hand-over in either
// direction sees the state the step kernels would leave.
constexpr int kInsLoopR = kInsLoopSlots / kLoopBlock;   // slab slots per thread

// Index i of the last prefix entry pre[i] <= j (pre[0] = 0, ascending; n entries).
__device__ __forceinline__ int32_t prefix_owner(const int32_t *pre, int32_t n, int32_t j) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kLoopBlock) k_ins_loop(Dev d) {
    __shared__ int32_t sh1[2];
    __shared__ int32_t red[kLoopBlock / kWave + 2];
    __shared__ int32_t s_pre[kInsLoopMovers + 1];   // exclusive prefix sums of the movers' slab sizes
    __shared__ int32_t s_mv[kInsLoopMovers];
    __shared__ int64_t s_off[kInsLoopMovers];
    __shared__ int32_t s_stay[kInsLoopMovers];
    __shared__ int32_t s_p, s_stop, s_nc, s_nsl, s_slbase;
    Ctl *c = d.ctl;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int32_t p = c->ins_p;
        if (c->ins_big) {   // the step kernels ran the step this loop left them
            c->ins_big = 0;
            p ^= 1;
            c->ins_p = p;
        }
        s_p = p;
        s_stop = c->done || ld_dev(&c->err) != 0;
        if (!s_stop) c->ins_trips++;
    }
    __syncthreads();
    while (!s_stop) {   // block-uniform
        const int p = s_p;
        const int32_t Mp = p ? kMover1 : kMover0, Mn = p ? kMover0 : kMover1;
        const InsStep prv = c->st[p ^ 1];
        bool hand = !prv.fresh && prv.mode != kPull;
        InsStep cur = prv;
        int32_t movers = 0, occz = 0, a0 = 0, nA = 0, nB = 0;
        if (!hand) {
            if (prv.fresh) {
                cur.fresh = 0;
                if (!cur.done) {
                    a0 = d.lvl_start[cur.phys];
                    movers = d.lvl_start[cur.phys + 1] - a0;
                    occz = d.occ[cur.phys];
                }
                nA = movers;
                nB = c->casc_n[cur.cur];
            } else {
                const int32_t cn = c->casc_n[prv.cur ^ 1];
                cur = ins_decide(d, prv, c->nmove[p ^ 1], cn, sh1, &movers, &occz, &a0);
                nA = movers - cn;
                nB = cn;
            }
            if (d.climb_ok && !cur.done && !cur.jump && cur.l == cur.phys && cur.l + 2 <= d.K &&
                movers >= d.climb_min && !group_start(d, cur.l + 1)) {
                const int32_t work = occz - movers + d.occ[cur.l + 1] + d.occ[cur.l + 2];
                if ((int64_t)work * 2 <= movers) hand = true;   // a climbing step: the step kernels run it
            }
        }
        const int32_t nm = nA + nB;
        int32_t slots = 0;
        if (!hand && !cur.done) {
            if (cur.phys < 0 || cur.phys > cur.l || cur.l + 1 >= d.K || nm > d.n) {
                if (tid == 0) {
                    latch(c, kErrLevel);
                    s_stop = 1;
                }
                __syncthreads();
                break;
            }
            if (nm > kInsLoopMovers) {
                hand = true;
            } else {
                // the movers, their slabs and slab sizes (two per thread)
                const int32_t *casc = cur.cur ? d.casc1 : d.casc0;
                int32_t cap2 = 0;
                for (int i = 2 * tid; i < 2 * tid + 2; i++) {
                    if (i >= nm) break;
                    const int32_t v = i < nA ? d.sorted[a0 + i] : casc[i - nA];
                    const int32_t cp = d.cap[v];
                    s_mv[i] = v;
                    s_off[i] = d.off[v];
                    s_stay[i] = 0;
                    s_pre[i] = cp;
                    cap2 += cp;
                }
                int32_t first = 0;
                const int32_t base = block_excl(cap2, &slots, red);
                if (2 * tid < nm) {
                    first = s_pre[2 * tid];
                    s_pre[2 * tid] = base;
                    if (2 * tid + 1 < nm) s_pre[2 * tid + 1] = base + first;
                }
                if (tid == 0) s_pre[nm] = slots;
                __syncthreads();
                if (slots > kInsLoopSlots) hand = true;
            }
        }
        if (hand) {
            if (tid == 0) {
                c->ins_big = 1;
                c->ins_p = p;
                s_stop = 1;
            }
            __syncthreads();
            break;
        }
        // commit: the previous step's bookkeeping and occupancy change, the
        // step state, the work-list counters (as k_ins_prep's writer and
        // k_ins_scan's keeper)
        if (tid == 0) {
            if (!prv.fresh) {
                const int32_t nm0 = c->nmove[p ^ 1];
                ins_account(d, prv, nm0, ins_items(c, p ^ 1));
                if (nm0) {
                    d.occ[prv.phys] -= nm0;
                    d.occ[prv.l + 1] += nm0;
                }
            }
            c->st[p] = cur;
            ins_store(c, cur);
            c->n_chunks2[p ^ 1] = 0;
            c->n_cls2[p ^ 1][0] = c->n_cls2[p ^ 1][1] = c->n_cls2[p ^ 1][2] = c->n_cls2[p ^ 1][3] = 0;
            c->n_cw[p ^ 1] = 0;
            c->step_dec[p] = 0;
            c->n_sl[p ^ 1] = 0;
            c->n_cl_snap = c->n_cl;
            s_nc = 0;
            s_nsl = 0;
            s_slbase = c->n_sl[p];
        }
        {   // the previous step's movers lose its flag (a mover that moves again keeps this step's)
            const int32_t np = c->nmvb[p ^ 1];
            const int32_t *prev = p ? d.mv : d.mv1;
            for (int i = tid; i < np; i += kLoopBlock) {
                const int32_t u = prev[i];
                const int32_t raw = d.level[u];
                d.level[u] = (raw & (kLevelMask | kClimb)) | ((raw & Mp) ? Mp : 0);
            }
        }
        __syncthreads();
        if (cur.done) {
            if (tid == 0) s_stop = 1;
            __syncthreads();
            break;
        }
        // prepare: flag the movers, list them for the next step's clearing,
        // and count them by slab-size class (the step log's work items)
        int32_t *mvp = p ? d.mv1 : d.mv;
        int32_t k0 = 0, k1 = 0, k2 = 0, k3 = 0, kch = 0;
        for (int i = tid; i < nm; i += kLoopBlock) {
            const int32_t v = s_mv[i];
            const int32_t cp = s_pre[i + 1] - s_pre[i];
            mvp[i] = v;
            d.level[v] = cur.phys | Mp;
            k0 += cp <= 8;
            k1 += cp > 8 && cp <= 16;
            k2 += cp > 16 && cp <= 32;
            k3 += cp > 32 && cp <= 64;
            kch += cp > 64 ? (cp + kChunk - 1) / kChunk : 0;
        }
        k0 = block_sum32(k0, red);
        k1 = block_sum32(k1, red);
        k2 = block_sum32(k2, red);
        k3 = block_sum32(k3, red);
        kch = block_sum32(kch, red);   // (its barriers also order the flagging before the scan)
        if (tid == 0) {
            c->n_cls2[p][0] = k0;
            c->n_cls2[p][1] = k1;
            c->n_cls2[p][2] = k2;
            c->n_cls2[p][3] = k3;
            c->n_chunks2[p] = kch;
            c->nmvb[p] = c->nmove[p] = nm;
        }
        // scan: the slots of all movers' slabs, kInsLoopR per thread, their
        // loads issued together
        const int32_t l = cur.l, nxt = cur.cur ^ 1;
        int32_t *casc = nxt ? d.casc1 : d.casc0;
        const int32_t ub1_all = d.ng == 1 ? d.up_max[(l + 1) / d.L] : 0;
        int32_t wv[kInsLoopR], mo[kInsLoopR];
#pragma unroll
        for (int k = 0; k < kInsLoopR; k++) {
            const int32_t j = tid + k * kLoopBlock;
            wv[k] = -1;
            mo[k] = 0;
            if (j < slots) {
                const int32_t mi = prefix_owner(s_pre, nm, j);
                mo[k] = mi;
                wv[k] = d.pool[s_off[mi] + (j - s_pre[mi])];
            }
        }
        int32_t rw[kInsLoopR];
#pragma unroll
        for (int k = 0; k < kInsLoopR; k++) rw[k] = wv[k] >= 0 ? d.level[wv[k]] : 0;
        int32_t nU = 0, n1 = 0;
#pragma unroll
        for (int k = 0; k < kInsLoopR; k++) {
            const int32_t w = wv[k], raw = rw[k];
            const bool comover = w >= 0 && (raw & Mp);
            const int32_t lw = (w < 0 || comover) ? -1 : (raw & kLevelMask);
            nU += comover || lw >= l;
            if (lw == l) {
                atomicAdd(&s_stay[mo[k]], 1);
            } else if (lw == l + 1) {
                n1++;
                const int32_t ub1 = d.ng == 1 ? ub1_all : up_cap(d, gp(d, w), l + 1);
                const int32_t old = atomicAdd(&d.up[w], 1);
                if (cur.jump) atomicAdd(&d.ups[w], 1);
                if (old == ub1) {
                    const int32_t pos = atomicAdd(&s_nc, 1);
                    if (pos < d.n) casc[pos] = w;
                    else latch(c, kErrPool);
                }
            } else if (lw == l + 2) {
                atomicAdd(&d.ups[w], 1);
            }
        }
        nU = block_sum32(nU, red);
        n1 = block_sum32(n1, red);
        // finish the movers: level l+1, up*(v) = old up(v), up(v) = old up(v) - stay;
        // a mover still above the cap of l+1 keeps moving (next step's flag, cascade list)
        int32_t *slist = p ? d.sl1 : d.sl0;
        for (int i = tid; i < nm; i += kLoopBlock) {
            const int32_t v = s_mv[i];
            int32_t u = ld_dev(&d.up[v]);   // atomics of earlier steps of this launch may have changed it
            d.ups[v] = u;
            u -= s_stay[i];
            d.up[v] = u;
            const int32_t ub1 = d.ng == 1 ? ub1_all : up_cap(d, gp(d, v), l + 1);
            const bool viol = u > ub1;
            d.level[v] = (l + 1) | Mp | (viol ? Mn : 0);
            if (viol) {
                const int32_t pos = atomicAdd(&s_nc, 1);
                if (pos < d.n) casc[pos] = v;
                else latch(c, kErrPool);
            } else if (d.climb_ok) {
                const int32_t pos = s_slbase + atomicAdd(&s_nsl, 1);
                if (pos < d.n) slist[pos] = v;
                else latch(c, kErrPool);
            }
        }
        __syncthreads();
        if (tid == 0) {
            c->casc_n[nxt] = s_nc;
            c->n_sl[p] = s_slbase + s_nsl;
            c->lp_scanned += slots;
            c->lp_U += nU;
            c->lp_up1 += n1;
            c->lp_moves += (int64_t)nm * (l + 1 - cur.phys);
            c->lp_steps++;
            s_p = p ^ 1;
            c->ins_p = p ^ 1;
            if (c->n_steps > 2 * d.K + 2) latch(c, kErrLevel);   // a level gets at most an exit and a moving step
            s_stop = ld_dev(&c->err) != 0;
        }
        __syncthreads();
    }
}

// ------------------------------------------------- insertions with jumps
// The implementation's insertion procedure (PLDS implementation details):
// levels are processed upwards from the lowest one holding an Invariant-1
// violator; the violators S_l of level l each take their desire-level (the
// first level above l where Invariant 1 holds, counted from the levels
// before any of them moves; Invariant 2 then holds there too, since the
// count one level down exceeds the cap, which is at least the floor less
// one), and all of S_l move there together.  A neighbour w that stays
// gains an up-neighbour for a mover v going from l to t_v if l < level(w)
// <= t_v, and an up*-neighbour if l+1 < level(w) <= t_v+1; one whose count
// crosses its cap becomes pending at its level; a mover that still violates
// at t_v (co-movers landed above it) becomes pending at t_v.  Pending
// vertices sit in the ping-pong lists p0/p1 (idle during insertions), the
// round's movers' targets in dl[] (-1 elsewhere).

// Initial pending list: the violators among the touched endpoints (listed
// by k_ins_seed in cand).
__global__ void k_jmp_init(Dev d) {
    Ctl *c = d.ctl;
    const int32_t nc = c->n_cand;
    int32_t *P = c->cur ? d.p1 : d.p0;
    int32_t best = kInf;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        const int32_t v = d.cand[i];
        P[i] = v;
        best = min(best, d.level[v]);
    }
    block_min_to(best, &c->nm);
    if (blockIdx.x == 0 && threadIdx.x == 0) c->p_n[c->cur] = nc;
}

// Round at level l, part 1: movers (pending at l) to mv with their slab
// chunks; the rest stay pending.
__global__ void k_jmp_select(Dev d) {
    Ctl *c = d.ctl;
    if (c->done) return;
    const int32_t l = c->l, cur = c->cur, nxt = cur ^ 1, np = c->p_n[cur];
    const int32_t *P = cur ? d.p1 : d.p0;
    int32_t *Q = nxt ? d.p1 : d.p0;
    const int lane = threadIdx.x % kWave;
    const int stride = gridDim.x * blockDim.x;
    int32_t best = kInf;
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < np; i0 += stride) {
        const int i = i0 + lane;
        int32_t v = -1, lv = -1;
        if (i < np) {
            v = P[i];
            lv = d.level[v];
            if (lv < l) latch(c, kErrOrder);
            else if (lv > l) best = min(best, lv);
        }
        const bool mover = i < np && lv == l;
        wpush(d.mv, &c->n_mv, d.n, mover, v, c);
        wpush(Q, &c->p_n[nxt], d.n, i < np && lv > l, v, c);
        add_chunks_w(d, mover ? v : -1);
    }
    block_min_to(best, &c->nm);
}

// Part 2: each mover's desire-level into dl[]: a wavefront per slab that fits
// its registers, the rest listed (casc1, n_big) for k_jmp_dl_big.
__global__ void __launch_bounds__(kBlock) k_jmp_dl(Dev d) {
    Ctl *c = d.ctl;
    if (c->done) return;
    const int32_t l = c->l, nmv = c->n_mv;
    const int lane = threadIdx.x % kWave;
    const int nw = gridDim.x * (kBlock / kWave);
    for (int i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < nmv; i += nw) {   // wave-uniform
        const int32_t v = d.mv[i];
        const int32_t cap = d.cap[v];
        if (cap > kDlWaveCap) {
            if (lane == 0) push(d.casc1, &c->n_big, d.n, v, c);
            continue;
        }
        const int32_t t = wave_srch(d, v, cap, Srch{l, d.K - 2, d.K - 1, 1}) + 1;
        if (lane == 0) {
            if (t <= l) latch(c, kErrOrder);
            d.dl[v] = t;
        }
    }
}

__global__ void __launch_bounds__(kBigBlock) k_jmp_dl_big(Dev d, int32_t nbins) {
    extern __shared__ int32_t hist[];
    __shared__ int32_t red[kBigBlock / kWave + 2];
    Ctl *c = d.ctl;
    if (c->done) return;
    const int32_t l = c->l, cnt = c->n_big;
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {   // block-uniform
        const int32_t v = d.casc1[i];
        const int32_t t = block_srch(d, v, Srch{l, d.K - 2, d.K - 1, 1}, hist, nbins, red) + 1;
        if (threadIdx.x == 0) {
            if (t <= l) latch(c, kErrOrder);
            d.dl[v] = t;
        }
    }
}

// Part 3: every mover v (l -> t = dl[v]) scans its slab by chunks.  A
// co-mover w counts at its own target dl[w]; another w keeps its level lw,
// gains an up-neighbour if l < lw <= t (the one whose count reaches cap + 1
// makes it pending) and an up*-neighbour if l+1 < lw <= t+1.  v's own up and
// up* at t are counted on the way (stay, cnt2).
__global__ void k_jmp_scan(Dev d) {
    Ctl *c = d.ctl;
    if (c->done) return;
    const int32_t l = c->l, nch = c->n_chunks, nxt = c->cur ^ 1;
    int32_t *Q = nxt ? d.p1 : d.p0;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    int32_t scanned = 0, bumps = 0, best = kInf;
    for (int ci = wid; ci < nch; ci += nw) {
        const int64_t desc = d.chunks[ci];
        const int32_t v = (int32_t)(desc >> 32), k = (int32_t)(desc & 0xffffffff);
        const int32_t cap = d.cap[v], t = d.dl[v];
        const int32_t *sl = d.pool + d.off[v];
        const int32_t lo = k * kChunk, hi = min(lo + kChunk, cap);
        int32_t cu = 0, cus = 0;
        for (int32_t e0 = lo; e0 < hi; e0 += kWave) {
            const int32_t e = e0 + lane;
            const int32_t w = e < hi ? sl[e] : -1;
            bool pend = false;
            if (w >= 0) {
                const int32_t tw = d.dl[w];
                const int32_t lw = tw >= 0 ? tw : d.level[w];   // a co-mover counts at its target
                cu += lw >= t;
                cus += lw >= t - 1;
                if (tw < 0) {
                    if (lw > l && lw <= t) {
                        const int32_t old = atomicAdd(&d.up[w], 1);
                        bumps++;
                        if (old == up_cap(d, gp(d, w), lw)) {
                            pend = true;
                            best = min(best, lw);
                        }
                    }
                    if (lw > l + 1 && lw <= t + 1) {
                        atomicAdd(&d.ups[w], 1);
                        bumps++;
                    }
                }
            }
            wpush(Q, &c->p_n[nxt], d.n, pend, w, c);
        }
        scanned += hi - lo;
        cu = wave_sum(cu);
        cus = wave_sum(cus);
        if (lane == 0) {
            if (cu) atomicAdd(&d.stay[v], cu);
            if (cus) atomicAdd(&d.cnt2[v], cus);
        }
    }
    // scanned is wave-uniform; count it once per wavefront
    block_min_to(best, &c->nm);
    block_add64_to(lane == 0 ? scanned : 0, (unsigned long long *)&c->scanned);
    block_add64_to(bumps, (unsigned long long *)&c->alg_up1);
}

// Part 4: movers take their targets with their recounted degrees; one that
// still violates becomes pending at its new level.
__global__ void k_jmp_fin(Dev d) {
    Ctl *c = d.ctl;
    if (c->done) return;
    const int32_t nmv = c->n_mv, nxt = c->cur ^ 1;
    int32_t *Q = nxt ? d.p1 : d.p0;
    const int lane = threadIdx.x % kWave;
    const int stride = gridDim.x * blockDim.x;
    int32_t best = kInf, top = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicSub(&d.occ[c->l], nmv);   // every mover leaves level l
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < nmv; i0 += stride) {
        const int i = i0 + lane;
        bool pend = false;
        int32_t v = -1, t = -1;
        if (i < nmv) {
            v = d.mv[i];
            t = d.dl[v];
        }
        wave_add_key(d.occ, t, 1);
        if (i < nmv) {
            d.level[v] = t;
            d.up[v] = d.stay[v];
            d.ups[v] = d.cnt2[v];
            d.stay[v] = 0;
            d.cnt2[v] = 0;
            d.dl[v] = -1;
            top = max(top, t);
            if (d.up[v] > up_cap(d, gp(d, v), t)) {
                pend = true;
                best = min(best, t);
            }
        }
        wpush(Q, &c->p_n[nxt], d.n, pend, v, c);
    }
    block_min_to(best, &c->nm);
    top = wave_max(top);
    if (lane == 0 && top) atomicMax((unsigned long long *)&c->top, (unsigned long long)top);
}

// One thread: close a round (mode 1) or the seeding (mode 0), and take the
// lowest pending level next.
__global__ void k_jmp_next(Dev d, int mode) {
    Ctl *c = d.ctl;
    if (mode == 1 && c->done) return;
    if (mode == 1) {
        if (c->n_log < 4 * d.K) {
            int64_t *row = d.steplog + 4 * c->n_log++;
            row[0] = c->l;
            row[1] = c->l;
            row[2] = c->n_mv;
            row[3] = (int64_t)c->n_chunks + ((int64_t)3 << 48);   // kind 3: a round of jumps
        }
        c->sweeps += 1;
        c->moves += c->n_mv;
        c->p_n[c->cur] = 0;
        c->cur ^= 1;
        c->n_mv = 0;
        c->n_chunks = 0;
    }
    c->n_big = 0;
    const int32_t nm = c->nm;
    c->nm = kInf;
    if (nm == kInf) c->done = 1;
    else c->l = nm;
}

// ------------------------------------------------------------- queries
// Def. coreness estimate: (1+delta)^max(floor((l+1)/L)-1, 0), 0 if isolated.
__global__ void k_coreness(Dev d, const int32_t *vs, int64_t cnt, double *out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
        int32_t v = vs ? vs[i] : (int32_t)i;
        if (v < 0 || v >= d.n) {
            out[i] = -1.0;
            latch(d.ctl, kErrRange);
            continue;
        }
        const GP p = gp(d, v);
        int32_t e = (d.level[v] + 1) / p.L - 1;
        out[i] = d.deg[v] == 0 ? 0.0 : d.pow_tab[p.tab + (e > 0 ? e : 0)];
    }
}

// Full check, one wave per vertex; bad[0..5] count violations of:
// counters, Invariant 1, Invariant 2, isolated at level 0, level range,
// slab live count == degree.
// ---- orientation (the orientation section, Algorithm 5): an edge points
// from the endpoint at the lower level to the one at the higher level; on
// equal levels the edge {u, v}, u < v, points u -> v.
__device__ __forceinline__ bool points_up(int32_t u, int32_t v, int32_t lu, int32_t lv) {
    // true: min(u, v) -> max(u, v)
    return u < v ? lu <= lv : lv <= lu;
}

// (tail, head) of each edge under the levels lv; ids out of range give
// (-1, -1) and latch a range error.
__global__ void k_orient(Dev d, const int32_t *e, int64_t cnt, const int32_t *lv, int32_t *out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const int32_t a = e[2 * i], b = e[2 * i + 1];
        if (a < 0 || a >= d.n || b < 0 || b >= d.n) {
            out[2 * i] = out[2 * i + 1] = -1;
            latch(d.ctl, kErrRange);
            continue;
        }
        const int32_t u = min(a, b), v = max(a, b);
        const bool fwd = points_up(u, v, lv[u], lv[v]);
        out[2 * i] = fwd ? u : v;
        out[2 * i + 1] = fwd ? v : u;
    }
}

// ---- slab traversal by slab size (flip scan, static peeling)
// A pass that visits every slot of the slabs of a list of vertices keeps
// many searches in flight per wavefront when the vertices are sorted by slab
// size first: class 0 (at most 8 slots) and 1 (9..16) take lane groups of
// 8 and 16 lanes, class 2 (up to kSlabHub) a wavefront each, class 3 (hubs)
// is cut into 256-slot chunks dealt out over all wavefronts.  Classes 0 and
// 1 are listed from the front and the back of one array of n entries,
// classes 2 and 3 likewise in a second one; the lists hold distinct
// vertices, so two lists that share an array never meet.
constexpr int32_t kSlabHub = 2048;
constexpr int kSlabQ = 1024;
constexpr int kSlabChunk = 4;   // 64-slot pieces per wavefront pass

__device__ __forceinline__ int slab_class(int32_t cap) {
    return cap <= 8 ? 0 : cap <= 16 ? 1 : cap <= kSlabHub ? 2 : 3;
}

struct SlabQ {
    StageT<int32_t, kSlabQ> q[4];
};

__device__ __forceinline__ void slabq_init(SlabQ &s) {
    for (int k = 0; k < 4; k++) st_init(s.q[k]);
}

// every thread of the block calls both; cls < 0 lists nothing
__device__ __forceinline__ void slabq_push(SlabQ &s, int cls, int32_t v) {
    for (int k = 0; k < 4; k++) st_push(s.q[k], cls == k, v);
}

// Moves every queue with fewer than `room` free entries to its list (all
// non-empty ones when room = kSlabQ), deciding for the four queues at once,
// so that a round without a flush costs two barriers.
__device__ void slabq_flush(SlabQ &s, int32_t room, int32_t *lo, int32_t *hi, int32_t *cnt, int32_t n, Ctl *c) {
    __shared__ int32_t base[4];
    __syncthreads();
    int32_t k[4];
    bool any = false;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        k[q] = s.q[q].n;
        if (k[q] == 0 || k[q] + room <= kSlabQ) k[q] = 0;   // not flushed this time
        any |= k[q] != 0;
    }
    __syncthreads();
    if (!any) return;   // block-uniform
    if (threadIdx.x < 4 && k[threadIdx.x]) {
        base[threadIdx.x] = atomicAdd(&cnt[threadIdx.x], k[threadIdx.x]);
        if (base[threadIdx.x] + k[threadIdx.x] > n) latch(c, kErrLevel);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int32_t b = base[q];
        for (int i = threadIdx.x; i < k[q]; i += blockDim.x) {
            if (b + i >= n) continue;
            const int32_t x = s.q[q].buf[i];
            if (q == 0) lo[b + i] = x;
            else if (q == 1) lo[n - 1 - (b + i)] = x;
            else if (q == 2) hi[b + i] = x;
            else hi[n - 1 - (b + i)] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 && k[threadIdx.x]) s.q[threadIdx.x].n = 0;
    __syncthreads();
}

// Every slot of every listed vertex's slab.  Every lane of the wavefront
// calls it with the same lists and counts.  Per vertex u, hu = head(u) is
// loaded once; the slots are taken in groups, gather(w) (w = -1: no slot)
// is issued for the whole group before apply(u, hu, w, g) runs for each slot
// of it, with every lane of the wavefront together.
template <class Head, class Gather, class Apply>
__device__ void visit_slabs(const Dev &d, const int32_t *lo, const int32_t *hi, const int32_t cnt[4], Head head,
                            Gather gather, Apply apply) {
    using G = decltype(gather(0));
    const int lane = threadIdx.x % kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    // (the counts never exceed n by construction; clamped so that a list
    // read from the back of its array stays inside it in any case)
    const int32_t nn = d.n, n0 = min(cnt[0], nn), n1 = min(cnt[1], nn), n2 = min(cnt[2], nn), n3 = min(cnt[3], nn);
    // kSlabChunk * 64 slots of u's slab from slot e0
    auto chunk = [&](int32_t u, int2 hu, const int32_t *sl, int32_t cu, int32_t e0) {
        int32_t w[kSlabChunk];
        G g[kSlabChunk];
#pragma unroll
        for (int k = 0; k < kSlabChunk; k++) {
            const int32_t e = e0 + k * kWave + lane;
            w[k] = e < cu ? sl[e] : -1;
        }
#pragma unroll
        for (int k = 0; k < kSlabChunk; k++) g[k] = gather(w[k]);
#pragma unroll
        for (int k = 0; k < kSlabChunk; k++) apply(u, hu, w[k], g[k]);
    };
    // hubs: chunks numbered across the hubs, 64 hubs at a time (a lane
    // loads one hub's header); a wavefront takes the chunks whose number is
    // its own modulo the number of wavefronts
    int64_t before = 0;
    for (int32_t hb = 0; hb < n3; hb += kWave) {
        int32_t hv = -1, hc = 0;
        int2 hh = make_int2(0, 0);
        int64_t ho = 0;
        if (hb + lane < n3) {
            hv = hi[nn - 1 - (hb + lane)];
            hh = head(hv);
            hc = d.cap[hv];
            ho = d.off[hv];
        }
        const int32_t nch = (hc + kSlabChunk * kWave - 1) / (kSlabChunk * kWave);
        int32_t tot;
        const int32_t ex = wave_excl(nch, &tot);
        for (int64_t f = before + ((wid - before) % nw + nw) % nw; f < before + tot; f += nw) {
            const int32_t r = (int32_t)(f - before);
            const int j = __popcll(__ballot(ex + nch <= r));   // the hub holding chunk r
            const int32_t u = __shfl(hv, j, kWave), cu = __shfl(hc, j, kWave);
            const int2 hu = make_int2(__shfl(hh.x, j, kWave), __shfl(hh.y, j, kWave));
            const int64_t o = __shfl(ho, j, kWave);
            chunk(u, hu, d.pool + o, cu, (r - __shfl(ex, j, kWave)) * kSlabChunk * kWave);
        }
        before += tot;
    }
    // class 2: a wavefront each
    for (int32_t i = wid; i < n2; i += nw) {
        const int32_t u = hi[i];
        const int2 hu = head(u);
        const int32_t cu = d.cap[u];
        const int32_t *sl = d.pool + d.off[u];
        for (int32_t e0 = 0; e0 < cu; e0 += kSlabChunk * kWave) chunk(u, hu, sl, cu, e0);
    }
    // classes 1 and 0: lane groups, a vertex each, two passes of the grid in flight
    auto groups = [&](auto GS, int32_t cnt_c, bool from_back) {
        constexpr int gs = decltype(GS)::value, per = kWave / gs;
        const int gi = lane / gs, gl = lane % gs;
        for (int32_t base = wid * per; base < cnt_c; base += 2 * nw * per) {
            int32_t u[2], w[2];
            int2 hu[2];
            G g[2];
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int32_t i = base + k * nw * per + gi;
                u[k] = i < cnt_c ? (from_back ? lo[nn - 1 - i] : lo[i]) : -1;
            }
#pragma unroll
            for (int k = 0; k < 2; k++) {
                hu[k] = make_int2(0, 0);
                w[k] = -1;
                if (u[k] >= 0) {
                    hu[k] = head(u[k]);
                    if (gl < d.cap[u[k]]) w[k] = d.pool[d.off[u[k]] + gl];
                }
            }
#pragma unroll
            for (int k = 0; k < 2; k++) g[k] = gather(w[k]);
#pragma unroll
            for (int k = 0; k < 2; k++) apply(u[k], hu[k], w[k], g[k]);
        }
    };
    groups(std::integral_constant<int, 16>{}, n1, true);
    groups(std::integral_constant<int, 8>{}, n0, false);
}

// Both levels of every vertex side by side (d.lvp), so that the edge scan
// gathers one 8-byte pair per neighbour instead of two 4-byte values from two
// arrays; and the vertices whose level differs from the call's starting
// level, by slab class (d.mv, d.mv1; counts n_fl).
__global__ void k_flip_moved(Dev d) {
    __shared__ SlabQ q;
    slabq_init(q);
    const int32_t nn = d.n;
    const int stride = gridDim.x * blockDim.x;
    for (int vb = blockIdx.x * blockDim.x; vb < nn; vb += stride) {
        const int v = vb + threadIdx.x;
        int cls = -1;
        if (v < nn) {
            const int32_t l0 = d.prevlvl[v], l1 = d.level[v];
            d.lvp[v] = make_int2(l0, l1);
            if (l0 != l1) cls = slab_class(d.cap[v]);
        }
        slabq_push(q, cls, v);
        slabq_flush(q, blockDim.x, d.mv, d.mv1, d.ctl->n_fl, nn, d.ctl);
    }
    slabq_flush(q, kSlabQ, d.mv, d.mv1, d.ctl->n_fl, nn, d.ctl);
}

// The call's applied insertions into the batch hash set (empty before).
__global__ void k_flip_inserted(Dev d, const int32_t *ins, int64_t cnt) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const uint64_t key = ((uint64_t)(uint32_t)ins[2 * i] << 32) | (uint32_t)ins[2 * i + 1];
        uint64_t j = mix64(key) & d.hmask;
        for (uint64_t p = 0; p <= d.hmask; p++) {
            const uint64_t prev =
                atomicCAS((unsigned long long *)&d.hset[j], (unsigned long long)kEmpty64, (unsigned long long)key);
            if (prev == kEmpty64 || prev == key) break;
            j = (j + 1) & d.hmask;
        }
    }
}

__device__ __forceinline__ bool flip_was_inserted(const Dev &d, uint64_t key) {
    uint64_t j = mix64(key) & d.hmask;
    for (uint64_t p = 0; p <= d.hmask; p++) {
        const uint64_t x = d.hset[j];
        if (x == key) return true;
        if (x == kEmpty64) return false;
        j = (j + 1) & d.hmask;
    }
    return false;
}

// Algorithm 5's first loop: the moved vertices search their edges; an edge
// whose orientation under the starting levels differs from the one under
// the current levels is a flip, reported as it was.  An edge with both
// endpoints moved is reported by its smaller endpoint; edges the call
// inserted (in the hash set when with_ins) had no orientation before.
// The slabs are visited by slab class.  Each wavefront stages its flips in
// LDS and appends them with one atomic per 256; positions at or beyond cap
// are counted, not written.
constexpr int kFlipStage = 256;
__global__ void __launch_bounds__(kBlock) k_flip_scan(Dev d, int with_ins, int32_t *out, int64_t cap) {
    __shared__ int32_t buf[kBlock / kWave][2 * (kFlipStage + kWave)];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int32_t *b = buf[wv];
    int32_t nb = 0;   // wave-uniform
    auto flush = [&]() {
        __threadfence_block();   // the wavefront's staged entries are visible to all its lanes
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long *)&d.ctl->n_flip, (unsigned long long)nb);
        base = __shfl(base, 0, kWave);
        for (int i = lane; i < 2 * nb; i += kWave)
            if ((int64_t)base + i / 2 < cap) out[2 * base + i] = b[i];
        nb = 0;
    };
    // one slot (w < 0: none) with both levels of both ends; stages the edge
    // (u, w) if it flipped
    auto slot = [&](int32_t u, int2 lu, int32_t w, int2 lw) {
        bool f = false;
        int32_t t = 0, hd = 0;
        if (w >= 0) {
            const bool b0 = points_up(u, w, lu.x, lw.x), b1 = points_up(u, w, lu.y, lw.y);
            const int32_t lo = min(u, w), hi = max(u, w);
            f = b0 != b1 && (lw.x == lw.y || u < w);
            if (f && with_ins) f = !flip_was_inserted(d, ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi);
            t = b0 ? lo : hi;
            hd = b0 ? hi : lo;
        }
        const uint64_t m = __ballot(f);
        if (f) {
            const int k = nb + __popcll(m & ((1ull << lane) - 1));
            b[2 * k] = t;
            b[2 * k + 1] = hd;
        }
        nb += __popcll(m);
        if (nb >= kFlipStage) flush();
    };
    const int2 *lvp = d.lvp;
    visit_slabs(
        d, d.mv, d.mv1, d.ctl->n_fl, [=](int32_t u) { return lvp[u]; },
        [=](int32_t w) { return w >= 0 ? lvp[w] : make_int2(0, 0); }, slot);
    if (nb) flush();
}

// Largest coreness estimate over the vertices [v0, v0 + cnt) (one graph).
__global__ void k_max_estimate(Dev d, int32_t v0, int32_t cnt) {
    uint64_t best = 0;
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const int32_t v = v0 + i;
        if (d.deg[v] == 0) continue;
        const GP p = gp(d, v);
        const int32_t e = (d.level[v] + 1) / p.L - 1;
        const double est = d.pow_tab[p.tab + (e > 0 ? e : 0)];
        best = max(best, (uint64_t)__double_as_longlong(est));
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor((unsigned long long)best, o, kWave);
        best = max(best, y);
    }
    if (threadIdx.x % kWave == 0 && best) atomicMax((unsigned long long *)&d.ctl->dv_bits, (unsigned long long)best);
}

// ---- static approximate k-core (the static section, Algorithm 6).  State:
// C[v] (the count), B[v] (bucket; -1: no edges or peeled, -2: peeled in
// the current round), r[v] (the round's peeled neighbours of v; zero
// between rounds), cnt[b] (alive vertices per bucket), pw[b] = (1+eps)^b by
// repeated double multiplication on the host; Ilo/Ihi list the round's
// peeled vertices by slab class, T the vertices the round touched.  A round
// peels bucket bp, lowers the counts of the peeled vertices' alive
// neighbours, re-buckets them, and picks the next bucket.
struct SK {
    int32_t *C, *B, *r, *cnt, *Ilo, *Ihi, *T;
    const double *pw;
    double *est;
    int32_t nbk, R;
    double eps;
};
constexpr int kSkBuckets = 4096;   // most buckets (LDS histogram of a block)

// least b with pw[b] >= c (c >= 1)
__device__ __forceinline__ int32_t sk_bucket(const SK &k, int32_t c) {
    int32_t lo = 0, hi = k.nbk - 1;
    const double x = (double)c;
    while (lo < hi) {
        const int32_t mid = (lo + hi) / 2;
        if (k.pw[mid] >= x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// flush a block's bucket-count changes (LDS histogram h, nbk entries)
__device__ void sk_flush_hist(const SK &k, int32_t *h) {
    __syncthreads();
    for (int b = threadIdx.x; b < k.nbk; b += blockDim.x)
        if (h[b]) atomicAdd(&k.cnt[b], h[b]);
}

// Powers of 1+eps (pw[b] = pw[b-1] * (1+eps) in double, from pw[0] = 1, the
// same repeated multiplication as the host's count of them) and cleared
// bucket counts.  One block.
__global__ void k_sk_setup(SK k) {
    double *pw = const_cast<double *>(k.pw);
    if (threadIdx.x == 0) {
        double x = 1.0;
        for (int32_t b = 0; b < k.nbk; b++) {
            if (b > 0) x *= 1.0 + k.eps;
            pw[b] = x;
        }
    }
    for (int i = threadIdx.x; i < kSkBuckets; i += blockDim.x) k.cnt[i] = 0;
}

__global__ void k_sk_init(Dev d, SK k) {
    extern __shared__ int32_t hist[];   // [nbk]
    for (int b = threadIdx.x; b < k.nbk; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    int64_t alive = 0;
    const int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n; v += stride) {
        const int32_t dg = d.deg[v];
        k.C[v] = dg;
        k.r[v] = 0;
        k.est[v] = 0.0;
        int32_t b = -1;
        if (dg > 0) {
            b = sk_bucket(k, dg);
            atomicAdd(&hist[b], 1);
            alive++;
        }
        k.B[v] = b;
    }
    alive = wave_sum64(alive);
    if (threadIdx.x % kWave == 0 && alive) atomicAdd((unsigned long long *)&d.ctl->sk_alive, (unsigned long long)alive);
    sk_flush_hist(k, hist);
}

// The smallest non-empty bucket, or -1 (one block).
__device__ int32_t sk_min_bucket(const SK &k, int32_t *red) {
    int32_t best = INT32_MAX;
    for (int b = threadIdx.x; b < k.nbk; b += blockDim.x)
        if (k.cnt[b] > 0) best = min(best, b);
    for (int o = kWave / 2; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, kWave));
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = best;
    __syncthreads();
    int32_t r = INT32_MAX;
    for (int i = 0; i < (int)blockDim.x / kWave; i++) r = min(r, red[i]);
    __syncthreads();
    return r == INT32_MAX ? -1 : r;
}

// the first threshold (one block)
__global__ void k_sk_first(Dev d, SK k) {
    __shared__ int32_t red[kBlock / kWave];
    Ctl *c = d.ctl;
    const int32_t b = sk_min_bucket(k, red);
    if (threadIdx.x == 0) {
        c->sk_t = c->sk_bp = b;
        c->sk_peels = 0;
        c->sk_round = 0;
        c->sk_nT = 0;
        c->sk_ncl[0] = c->sk_ncl[1] = c->sk_ncl[2] = c->sk_ncl[3] = 0;
        c->sk_done = b < 0 ? 1 : 0;
    }
}

// Part 1 of a round: the alive vertices of bucket bp are peeled (estimate
// (1+eps)^bp) and listed; the previous round's peeled vertices become dead.
__global__ void k_sk_peel(Dev d, SK k) {
    __shared__ SlabQ q;
    const Ctl *c = d.ctl;
    if (c->sk_done) return;
    const int32_t bp = c->sk_bp;
    const double e = k.pw[bp];
    slabq_init(q);
    const int stride = gridDim.x * blockDim.x;
    for (int vb = blockIdx.x * blockDim.x; vb < d.n; vb += stride) {
        const int v = vb + threadIdx.x;
        int cls = -1;
        if (v < d.n) {
            const int32_t b = k.B[v];
            if (b == -2) k.B[v] = -1;
            if (b == bp) {
                k.B[v] = -2;
                k.est[v] = e;
                cls = slab_class(d.cap[v]);
            }
        }
        slabq_push(q, cls, v);
        slabq_flush(q, blockDim.x, k.Ilo, k.Ihi, d.ctl->sk_ncl, d.n, d.ctl);
    }
    slabq_flush(q, kSlabQ, k.Ilo, k.Ihi, d.ctl->sk_ncl, d.n, d.ctl);
}

// Part 2: every alive neighbour w of a peeled vertex counts its peeled
// neighbours in r[w]; the first count in the round lists w.  The peeled
// vertices' slabs are visited by slab class; touched vertices are staged per
// wavefront.
__global__ void __launch_bounds__(kBlock) k_sk_relax(Dev d, SK k) {
    __shared__ int32_t buf[kBlock / kWave][kFlipStage + kWave];
    const Ctl *c = d.ctl;
    if (c->sk_done) return;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int32_t *b = buf[wv];
    int32_t nb = 0;   // wave-uniform
    auto flush = [&]() {
        __threadfence_block();
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&d.ctl->sk_nT, nb);
        base = __shfl(base, 0, kWave);
        for (int i = lane; i < nb; i += kWave)
            if (base + i < d.n) k.T[base + i] = b[i];
        if (lane == 0 && base + nb > d.n) latch(d.ctl, kErrLevel);
        nb = 0;
    };
    auto slot = [&](int32_t, int2, int32_t w, int32_t bw) {
        const bool first = w >= 0 && bw >= 0 && atomicAdd(&k.r[w], 1) == 0;
        const uint64_t m = __ballot(first);
        if (first) b[nb + __popcll(m & ((1ull << lane) - 1))] = w;
        nb += __popcll(m);
        if (nb >= kFlipStage) flush();
    };
    const int32_t *B = k.B;
    visit_slabs(
        d, k.Ilo, k.Ihi, c->sk_ncl, [](int32_t) { return make_int2(0, 0); },
        [=](int32_t w) { return w >= 0 ? B[w] : -1; }, slot);
    if (nb) flush();
}

// Part 3: the touched vertices: C = max(C - r, ceil((1+eps)^(t-1))), r = 0, bucket
// max(b(C), t); bucket counts moved through an LDS histogram per block.
__global__ void k_sk_fix(Dev d, SK k) {
    extern __shared__ int32_t hist[];   // [nbk]
    const Ctl *c = d.ctl;
    if (c->sk_done) return;
    for (int b = threadIdx.x; b < k.nbk; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const int32_t t = c->sk_t, nt = min(c->sk_nT, d.n);
    const int32_t floor_t = t >= 1 ? (int32_t)ceil(k.pw[t - 1]) : 1;
    const int stride = gridDim.x * blockDim.x;
    int64_t relaxed = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += stride) {
        const int32_t w = k.T[i];
        const int32_t ob = k.B[w];
        const int32_t rw = k.r[w];
        const int32_t cw = max(k.C[w] - rw, floor_t);
        relaxed += rw;
        k.C[w] = cw;
        k.r[w] = 0;
        const int32_t nb = max(sk_bucket(k, cw), t);
        if (nb != ob) {
            k.B[w] = nb;
            atomicSub(&hist[ob], 1);
            atomicAdd(&hist[nb], 1);
        }
    }
    relaxed = wave_sum64(relaxed);
    if (threadIdx.x % kWave == 0 && relaxed)
        atomicAdd((unsigned long long *)&d.ctl->sk_relaxed, (unsigned long long)relaxed);
    sk_flush_hist(k, hist);
}

// Part 4 (one block): the round's bookkeeping and the next bucket to peel:
// the smallest non-empty one, in the same threshold while it is within
// (2+eps)(1+eps)^t and fewer than R peels were made at t, else as the next
// threshold.
__global__ void k_sk_next(Dev d, SK k) {
    __shared__ int32_t red[kBlock / kWave];
    Ctl *c = d.ctl;
    if (c->sk_done) return;
    const int32_t bp = c->sk_bp, t = c->sk_t;
    const int32_t ni = c->sk_ncl[0] + c->sk_ncl[1] + c->sk_ncl[2] + c->sk_ncl[3];
    __syncthreads();
    if (threadIdx.x == 0) k.cnt[bp] -= ni;   // the peeled vertices (vertices re-bucketed to bp stay)
    __syncthreads();
    const int32_t nb = sk_min_bucket(k, red);
    if (threadIdx.x == 0) {
        c->sk_alive -= ni;
        c->sk_peels += 1;
        c->sk_round += 1;
        c->sk_ncl[0] = c->sk_ncl[1] = c->sk_ncl[2] = c->sk_ncl[3] = 0;
        c->sk_nT = 0;
        if (nb < 0 || c->sk_alive <= 0) {
            c->sk_done = 1;
        } else if (c->sk_peels < k.R && k.pw[nb] <= (2.0 + k.eps) * k.pw[t]) {
            c->sk_bp = nb;
        } else {
            c->sk_t = c->sk_bp = nb;
            c->sk_peels = 0;
        }
    }
}

// ---- vertex updates (the section on vertex insertions and deletions).
// Degrees of the listed vertices, summed (ids out of range latch an error).
__global__ void k_vd_deg(Dev d, const int32_t *vs, int64_t cnt) {
    int64_t sum = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const int32_t v = vs[i];
        if (v < 0 || v >= d.n) {
            latch(d.ctl, kErrRange);
            continue;
        }
        sum += d.deg[v];
    }
    sum = wave_sum64(sum);
    if (threadIdx.x % kWave == 0 && sum) atomicAdd((unsigned long long *)&d.ctl->vd_deg, (unsigned long long)sum);
}

// The listed vertices by slab class (d.mv, d.mv1; counts vd_ncl), for a
// list of at most n entries (repeats included), so that two class lists
// sharing an array never meet.
__global__ void k_vd_classify(Dev d, const int32_t *vs, int64_t cnt) {
    __shared__ SlabQ q;
    slabq_init(q);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ib = (int64_t)blockIdx.x * blockDim.x; ib < cnt; ib += stride) {
        const int64_t i = ib + threadIdx.x;
        const int cls = i < cnt ? slab_class(d.cap[vs[i]]) : -1;
        slabq_push(q, cls, i < cnt ? vs[i] : -1);
        slabq_flush(q, blockDim.x, d.mv, d.mv1, d.ctl->vd_ncl, d.n, d.ctl);
    }
    slabq_flush(q, kSlabQ, d.mv, d.mv1, d.ctl->vd_ncl, d.n, d.ctl);
}

// Every edge of the listed vertices as a pair (v, w): the slabs are visited
// by slab class (classified lists) or a wavefront per vertex (`vs`, when the
// list is longer than n).  Each wavefront stages its pairs in LDS and appends
// them with one atomic per kVdStage; same-address atomics serialise, so the
// grid is kept to about a thousand wavefronts.
constexpr int kVdStage = 256;
constexpr int kVdGrid = 256;
__global__ void __launch_bounds__(kBlock) k_vd_gather(Dev d, const int32_t *vs, int64_t cnt, int32_t *out,
                                                      int64_t cap) {
    __shared__ int32_t buf[kBlock / kWave][2 * (kVdStage + kWave)];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int32_t *b = buf[wv];
    int32_t nb = 0;   // wave-uniform
    auto flush = [&]() {
        __threadfence_block();   // the wavefront's staged pairs are visible to all its lanes
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long *)&d.ctl->vd_n, (unsigned long long)nb);
        base = __shfl(base, 0, kWave);
        for (int i = lane; i < 2 * nb; i += kWave)
            if ((int64_t)base + i / 2 < cap) out[2 * base + i] = b[i];
        if (lane == 0 && (int64_t)base + nb > cap) latch(d.ctl, kErrLevel);
        nb = 0;
    };
    // one slot (w < 0: none) of v's slab; every lane of the wavefront calls it together
    auto slot = [&](int32_t v, int2, int32_t w, int32_t) {
        const uint64_t m = __ballot(w >= 0);
        if (w >= 0) {
            const int k = nb + __popcll(m & ((1ull << lane) - 1));
            b[2 * k] = v;
            b[2 * k + 1] = w;
        }
        nb += __popcll(m);
        if (nb >= kVdStage) flush();
    };
    if (!vs) {
        visit_slabs(
            d, d.mv, d.mv1, d.ctl->vd_ncl, [](int32_t) { return make_int2(0, 0); }, [](int32_t) { return 0; },
            slot);
    } else {
        const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
        for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < cnt; i += nw) {
            const int32_t v = vs[i];
            const int32_t cv = d.cap[v];
            const int32_t *sl = d.pool + d.off[v];
            for (int32_t e0 = 0; e0 < cv; e0 += kWave) {
                const int32_t e = e0 + lane;
                slot(v, make_int2(0, 0), e < cv ? sl[e] : -1, 0);
            }
        }
    }
    if (nb) flush();
}

// A rebuild's edge list through the renumbering: an edge with a dropped end
// (new id < 0) becomes the self-loop (0, 0), which the batch drops.
__global__ void k_relabel(int32_t *e, int64_t m, const int32_t *relabel) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
        const int32_t a = relabel[e[2 * i]], b = relabel[e[2 * i + 1]];
        const bool keep = a >= 0 && b >= 0;
        e[2 * i] = keep ? a : 0;
        e[2 * i + 1] = keep ? b : 0;
    }
}

__global__ void k_check(Dev d, int32_t *bad) {
    int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    int nw = gridDim.x * blockDim.x / kWave;
    for (int v = wid; v < d.n; v += nw) {
        int32_t lv = d.level[v], cap = d.cap[v];
        const int32_t *s = d.pool + d.off[v];
        int32_t cu = 0, cus = 0, live = 0;
        for (int32_t e = lane; e < cap; e += kWave) {
            int32_t w = s[e];
            if (w < 0) continue;
            int32_t lw = d.level[w];
            live++;
            cu += lw >= lv;
            cus += lw >= lv - 1;
        }
        cu = wave_sum(cu);
        cus = wave_sum(cus);
        live = wave_sum(live);
        if (lane == 0) {
            const GP p = gp(d, v);
            if (lv < 0 || lv >= (d.ng == 1 ? d.K : d.gK[d.gid[v]])) {
                atomicAdd(&bad[4], 1);
            } else {
                if (cu != d.up[v] || cus != d.ups[v]) atomicAdd(&bad[0], 1);
                if (cu > up_cap(d, p, lv)) atomicAdd(&bad[1], 1);
                if (lv > 0 && cus < dn_floor(d, p, lv)) atomicAdd(&bad[2], 1);
                if (d.deg[v] == 0 && lv != 0) atomicAdd(&bad[3], 1);
                if (live != d.deg[v]) atomicAdd(&bad[5], 1);
            }
        }
    }
}

__global__ void k_dump_edges(Dev d, int32_t *out, int64_t cap_out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // thread per slot of the whole used pool is not available; walk vertices
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < d.n; v += stride) {
        int32_t cap = d.cap[v];
        const int32_t *s = d.pool + d.off[v];
        for (int32_t e = 0; e < cap; e++) {
            int32_t w = s[e];
            if (w > (int32_t)v) {
                int64_t k = (int64_t)atomicAdd((unsigned long long *)&d.ctl->m_out, 1ull);
                if (k < cap_out) {
                    out[2 * k] = (int32_t)v;
                    out[2 * k + 1] = w;
                }
            }
        }
    }
}

// number of vertices per level
// Vertices per level into occ: a histogram per block in LDS (dynamic, K bins)
// when K <= kHistMax, flushed with one atomic per non-empty bin; else
// atomics aggregated per wavefront over equal levels.
__global__ void k_count_levels(Dev d, int32_t *occ) {
    extern __shared__ int32_t hist[];
    const int stride = gridDim.x * blockDim.x;
    const bool lds = d.K <= kHistMax;
    if (lds) {
        for (int i = threadIdx.x; i < d.K; i += blockDim.x) hist[i] = 0;
        __syncthreads();
    }
    for (int v0 = blockIdx.x * blockDim.x; v0 < d.n; v0 += stride) {   // wave-uniform
        const int v = v0 + threadIdx.x;
        const int32_t x = v < d.n ? d.level[v] : -1;
        const bool ok = x >= 0 && x < d.K;
        if (lds) {
            if (ok) atomicAdd(&hist[x], 1);
        } else {
            wave_add_key(occ, ok ? x : -1, 1);
        }
    }
    if (lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < d.K; i += blockDim.x)
            if (hist[i]) atomicAdd(&occ[i], hist[i]);
    }
}

__global__ void k_compare(const int32_t *a, const int32_t *b, int32_t cnt, int32_t *bad) {
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        if (a[i] != b[i]) atomicAdd(bad, 1);
}

// after a load: the endpoints' new edges into deg, counts cleared
__global__ void k_clear_touch(Dev d) {
    int32_t nt = d.ctl->n_touch;
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += stride) {
        int32_t x = d.touch[i];
        const int32_t k = d.addc[x];   // the endpoint's new edges
        d.deg[x] += k;
        d.fill[x] += k;
        d.addc[x] = 0;
    }
}

// Empty the vertex range [v0, v0+cnt) (one graph of a multi-graph handle):
// its vertices lose their slabs (the pool space is reclaimed by the next
// compaction) and go to level 0 (occupancy moved with one atomic per
// distinct level of a wavefront); their degrees are summed into m_out.
__global__ void k_reset_range(Dev d, int32_t v0, int32_t cnt) {
    const int lane = threadIdx.x % kWave;
    int64_t deg = 0, up0 = 0;
    const int stride = gridDim.x * blockDim.x;
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < cnt; i0 += stride) {
        const int i = i0 + lane;
        const int32_t v = i < cnt ? v0 + i : -1;
        const int32_t lv = v >= 0 ? d.level[v] : -1;
        wave_add_key(d.occ, lv > 0 ? lv : -1, -1);
        if (v < 0) continue;
        up0 += lv > 0;
        deg += d.deg[v];
        d.level[v] = 0;
        d.deg[v] = d.up[v] = d.ups[v] = 0;
        d.cap[v] = d.fill[v] = 0;
        d.off[v] = 0;
        d.addc[v] = d.stay[v] = d.cnt2[v] = 0;
        d.dl[v] = -1;
        if (d.prevlvl) d.prevlvl[v] = 0;
    }
    block_add64_to(deg, (unsigned long long *)&d.ctl->m_out);
    block_add64_to(up0, (unsigned long long *)&d.ctl->sum_up);
}

// Applied pairs of the list just applied (valid[0..n_valid)), per graph of
// a multi-graph handle, into gapp[which][g]: an LDS histogram per block
// when the graphs are few, else one atomic per distinct graph of a wavefront.
constexpr int kGraphHist = 8192;
__global__ void k_graph_count(Dev d, int which) {
    __shared__ int32_t hist[kGraphHist];
    const bool lds = d.ng <= kGraphHist;
    if (lds) {
        for (int i = threadIdx.x; i < d.ng; i += blockDim.x) hist[i] = 0;
        __syncthreads();
    }
    const int32_t nv = d.ctl->n_valid;
    unsigned long long *out = d.gapp + (size_t)which * d.ng;
    const int lane = threadIdx.x % kWave;
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < nv; i0 += gridDim.x * blockDim.x) {
        const int i = i0 + lane;
        const int32_t g = i < nv ? d.gid[d.valid[2 * i]] : -1;
        if (lds) {
            if (g >= 0) atomicAdd(&hist[g], 1);
        } else {
            uint64_t todo = __ballot(g >= 0);
            while (todo) {
                const int leader = __ffsll((unsigned long long)todo) - 1;
                const int32_t k = __shfl(g, leader, kWave);
                const uint64_t same = __ballot(g == k) & todo;
                if (lane == leader) atomicAdd(&out[k], (unsigned long long)__popcll(same));
                todo &= ~same;
            }
        }
    }
    if (lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < d.ng; i += blockDim.x)
            if (hist[i]) atomicAdd(&out[i], (unsigned long long)hist[i]);
    }
}

__global__ void k_set_levels(Dev d, const int32_t *lv) {
    int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n; v += stride) {
        int32_t x = lv[v];
        if (x < 0 || x >= d.K) latch(d.ctl, kErrLevel);
        d.level[v] = x;
    }
}

// pool compaction: new offsets by exclusive scan of capacities
__global__ void k_scan_tiles(const int32_t *in, int64_t n, int64_t *tile_sum) {
    __shared__ int64_t sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kBlock * 4;
    int64_t s = 0;
    for (int j = 0; j < 4; j++) {
        int64_t i = base + j * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = sh[0];
}
__global__ void k_scan_tile_prefix(int64_t *tile_sum, int64_t ntiles) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t acc = 0;
        for (int64_t i = 0; i < ntiles; i++) {
            int64_t x = tile_sum[i];
            tile_sum[i] = acc;
            acc += x;
        }
        tile_sum[ntiles] = acc;
    }
}
__global__ void k_scan_apply(const int32_t *in, int64_t n, const int64_t *tile_sum, int64_t *out) {
    if (threadIdx.x != 0) return;
    int64_t base = (int64_t)blockIdx.x * kBlock * 4;
    int64_t acc = tile_sum[blockIdx.x];
    for (int64_t i = base; i < std::min<int64_t>(n, base + kBlock * 4); i++) {
        out[i] = acc;
        acc += in[i];
    }
}
__global__ void k_compact_copy(Dev d, const int64_t *newoff, int32_t *newpool) {
    int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    int nw = gridDim.x * blockDim.x / kWave;
    for (int v = wid; v < d.n; v += nw) {
        int32_t cap = d.cap[v];
        const int32_t *s = d.pool + d.off[v];
        int32_t *t = newpool + newoff[v];
        for (int32_t e = lane; e < cap; e += kWave) t[e] = s[e];
    }
}
__global__ void k_set_offsets(Dev d, const int64_t *newoff) {
    int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n; v += stride) d.off[v] = newoff[v];
}

// One graph's edge list of a multi-graph batch: `cnt` pairs at `src` (ids
// local to the graph), written from pair `dst` on with the graph's first
// vertex `base` added.
struct Seg {
    const int32_t *src;
    int64_t cnt, dst;
    int32_t base, n;
};

// Gather the per-graph lists of a multi-graph batch into one list of global
// ids; an id outside [0, n) of its own graph latches kErrRange.
__global__ void k_stage(const Seg *segs, int32_t nseg, int64_t total, int32_t *out, Ctl *ctl) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += stride) {
        int32_t lo = 0, hi = nseg - 1;   // last segment with dst <= i
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) / 2;
            if (segs[mid].dst <= i) lo = mid;
            else hi = mid - 1;
        }
        const Seg sg = segs[lo];
        int64_t j = i - sg.dst;
        int32_t a = sg.src[2 * j], b = sg.src[2 * j + 1];
        if (a < 0 || a >= sg.n || b < 0 || b >= sg.n) latch(ctl, kErrRange);
        out[2 * i] = a + sg.base;
        out[2 * i + 1] = b + sg.base;
    }
}

}  // namespace

// ===================================================================== host
// Levels, groups and thresholds of one graph (Section "Detailed PLDS
// Algorithm"): t = least integer with (1+delta)^t >= n, L = 4t (or the
// override, at least 1; or the experiments' PLDSOpt ceil(t/50), which is
// ceil(log_{1+delta} n / 50)), G = t+1, K = G*L; up_max[g] = floor((2+3/lambda)
// x_g) and dn_min[g] = ceil(x_g) as exact integer rewrites of Invariants
// 1-2, where x_g = (1+delta)^g is formed by repeated IEEE double
// multiplication.  Entry G of up_max/dn_min is INT32_MAX.
struct Tables {
    int32_t t = 0, L = 0, G = 0, K = 0;
    std::vector<int32_t> up, dn;
    std::vector<double> pw;
};

static Tables make_tables(int64_t n, double delta, double lambda, int32_t lpg, double up_coeff) {
    Tables T;
    double p = 1.0;
    while (p < (double)n) {
        p *= 1.0 + delta;
        T.t++;
    }
    T.L = lpg > 0 ? lpg : lpg == PLDS_LPG_OPT ? std::max(1, (T.t + 49) / 50) : std::max(1, 4 * T.t);
    T.G = T.t + 1;
    T.K = T.G * T.L;
    T.up.assign(T.G + 1, INT32_MAX);
    T.dn.assign(T.G + 1, INT32_MAX);
    T.pw.assign(T.G + 1, 0.0);
    double coeff = up_coeff > 0 ? up_coeff : 2.0 + 3.0 / lambda, x = 1.0;
    for (int32_t g = 0; g < T.G; g++) {
        if (g > 0) x *= 1.0 + delta;
        T.pw[g] = x;
        double ub = std::floor(coeff * x), lb = std::ceil(x);
        T.up[g] = ub >= (double)INT32_MAX ? INT32_MAX : (int32_t)ub;
        T.dn[g] = lb >= (double)INT32_MAX ? INT32_MAX : (int32_t)lb;
    }
    return T;
}
// Scratch memory of the allocation-free entry points (callers that cannot
// allocate device memory): one array per device, held until the process
// ends.  Host code never passes `scratch` itself to a kernel (in host code
// the name is only a stand-in for the symbol); it uses the device address
// looked up once per device by scratch_lookup().
constexpr size_t kScratchPw = (size_t)kSkBuckets * sizeof(double);    // powers of 1+eps
constexpr size_t kScratchCnt = (size_t)kSkBuckets * sizeof(int32_t);  // bucket counts
constexpr size_t kScratchBytes = kScratchPw + kScratchCnt + (size_t)3 * PLDS_NOALLOC_MAX_N * sizeof(int32_t);
static __device__ __align__(256) int32_t scratch[kScratchBytes / sizeof(int32_t)];

struct plds {
    int64_t n = 0, m = 0;
    double delta = 0, lambda = 0;
    int32_t t = 0, L = 0, G = 0, K = 0;
    int device = 0;
    std::vector<int32_t> h_up_max, h_dn_min;   // concatenated per graph (stride G_g + 1)
    std::vector<double> h_pow;
    // graphs of a multi-graph handle (one entry for a plain handle)
    std::vector<Tables> gt;
    std::vector<int64_t> gbase, gn;           // first vertex and vertex count of each graph
    std::vector<int64_t> gcap;                // vertices of each graph's range (its n at create)
    std::vector<int32_t> gcapG;               // groups of each graph's table region (its G at create)
    std::vector<int32_t> gtab;
    int32_t *stage = nullptr;                 // gathered multi-graph batch
    int64_t stage_cap = 0;                    // pairs
    Seg *d_segs = nullptr, *h_segs = nullptr;
    Dev d{};
    int64_t batch_cap = 0;
    int64_t pool_top = 0;
    int64_t *tile = nullptr;
    int64_t tile_cap = 0;
    int64_t *newoff = nullptr;
    int32_t *bad = nullptr;
    Ctl *h_ctl = nullptr;   // pinned host mirror
    plds_stats_t stats{};
    int32_t latched = 0;
    bool broken = false;
    // the call's range checks were launched but not yet read back (the first
    // batch application's sync reads them, before the state changes)
    bool range_pending = false;
    // steps of the last insertion sweep: that many are issued before the
    // first wait for the sweep's end
    int64_t ins_steps_hint = 0;
    int64_t ins_trips_hint = 0;   // launches of the single-block loop the last sweep needed
    bool ins_loop_on = true;      // the next insertion sweep runs its small steps in the single-block loop
    bool climb_hint = true;       // the last insertion sweep decided a step that could climb
    // insertion sweep as one cooperative launch (0 blocks = not available)
    int sweep_mode = 1;          // 0: cooperative when possible, 1: one kernel per part
    int coop_blocks = -1;        // -1 = not yet determined
    int scan_grid = kSweepGrid;  // blocks of the insertion scan: what the device holds at once
    int scan_grid_def = kSweepGrid;   // the device default of scan_grid
    int graph_steps = kGraphStepsDef; // insertion steps per prebuilt step graph
    int dl_grid = kDlGrid;            // blocks of the desire-level kernels of deletions and jumps
    int del_scan_grid = kSweepGrid;   // blocks of the deletion and jump scans
    Bar *bar = nullptr;
    // the insertion step sequence as a prebuilt graph of graph_steps steps
    hipGraph_t ins_graph = nullptr;
    hipGraphExec_t ins_exec = nullptr;
    Dev ins_graph_dev{};
    // the deletion step sequence as a prebuilt graph of kDelGraphSteps steps
    hipGraph_t del_graph = nullptr;
    hipGraphExec_t del_exec = nullptr;
    Dev del_graph_dev{};
    int64_t del_steps_hint = 0;   // steps of the last deletion sweep run by the grid kernels
    // the rounds of the jump procedure as a prebuilt graph
    hipGraph_t jmp_graph = nullptr;
    hipGraphExec_t jmp_exec = nullptr;
    Dev jmp_graph_dev{};
    int64_t jmp_steps_hint = 0;
    int32_t dl_nbins = 0;         // bins argument of the step graph's large-slab desire-level kernel
    // orientation tracking: the last update call's starting levels and its
    // applied updates (pairs (min, max))
    int32_t lpg = 0;              // levels_per_group as given at create
    double up_coeff = 0;          // Invariant-1 coefficient given at create (0: 2 + 3/lambda)
    int32_t up_jump = 0;          // insertions move violators straight to their desire-level
    int32_t *vd_buf = nullptr;    // incident edges of deleted vertices
    int64_t vd_cap = 0;
    // static approximate k-core scratch (allocated on first use)
    int32_t *sk_C = nullptr, *sk_B = nullptr, *sk_r = nullptr, *sk_cnt = nullptr;
    double *sk_pw = nullptr;
    bool track = false;
    bool tracked_call = false;
    int32_t *t_ins = nullptr, *t_del = nullptr;
    int64_t t_ins_cap = 0, t_del_cap = 0, n_tins = 0, n_tdel = 0;
    int par[2] = {0, 1};
    // optional event timing of one sweep kernel
    int32_t timed_kind = 0;
    std::vector<hipEvent_t> ev;   // pairs (start, stop)
    int32_t ev_used = 0;
};

namespace {

#define HIPCHK(x)                      \
    do {                               \
        if ((x) != hipSuccess) {       \
            return PLDS_EHIP;          \
        }                              \
    } while (0)

// Device address of each device's scratch array, looked up once per device
// (with that device current) when a handle is created there.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

void scratch_lookup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[dev] = p;
    else (void)hipGetLastError();
}

void *scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

// Failure injection (plds_inject_alloc_failure): allocations left on this
// thread before one fails, -1 = off.
thread_local int64_t t_alloc_fail_after = -1;

template <class T>
int dalloc(T **p, int64_t count) {
    *p = nullptr;
    if (t_alloc_fail_after >= 0 && t_alloc_fail_after-- == 0) return PLDS_ENOMEM;
    if (count <= 0) count = 1;
    if (hipMalloc((void **)p, (size_t)count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return PLDS_ENOMEM;
    }
    return PLDS_OK;
}

template <class T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

int grid_for(int64_t work, int block = kBlock, int cap = 4096) {
    int64_t g = (work + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Vertices per level of the handle into occ (k_count_levels).
void count_levels(const plds *h, int32_t *occ, hipStream_t s) {
    const bool lds = h->K <= kHistMax;
    hipLaunchKernelGGL(k_count_levels, dim3(lds ? std::min(grid_for(h->n), 512) : grid_for(h->n)), dim3(kBlock),
                       lds ? (size_t)h->K * sizeof(int32_t) : 0, s, h->d, occ);
}

// Tables of every graph of the handle, concatenated; the handle's t, L, G,
// K are the largest over its graphs.
void build_tables(plds *h, int32_t lpg) {
    h->gt.clear();
    h->gtab.clear();
    h->h_up_max.clear();
    h->h_dn_min.clear();
    h->h_pow.clear();
    h->t = h->L = h->G = h->K = 0;
    for (size_t g = 0; g < h->gn.size(); g++) {
        Tables T = make_tables(h->gn[g], h->delta, h->lambda, lpg, h->up_coeff);
        h->gtab.push_back((int32_t)h->h_up_max.size());
        h->h_up_max.insert(h->h_up_max.end(), T.up.begin(), T.up.end());
        h->h_dn_min.insert(h->h_dn_min.end(), T.dn.begin(), T.dn.end());
        h->h_pow.insert(h->h_pow.end(), T.pw.begin(), T.pw.end());
        h->t = std::max(h->t, T.t);
        h->L = std::max(h->L, T.L);
        h->G = std::max(h->G, T.G);
        h->K = std::max(h->K, T.K);
        h->gt.push_back(std::move(T));
    }
}

// Destroys the prebuilt step graphs; the next sweep rebuilds them.
void drop_graphs(plds *h) {
    if (h->ins_exec) (void)hipGraphExecDestroy(h->ins_exec);
    if (h->ins_graph) (void)hipGraphDestroy(h->ins_graph);
    h->ins_exec = nullptr;
    h->ins_graph = nullptr;
    if (h->del_exec) (void)hipGraphExecDestroy(h->del_exec);
    if (h->del_graph) (void)hipGraphDestroy(h->del_graph);
    h->del_exec = nullptr;
    h->del_graph = nullptr;
    if (h->jmp_exec) (void)hipGraphExecDestroy(h->jmp_exec);
    if (h->jmp_graph) (void)hipGraphDestroy(h->jmp_graph);
    h->jmp_exec = nullptr;
    h->jmp_graph = nullptr;
}

void free_all(plds *h) {
    Dev &d = h->d;
    dfree(d.up_max), dfree(d.dn_min), dfree(d.pow_tab);
    dfree(d.gid), dfree(d.gL), dfree(d.gK), dfree(d.gtab), dfree(d.Ls), dfree(d.gapp);
    dfree(h->stage), dfree(h->d_segs);
    if (h->h_segs) (void)hipHostFree(h->h_segs);
    h->h_segs = nullptr;
    dfree(d.level), dfree(d.deg), dfree(d.up), dfree(d.ups), dfree(d.cap), dfree(d.fill), dfree(d.off);
    dfree(d.pool), dfree(d.stay), dfree(d.cnt2), dfree(d.addc), dfree(d.dl), dfree(d.rcstamp), dfree(d.ctl);
    dfree(d.hset), dfree(d.valid), dfree(d.touch), dfree(d.grow), dfree(d.newcap), dfree(d.oldoff),
        dfree(d.oldcap);
    dfree(d.cand), dfree(d.sorted), dfree(d.lvl_cnt), dfree(d.lvl_start), dfree(d.next_nz), dfree(d.occ), dfree(d.lvl_fill), dfree(d.steplog), dfree(d.part);
    for (int k = 0; k < 4; k++) dfree(d.cls[k]);
    dfree(d.casc0), dfree(d.casc1), dfree(d.mv), dfree(d.mv1), dfree(d.sp), dfree(d.chunks), dfree(d.p0), dfree(d.p1), dfree(d.rc);
    dfree(d.lvb_start), dfree(d.lvb_fill), dfree(d.lvb), dfree(d.cl), dfree(d.sl0), dfree(d.sl1), dfree(d.cw);
    dfree(h->tile), dfree(h->newoff), dfree(h->bad), dfree(h->bar);
    dfree(d.prevlvl), dfree(d.lvp), dfree(h->t_ins), dfree(h->t_del);
    dfree(h->sk_C), dfree(h->sk_B), dfree(h->sk_r), dfree(h->sk_cnt), dfree(h->sk_pw);
    dfree(h->vd_buf);
    drop_graphs(h);
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    h->ev.clear();
    if (h->h_ctl) (void)hipHostFree(h->h_ctl);
    h->h_ctl = nullptr;
}

hipStream_t S(void *s) { return (hipStream_t)s; }

constexpr int kEvPairs = 512;

// record the start event of a timed launch of `kind` (no-op otherwise);
// for launches that hipExtLaunchKernel cannot make (cooperative ones)
inline void tstart(plds *h, int kind, hipStream_t s) {
    if (h->timed_kind != kind || h->ev_used >= kEvPairs) return;
    (void)hipEventRecord(h->ev[2 * h->ev_used], s);
}
inline void tstop(plds *h, int kind, hipStream_t s) {
    if (h->timed_kind != kind || h->ev_used >= kEvPairs) return;
    (void)hipEventRecord(h->ev[2 * h->ev_used + 1], s);
    h->ev_used++;
}

// Launch a kernel; when it is the timed kind, with an event pair that the
// runtime stamps at the dispatch's own start and end (no queue gap inside).
template <class F, class... A>
inline void tlaunch(plds *h, int kind, F f, dim3 grid, dim3 block, size_t lds, hipStream_t s, A... a) {
    if (h->timed_kind == kind && h->ev_used < kEvPairs) {
        hipExtLaunchKernelGGL(f, grid, block, (uint32_t)lds, s, h->ev[2 * h->ev_used], h->ev[2 * h->ev_used + 1], 0,
                              a...);
        h->ev_used++;
    } else {
        hipLaunchKernelGGL(f, grid, block, lds, s, a...);
    }
}

// Add the durations of the first `count` recorded launches (the ones that
// did work) to the statistics and free the event pairs.  After sync only.
void take_timing(plds *h, int count) {
    for (int i = 0; i < std::min(count, h->ev_used); i++) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) == hipSuccess) {
            h->stats.timed_ms += ms;
            h->stats.timed_launches++;
        }
    }
    h->ev_used = 0;
}

int sync_ctl(plds *h, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(h->h_ctl, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->stats.host_syncs++;
    return PLDS_OK;
}

int ensure_batch(plds *h, int64_t count) {
    if (count <= h->batch_cap) return PLDS_OK;
    int64_t cap = std::max<int64_t>(count, 1024);
    Dev &d = h->d;
    dfree(d.hset), dfree(d.valid);
    uint64_t hs = 1;
    while (hs < (uint64_t)(2 * cap)) hs <<= 1;
    int rc = dalloc(&d.hset, (int64_t)hs);
    if (!rc) rc = dalloc(&d.valid, 2 * cap);
    if (rc) {
        dfree(d.hset), dfree(d.valid);
        h->batch_cap = 0;
        return rc;
    }
    d.hmask = hs - 1;
    h->batch_cap = cap;
    return PLDS_OK;
}

int ensure_chunks(plds *h) {
    // one descriptor per kChunk (kCw) slots of any slab plus one per vertex
    int64_t need = h->n + h->d.pool_cap / kChunk + 1;
    if (need > h->d.chunk_cap) {
        dfree(h->d.chunks);
        int rc = dalloc(&h->d.chunks, need);
        h->d.chunk_cap = rc ? 0 : need;
        if (rc) return rc;
    }
    need = h->n + h->d.pool_cap / kCw + 1;
    if (need > h->d.cw_cap) {
        dfree(h->d.cw);
        int rc = dalloc(&h->d.cw, need);
        h->d.cw_cap = rc ? 0 : need;
        if (rc) return rc;
    }
    return PLDS_OK;
}

// exclusive scan of d.cap into newoff (int64), returns the total
int scan_caps(plds *h, hipStream_t s, int64_t *total) {
    int64_t n = h->n, ntiles = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (ntiles + 1 > h->tile_cap) {
        dfree(h->tile);
        if (dalloc(&h->tile, ntiles + 1)) return PLDS_ENOMEM;
        h->tile_cap = ntiles + 1;
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, s, h->d.cap, n, h->tile);
    hipLaunchKernelGGL(k_scan_tile_prefix, dim3(1), dim3(64), 0, s, h->tile, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(64), 0, s, h->d.cap, n, h->tile, h->newoff);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(total, h->tile + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PLDS_OK;
}

// Make room for `extra` more pool slots: compact live slabs into a new pool
// sized for the live total plus `extra`, with headroom.
int ensure_pool(plds *h, hipStream_t s, int64_t extra) {
    if (h->pool_top + extra <= h->d.pool_cap) return PLDS_OK;
    int64_t live = 0;
    int rc = scan_caps(h, s, &live);
    if (rc) return rc;
    int64_t want = std::max<int64_t>((live + extra) * 3 / 2, h->d.pool_cap);
    want = std::max<int64_t>(want, live + extra + (1 << 20));
    int32_t *np = nullptr;
    if (dalloc(&np, want)) return PLDS_ENOMEM;
    hipLaunchKernelGGL(k_compact_copy, dim3(grid_for(h->n * kWave)), dim3(kBlock), 0, s, h->d, h->newoff, np);
    hipLaunchKernelGGL(k_set_offsets, dim3(grid_for(h->n)), dim3(kBlock), 0, s, h->d, h->newoff);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    dfree(h->d.pool);
    h->d.pool = np;
    h->d.pool_cap = want;
    h->pool_top = live;
    h->h_ctl->pool_top = live;
    HIPCHK(hipMemcpyAsync(&h->d.ctl->pool_top, &h->h_ctl->pool_top, sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return ensure_chunks(h);
}

// reset the per-call fields of the control block (host mirror -> device)
int ctl_reset_batch(plds *h, hipStream_t s) {
    Ctl *c = h->h_ctl;
    c->n_valid = c->n_touch = c->n_grow = c->n_cand = c->n_pieces = 0;
    c->grow_req = 0;
    c->l = 0;
    c->done = 0;
    c->cur = 0;
    c->n_mv = 0;
    c->casc_n[0] = c->casc_n[1] = 0;
    c->p_n[0] = c->p_n[1] = 0;
    c->n_chunks = c->n_rc = 0;
    c->n_cls[0] = c->n_cls[1] = c->n_cls[2] = c->n_cls[3] = 0;
    for (int q = 0; q < 2; q++) {
        c->n_chunks2[q] = 0;
        c->n_cls2[q][0] = c->n_cls2[q][1] = c->n_cls2[q][2] = c->n_cls2[q][3] = 0;
    }
    c->nm = kInf;
    c->blocks_done = 0;
    c->nmove[0] = c->nmove[1] = 0;
    c->n_cl = 0;
    c->n_sl[0] = c->n_sl[1] = 0;
    c->n_cw[0] = c->n_cw[1] = 0;
    c->step_dec[0] = c->step_dec[1] = 0;
    c->del_big = 0;
    c->n_big = 0;
    c->big_steps = 0;
    c->sum_up = 0;
    c->sweeps = c->moves = c->scanned = c->dl_calcs = 0;
    c->alg_U = c->alg_up1 = 0;
    c->top = 0;
    c->m_out = 0;
    c->pool_top = h->pool_top;
    // everything but err, which may hold the call's range-check result
    const size_t e0 = offsetof(Ctl, err), e1 = e0 + sizeof(c->err);
    HIPCHK(hipMemcpyAsync(h->d.ctl, c, e0, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((char *)h->d.ctl + e1, (const char *)c + e1, sizeof(Ctl) - e1, hipMemcpyHostToDevice, s));
    return PLDS_OK;
}

int check_err(plds *h) {
    int32_t e = h->h_ctl->err;
    if (e & (kErrFull | kErrLevel | kErrOrder | kErrHang)) {
        h->broken = true;
        return PLDS_ESTATE;
    }
    if (e & kErrPool) {
        h->broken = true;
        return PLDS_ENOMEM;
    }
    return PLDS_OK;
}

// Orientation tracking: keep a copy of the call's applied list (pairs
// (min, max)) for plds_oriented_updates and plds_flips.
int track_list(plds *h, int insert, int64_t applied, hipStream_t s) {
    int32_t *&buf = insert ? h->t_ins : h->t_del;
    int64_t &cap = insert ? h->t_ins_cap : h->t_del_cap;
    if (applied > cap) {
        dfree(buf);
        cap = 0;
        if (dalloc(&buf, 2 * applied)) return PLDS_ENOMEM;
        cap = applied;
    }
    if (applied)
        HIPCHK(hipMemcpyAsync(buf, h->d.valid, (size_t)applied * 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    (insert ? h->n_tins : h->n_tdel) = applied;
    return PLDS_OK;
}

// Preprocess one list and apply it to the slabs.  insert=1: keep absent
// pairs, regrow slabs, insert; insert=0: keep present pairs, delete.
// On return the touched endpoints are in d.touch (count in ctl).
int apply_list(plds *h, const int32_t *e, int64_t cnt, int insert, hipStream_t s, int64_t *applied) {
    Dev &d = h->d;
    *applied = 0;
    int rc = ensure_batch(h, cnt);
    if (rc) return rc;
    rc = ctl_reset_batch(h, s);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(d.hset, 0xff, (size_t)(d.hmask + 1) * sizeof(uint64_t), s));
    hipLaunchKernelGGL(k_dedupe, dim3(grid_for(cnt, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d, e, cnt,
                       insert ? 0 : 1);
    if (insert)
        hipLaunchKernelGGL(k_plan_growth, dim3(grid_for(2 * cnt, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d);
    HIPCHK(hipGetLastError());
    rc = sync_ctl(h, s);
    if (rc) return rc;
    if (h->range_pending) {
        h->range_pending = false;
        if (h->h_ctl->err & kErrRange) {
            // nothing is applied yet: only the endpoint counts of this list are undone
            h->h_ctl->err = 0;
            HIPCHK(hipMemsetAsync(d.addc, 0, (size_t)h->n * sizeof(int32_t), s));
            HIPCHK(hipMemcpyAsync(&d.ctl->err, &h->h_ctl->err, sizeof(int32_t), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            return PLDS_ERANGE;
        }
    }
    *applied = h->h_ctl->n_valid;
    if (d.ng > 1 && *applied)
        hipLaunchKernelGGL(k_graph_count, dim3(grid_for(*applied, kBlock, 256)), dim3(kBlock), 0, s, d, insert ? 0 : 1);
    // From here on the dedupe pass has counted this list's edges per
    // endpoint (addc) and listed the endpoints: a failure leaves the handle
    // unusable rather than half-applied.
    if (h->track) {
        rc = track_list(h, insert, *applied, s);
        if (rc) {
            h->broken = true;
            return rc;
        }
    }
    if (insert) {
        if (h->h_ctl->n_grow > 0) {
            int64_t req = h->h_ctl->grow_req;
            rc = ensure_pool(h, s, req);
            if (rc) {
                h->broken = true;
                return rc;
            }
            HIPCHK(hipMemsetAsync(d.pool + h->pool_top, 0xff, (size_t)req * sizeof(int32_t), s));
            hipLaunchKernelGGL(k_grow_alloc, dim3(grid_for(h->h_ctl->n_grow)), dim3(kBlock), 0, s, d);
            // a wavefront per slab (at least 256 blocks, for the pieces of large slabs)
            int gm = std::max(grid_for((int64_t)h->h_ctl->n_grow * kWave, kBlock, 2048), 256);
            hipLaunchKernelGGL(k_grow_move, dim3(gm), dim3(kBlock), 0, s, d);
            h->pool_top += req;
        }
        hipLaunchKernelGGL(k_apply_ins, dim3(grid_for(*applied)), dim3(kBlock), 0, s, d);
    } else {
        tlaunch(h, 8, k_apply_del, dim3(grid_for(*applied)), dim3(kBlock), 0, s, d);
    }
    HIPCHK(hipGetLastError());
    h->m += insert ? *applied : -*applied;
    return PLDS_OK;
}

// The insertion step sequence (prep, scan) x graph_steps as one graph of
// kernel nodes, each pair preceded by the single-block loop when it runs the
// small steps (then a pair runs only a step the loop leaves); rebuilt when
// the device buffers move.
int ins_graph(plds *h) {
    if (h->ins_exec && !memcmp(&h->ins_graph_dev, &h->d, sizeof(Dev))) return 0;
    if (h->ins_exec) (void)hipGraphExecDestroy(h->ins_exec);
    if (h->ins_graph) (void)hipGraphDestroy(h->ins_graph);
    h->ins_exec = nullptr;
    h->ins_graph = nullptr;
    h->ins_graph_dev = h->d;
    if (hipGraphCreate(&h->ins_graph, 0) != hipSuccess) return PLDS_EHIP;
    Dev *dv = &h->ins_graph_dev;
    void *a0[] = {(void *)dv, (void *)&h->par[0]};
    void *a1[] = {(void *)dv, (void *)&h->par[1]};
    struct K {
        const void *f;
        int grid, block;
    } ks[3] = {{(const void *)k_ins_loop, 1, kLoopBlock},
               {(const void *)k_ins_prep, kListGrid, kBlock},
               {(const void *)k_ins_scan, h->scan_grid, kBlock}};
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < h->graph_steps; i++) {
        for (int k = h->d.ins_loop ? 0 : 1; k < 3; k++) {
            hipGraphNode_t node;
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(ks[k].f);
            p.gridDim = dim3(ks[k].grid);
            p.blockDim = dim3(ks[k].block);
            p.sharedMemBytes = 0;
            p.kernelParams = (i & 1) ? a1 : a0;   // (the loop takes the Dev alone)
            p.extra = nullptr;
            if (hipGraphAddKernelNode(&node, h->ins_graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
                return PLDS_EHIP;
            prev = node;
        }
    }
    {   // the sweep's totals of the scan statistics, recomputed at the end of every graph, so
        // that they are ready when the host sees the sweep done
        hipGraphNode_t node;
        hipKernelNodeParams p{};
        void *at[] = {(void *)dv, (void *)&h->scan_grid};
        p.func = (void *)k_ins_totals;
        p.gridDim = dim3(1);
        p.blockDim = dim3(kBlock);
        p.sharedMemBytes = 0;
        p.kernelParams = at;
        p.extra = nullptr;
        if (hipGraphAddKernelNode(&node, h->ins_graph, &prev, 1, &p) != hipSuccess) return PLDS_EHIP;
    }
    if (hipGraphInstantiate(&h->ins_exec, h->ins_graph, nullptr, nullptr, 0) != hipSuccess) return PLDS_EHIP;
    return 0;
}

constexpr int kDelGraphSteps = 4;

// bins of the large-slab desire-level histogram: one per level when the
// handle has at most kHistMax levels
int32_t dl_bins(const plds *h) { return std::max<int32_t>(std::min<int32_t>(h->K, kHistMax), 64); }

// The deletion steps too large for the single-block loop, as one graph of
// kernel nodes: (select, scan, fin, desire-levels (two phases), next, loop) x
// kDelGraphSteps; rebuilt when the device buffers move.
int del_graph(plds *h) {
    if (h->del_exec && !memcmp(&h->del_graph_dev, &h->d, sizeof(Dev))) return 0;
    if (h->del_exec) (void)hipGraphExecDestroy(h->del_exec);
    if (h->del_graph) (void)hipGraphDestroy(h->del_graph);
    h->del_exec = nullptr;
    h->del_graph = nullptr;
    h->del_graph_dev = h->d;
    if (hipGraphCreate(&h->del_graph, 0) != hipSuccess) return PLDS_EHIP;
    Dev *dv = &h->del_graph_dev;
    void *a0[] = {(void *)dv};
    void *a1[] = {(void *)dv, (void *)&h->par[1]};                          // mode 1
    h->dl_nbins = dl_bins(h);
    void *ab[] = {(void *)dv, (void *)&h->par[1], (void *)&h->dl_nbins};   // mode 1, bins
    const unsigned blds = (unsigned)h->dl_nbins * sizeof(int32_t);
    struct K {
        const void *f;
        int grid, block;
        unsigned lds;
        void **args;
    } ks[7] = {{(const void *)k_del_select, kSweepGrid / 4, kBlock, 0, a0},
               {(const void *)k_del_scan, h->del_scan_grid, kBlock, 0, a0},
               {(const void *)k_del_fin, kSweepGrid / 4, kBlock, 0, a0},
               {(const void *)k_dl, h->dl_grid, kBlock, 0, a1},
               {(const void *)k_dl_big, kBigGrid, kBigBlock, blds, ab},
               {(const void *)k_del_next, 1, 1, 0, a1},
               {(const void *)k_del_loop, 1, kLoopBlock, 0, a0}};
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < kDelGraphSteps; i++) {
        for (int k = 0; k < 7; k++) {
            hipGraphNode_t node;
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(ks[k].f);
            p.gridDim = dim3(ks[k].grid);
            p.blockDim = dim3(ks[k].block);
            p.sharedMemBytes = ks[k].lds;
            p.kernelParams = ks[k].args;
            p.extra = nullptr;
            if (hipGraphAddKernelNode(&node, h->del_graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
                return PLDS_EHIP;
            prev = node;
        }
    }
    if (hipGraphInstantiate(&h->del_exec, h->del_graph, nullptr, nullptr, 0) != hipSuccess) return PLDS_EHIP;
    return 0;
}

// Blocks of the cooperative sweep: up to 4 resident blocks per compute unit
// (fewer if the occupancy calculator says so), at most kSweepGrid.
int coop_blocks(plds *h) {
    if (h->coop_blocks >= 0) return h->coop_blocks;
    h->coop_blocks = 0;
    int coop = 0, ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->device) != hipSuccess || !coop)
        return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || ncu <= 0)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_ins_sweep, kBlock, 0) != hipSuccess ||
        per <= 0)
        return 0;
    if (!h->bar && dalloc(&h->bar, 1)) return 0;
    h->coop_blocks = std::min(std::min(per, 4) * ncu, kSweepGrid);
    return h->coop_blocks;
}

// Algorithm 2 after the edges are in: seed, bucket by level, then run the
// level loop: one cooperative launch, or (fallback) one kernel per part in
// growing runs until the control block reports done.
int insertion_sweep(plds *h, hipStream_t s) {
    Dev &d = h->d;
    int nt = h->h_ctl->n_touch;
    // climbing steps: per-part kernels, level histograms in LDS, and a batch
    // with enough touched endpoints that a step could have kClimbMin movers,
    // after a sweep that had such a step (mode 3: always); otherwise the
    // sweep skips the O(n) resident buckets they need (climbing is exact,
    // so results do not depend on it)
    d.climb_ok = (h->sweep_mode == 1 || h->sweep_mode == 3) && h->K <= kHistMax &&
                 (h->sweep_mode == 3 || (nt >= kClimbMin && h->climb_hint)) ? 1 : 0;
    d.climb_min = h->sweep_mode == 3 ? 1 : kClimbMin;
    // small steps in the single-block loop: per-part kernels (mode 2 sends
    // every step to them), when most steps of the last sweep were small
    d.ins_loop = (h->sweep_mode == 1 || h->sweep_mode == 3) && h->ins_loop_on ? 1 : 0;
    HIPCHK(hipMemsetAsync(d.lvl_cnt, 0, (size_t)(h->K + 1) * sizeof(int32_t), s));
    size_t hist = (size_t)(h->K <= kHistMax ? h->K : 0) * sizeof(int32_t);
    hipLaunchKernelGGL(k_ins_seed, dim3(grid_for(nt, kBlock, kApplyGrid)), dim3(kBlock), hist, s, d);
    hipLaunchKernelGGL(k_level_scan, dim3(1), dim3(1024), 0, s, d);
    hipLaunchKernelGGL(k_level_scatter, dim3(grid_for(nt, kBlock, kApplyGrid)), dim3(kBlock), hist, s, d);
    HIPCHK(hipGetLastError());
    // After a sweep of many steps the next one is expected to have
    // candidates too: the buckets and the first step graphs follow the
    // seeding without a wait (the steps of a sweep without candidates return
    // at once).  Otherwise, and for the cooperative or timed forms, wait.
    const bool eager = h->sweep_mode != 0 && h->sweep_mode != 4 && h->timed_kind != 1 && h->timed_kind != 4 &&
                       h->timed_kind != 11 && h->ins_steps_hint >= 32;
    int rc = PLDS_OK;
    if (!eager) {
        rc = sync_ctl(h, s);
        if (rc) return rc;
    }
    HIPCHK(hipMemsetAsync(d.part, 0, 3 * kSweepGrid * sizeof(int64_t), s));
    if (d.climb_ok && (eager || !h->h_ctl->done)) {
        HIPCHK(hipMemsetAsync(d.lvb_fill, 0, (size_t)(h->K + 2) * sizeof(int32_t), s));
        size_t lds = (size_t)h->K * sizeof(int32_t);
        hipLaunchKernelGGL(k_bucket_count, dim3(grid_for(h->n, kBlock, kApplyGrid)), dim3(kBlock), lds, s, d);
        hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, d);
        hipLaunchKernelGGL(k_bucket_scatter, dim3(grid_for(h->n, kBlock, kApplyGrid)), dim3(kBlock), lds, s, d);
        HIPCHK(hipGetLastError());
    }
    if (!h->h_ctl->done && (h->sweep_mode == 0 || h->sweep_mode == 4) && coop_blocks(h) > 0) {
        HIPCHK(hipMemsetAsync(h->bar, 0, sizeof(Bar), s));
        if (h->sweep_mode == 4) {   // every block leaves at its first barrier
            static const int one = 1;
            HIPCHK(hipMemcpyAsync(&h->bar->abort, &one, sizeof(int), hipMemcpyHostToDevice, s));
        }
        Bar *bar = h->bar;
        void *args[] = {(void *)&d, (void *)&bar};
        tstart(h, 6, s);
        hipError_t e = hipLaunchCooperativeKernel((const void *)k_ins_sweep, dim3(h->coop_blocks), dim3(kBlock), args,
                                                  0, s);
        tstop(h, 6, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->coop_blocks = 0;          // use the per-part kernels from now on
        } else {
            rc = sync_ctl(h, s);
            if (rc) return rc;
            take_timing(h, 1);
        }
    }
    int64_t steps = 0;
    bool totals = false;
    // a timed step kernel is launched directly, so that its events bracket the dispatch alone
    bool use_graph = h->timed_kind != 1 && h->timed_kind != 4 && h->timed_kind != 11;
    // launched one by one: a first run of 7/8 of the steps the last sweep
    // took (even, so that every run starts at parity 0), then runs of 16,
    // 32, ... (a step launched after the sweep's end still costs its launches
    // on the host)
    // with the single-block loop, a step slot of the sequence is (loop,
    // prep, scan), and the sweep needs about as many slots as the loop's
    // launches that found it running
    const int64_t hint = d.ins_loop ? h->ins_trips_hint : h->ins_steps_hint;
    int run = use_graph ? h->graph_steps : (int)std::min<int64_t>(std::max<int64_t>((hint * 7 / 8) & ~1LL, 8), 256);
    int next_run = 16;
    // before the first wait, issue about as many steps as the last sweep
    // took (rounded down to whole step graphs); steps issued after the
    // sweep's end return at once
    int64_t first = std::min<int64_t>(std::max<int64_t>(hint / h->graph_steps, 1), 8);
    while (!h->h_ctl->done && !h->h_ctl->err) {
        if (steps > 2 * (int64_t)h->K + 2) {   // a level gets at most an exit step and a moving step
            h->broken = true;
            return PLDS_ESTATE;
        }
        if (use_graph) {
            rc = ins_graph(h);
            if (rc) return rc;
            for (int64_t i = 0; i < first; i++) HIPCHK(hipGraphLaunch(h->ins_exec, s));
            steps += first * h->graph_steps;
            first = 1;
        } else {
            steps += run;
            for (int i = 0; i < run; i++) {      // run is even: every run starts at parity 0
                int par = i & 1;
                if (d.ins_loop) tlaunch(h, 11, k_ins_loop, dim3(1), dim3(kLoopBlock), 0, s, d);
                tlaunch(h, 4, k_ins_prep, dim3(kListGrid), dim3(kBlock), 0, s, d, par);
                tlaunch(h, 1, k_ins_scan, dim3(h->scan_grid), dim3(kBlock), 0, s, d, par);
            }
            run = next_run;
            next_run = std::min(next_run * 2, 256);
            hipLaunchKernelGGL(k_ins_totals, dim3(1), dim3(kBlock), 0, s, d, h->scan_grid);
        }
        HIPCHK(hipGetLastError());
        rc = sync_ctl(h, s);
        if (rc) return rc;
        take_timing(h, h->ev_used);
        totals = true;   // each run of steps ends with the totals (the graph's last node)
    }
    if (!totals) {   // no step run by this loop (none needed, or the cooperative sweep ran them)
        hipLaunchKernelGGL(k_ins_totals, dim3(1), dim3(kBlock), 0, s, d, h->scan_grid);
        HIPCHK(hipGetLastError());
        rc = sync_ctl(h, s);
        if (rc) return rc;
    }
    // up* of the climbers that stopped; nothing the host reads depends on it
    if (h->h_ctl->n_rc > 0)
        hipLaunchKernelGGL(k_ups_recount, dim3(grid_for((int64_t)h->h_ctl->n_rc * kWave, kBlock, 2048)),
                           dim3(kBlock), 0, s, d);
    HIPCHK(hipGetLastError());
    Ctl *c = h->h_ctl;
    h->stats.viol_ins0 = c->n_cand;
    h->ins_steps_hint = c->n_steps + 1;   // the steps and the one that found the sweep done
    h->ins_trips_hint = c->ins_trips + 1;
    h->climb_hint = c->n_climbable > 0 || c->n_steps == 0;
    // the loop pays off when most steps are small (it decides a large step
    // before leaving it to the step kernels, and costs a launch per step
    // slot): on when at least 4/5 of the step kernels' steps had few movers
    // (the loop would also need their slabs to be small), off again when it
    // ran less than half of the steps
    if (c->n_steps > 0)
        h->ins_loop_on = d.ins_loop ? 2 * c->lp_steps >= c->n_steps : 5 * (int64_t)c->n_small >= 4 * (int64_t)c->n_steps;
    h->stats.sweeps_ins += c->sweeps;
    h->stats.moves_up += c->moves;
    h->stats.alg_bytes_up += 8 * (c->alg_U + c->alg_up1) + 4 * c->moves;
    h->stats.alg_bytes_up_loop += 8 * (c->lp_U + c->lp_up1) + 4 * c->lp_moves;
    h->stats.ins_steps += c->n_steps;
    h->stats.ins_loop_steps += c->lp_steps;
    h->stats.ins_loop_launches += c->ins_trips;
    h->stats.slots_scanned += c->scanned;
    h->stats.top_level = std::max(h->stats.top_level, c->top);
    return check_err(h);
}

constexpr int kJmpGraphSteps = 4;

// Rounds of the jump procedure as one graph of kernel nodes: (select,
// desire-levels (two kernels), scan, fin, next) x kJmpGraphSteps; rebuilt
// when the device buffers move.
int jmp_graph(plds *h) {
    if (h->jmp_exec && !memcmp(&h->jmp_graph_dev, &h->d, sizeof(Dev))) return 0;
    if (h->jmp_exec) (void)hipGraphExecDestroy(h->jmp_exec);
    if (h->jmp_graph) (void)hipGraphDestroy(h->jmp_graph);
    h->jmp_exec = nullptr;
    h->jmp_graph = nullptr;
    h->jmp_graph_dev = h->d;
    if (hipGraphCreate(&h->jmp_graph, 0) != hipSuccess) return PLDS_EHIP;
    Dev *dv = &h->jmp_graph_dev;
    h->dl_nbins = dl_bins(h);
    void *a0[] = {(void *)dv};
    void *a1[] = {(void *)dv, (void *)&h->par[1]};
    void *ab[] = {(void *)dv, (void *)&h->dl_nbins};
    const unsigned blds = (unsigned)h->dl_nbins * sizeof(int32_t);
    struct K {
        const void *f;
        int grid, block;
        unsigned lds;
        void **args;
    } ks[6] = {{(const void *)k_jmp_select, kSweepGrid / 4, kBlock, 0, a0},
               {(const void *)k_jmp_dl, h->dl_grid, kBlock, 0, a0},
               {(const void *)k_jmp_dl_big, kJmpBigGrid, kBigBlock, blds, ab},
               {(const void *)k_jmp_scan, h->del_scan_grid, kBlock, 0, a0},
               {(const void *)k_jmp_fin, kSweepGrid / 4, kBlock, 0, a0},
               {(const void *)k_jmp_next, 1, 1, 0, a1}};
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < kJmpGraphSteps; i++) {
        for (int k = 0; k < 6; k++) {
            hipGraphNode_t node;
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(ks[k].f);
            p.gridDim = dim3(ks[k].grid);
            p.blockDim = dim3(ks[k].block);
            p.sharedMemBytes = ks[k].lds;
            p.kernelParams = ks[k].args;
            p.extra = nullptr;
            if (hipGraphAddKernelNode(&node, h->jmp_graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
                return PLDS_EHIP;
            prev = node;
        }
    }
    if (hipGraphInstantiate(&h->jmp_exec, h->jmp_graph, nullptr, nullptr, 0) != hipSuccess) return PLDS_EHIP;
    return 0;
}

// The insertion rebalance with desire-level jumps (handles created with
// up_jump): seed the pending list with the batch's violating endpoints,
// then run rounds until no vertex is pending.
int jump_sweep(plds *h, hipStream_t s) {
    Dev &d = h->d;
    const int nt = h->h_ctl->n_touch;
    HIPCHK(hipMemsetAsync(d.lvl_cnt, 0, (size_t)(h->K + 1) * sizeof(int32_t), s));
    const size_t hist = (size_t)(h->K <= kHistMax ? h->K : 0) * sizeof(int32_t);
    hipLaunchKernelGGL(k_ins_seed, dim3(grid_for(nt, kBlock, kApplyGrid)), dim3(kBlock), hist, s, d);
    hipLaunchKernelGGL(k_jmp_init, dim3(kListGrid), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_jmp_next, dim3(1), dim3(1), 0, s, d, 0);
    HIPCHK(hipGetLastError());
    const bool timed = h->timed_kind != 0;
    int64_t first = std::min<int64_t>(std::max<int64_t>(h->jmp_steps_hint / kJmpGraphSteps, 1), 8);
    int64_t steps = 0;
    int rc = PLDS_OK;
    const int32_t nbins = dl_bins(h);
    do {
        if (steps > (int64_t)h->K + 1) {   // every round moves to a higher level
            h->broken = true;
            return PLDS_ESTATE;
        }
        if (!timed) {
            rc = jmp_graph(h);
            if (rc) return rc;
            for (int64_t i = 0; i < first; i++) HIPCHK(hipGraphLaunch(h->jmp_exec, s));
        } else {
            for (int64_t i = 0; i < first * kJmpGraphSteps; i++) {
                hipLaunchKernelGGL(k_jmp_select, dim3(kSweepGrid / 4), dim3(kBlock), 0, s, d);
                hipLaunchKernelGGL(k_jmp_dl, dim3(h->dl_grid), dim3(kBlock), 0, s, d);
                hipLaunchKernelGGL(k_jmp_dl_big, dim3(kJmpBigGrid), dim3(kBigBlock), (size_t)nbins * sizeof(int32_t),
                                   s, d, nbins);
                tlaunch(h, 10, k_jmp_scan, dim3(h->del_scan_grid), dim3(kBlock), 0, s, d);
                hipLaunchKernelGGL(k_jmp_fin, dim3(kSweepGrid / 4), dim3(kBlock), 0, s, d);
                hipLaunchKernelGGL(k_jmp_next, dim3(1), dim3(1), 0, s, d, 1);
            }
        }
        steps += first * kJmpGraphSteps;
        first = std::min<int64_t>(first * 2, 16);   // rounds issued after a sweep's end return at once
        HIPCHK(hipGetLastError());
        rc = sync_ctl(h, s);
        if (rc) return rc;
        take_timing(h, h->ev_used);
    } while (!h->h_ctl->done && !h->h_ctl->err);
    Ctl *c = h->h_ctl;
    h->stats.viol_ins0 = c->n_cand;
    h->jmp_steps_hint = c->sweeps + 1;
    h->stats.sweeps_ins += c->sweeps;
    h->stats.moves_up += c->moves;
    h->stats.alg_bytes_up += 8 * c->scanned + 8 * c->alg_up1 + 4 * c->moves;
    h->stats.slots_scanned += c->scanned;
    h->stats.top_level = std::max(h->stats.top_level, c->top);
    return check_err(h);
}

int deletion_sweep(plds *h, hipStream_t s) {
    Dev &d = h->d;
    d.loop_slots = h->sweep_mode == 2 ? 0 : kLoopSlots;
    hipLaunchKernelGGL(k_del_cand, dim3(grid_for(h->h_ctl->n_touch, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d);
    const int32_t nbins = dl_bins(h);
    tlaunch(h, 3, k_dl, dim3(h->dl_grid), dim3(kBlock), 0, s, d, 0);
    hipLaunchKernelGGL(k_dl_big, dim3(kBigGrid), dim3(kBigBlock), (size_t)nbins * sizeof(int32_t), s, d, 0, nbins);
    hipLaunchKernelGGL(k_del_next, dim3(1), dim3(1), 0, s, d, 0);
    // the level loop in one block; it stops at a step too large for it
    tlaunch(h, 9, k_del_loop, dim3(1), dim3(kLoopBlock), 0, s, d);
    HIPCHK(hipGetLastError());
    int rc = sync_ctl(h, s);
    if (rc) return rc;
    take_timing(h, h->ev_used);
    // Large steps: the grid kernels run the step, then the single-block loop
    // goes on; a step graph holds kDelGraphSteps such pairs (the kernels of
    // a pair not needed return at once).  Timed step kernels are launched one
    // by one.
    const bool use_graph = h->timed_kind != 2 && h->timed_kind != 3 && h->timed_kind != 9;
    int run = 4;
    int64_t steps = 0;
    // before the next wait, as many step graphs as the last sweep had large
    // steps (at most 8; steps issued after the sweep's end return at once)
    int64_t first = std::min<int64_t>(std::max<int64_t>((h->del_steps_hint + kDelGraphSteps - 1) / kDelGraphSteps, 1), 8);
    while (!h->h_ctl->done && !h->h_ctl->err) {
        if (steps > (int64_t)h->K + 1) {
            h->broken = true;
            return PLDS_ESTATE;
        }
        if (use_graph) {
            rc = del_graph(h);
            if (rc) return rc;
            for (int64_t i = 0; i < first; i++) HIPCHK(hipGraphLaunch(h->del_exec, s));
            steps += first * kDelGraphSteps;
            first = 1;
        } else {
            steps += run;
            for (int i = 0; i < run; i++) {
                hipLaunchKernelGGL(k_del_select, dim3(kSweepGrid / 4), dim3(kBlock), 0, s, d);
                tlaunch(h, 2, k_del_scan, dim3(h->del_scan_grid), dim3(kBlock), 0, s, d);
                hipLaunchKernelGGL(k_del_fin, dim3(kSweepGrid / 4), dim3(kBlock), 0, s, d);
                tlaunch(h, 3, k_dl, dim3(h->dl_grid), dim3(kBlock), 0, s, d, 1);
                hipLaunchKernelGGL(k_dl_big, dim3(kBigGrid), dim3(kBigBlock), (size_t)nbins * sizeof(int32_t), s, d, 1,
                                   nbins);
                hipLaunchKernelGGL(k_del_next, dim3(1), dim3(1), 0, s, d, 1);
                tlaunch(h, 9, k_del_loop, dim3(1), dim3(kLoopBlock), 0, s, d);
            }
            run = std::min(run * 2, 128);
        }
        HIPCHK(hipGetLastError());
        rc = sync_ctl(h, s);
        if (rc) return rc;
        take_timing(h, h->ev_used);
    }
    Ctl *c = h->h_ctl;
    h->stats.viol_del0 = c->viol_del0;
    h->del_steps_hint = c->big_steps;
    h->stats.sweeps_del += c->sweeps;
    h->stats.moves_down += c->moves;
    h->stats.slots_scanned += c->scanned;
    h->stats.dl_calcs += c->dl_calcs;
    return check_err(h);
}

// Checks of a static k-core call; *nbk receives the number of powers of
// 1+eps up to the first one past n (plus one), *R the peels per threshold,
// ceil(log_{1+delta} n) with delta = 2/eps.
int static_kcore_args(const plds *h, double eps, const double *est_out, int32_t *nbk, int32_t *R) {
    if (!est_out || !(eps > 0) || !std::isfinite(eps) || h->d.ng != 1) return PLDS_EINVAL;
    int32_t k = 1;
    for (double x = 1.0; x < (double)h->n; x *= 1.0 + eps) {
        if (k >= kSkBuckets) return PLDS_EINVAL;   // eps too small for the bucket table
        k++;
    }
    if (k + 1 > kSkBuckets) return PLDS_EINVAL;
    *nbk = k + 1;
    int32_t r = 0;
    for (double x = 1.0; x < (double)h->n; x *= 1.0 + 2.0 / eps) r++;
    *R = r;
    return PLDS_OK;
}

// Algorithm 6 with the scratch arrays of k (allocates nothing).
int static_kcore_run(plds *h, const SK &k, hipStream_t s) {
    Dev &d = h->d;
    hipLaunchKernelGGL(k_sk_setup, dim3(1), dim3(kBlock), 0, s, k);
    h->h_ctl->sk_alive = 0;
    h->h_ctl->sk_relaxed = 0;
    HIPCHK(hipMemcpyAsync(&d.ctl->sk_alive, &h->h_ctl->sk_alive, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
    const size_t hist = (size_t)k.nbk * sizeof(int32_t);
    hipLaunchKernelGGL(k_sk_init, dim3(grid_for(h->n, kBlock, kApplyGrid)), dim3(kBlock), hist, s, d, k);
    hipLaunchKernelGGL(k_sk_first, dim3(1), dim3(kBlock), 0, s, d, k);
    HIPCHK(hipGetLastError());
    int rc = sync_ctl(h, s);
    if (rc) return rc;
    int run = 8;
    int64_t rounds = 0;
    while (!h->h_ctl->sk_done && !h->h_ctl->err) {
        if (rounds > h->n + 1) {   // every round peels at least one vertex
            h->broken = true;
            return PLDS_ESTATE;
        }
        for (int i = 0; i < run; i++) {
            hipLaunchKernelGGL(k_sk_peel, dim3(grid_for(h->n, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d, k);
            tlaunch(h, 7, k_sk_relax, dim3(grid_for((int64_t)h->n * kWave, kBlock, 2048)), dim3(kBlock), 0, s, d, k);
            hipLaunchKernelGGL(k_sk_fix, dim3(grid_for(h->n, kBlock, kApplyGrid)), dim3(kBlock), hist, s, d, k);
            hipLaunchKernelGGL(k_sk_next, dim3(1), dim3(kBlock), 0, s, d, k);
        }
        rounds += run;
        HIPCHK(hipGetLastError());
        rc = sync_ctl(h, s);
        if (rc) return rc;
        take_timing(h, h->ev_used);
        run = std::min(run * 2, 256);
    }
    // the relax kernel's algorithmic bytes: every vertex's adjacency is read
    // once (4-byte id and 4-byte bucket per slot of its 2m), plus an 8-byte
    // count update per alive neighbour of a peeled vertex
    h->stats.alg_bytes_peel += 16 * h->m + 8 * h->h_ctl->sk_relaxed;
    return check_err(h);
}

int guard(const plds *h) {
    if (!h) return PLDS_EINVAL;
    if (h->broken) return PLDS_ESTATE;
    if (hipSetDevice(h->device) != hipSuccess) return PLDS_EHIP;
    return PLDS_OK;
}

}  // namespace

extern "C" {

const char *plds_strerror(int code) {
    switch (code) {
        case PLDS_OK: return "ok";
        case PLDS_EINVAL: return "invalid argument";
        case PLDS_ERANGE: return "vertex id out of range";
        case PLDS_ENOMEM: return "out of memory";
        case PLDS_EHIP: return "HIP runtime error";
        case PLDS_ESTATE: return "internal consistency check failed";
        default: return "unknown error";
    }
}

}  // extern "C"

namespace {

int create_impl(int32_t ngraphs, const int64_t *ns, double delta, double lambda, int32_t levels_per_group,
                int64_t edge_capacity_hint, double up_coeff, int32_t up_jump, plds_t **out) {
    if (!out) return PLDS_EINVAL;
    *out = nullptr;
    if (ngraphs < 1 || !ns || !(delta > 0) || !(lambda > 0) || !std::isfinite(delta) || !std::isfinite(lambda) ||
        (levels_per_group < 0 && levels_per_group != PLDS_LPG_OPT) || edge_capacity_hint < 0)
        return PLDS_EINVAL;
    if (up_coeff != 0 && !(up_coeff >= 1.0 && std::isfinite(up_coeff))) return PLDS_EINVAL;
    int64_t n = 0;
    for (int32_t g = 0; g < ngraphs; g++) {
        if (ns[g] < 1 || ns[g] > INT32_MAX) return PLDS_EINVAL;
        n += ns[g];
        if (n > INT32_MAX) return PLDS_EINVAL;
    }
    plds *h = new (std::nothrow) plds();
    if (!h) return PLDS_ENOMEM;
    h->n = n;
    h->delta = delta;
    h->lambda = lambda;
    h->lpg = levels_per_group;
    h->up_coeff = up_coeff;
    h->up_jump = up_jump ? 1 : 0;
    for (int32_t g = 0, b = 0; g < ngraphs; b += (int32_t)ns[g], g++) {
        h->gbase.push_back(b);
        h->gn.push_back(ns[g]);
        h->gcap.push_back(ns[g]);
    }
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return PLDS_EHIP;
    }
    scratch_lookup(h->device);
    {   // scan blocks: at most one resident round (a scan launched with more
        // blocks than the device holds at once runs its latency chain once
        // per round of blocks), and at most kScanPerCU per compute unit
        int per = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_ins_scan, kBlock, 0) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
            per > 0 && ncu > 0)
            h->scan_grid = std::max(256, std::min(std::min(per, kScanPerCU) * ncu, kSweepGrid));
        h->scan_grid_def = h->scan_grid;
    }
    build_tables(h, levels_per_group);
    for (auto &t : h->gt) h->gcapG.push_back(t.G);
    if ((int64_t)h->G * h->L >= (int64_t)kLevelMask) {   // levels must fit under the mover flags
        delete h;
        return PLDS_EINVAL;
    }
    Dev &d = h->d;
    d.n = (int32_t)n;
    d.L = h->L;
    d.G = h->G;
    d.K = h->K;
    d.ng = ngraphs;
    int64_t ntab = (int64_t)h->h_up_max.size();
    std::vector<int32_t> hL, hK, hLs;
    for (auto &T : h->gt) {
        hL.push_back(T.L);
        hK.push_back(T.K);
        if (std::find(hLs.begin(), hLs.end(), T.L) == hLs.end()) hLs.push_back(T.L);
    }
    d.nLs = (int32_t)hLs.size();
    int rc = 0;
    rc |= dalloc(&d.up_max, ntab) | dalloc(&d.dn_min, ntab) | dalloc(&d.pow_tab, ntab);
    rc |= dalloc(&d.gL, ngraphs) | dalloc(&d.gK, ngraphs) | dalloc(&d.gtab, ngraphs) | dalloc(&d.Ls, d.nLs);
    if (ngraphs > 1) rc |= dalloc(&d.gid, n) | dalloc(&d.gapp, 2 * (int64_t)ngraphs);
    rc |= dalloc(&d.level, n) | dalloc(&d.deg, n) | dalloc(&d.up, n) | dalloc(&d.ups, n);
    rc |= dalloc(&d.cap, n) | dalloc(&d.fill, n) | dalloc(&d.off, n);
    rc |= dalloc(&d.stay, n) | dalloc(&d.cnt2, n) | dalloc(&d.addc, n) | dalloc(&d.dl, n) | dalloc(&d.rcstamp, n);
    rc |= dalloc(&d.ctl, 1);
    rc |= dalloc(&d.touch, n) | dalloc(&d.grow, n) | dalloc(&d.newcap, n) | dalloc(&d.oldoff, n) |
          dalloc(&d.oldcap, n);
    rc |= dalloc(&d.cand, n) | dalloc(&d.sorted, n);
    rc |= dalloc(&d.lvl_cnt, h->K + 1) | dalloc(&d.lvl_start, h->K + 1) | dalloc(&d.next_nz, h->K + 1);
    rc |= dalloc(&d.occ, h->K + 1) | dalloc(&d.lvl_fill, h->K + 1);
    rc |= dalloc(&d.steplog, 16 * (int64_t)h->K) | dalloc(&d.part, 3 * kSweepGrid);
    rc |= dalloc(&d.casc0, n) | dalloc(&d.casc1, n) | dalloc(&d.mv, n) | dalloc(&d.mv1, n) | dalloc(&d.sp, n);
    for (int k = 0; k < 4; k++) rc |= dalloc(&d.cls[k], n);
    rc |= dalloc(&d.p0, n) | dalloc(&d.p1, n) | dalloc(&d.rc, n);
    rc |= dalloc(&d.lvb_start, h->K + 2) | dalloc(&d.lvb_fill, h->K + 2) | dalloc(&d.lvb, n) | dalloc(&d.cl, n) |
          dalloc(&d.sl0, n) | dalloc(&d.sl1, n);
    rc |= dalloc(&h->newoff, n) | dalloc(&h->bad, 8);
    int64_t pool = std::max<int64_t>(1 << 20, 12 * n + (edge_capacity_hint * 2 * 5) / 3);
    rc |= dalloc(&d.pool, pool);
    if (!rc) {
        d.pool_cap = pool;
        rc = ensure_chunks(h);
    }
    if (!rc && hipHostMalloc((void **)&h->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) rc = PLDS_ENOMEM;
    if (rc) {
        free_all(h);
        delete h;
        return PLDS_ENOMEM;
    }
    memset(h->h_ctl, 0, sizeof(Ctl));
    h->h_ctl->nm = kInf;
    hipStream_t s = 0;
    int32_t n32 = (int32_t)n;
    bool ok = hipMemcpy(d.up_max, h->h_up_max.data(), ntab * sizeof(int32_t), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(d.dn_min, h->h_dn_min.data(), ntab * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.pow_tab, h->h_pow.data(), ntab * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.gL, hL.data(), ngraphs * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.gK, hK.data(), ngraphs * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.gtab, h->gtab.data(), ngraphs * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.Ls, hLs.data(), d.nLs * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemsetAsync(d.level, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.deg, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.up, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.ups, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.cap, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.fill, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.off, 0, n * sizeof(int64_t), s) == hipSuccess &&
              hipMemsetAsync(d.stay, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.cnt2, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.addc, 0, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.dl, 0xff, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.rcstamp, 0xff, n * sizeof(int32_t), s) == hipSuccess &&
              hipMemsetAsync(d.sp, 0, n * sizeof(int64_t), s) == hipSuccess &&
              hipMemsetAsync(d.occ, 0, (h->K + 1) * sizeof(int32_t), s) == hipSuccess &&
              hipMemcpy(d.occ, &n32, sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.ctl, h->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    for (int32_t g = 0; ok && ngraphs > 1 && g < ngraphs; g++)
        ok = hipMemsetD32Async((hipDeviceptr_t)(d.gid + h->gbase[g]), g, (size_t)h->gn[g], s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        free_all(h);
        delete h;
        return PLDS_EHIP;
    }
    *out = h;
    return PLDS_OK;
}

}  // namespace

extern "C" {

int plds_create_multi(int32_t ngraphs, const int64_t *ns, double delta, double lambda, int32_t levels_per_group,
                      int64_t edge_capacity_hint, plds_t **out) {
    return create_impl(ngraphs, ns, delta, lambda, levels_per_group, edge_capacity_hint, 0.0, 0, out);
}

int plds_create_opts(int64_t n, double delta, double lambda, const plds_options_t *opts, plds_t **out) {
    if (out) *out = nullptr;
    if (!opts || n < 1 || n > INT32_MAX) return PLDS_EINVAL;
    return create_impl(1, &n, delta, lambda, opts->levels_per_group, opts->edge_capacity_hint, opts->up_coeff,
                       opts->up_jump, out);
}

int plds_create_ex(int64_t n, double delta, double lambda, int32_t levels_per_group, int64_t edge_capacity_hint,
                   plds_t **out) {
    if (n < 1 || n > INT32_MAX) {
        if (out) *out = nullptr;
        return PLDS_EINVAL;
    }
    return plds_create_multi(1, &n, delta, lambda, levels_per_group, edge_capacity_hint, out);
}

int plds_create(int64_t n, double delta, double lambda, plds_t **out) {
    return plds_create_ex(n, delta, lambda, 0, 0, out);
}

int plds_destroy(plds_t *h) {
    if (!h) return PLDS_EINVAL;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
    return PLDS_OK;
}

}  // extern "C"

namespace {

// Start of a batch call: clear the statistics, the step log and the error
// bits (host mirror and device).
int begin_call(plds *h, hipStream_t s) {
    memset(&h->stats, 0, sizeof(h->stats));
    h->range_pending = false;
    h->h_ctl->err = 0;
    h->h_ctl->n_log = 0;
    HIPCHK(hipMemcpyAsync(&h->d.ctl->n_log, &h->h_ctl->n_log, sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(&h->d.ctl->err, &h->h_ctl->err, sizeof(int32_t), hipMemcpyHostToDevice, s));
    return PLDS_OK;
}

// After the range checks of a call: PLDS_ERANGE (nothing applied) if any id
// was out of range.

// Algorithm 1 on range-checked lists of global ids: insertions and their
// sweep, then deletions and theirs.
// A call without updates: its flips and oriented updates are empty.
int track_empty(plds *h, hipStream_t s) {
    if (!h->track) return PLDS_OK;
    h->n_tins = h->n_tdel = 0;
    HIPCHK(hipMemcpyAsync(h->d.prevlvl, h->d.level, (size_t)h->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    h->tracked_call = true;
    return PLDS_OK;
}

int run_update_body(plds *h, const int32_t *ins, int64_t n_ins, const int32_t *del, int64_t n_del, hipStream_t s) {
    int rc;
    bool synced = false;   // the last step ended with a wait, nothing launched since
    h->tracked_call = false;
    if (h->track) {   // the levels the call starts from (the range checks are ahead on the stream)
        h->n_tins = h->n_tdel = 0;
        HIPCHK(hipMemcpyAsync(h->d.prevlvl, h->d.level, (size_t)h->n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              s));
    }
    if (n_ins) {
        int64_t applied = 0;
        rc = apply_list(h, ins, n_ins, 1, s, &applied);
        if (rc) return rc;
        h->stats.applied_ins = applied;
        synced = false;
        if (applied) {
            rc = h->up_jump ? jump_sweep(h, s) : insertion_sweep(h, s);
            if (rc) return rc;
            synced = true;
        }
    }
    if (n_del) {
        int64_t applied = 0;
        rc = apply_list(h, del, n_del, 0, s, &applied);
        if (rc) return rc;
        h->stats.applied_del = applied;
        synced = false;
        if (applied) {
            rc = deletion_sweep(h, s);
            if (rc) return rc;
            synced = true;
        }
    }
    if (!synced) {
        rc = sync_ctl(h, s);
        if (rc) return rc;
    }
    take_timing(h, h->ev_used);   // launches timed since the last collection (complete by now)
    return check_err(h);
}

int run_update(plds *h, const int32_t *ins, int64_t n_ins, const int32_t *del, int64_t n_del, hipStream_t s) {
    int rc = run_update_body(h, ins, n_ins, del, n_del, s);
    h->tracked_call = h->track && rc == PLDS_OK;
    return rc;
}

}  // namespace

extern "C" {

int plds_update(plds_t *h, const int32_t *ins, int64_t n_ins, const int32_t *del, int64_t n_del, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (n_ins < 0 || n_del < 0 || (n_ins && !ins) || (n_del && !del)) return PLDS_EINVAL;
    if ((uint64_t)n_ins > (uint64_t)INT32_MAX / 2 || (uint64_t)n_del > (uint64_t)INT32_MAX / 2) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    memset(&h->stats, 0, sizeof(h->stats));
    if (n_ins + n_del == 0) return track_empty(h, s);
    rc = begin_call(h, s);
    if (rc) return rc;
    // range check of both lists before anything changes
    if (n_ins) hipLaunchKernelGGL(k_range_check, dim3(grid_for(2 * n_ins)), dim3(kBlock), 0, s, ins, n_ins, h->d.n, h->d.ctl);
    if (n_del) hipLaunchKernelGGL(k_range_check, dim3(grid_for(2 * n_del)), dim3(kBlock), 0, s, del, n_del, h->d.n, h->d.ctl);
    HIPCHK(hipGetLastError());
    h->range_pending = true;   // read back by the first batch application
    return run_update(h, ins, n_ins, del, n_del, s);
}

int plds_update_multi(plds_t *h, const int32_t *const *ins, const int64_t *n_ins, const int32_t *const *del,
                      const int64_t *n_del, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    int32_t ng = h->d.ng;
    int64_t ti = 0, td = 0;
    for (int32_t g = 0; g < ng; g++) {
        int64_t a = n_ins ? n_ins[g] : 0, b = n_del ? n_del[g] : 0;
        if (a < 0 || b < 0 || (a && (!ins || !ins[g])) || (b && (!del || !del[g]))) return PLDS_EINVAL;
        ti += a;
        td += b;
    }
    if ((uint64_t)ti > (uint64_t)INT32_MAX / 2 || (uint64_t)td > (uint64_t)INT32_MAX / 2) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    memset(&h->stats, 0, sizeof(h->stats));
    if (ti + td == 0) return track_empty(h, s);
    if (ti + td > h->stage_cap) {
        dfree(h->stage);
        h->stage_cap = 0;
        if (dalloc(&h->stage, 2 * (ti + td))) return PLDS_ENOMEM;
        h->stage_cap = ti + td;
    }
    if (!h->d_segs) {
        if (dalloc(&h->d_segs, 2 * (int64_t)ng)) return PLDS_ENOMEM;
        if (hipHostMalloc((void **)&h->h_segs, 2 * (size_t)ng * sizeof(Seg), hipHostMallocDefault) != hipSuccess) {
            h->h_segs = nullptr;
            return PLDS_ENOMEM;
        }
    }
    // the insertion lists, then the deletion lists, each in graph order
    int32_t nseg = 0;
    int64_t at = 0;
    for (int pass = 0; pass < 2; pass++)
        for (int32_t g = 0; g < ng; g++) {
            int64_t c = pass == 0 ? (n_ins ? n_ins[g] : 0) : (n_del ? n_del[g] : 0);
            if (!c) continue;
            h->h_segs[nseg++] = Seg{pass == 0 ? ins[g] : del[g], c, at, (int32_t)h->gbase[g], (int32_t)h->gn[g]};
            at += c;
        }
    rc = begin_call(h, s);
    if (rc) return rc;
    if (h->d.gapp) HIPCHK(hipMemsetAsync(h->d.gapp, 0, 2 * (size_t)ng * sizeof(unsigned long long), s));
    HIPCHK(hipMemcpyAsync(h->d_segs, h->h_segs, nseg * sizeof(Seg), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_stage, dim3(grid_for(ti + td)), dim3(kBlock), 0, s, h->d_segs, nseg, ti + td, h->stage,
                       h->d.ctl);
    HIPCHK(hipGetLastError());
    h->range_pending = true;   // read back by the first batch application
    return run_update(h, h->stage, ti, h->stage + 2 * ti, td, s);
}

int plds_graph_applied(plds_t *h, int64_t *ins, int64_t *del, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!ins || !del) return PLDS_EINVAL;
    const int32_t ng = h->d.ng;
    if (ng == 1) {
        ins[0] = h->stats.applied_ins;
        del[0] = h->stats.applied_del;
        return PLDS_OK;
    }
    std::vector<unsigned long long> buf(2 * (size_t)ng);
    HIPCHK(hipMemcpyAsync(buf.data(), h->d.gapp, buf.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          S(stream)));
    HIPCHK(hipStreamSynchronize(S(stream)));
    for (int32_t g = 0; g < ng; g++) {
        ins[g] = (int64_t)buf[g];
        del[g] = (int64_t)buf[ng + g];
    }
    return PLDS_OK;
}

int plds_reset_graph(plds_t *h, int32_t g, int64_t n_new, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (g < 0 || g >= h->d.ng || n_new < 1 || n_new > h->gcap[g]) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    Dev &d = h->d;
    // the tables of a handle of n_new vertices, in the graph's table region
    // (sized for its capacity: G and K only grow with n)
    Tables T = make_tables(n_new, h->delta, h->lambda, h->lpg, h->up_coeff);
    if (T.G > h->gcapG[g]) return PLDS_EINVAL;
    const int32_t tab = h->gtab[g];
    HIPCHK(hipMemcpyAsync(d.up_max + tab, T.up.data(), T.up.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.dn_min + tab, T.dn.data(), T.dn.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.pow_tab + tab, T.pw.data(), T.pw.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.gL + g, &T.L, sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.gK + g, &T.K, sizeof(int32_t), hipMemcpyHostToDevice, s));
    h->h_ctl->m_out = 0;
    h->h_ctl->sum_up = 0;
    HIPCHK(hipMemcpyAsync(&d.ctl->m_out, &h->h_ctl->m_out, sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(&d.ctl->sum_up, &h->h_ctl->sum_up, sizeof(int64_t), hipMemcpyHostToDevice, s));
    const int32_t cnt = (int32_t)h->gcap[g];
    hipLaunchKernelGGL(k_reset_range, dim3(grid_for(cnt)), dim3(kBlock), 0, s, d, (int32_t)h->gbase[g], cnt);
    HIPCHK(hipGetLastError());
    rc = sync_ctl(h, s);
    if (rc) return rc;
    int32_t moved = (int32_t)h->h_ctl->sum_up;   // vertices that came down to level 0
    if (moved) {
        int32_t occ0 = 0;
        HIPCHK(hipMemcpy(&occ0, d.occ, sizeof(int32_t), hipMemcpyDeviceToHost));
        occ0 += moved;
        HIPCHK(hipMemcpy(d.occ, &occ0, sizeof(int32_t), hipMemcpyHostToDevice));
    }
    h->m -= h->h_ctl->m_out / 2;
    h->gn[g] = n_new;
    h->gt[g] = std::move(T);
    // the distinct levels-per-group values of the graphs (multi-level step bounds)
    std::vector<int32_t> hLs;
    for (auto &t : h->gt)
        if (std::find(hLs.begin(), hLs.end(), t.L) == hLs.end()) hLs.push_back(t.L);
    if ((int32_t)hLs.size() > d.nLs) {
        dfree(d.Ls);
        if (dalloc(&d.Ls, (int64_t)hLs.size())) {
            h->broken = true;
            return PLDS_ENOMEM;
        }
    }
    d.nLs = (int32_t)hLs.size();
    HIPCHK(hipMemcpy(d.Ls, hLs.data(), hLs.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    memset(&h->stats, 0, sizeof(h->stats));
    return PLDS_OK;
}

int plds_graph_info(const plds_t *h, int32_t g, int64_t *vertex_base, plds_info_t *out) {
    if (!h || g < 0 || g >= h->d.ng) return PLDS_EINVAL;
    if (vertex_base) *vertex_base = h->gbase[g];
    if (out) {
        const Tables &T = h->gt[g];
        plds_info(h, out);
        out->n = h->gn[g];
        out->t = T.t;
        out->L = T.L;
        out->G = T.G;
        out->K = T.K;
    }
    return PLDS_OK;
}

int plds_batch_insert(plds_t *h, const int32_t *edges, int64_t count, void *stream) {
    return plds_update(h, edges, count, nullptr, 0, stream);
}

int plds_batch_delete(plds_t *h, const int32_t *edges, int64_t count, void *stream) {
    return plds_update(h, nullptr, 0, edges, count, stream);
}

int plds_coreness(plds_t *h, const int32_t *vertices, int64_t count, double *out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!out || (vertices && count < 0)) return PLDS_EINVAL;
    int64_t cnt = vertices ? count : h->n;
    if (cnt == 0) return PLDS_OK;
    hipLaunchKernelGGL(k_coreness, dim3(grid_for(cnt)), dim3(kBlock), 0, S(stream), h->d, vertices, cnt, out);
    HIPCHK(hipGetLastError());
    return PLDS_OK;
}

int plds_track_orientation(plds_t *h, int32_t on) {
    int rc = guard(h);
    if (rc) return rc;
    if (on && !h->d.prevlvl) {
        if (dalloc(&h->d.prevlvl, h->n)) return PLDS_ENOMEM;
        if (dalloc(&h->d.lvp, h->n)) {
            dfree(h->d.prevlvl);
            h->d.prevlvl = nullptr;
            return PLDS_ENOMEM;
        }
    }
    h->track = on != 0;
    h->tracked_call = false;
    return PLDS_OK;
}

int plds_orient(plds_t *h, const int32_t *edges, int64_t count, int32_t *out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (count < 0 || (count && (!edges || !out))) return PLDS_EINVAL;
    if (count == 0) return PLDS_OK;
    hipLaunchKernelGGL(k_orient, dim3(grid_for(count)), dim3(kBlock), 0, S(stream), h->d, edges, count, h->d.level,
                       out);
    HIPCHK(hipGetLastError());
    return PLDS_OK;
}

int plds_oriented_updates(plds_t *h, int32_t *ins_out, int64_t ins_cap, int64_t *n_ins, int32_t *del_out,
                          int64_t del_cap, int64_t *n_del, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!n_ins || !n_del || ins_cap < 0 || del_cap < 0 || (ins_cap && !ins_out) || (del_cap && !del_out))
        return PLDS_EINVAL;
    if (!h->tracked_call) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    *n_ins = h->n_tins;
    *n_del = h->n_tdel;
    int64_t ki = std::min(h->n_tins, ins_cap), kd = std::min(h->n_tdel, del_cap);
    if (ki) hipLaunchKernelGGL(k_orient, dim3(grid_for(ki)), dim3(kBlock), 0, s, h->d, h->t_ins, ki, h->d.level, ins_out);
    if (kd)
        hipLaunchKernelGGL(k_orient, dim3(grid_for(kd)), dim3(kBlock), 0, s, h->d, h->t_del, kd, h->d.prevlvl, del_out);
    HIPCHK(hipGetLastError());
    return PLDS_OK;
}

int plds_flips(plds_t *h, int32_t *out, int64_t cap, int64_t *count, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!count || cap < 0 || (cap && !out)) return PLDS_EINVAL;
    if (!h->tracked_call) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    Dev &d = h->d;
    for (int k = 0; k < 4; k++) h->h_ctl->n_fl[k] = 0;
    h->h_ctl->n_flip = 0;
    HIPCHK(hipMemcpyAsync(d.ctl->n_fl, h->h_ctl->n_fl, sizeof(h->h_ctl->n_fl), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(&d.ctl->n_flip, &h->h_ctl->n_flip, sizeof(int64_t), hipMemcpyHostToDevice, s));
    const int with_ins = h->n_tins > 0;
    if (with_ins) {   // the call's insertions had no orientation before it
        rc = ensure_batch(h, h->n_tins);
        if (rc) return rc;
        HIPCHK(hipMemsetAsync(d.hset, 0xff, (size_t)(d.hmask + 1) * sizeof(uint64_t), s));
        hipLaunchKernelGGL(k_flip_inserted, dim3(grid_for(h->n_tins)), dim3(kBlock), 0, s, d, h->t_ins, h->n_tins);
    }
    hipLaunchKernelGGL(k_flip_moved, dim3(grid_for(h->n, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d);
    tlaunch(h, 5, k_flip_scan, dim3(grid_for((int64_t)h->n * kWave, kBlock, 2048)), dim3(kBlock), 0, s, d, with_ins,
            out, cap);
    HIPCHK(hipGetLastError());
    rc = sync_ctl(h, s);
    if (rc) return rc;
    take_timing(h, h->ev_used);
    *count = h->h_ctl->n_flip;
    return check_err(h);
}

int plds_densest_value(plds_t *h, int32_t graph, double *out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!out || graph < 0 || graph >= h->d.ng) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    int64_t v0 = h->d.ng > 1 ? h->gbase[graph] : 0, cnt = h->d.ng > 1 ? h->gn[graph] : h->n;
    h->h_ctl->dv_bits = 0;
    HIPCHK(hipMemcpyAsync(&h->d.ctl->dv_bits, &h->h_ctl->dv_bits, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    if (cnt)
        hipLaunchKernelGGL(k_max_estimate, dim3(grid_for(cnt, kBlock, kApplyGrid)), dim3(kBlock), 0, s, h->d,
                           (int32_t)v0, (int32_t)cnt);
    HIPCHK(hipGetLastError());
    uint64_t bits = 0;
    HIPCHK(hipMemcpyAsync(&h->h_ctl->dv_bits, &h->d.ctl->dv_bits, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bits = h->h_ctl->dv_bits;
    memcpy(out, &bits, sizeof(double));
    return PLDS_OK;
}

int plds_static_kcore(plds_t *h, double eps, double *est_out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    int32_t nbk = 0, R = 0;
    rc = static_kcore_args(h, eps, est_out, &nbk, &R);
    if (rc) return rc;
    hipStream_t s = S(stream);
    Dev &d = h->d;
    if (!h->sk_C) {
        if (dalloc(&h->sk_C, h->n) || dalloc(&h->sk_B, h->n) || dalloc(&h->sk_r, h->n) ||
            dalloc(&h->sk_cnt, kSkBuckets) || dalloc(&h->sk_pw, kSkBuckets)) {
            dfree(h->sk_C), dfree(h->sk_B), dfree(h->sk_r), dfree(h->sk_cnt), dfree(h->sk_pw);
            return PLDS_ENOMEM;
        }
    }
    // the peeled and touched lists use arrays of n entries that are idle
    // outside update calls
    SK k{h->sk_C, h->sk_B, h->sk_r, h->sk_cnt, d.mv, d.casc0, d.mv1, h->sk_pw, est_out, nbk, R, eps};
    return static_kcore_run(h, k, s);
}

int plds_static_kcore_noalloc(plds_t *h, double eps, double *est_out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    int32_t nbk = 0, R = 0;
    rc = static_kcore_args(h, eps, est_out, &nbk, &R);
    if (rc) return rc;
    if (h->n > PLDS_NOALLOC_MAX_N) return PLDS_EINVAL;
    char *base = (char *)scratch_ptr(h->device);
    if (!base) return PLDS_EHIP;   // the symbol lookup at create failed
    // layout of the scratch array: powers, bucket counts, then C, B, r
    double *pw = (double *)base;
    int32_t *cnt = (int32_t *)(base + kScratchPw);
    int32_t *C = (int32_t *)(base + kScratchPw + kScratchCnt);
    int32_t *B = C + PLDS_NOALLOC_MAX_N, *r = B + PLDS_NOALLOC_MAX_N;
    Dev &d = h->d;
    SK k{C, B, r, cnt, d.mv, d.casc0, d.mv1, pw, est_out, nbk, R, eps};
    return static_kcore_run(h, k, S(stream));
}

int plds_delete_vertices(plds_t *h, const int32_t *vertices, int64_t count, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (count < 0 || (count && !vertices)) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    Dev &d = h->d;
    if (count == 0) return plds_update(h, nullptr, 0, nullptr, 0, stream);
    h->h_ctl->err = 0;
    h->h_ctl->vd_deg = h->h_ctl->vd_n = 0;
    for (int c = 0; c < 4; c++) h->h_ctl->vd_ncl[c] = 0;
    HIPCHK(hipMemcpyAsync(&d.ctl->err, &h->h_ctl->err, sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(&d.ctl->vd_deg, &h->h_ctl->vd_deg, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.ctl->vd_ncl, h->h_ctl->vd_ncl, sizeof(h->h_ctl->vd_ncl), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_vd_deg, dim3(grid_for(count, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d, vertices, count);
    HIPCHK(hipGetLastError());
    rc = sync_ctl(h, s);
    if (rc) return rc;
    if (h->h_ctl->err & kErrRange) {
        h->h_ctl->err = 0;
        HIPCHK(hipMemcpyAsync(&d.ctl->err, &h->h_ctl->err, sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        return PLDS_ERANGE;
    }
    const int64_t k = h->h_ctl->vd_deg;
    if ((uint64_t)k > (uint64_t)INT32_MAX / 2) return PLDS_EINVAL;
    if (k > h->vd_cap) {
        dfree(h->vd_buf);
        h->vd_cap = 0;
        if (dalloc(&h->vd_buf, 2 * k)) return PLDS_ENOMEM;
        h->vd_cap = k;
    }
    if (k) {
        // sorted by slab class when the list fits the class lists (ids are in range by now)
        const bool by_class = count <= h->n;
        if (by_class)
            hipLaunchKernelGGL(k_vd_classify, dim3(grid_for(count, kBlock, kApplyGrid)), dim3(kBlock), 0, s, d,
                               vertices, count);
        hipLaunchKernelGGL(k_vd_gather, dim3(grid_for(count * kWave, kBlock, kVdGrid)), dim3(kBlock), 0, s, d,
                           by_class ? nullptr : vertices, count, h->vd_buf, k);
        HIPCHK(hipGetLastError());
        rc = sync_ctl(h, s);
        if (rc) return rc;
        if (h->h_ctl->vd_n != k) return PLDS_ESTATE;
    }
    // one batch of edge deletions (duplicates, from vertices listed twice or
    // edges between two listed vertices, collapse)
    return plds_update(h, nullptr, 0, h->vd_buf, k, stream);
}

int plds_rebuild(plds_t *h, int64_t new_n, const int32_t *relabel, plds_t **out, void *stream) {
    if (!out) return PLDS_EINVAL;
    *out = nullptr;
    int rc = guard(h);
    if (rc) return rc;
    if (h->d.ng != 1 || new_n < 1 || new_n > INT32_MAX || (!relabel && new_n < h->n)) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    int32_t *e = nullptr;
    const int64_t m = h->m;
    if (m && dalloc(&e, 2 * m)) return PLDS_ENOMEM;
    int64_t got = 0;
    rc = m ? plds_dump_state(h, e, m, &got, nullptr, stream) : PLDS_OK;
    if (!rc && m && relabel) {
        hipLaunchKernelGGL(k_relabel, dim3(grid_for(m)), dim3(kBlock), 0, s, e, m, relabel);
        if (hipGetLastError() != hipSuccess) rc = PLDS_EHIP;
    }
    plds_t *nh = nullptr;
    if (!rc) rc = create_impl(1, &new_n, h->delta, h->lambda, h->lpg, 2 * m, h->up_coeff, h->up_jump, &nh);
    if (!rc) {
        nh->sweep_mode = h->sweep_mode;
        nh->scan_grid = h->scan_grid;
        nh->graph_steps = h->graph_steps;
        nh->dl_grid = h->dl_grid;
        nh->del_scan_grid = h->del_scan_grid;
        if (m) rc = plds_update(nh, e, m, nullptr, 0, stream);   // Algorithm 2 on every edge
    }
    dfree(e);
    if (rc) {
        if (nh) plds_destroy(nh);
        return rc;
    }
    *out = nh;
    return PLDS_OK;
}

int plds_levels(plds_t *h, int32_t *out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!out) return PLDS_EINVAL;
    HIPCHK(hipMemcpyAsync(out, h->d.level, h->n * sizeof(int32_t), hipMemcpyDeviceToDevice, S(stream)));
    return PLDS_OK;
}

int plds_degrees(plds_t *h, int32_t *out, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!out) return PLDS_EINVAL;
    HIPCHK(hipMemcpyAsync(out, h->d.deg, h->n * sizeof(int32_t), hipMemcpyDeviceToDevice, S(stream)));
    return PLDS_OK;
}

int plds_info(const plds_t *h, plds_info_t *out) {
    if (!h || !out) return PLDS_EINVAL;
    out->n = h->n;
    out->m = h->m;
    out->t = h->t;
    out->L = h->L;
    out->G = h->G;
    out->K = h->K;
    out->delta = h->delta;
    out->lambda = h->lambda;
    out->slab_slots = h->d.pool_cap;
    out->slab_used = h->pool_top;
    out->ngraphs = h->d.ng;
    out->reserved32 = 0;
    return PLDS_OK;
}

int plds_thresholds(const plds_t *h, int32_t *up_max, int32_t *dn_min, double *pow_tab) {
    if (!h) return PLDS_EINVAL;
    for (int32_t g = 0; g < h->gt[0].G; g++) {   // graph 0 (the only one of a plain handle)
        if (up_max) up_max[g] = h->h_up_max[g];
        if (dn_min) dn_min[g] = h->h_dn_min[g];
        if (pow_tab) pow_tab[g] = h->h_pow[g];
    }
    return PLDS_OK;
}

int plds_set_sweep_mode(plds_t *h, int32_t mode) {
    if (!h || mode < 0 || mode > 4) return PLDS_EINVAL;
    h->sweep_mode = mode;
    return PLDS_OK;
}

int plds_set_launch(plds_t *h, const plds_launch_t *cfg) {
    if (!h || !cfg) return PLDS_EINVAL;
    for (int k = 0; k < 4; k++)
        if (cfg->reserved[k]) return PLDS_EINVAL;
    auto in = [](int32_t v, int32_t lo, int32_t hi) { return v == 0 || (v >= lo && v <= hi); };
    if (!in(cfg->scan_blocks, 64, kSweepGrid) || !in(cfg->graph_steps, 2, 64) || (cfg->graph_steps & 1) ||
        !in(cfg->dl_blocks, 64, 4096) || !in(cfg->del_scan_blocks, 64, 8192))
        return PLDS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return PLDS_EHIP;
    h->scan_grid = cfg->scan_blocks ? cfg->scan_blocks : h->scan_grid_def;
    h->graph_steps = cfg->graph_steps ? cfg->graph_steps : kGraphStepsDef;
    h->dl_grid = cfg->dl_blocks ? cfg->dl_blocks : kDlGrid;
    h->del_scan_grid = cfg->del_scan_blocks ? cfg->del_scan_blocks : kSweepGrid;
    drop_graphs(h);   // the step graphs carry the grids
    return PLDS_OK;
}

int plds_get_launch(const plds_t *h, plds_launch_t *out) {
    if (!h || !out) return PLDS_EINVAL;
    *out = plds_launch_t{};
    out->scan_blocks = h->scan_grid;
    out->graph_steps = h->graph_steps;
    out->dl_blocks = h->dl_grid;
    out->del_scan_blocks = h->del_scan_grid;
    return PLDS_OK;
}

int plds_inject_alloc_failure(int64_t after) {
    t_alloc_fail_after = after < 0 ? -1 : after;
    return PLDS_OK;
}

int plds_set_timing(plds_t *h, int32_t kernel) {
    if (!h || kernel < 0 || kernel > 11) return PLDS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return PLDS_EHIP;
    if (kernel && h->ev.empty()) {
        h->ev.assign(2 * kEvPairs, nullptr);
        for (auto &e : h->ev)
            if (hipEventCreate(&e) != hipSuccess) return PLDS_EHIP;
    }
    h->timed_kind = kernel;
    h->ev_used = 0;
    return PLDS_OK;
}

int plds_step_log(plds_t *h, int64_t *out, int64_t cap, int64_t *rows) {
    if (!h || !rows || cap < 0 || (cap && !out)) return PLDS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return PLDS_EHIP;
    int64_t k = std::min<int64_t>(h->h_ctl->n_log, cap);
    *rows = h->h_ctl->n_log;
    if (k > 0) HIPCHK(hipMemcpy(out, h->d.steplog, (size_t)k * 4 * sizeof(int64_t), hipMemcpyDeviceToHost));
    return PLDS_OK;
}

int plds_stats(const plds_t *h, plds_stats_t *out) {
    if (!h || !out) return PLDS_EINVAL;
    *out = h->stats;
    return PLDS_OK;
}

int plds_check(plds_t *h, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    hipStream_t s = S(stream);
    HIPCHK(hipMemsetAsync(h->bad, 0, 8 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_check, dim3(grid_for(h->n * kWave)), dim3(kBlock), 0, s, h->d, h->bad);
    HIPCHK(hipMemsetAsync(h->d.lvl_cnt, 0, (h->K + 1) * sizeof(int32_t), s));
    count_levels(h, h->d.lvl_cnt, s);
    hipLaunchKernelGGL(k_compare, dim3(grid_for(h->K)), dim3(kBlock), 0, s, h->d.lvl_cnt, h->d.occ, h->K,
                       h->bad + 6);
    HIPCHK(hipGetLastError());
    int32_t bad[8];
    HIPCHK(hipMemcpyAsync(bad, h->bad, sizeof(bad), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < 7; i++)
        if (bad[i]) return PLDS_ESTATE;
    return PLDS_OK;
}

int plds_dump_state(plds_t *h, int32_t *edges, int64_t cap, int64_t *m_out, int32_t *levels, void *stream) {
    int rc = guard(h);
    if (rc) return rc;
    if (!m_out || cap < 0 || (cap && !edges)) return PLDS_EINVAL;
    *m_out = h->m;
    if (cap < h->m) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    h->h_ctl->m_out = 0;
    HIPCHK(hipMemcpyAsync(&h->d.ctl->m_out, &h->h_ctl->m_out, sizeof(int64_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_dump_edges, dim3(grid_for(h->n)), dim3(kBlock), 0, s, h->d, edges, cap);
    HIPCHK(hipGetLastError());
    if (levels) HIPCHK(hipMemcpyAsync(levels, h->d.level, h->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    rc = sync_ctl(h, s);
    if (rc) return rc;
    if (h->h_ctl->m_out != h->m) return PLDS_ESTATE;
    return PLDS_OK;
}

int plds_load_state(plds_t *h, const int32_t *edges, int64_t m, const int32_t *levels, void *stream) {
    if (!h) return PLDS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return PLDS_EHIP;
    if (m < 0 || (m && !edges) || !levels || (uint64_t)m > (uint64_t)INT32_MAX / 2) return PLDS_EINVAL;
    hipStream_t s = S(stream);
    Dev &d = h->d;
    h->tracked_call = false;   // a loaded state has no last update call
    // validate ids and levels before touching the state
    h->h_ctl->err = 0;
    HIPCHK(hipMemcpyAsync(&d.ctl->err, &h->h_ctl->err, sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (m) hipLaunchKernelGGL(k_range_check, dim3(grid_for(2 * m)), dim3(kBlock), 0, s, edges, m, d.n, d.ctl);
    HIPCHK(hipGetLastError());
    int rc = sync_ctl(h, s);
    if (rc) return rc;
    if (h->h_ctl->err & kErrRange) return PLDS_ERANGE;
    // wipe
    h->broken = false;
    h->pool_top = 0;
    h->m = 0;
    size_t n4 = h->n * sizeof(int32_t);
    HIPCHK(hipMemsetAsync(d.deg, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.up, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.ups, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.cap, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.fill, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.off, 0, h->n * sizeof(int64_t), s));
    HIPCHK(hipMemsetAsync(d.addc, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.stay, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.cnt2, 0, n4, s));
    HIPCHK(hipMemsetAsync(d.sp, 0, h->n * sizeof(int64_t), s));
    HIPCHK(hipMemsetAsync(d.dl, 0xff, n4, s));
    hipLaunchKernelGGL(k_set_levels, dim3(grid_for(h->n)), dim3(kBlock), 0, s, d, levels);
    HIPCHK(hipMemsetAsync(d.occ, 0, (h->K + 1) * sizeof(int32_t), s));
    count_levels(h, d.occ, s);
    HIPCHK(hipGetLastError());
    int64_t applied = 0;
    if (m) {
        rc = apply_list(h, edges, m, 1, s, &applied);
        if (rc) return rc;
        hipLaunchKernelGGL(k_clear_touch, dim3(grid_for(h->h_ctl->n_touch)), dim3(kBlock), 0, s, d);
    }
    rc = sync_ctl(h, s);
    if (rc) return rc;
    if (h->h_ctl->err & kErrLevel) {
        h->broken = true;
        return PLDS_EINVAL;
    }
    rc = check_err(h);
    if (rc) return rc;
    return plds_check(h, stream);
}

int plds_sync(plds_t *h, void *stream) {
    if (!h) return PLDS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return PLDS_EHIP;
    int rc = sync_ctl(h, S(stream));
    if (rc) return rc;
    if (h->h_ctl->err & kErrRange) {
        h->h_ctl->err &= ~kErrRange;
        HIPCHK(hipMemcpyAsync(&h->d.ctl->err, &h->h_ctl->err, sizeof(int32_t), hipMemcpyHostToDevice, S(stream)));
        HIPCHK(hipStreamSynchronize(S(stream)));
        return PLDS_ERANGE;
    }
    return h->broken ? PLDS_ESTATE : PLDS_OK;
}

}  // extern "C"
