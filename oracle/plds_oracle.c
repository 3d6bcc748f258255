/*
 * plds_oracle.c -- sequential CPU oracle of the parallel level data structure
 * (PLDS) of "Parallel Batch-Dynamic Algorithms for k-Core Decomposition and
 * Related Graph Problems" (Liu, Shi, Yu, Dhulipala, Shun; SPAA'22).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark.  The GPU library never links or calls it.
 *
 * The oracle runs the paper's algorithm step by step, sequentially:
 *   - levels, groups, Invariants 1-2, up/up* degrees and the desire-level
 *     (Section "Detailed PLDS Algorithm", Invariants 1-2, Def. desire-level);
 *   - Update(B) = RebalanceInsertions then RebalanceDeletions (Algorithm 1);
 *   - RebalanceInsertions: level by level from 0 upwards, all Invariant-1
 *     violators of the level move up one level together (Algorithm 2);
 *   - RebalanceDeletions: desire-levels of Invariant-2 violators, then level
 *     by level from 0 upwards all vertices whose desire-level is that level
 *     move there together, and violating neighbours get a new desire-level
 *     (Algorithm 3);
 *   - the coreness estimate from the level (Def. coreness estimate);
 *   - batch preprocessing: unique, canonical, valid updates (framework
 *     section, preprocessing paragraph).
 * Readings of garbled or silent passages:
 *   - L = 4*ceil(log_{1+delta} n) levels per group, groups 0..ceil(log n), so
 *     G = t+1 groups and K = G*L levels, t the least integer with
 *     (1+delta)^t >= n;
 *   - Invariant 1 is violated iff up > floor((2+3/lambda)(1+delta)^g) and
 *     Invariant 2 iff up* < ceil((1+delta)^g): exact rewrites for integer
 *     degrees; (1+delta)^g is formed by repeated IEEE double multiplication;
 *   - the desire-level follows its definition (the printed search procedure
 *     has garbled indices);
 *   - estimate = (1+delta)^max(floor((level+1)/L)-1, 0), and 0 for a vertex of
 *     degree 0 (the experiments state isolated vertices get estimate 0);
 *   - a batch: ids outside [0,n) reject the whole call; self-loops are
 *     dropped; duplicates collapse; inserting a present edge or deleting an
 *     absent one does nothing; insertions of a call are applied before its
 *     deletions.
 * Statistics (ora_stats, per call):
 *   0 applied insertions   1 applied deletions   2 insertion sweeps (levels
 *   with movers)   3 deletion sweeps   4 up-moves (one level each)
 *   5 down-moves   6 desire-level computations   7 sum of deg(v) over up-moves
 *   8 sum of up(v) over up-moves   9 sum of deg over desire-level computations
 *   10 sum of deg over down-moves   11 highest level after the call
 *   12 initial Invariant-1 violators   13 initial Invariant-2 violators
 */
#include "plds_oracle.h"

#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORA_EINVAL -1
#define ORA_ERANGE -2
#define ORA_ENOMEM -3
#define ORA_ESTATE -5

/* assertion codes recorded in o->assert_code */
#define A_T1_LEVEL_RANGE 1   /* a level left [0,K) (Lemma good-level)          */
#define A_T2_INV2_INSERT 2   /* Invariant 2 broken during insertions (Obs.)     */
#define A_T3_INV1_DELETE 3   /* Invariant 1 broken during deletions (Obs.)      */
#define A_T4_MOVE_UP     4   /* a violator at an already processed level        */
#define A_T5_SMALLER     5   /* a desire-level <= the level being processed     */
#define A_MOVER_VIOL     6   /* a vertex violates right after its down-move     */
#define A_FINAL          7   /* invariants do not hold after the call           */

typedef struct {
    int32_t *a;
    int64_t n, cap;
} vec_t;

struct ora {
    int64_t n, m;
    double delta, lambda;
    double coeff;           /* Invariant 1 coefficient: 2 + 3/lambda, or the caller's */
    int32_t jump;           /* insertions move violators to their desire-level at once */
    int32_t t, L, G, K, mode;
    int32_t *up_max, *dn_min;
    double *pow_tab;
    /* adjacency: sorted neighbour arrays */
    int32_t **adj;
    int32_t *deg, *acap;
    int32_t *level;
    int32_t *up, *ups;      /* counters: up-degree, up*-degree (mode 0)   */
    int32_t *dl;            /* desire-level of pending vertices, else -1  */
    int32_t *qlev;          /* level of the list a vertex is queued in    */
    uint8_t *inset;         /* member of the set moving at this level     */
    int32_t *old;           /* previous level of a mover                  */
    int32_t *hist;          /* scratch [K+1]                              */
    vec_t *bucket;          /* per-level candidate lists [K]              */
    vec_t movers;
    int64_t stats[16];
    int assert_code;
};

/* ------------------------------------------------------------------ vectors */
static int vec_push(vec_t *v, int32_t x) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 16;
        int32_t *na = (int32_t *)realloc(v->a, (size_t)nc * sizeof(int32_t));
        if (!na) return ORA_ENOMEM;
        v->a = na;
        v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------ parameters */
/* Levels and groups (Section "Detailed PLDS Algorithm"): groups
 * g_0..g_t with t = ceil(log_{1+delta} n), 4t levels per group; the
 * experiments' PLDSOpt variant has ceil(log_{1+delta} n / 50) levels per
 * group (levels_per_group == -1). */
static void build_tables(ora_t *o, int32_t levels_per_group) {
    double p = 1.0;
    int32_t t = 0;
    while (p < (double)o->n) {          /* least t with (1+delta)^t >= n */
        p *= 1.0 + o->delta;
        t++;
    }
    o->t = t;
    if (levels_per_group > 0)
        o->L = levels_per_group;
    else if (levels_per_group == -1)            /* PLDSOpt: ceil(log_{1+delta} n / 50) = ceil(t / 50) */
        o->L = (t + 49) / 50 > 1 ? (t + 49) / 50 : 1;
    else
        o->L = 4 * t > 1 ? 4 * t : 1;
    o->G = t + 1;
    o->K = o->G * o->L;
    o->up_max = (int32_t *)malloc((size_t)o->G * sizeof(int32_t));
    o->dn_min = (int32_t *)malloc((size_t)o->G * sizeof(int32_t));
    o->pow_tab = (double *)malloc((size_t)o->G * sizeof(double));
    double coeff = o->coeff;                    /* Invariant 1 coefficient */
    double x = 1.0;
    for (int32_t g = 0; g < o->G; g++) {
        if (g > 0) x *= 1.0 + o->delta;
        o->pow_tab[g] = x;
        double ub = floor(coeff * x);           /* Invariant 1: up <= ub      */
        double lb = ceil(x);                    /* Invariant 2: up* >= lb     */
        o->up_max[g] = ub >= (double)INT32_MAX ? INT32_MAX : (int32_t)ub;
        o->dn_min[g] = lb >= (double)INT32_MAX ? INT32_MAX : (int32_t)lb;
    }
}

static inline int32_t gn(const ora_t *o, int32_t lvl) { return lvl / o->L; }

/* coeff > 0 replaces the Invariant-1 coefficient 2 + 3/lambda (the
 * experiments' heuristic parameters use 1.1); it must be at least 1, so that
 * floor(coeff x) >= ceil(x) - 1 for every x >= 1 and an integer count below
 * the Invariant-2 floor never exceeds the Invariant-1 cap.  jump != 0 selects
 * the implementation's insertion procedure (PLDS implementation details):
 * violators move straight to their desire-level instead of one level at a
 * time. */
ora_t *ora_create_ex(int64_t n, double delta, double lambda, int32_t levels_per_group, int32_t mode, double coeff,
                     int32_t jump) {
    if (n < 1 || n > INT32_MAX || !(delta > 0) || !(lambda > 0) || (mode != 0 && mode != 1))
        return NULL;
    if (coeff > 0 && coeff < 1.0) return NULL;
    ora_t *o = (ora_t *)calloc(1, sizeof(ora_t));
    if (!o) return NULL;
    o->n = n;
    o->delta = delta;
    o->lambda = lambda;
    o->coeff = coeff > 0 ? coeff : 2.0 + 3.0 / lambda;
    o->jump = jump != 0;
    o->mode = mode;
    build_tables(o, levels_per_group);
    o->adj = (int32_t **)calloc((size_t)n, sizeof(int32_t *));
    o->deg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    o->acap = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    o->level = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    o->up = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    o->ups = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    o->dl = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    o->qlev = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    o->inset = (uint8_t *)calloc((size_t)n, 1);
    o->old = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    o->hist = (int32_t *)calloc((size_t)o->K + 1, sizeof(int32_t));
    o->bucket = (vec_t *)calloc((size_t)o->K + 1, sizeof(vec_t));
    if (!o->adj || !o->deg || !o->acap || !o->level || !o->up || !o->ups || !o->dl || !o->qlev ||
        !o->inset || !o->old || !o->hist || !o->bucket || !o->up_max || !o->dn_min || !o->pow_tab) {
        ora_destroy(o);
        return NULL;
    }
    for (int64_t i = 0; i < n; i++) {
        o->dl[i] = -1;
        o->qlev[i] = -1;
    }
    return o;
}

ora_t *ora_create(int64_t n, double delta, double lambda, int32_t levels_per_group, int32_t mode) {
    return ora_create_ex(n, delta, lambda, levels_per_group, mode, 0.0, 0);
}

void ora_destroy(ora_t *o) {
    if (!o) return;
    if (o->adj)
        for (int64_t i = 0; i < o->n; i++) free(o->adj[i]);
    free(o->adj);
    free(o->deg);
    free(o->acap);
    free(o->level);
    free(o->up);
    free(o->ups);
    free(o->dl);
    free(o->qlev);
    free(o->inset);
    free(o->old);
    free(o->hist);
    if (o->bucket)
        for (int32_t l = 0; l <= o->K; l++) free(o->bucket[l].a);
    free(o->bucket);
    free(o->movers.a);
    free(o->up_max);
    free(o->dn_min);
    free(o->pow_tab);
    free(o);
}

void ora_info(const ora_t *o, int64_t *out) {
    out[0] = o->n;
    out[1] = o->m;
    out[2] = o->t;
    out[3] = o->L;
    out[4] = o->G;
    out[5] = o->K;
    out[6] = o->mode;
    out[7] = 0;
}

void ora_tables(const ora_t *o, int32_t *up_max, int32_t *dn_min, double *pow_tab) {
    for (int32_t g = 0; g < o->G; g++) {
        if (up_max) up_max[g] = o->up_max[g];
        if (dn_min) dn_min[g] = o->dn_min[g];
        if (pow_tab) pow_tab[g] = o->pow_tab[g];
    }
}

/* ------------------------------------------------------------- adjacency */
static int has_edge(const ora_t *o, int32_t u, int32_t v) {
    const int32_t *a = o->adj[u];
    int32_t lo = 0, hi = o->deg[u];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo < o->deg[u] && a[lo] == v;
}

/* merge k sorted ids (all absent) into the sorted array of u */
static int adj_merge(ora_t *o, int32_t u, const int32_t *vs, int32_t k) {
    int32_t d = o->deg[u];
    if (d + k > o->acap[u]) {
        int32_t nc = o->acap[u] ? o->acap[u] : 4;
        while (nc < d + k) nc = nc > INT32_MAX / 2 ? INT32_MAX : 2 * nc;
        int32_t *na = (int32_t *)realloc(o->adj[u], (size_t)nc * sizeof(int32_t));
        if (!na) return ORA_ENOMEM;
        o->adj[u] = na;
        o->acap[u] = nc;
    }
    int32_t *a = o->adj[u];
    int32_t i = d - 1, j = k - 1, w = d + k - 1;
    while (j >= 0) {
        if (i >= 0 && a[i] > vs[j]) a[w--] = a[i--];
        else a[w--] = vs[j--];
    }
    o->deg[u] = d + k;
    return 0;
}

/* remove k sorted ids (all present) from the sorted array of u */
static void adj_remove(ora_t *o, int32_t u, const int32_t *vs, int32_t k) {
    int32_t *a = o->adj[u];
    int32_t d = o->deg[u], w = 0, j = 0;
    for (int32_t i = 0; i < d; i++) {
        if (j < k && a[i] == vs[j]) {
            j++;
            continue;
        }
        a[w++] = a[i];
    }
    o->deg[u] = w;
}

/* apply a list of canonical edge keys (u<<32|v) to the adjacency, add=1
 * inserts, add=0 removes.  Both directed copies are stored. */
static int adj_apply(ora_t *o, const uint64_t *keys, int64_t k, int add) {
    if (k == 0) return 0;
    uint64_t *dir = (uint64_t *)malloc((size_t)(2 * k) * sizeof(uint64_t));
    int32_t *tmp = NULL;
    if (!dir) return ORA_ENOMEM;
    for (int64_t i = 0; i < k; i++) {
        uint64_t a = keys[i] >> 32, b = keys[i] & 0xffffffffu;
        dir[2 * i] = (a << 32) | b;
        dir[2 * i + 1] = (b << 32) | a;
    }
    qsort(dir, (size_t)(2 * k), sizeof(uint64_t), cmp_u64);
    tmp = (int32_t *)malloc((size_t)(2 * k) * sizeof(int32_t));
    if (!tmp) {
        free(dir);
        return ORA_ENOMEM;
    }
    int rc = 0;
    for (int64_t i = 0; i < 2 * k && rc == 0;) {
        int32_t u = (int32_t)(dir[i] >> 32);
        int32_t c = 0;
        while (i < 2 * k && (int32_t)(dir[i] >> 32) == u) tmp[c++] = (int32_t)(dir[i++] & 0xffffffffu);
        if (add) rc = adj_merge(o, u, tmp, c);
        else adj_remove(o, u, tmp, c);
    }
    free(tmp);
    free(dir);
    if (rc == 0) o->m += add ? k : -k;
    return rc;
}

/* ---------------------------------------------------------------- degrees */
/* up(v) = #neighbours in Z_{level(v)}; up*(v) = #neighbours in Z_{level(v)-1}
 * (Section "Detailed PLDS Algorithm", definitions of up- and up*-degree). */
static int32_t count_up(const ora_t *o, int32_t v) {
    int32_t c = 0, lv = o->level[v];
    for (int32_t i = 0; i < o->deg[v]; i++) c += o->level[o->adj[v][i]] >= lv;
    return c;
}
static int32_t count_ups(const ora_t *o, int32_t v) {
    int32_t c = 0, lv = o->level[v];
    for (int32_t i = 0; i < o->deg[v]; i++) c += o->level[o->adj[v][i]] >= lv - 1;
    return c;
}
static int32_t up_of(const ora_t *o, int32_t v) { return o->mode == 0 ? o->up[v] : count_up(o, v); }
static int32_t ups_of(const ora_t *o, int32_t v) { return o->mode == 0 ? o->ups[v] : count_ups(o, v); }

/* Invariant 1: v in V_l, l in g_i  =>  up(v) <= (2+3/lambda)(1+delta)^i */
static int viol1(const ora_t *o, int32_t v) { return up_of(o, v) > o->up_max[gn(o, o->level[v])]; }
/* Invariant 2: v in V_l, l > 0, l-1 in g_i  =>  up*(v) >= (1+delta)^i */
static int viol2(const ora_t *o, int32_t v) {
    int32_t lv = o->level[v];
    return lv > 0 && ups_of(o, v) < o->dn_min[gn(o, lv - 1)];
}

/* counter change of a non-moving vertex w when its neighbour goes from level
 * a to level b: up(w) counts the neighbour iff its level >= level(w), up*(w)
 * iff its level >= level(w)-1. */
static void adjust(ora_t *o, int32_t w, int32_t a, int32_t b) {
    int32_t lw = o->level[w];
    o->up[w] += (b >= lw) - (a >= lw);
    o->ups[w] += (b >= lw - 1) - (a >= lw - 1);
}

static void recount(ora_t *o, int32_t v) {
    o->up[v] = count_up(o, v);
    o->ups[v] = count_ups(o, v);
}

/* edge (a,b) inserted (sign +1) or removed (sign -1) with levels unchanged */
static void edge_counters(ora_t *o, int32_t a, int32_t b, int32_t sign) {
    int32_t la = o->level[a], lb = o->level[b];
    o->up[a] += sign * (lb >= la);
    o->ups[a] += sign * (lb >= la - 1);
    o->up[b] += sign * (la >= lb);
    o->ups[b] += sign * (la >= lb - 1);
}

/* ----------------------------------------------------------- desire-level */
/* Def. desire-level: the level l' closest to level(v) at which both
 * invariants hold, with up(v), up*(v) counted as if v were at l'.  For an
 * Invariant-2 violator every level >= level(v) fails Invariant 2 (its
 * up*-count can only shrink and its floor only grow), so the search runs
 * downwards from level(v)-1 and takes the first level where both hold.
 * cnt(j) = #neighbours at level >= j is built from a histogram of neighbour
 * levels. */
static int32_t desire_level(ora_t *o, int32_t v) {
    int32_t lv = o->level[v];
    int32_t *h = o->hist;
    for (int32_t j = 0; j <= lv; j++) h[j] = 0;
    for (int32_t i = 0; i < o->deg[v]; i++) {
        int32_t lw = o->level[o->adj[v][i]];
        h[lw < lv ? lw : lv]++;                /* bin lv = "at level >= lv" */
    }
    o->stats[6]++;
    o->stats[9] += o->deg[v];
    /* cnt_at(l') = #nbrs >= l' ; walk l' = lv-1 .. 0 keeping cnt(l') and cnt(l'-1) */
    int32_t cnt_ge = h[lv];                      /* cnt(lv) */
    for (int32_t lp = lv - 1; lp >= 0; lp--) {
        cnt_ge += h[lp];                         /* now cnt(lp)   */
        int32_t up_here = cnt_ge;                /* up(v) if v were at lp */
        int ok1 = up_here <= o->up_max[gn(o, lp)];
        int ok2 = 1;
        if (lp > 0) {
            int32_t ups_here = cnt_ge + h[lp - 1];   /* cnt(lp-1) */
            ok2 = ups_here >= o->dn_min[gn(o, lp - 1)];
        }
        if (ok1 && ok2) return lp;
    }
    return 0;   /* unreachable for a violator: level 0 holds when deg(v) = 0 */
}

/* -------------------------------------------------------- preprocessing */
/* Batch preprocessing (framework section): canonical (min,max) keys, no
 * self-loops, sorted, unique.  Returns the count written to keys. */
static int64_t canon_unique(const int32_t *e, int64_t cnt, uint64_t *keys) {
    int64_t k = 0;
    for (int64_t i = 0; i < cnt; i++) {
        int32_t u = e[2 * i], v = e[2 * i + 1];
        if (u == v) continue;
        uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
        keys[k++] = (a << 32) | b;
    }
    qsort(keys, (size_t)k, sizeof(uint64_t), cmp_u64);
    int64_t w = 0;
    for (int64_t i = 0; i < k; i++)
        if (w == 0 || keys[i] != keys[w - 1]) keys[w++] = keys[i];
    return w;
}

static int in_range(const ora_t *o, const int32_t *e, int64_t cnt) {
    for (int64_t i = 0; i < 2 * cnt; i++)
        if (e[i] < 0 || (int64_t)e[i] >= o->n) return 0;
    return 1;
}

static void fail(ora_t *o, int code) {
    if (!o->assert_code) o->assert_code = code;
}

static void queue(ora_t *o, int32_t lvl, int32_t v) {
    if (lvl < 0 || lvl >= o->K) {
        fail(o, A_T1_LEVEL_RANGE);
        return;
    }
    if (vec_push(&o->bucket[lvl], v)) fail(o, A_T1_LEVEL_RANGE);
}

/* ----------------------------------------------------------- insertions */
/* Algorithm 2 (RebalanceInsertions), counter mode.  Candidates of level l
 * are the vertices incident to the batch or marked; the set S_l of those at
 * level l violating Invariant 1 is fixed before any of them moves, then all
 * of S_l move to l+1 together. */
static void insert_phase_counters(ora_t *o, const uint64_t *keys, int64_t k) {
    for (int64_t i = 0; i < k; i++)
        edge_counters(o, (int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu), +1);
    for (int64_t i = 0; i < k; i++) {
        int32_t ends[2] = {(int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu)};
        for (int e = 0; e < 2; e++) {
            int32_t x = ends[e];
            if (viol2(o, x)) fail(o, A_T2_INV2_INSERT);
            if (viol1(o, x) && o->qlev[x] != o->level[x]) {
                o->qlev[x] = o->level[x];
                queue(o, o->level[x], x);
                o->stats[12]++;
            }
        }
    }
    for (int32_t l = 0; l < o->K; l++) {
        vec_t *b = &o->bucket[l];
        if (b->n == 0) continue;
        o->movers.n = 0;
        for (int64_t i = 0; i < b->n; i++) {
            int32_t v = b->a[i];
            o->qlev[v] = -1;
            if (o->level[v] == l && !o->inset[v] && viol1(o, v)) {
                o->inset[v] = 1;
                vec_push(&o->movers, v);
            }
        }
        b->n = 0;
        if (o->movers.n == 0) continue;
        o->stats[2]++;
        o->stats[4] += o->movers.n;
        /* neighbours that stay see the mover go from l to l+1 */
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->stats[7] += o->deg[v];
            o->stats[8] += o->up[v];
            for (int32_t j = 0; j < o->deg[v]; j++) {
                int32_t w = o->adj[v][j];
                if (!o->inset[w]) adjust(o, w, l, l + 1);
            }
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->level[o->movers.a[i]] = l + 1;
        for (int64_t i = 0; i < o->movers.n; i++) recount(o, o->movers.a[i]);
        /* mark: movers and their neighbours that now violate Invariant 1 */
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            for (int32_t j = -1; j < o->deg[v]; j++) {
                int32_t x = j < 0 ? v : o->adj[v][j];
                if (viol2(o, x)) fail(o, A_T2_INV2_INSERT);
                if (!viol1(o, x)) continue;
                if (o->level[x] <= l) fail(o, A_T4_MOVE_UP);     /* Lemma move-up */
                if (o->qlev[x] != o->level[x]) {
                    o->qlev[x] = o->level[x];
                    queue(o, o->level[x], x);
                }
            }
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->inset[o->movers.a[i]] = 0;
    }
}

/* Algorithm 2, full-scan mode: every level 0..K-1, every vertex, degrees
 * recounted.  S_l = all vertices of level l violating Invariant 1. */
static void insert_phase_scan(ora_t *o) {
    for (int32_t l = 0; l < o->K; l++) {
        o->movers.n = 0;
        for (int32_t v = 0; v < (int32_t)o->n; v++) {
            if (o->level[v] < l && viol1(o, v)) fail(o, A_T4_MOVE_UP);
            if (o->level[v] == l && viol1(o, v)) vec_push(&o->movers, v);
        }
        if (o->movers.n == 0) continue;
        o->stats[2]++;
        o->stats[4] += o->movers.n;
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->stats[7] += o->deg[v];
            o->stats[8] += count_up(o, v);
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->level[o->movers.a[i]] = l + 1;
        for (int32_t v = 0; v < (int32_t)o->n; v++)
            if (viol2(o, v)) fail(o, A_T2_INV2_INSERT);
    }
}

/* Upward desire-level (Def. desire-level, for an Invariant-1 violator): the
 * level closest to level(v) at which both invariants hold.  Below level(v)
 * Invariant 1 keeps failing (the count of neighbours at or above a level only
 * grows downwards, the cap only shrinks), so the search runs upwards from
 * level(v)+1 and takes the first level where both hold; up(v) and up*(v) are
 * counted from the neighbours' current levels. */
static int32_t up_desire_level(ora_t *o, int32_t v) {
    int32_t lv = o->level[v];
    int32_t *h = o->hist;
    for (int32_t j = 0; j <= o->K; j++) h[j] = 0;
    for (int32_t i = 0; i < o->deg[v]; i++) h[o->level[o->adj[v][i]]]++;
    o->stats[6]++;
    o->stats[9] += o->deg[v];
    int32_t cnt_ge = 0;                          /* cnt(j) = #neighbours at level >= j */
    for (int32_t j = o->K - 1; j > lv; j--) cnt_ge += h[j];
    /* cnt_ge = cnt(lv+1); walk j = lv+1, lv+2, ... keeping cnt(j) and cnt(j-1) */
    for (int32_t j = lv + 1; j < o->K; j++) {
        int32_t cnt_prev = cnt_ge + h[j - 1];    /* cnt(j-1) */
        int ok1 = cnt_ge <= o->up_max[gn(o, j)];
        int ok2 = cnt_prev >= o->dn_min[gn(o, j - 1)];
        if (ok1 && ok2) return j;
        cnt_ge -= h[j];                          /* cnt(j+1) */
    }
    fail(o, A_T1_LEVEL_RANGE);                   /* no level above satisfies both */
    return lv;
}

/* The implementation's insertion procedure (PLDS implementation details:
 * a filter and sort computes the desire-level of the vertices that move up),
 * counter mode.  Levels are processed from the lowest one holding an
 * Invariant-1 violator: the set S_l of violators at l is fixed, the
 * desire-level of each is computed from the levels before any of them moves,
 * and all of S_l move to their desire-levels together; the neighbours that
 * start to violate (at levels above l) and the movers that still violate at
 * their new level are processed when the loop reaches their level. */
static void insert_phase_jump(ora_t *o, const uint64_t *keys, int64_t k) {
    for (int64_t i = 0; i < k; i++)
        edge_counters(o, (int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu), +1);
    for (int64_t i = 0; i < k; i++) {
        int32_t ends[2] = {(int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu)};
        for (int e = 0; e < 2; e++) {
            int32_t x = ends[e];
            if (viol2(o, x)) fail(o, A_T2_INV2_INSERT);
            if (viol1(o, x) && o->qlev[x] != o->level[x]) {
                o->qlev[x] = o->level[x];
                queue(o, o->level[x], x);
                o->stats[12]++;
            }
        }
    }
    for (int32_t l = 0; l < o->K; l++) {
        vec_t *b = &o->bucket[l];
        if (b->n == 0) continue;
        o->movers.n = 0;
        for (int64_t i = 0; i < b->n; i++) {
            int32_t v = b->a[i];
            o->qlev[v] = -1;
            if (o->level[v] == l && !o->inset[v] && viol1(o, v)) {
                o->inset[v] = 1;
                vec_push(&o->movers, v);
            }
        }
        b->n = 0;
        if (o->movers.n == 0) continue;
        o->stats[2]++;
        o->stats[4] += o->movers.n;
        /* desire-levels of all movers from the levels before the round */
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->dl[v] = up_desire_level(o, v);
            if (o->dl[v] <= l) fail(o, A_T4_MOVE_UP);
        }
        /* neighbours that stay see each mover go from l to its desire-level */
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->stats[7] += o->deg[v];
            o->stats[8] += o->up[v];
            for (int32_t j = 0; j < o->deg[v]; j++) {
                int32_t w = o->adj[v][j];
                if (!o->inset[w]) adjust(o, w, l, o->dl[v]);
            }
        }
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->level[v] = o->dl[v];
            o->dl[v] = -1;
        }
        for (int64_t i = 0; i < o->movers.n; i++) recount(o, o->movers.a[i]);
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            for (int32_t j = -1; j < o->deg[v]; j++) {
                int32_t x = j < 0 ? v : o->adj[v][j];
                if (viol2(o, x)) fail(o, A_T2_INV2_INSERT);
                if (!viol1(o, x)) continue;
                if (o->level[x] <= l) fail(o, A_T4_MOVE_UP);
                if (o->qlev[x] != o->level[x]) {
                    o->qlev[x] = o->level[x];
                    queue(o, o->level[x], x);
                }
            }
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->inset[o->movers.a[i]] = 0;
    }
}

/* The same, full-scan mode: every level, every vertex, degrees recounted;
 * S_l = all vertices of level l violating Invariant 1. */
static void insert_phase_jump_scan(ora_t *o) {
    for (int32_t l = 0; l < o->K; l++) {
        o->movers.n = 0;
        for (int32_t v = 0; v < (int32_t)o->n; v++) {
            if (o->level[v] < l && viol1(o, v)) fail(o, A_T4_MOVE_UP);
            if (o->level[v] == l && viol1(o, v)) vec_push(&o->movers, v);
        }
        if (o->movers.n == 0) continue;
        o->stats[2]++;
        o->stats[4] += o->movers.n;
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->stats[7] += o->deg[v];
            o->stats[8] += count_up(o, v);
            o->old[v] = up_desire_level(o, v);
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->level[o->movers.a[i]] = o->old[o->movers.a[i]];
        for (int32_t v = 0; v < (int32_t)o->n; v++)
            if (viol2(o, v)) fail(o, A_T2_INV2_INSERT);
    }
}

/* ------------------------------------------------------------ deletions */
/* Algorithm 3 (RebalanceDeletions), counter mode.  Invariant-2 violators get
 * their desire-level; for l = 0,1,... every pending vertex whose
 * desire-level is l moves to l at once; afterwards every neighbour at level
 * >= l that violates Invariant 2 gets its desire-level recomputed. */
static void delete_phase_counters(ora_t *o, const uint64_t *keys, int64_t k) {
    for (int64_t i = 0; i < k; i++)
        edge_counters(o, (int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu), -1);
    for (int64_t i = 0; i < k; i++) {
        int32_t ends[2] = {(int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu)};
        for (int e = 0; e < 2; e++) {
            int32_t x = ends[e];
            if (viol1(o, x)) fail(o, A_T3_INV1_DELETE);
            if (o->dl[x] < 0 && viol2(o, x)) {
                o->dl[x] = desire_level(o, x);
                queue(o, o->dl[x], x);
                o->stats[13]++;
            }
        }
    }
    for (int32_t l = 0; l < o->K; l++) {
        vec_t *b = &o->bucket[l];
        if (b->n == 0) continue;
        o->movers.n = 0;
        for (int64_t i = 0; i < b->n; i++) {
            int32_t v = b->a[i];
            if (o->dl[v] == l && !o->inset[v]) {       /* stale entries skipped */
                o->inset[v] = 1;
                vec_push(&o->movers, v);
            }
        }
        b->n = 0;
        if (o->movers.n == 0) continue;
        o->stats[3]++;
        o->stats[5] += o->movers.n;
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            o->old[v] = o->level[v];
            o->stats[10] += o->deg[v];
            if (o->dl[v] >= o->level[v]) fail(o, A_T5_SMALLER);
        }
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            for (int32_t j = 0; j < o->deg[v]; j++) {
                int32_t w = o->adj[v][j];
                if (!o->inset[w]) adjust(o, w, o->old[v], l);
            }
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->level[o->movers.a[i]] = l;
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            recount(o, v);
            o->dl[v] = -1;
        }
        for (int64_t i = 0; i < o->movers.n; i++) {
            int32_t v = o->movers.a[i];
            if (viol1(o, v) || viol2(o, v)) fail(o, A_MOVER_VIOL);
            for (int32_t j = 0; j < o->deg[v]; j++) {
                int32_t w = o->adj[v][j];
                if (viol1(o, w)) fail(o, A_T3_INV1_DELETE);
                if (o->level[w] < l || !viol2(o, w)) continue;
                int32_t d = desire_level(o, w);
                if (d <= l) fail(o, A_T5_SMALLER);          /* Lemma smaller-level */
                if (o->dl[w] != d) {
                    o->dl[w] = d;
                    queue(o, d, w);
                }
            }
        }
        for (int64_t i = 0; i < o->movers.n; i++) o->inset[o->movers.a[i]] = 0;
    }
}

/* Algorithm 3, full-scan mode: at every level l the desire-level of every
 * Invariant-2 violator is recomputed from scratch and those equal to l move. */
static void delete_phase_scan(ora_t *o) {
    int32_t *d = (int32_t *)malloc((size_t)o->n * sizeof(int32_t));
    if (!d) {
        fail(o, A_FINAL);
        return;
    }
    for (int32_t l = 0; l < o->K; l++) {
        o->movers.n = 0;
        for (int32_t v = 0; v < (int32_t)o->n; v++) {
            if (viol1(o, v)) fail(o, A_T3_INV1_DELETE);
            d[v] = viol2(o, v) ? desire_level(o, v) : -1;
            if (d[v] >= 0 && d[v] < l) fail(o, A_T5_SMALLER);
            if (d[v] == l) vec_push(&o->movers, v);
        }
        if (o->movers.n == 0) continue;
        o->stats[3]++;
        o->stats[5] += o->movers.n;
        for (int64_t i = 0; i < o->movers.n; i++) o->stats[10] += o->deg[o->movers.a[i]];
        for (int64_t i = 0; i < o->movers.n; i++) o->level[o->movers.a[i]] = l;
    }
    free(d);
}

/* ---------------------------------------------------------------- update */
int ora_check(const ora_t *o) {
    for (int32_t v = 0; v < (int32_t)o->n; v++) {
        int32_t lv = o->level[v];
        if (lv < 0 || lv >= o->K) return -1;
        if (o->deg[v] == 0 && lv != 0) return -2;
        int32_t u = count_up(o, v), us = count_ups(o, v);
        if (o->mode == 0 && (u != o->up[v] || us != o->ups[v])) return -3;
        if (u > o->up_max[gn(o, lv)]) return -4;                       /* Inv. 1 */
        if (lv > 0 && us < o->dn_min[gn(o, lv - 1)]) return -5;       /* Inv. 2 */
    }
    return 0;
}

int ora_last_assert(const ora_t *o) { return o->assert_code; }

/* Algorithm 1: preprocess both lists, then RebalanceInsertions, then
 * RebalanceDeletions.  Ids are range-checked before anything changes. */
int ora_update(ora_t *o, const int32_t *ins, int64_t n_ins, const int32_t *del, int64_t n_del) {
    if (!o || n_ins < 0 || n_del < 0 || (n_ins && !ins) || (n_del && !del)) return ORA_EINVAL;
    if ((n_ins && !in_range(o, ins, n_ins)) || (n_del && !in_range(o, del, n_del))) return ORA_ERANGE;
    memset(o->stats, 0, sizeof(o->stats));
    o->assert_code = 0;
    int64_t cap = n_ins > n_del ? n_ins : n_del;
    uint64_t *keys = (uint64_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(uint64_t));
    if (!keys) return ORA_ENOMEM;
    int rc = 0;

    /* insertions: unique, then keep edges not yet present */
    int64_t k = canon_unique(ins, n_ins, keys), w = 0;
    for (int64_t i = 0; i < k; i++)
        if (!has_edge(o, (int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu))) keys[w++] = keys[i];
    o->stats[0] = w;
    rc = adj_apply(o, keys, w, 1);
    if (rc == 0 && w > 0) {
        if (o->jump) {
            if (o->mode == 0) insert_phase_jump(o, keys, w);
            else insert_phase_jump_scan(o);
        } else if (o->mode == 0) {
            insert_phase_counters(o, keys, w);
        } else {
            insert_phase_scan(o);
        }
    }

    /* deletions: unique, then keep edges present (after the insertions) */
    if (rc == 0) {
        k = canon_unique(del, n_del, keys);
        w = 0;
        for (int64_t i = 0; i < k; i++)
            if (has_edge(o, (int32_t)(keys[i] >> 32), (int32_t)(keys[i] & 0xffffffffu))) keys[w++] = keys[i];
        o->stats[1] = w;
        rc = adj_apply(o, keys, w, 0);
        if (rc == 0 && w > 0) {
            if (o->mode == 0) delete_phase_counters(o, keys, w);
            else delete_phase_scan(o);
        }
    }
    free(keys);
    if (rc) return rc;
    int32_t top = 0;
    for (int32_t v = 0; v < (int32_t)o->n; v++) top = o->level[v] > top ? o->level[v] : top;
    o->stats[11] = top;
    if (o->assert_code) return ORA_ESTATE;
    return 0;
}

void ora_levels(const ora_t *o, int32_t *out) { memcpy(out, o->level, (size_t)o->n * sizeof(int32_t)); }
void ora_degrees(const ora_t *o, int32_t *out) { memcpy(out, o->deg, (size_t)o->n * sizeof(int32_t)); }
void ora_stats(const ora_t *o, int64_t *out) { memcpy(out, o->stats, sizeof(o->stats)); }

/* Def. coreness estimate: (1+delta)^max(floor((level+1)/L) - 1, 0); an
 * isolated vertex gets 0 (experiments: coreness-0 vertices get estimate 0). */
void ora_estimate_exponent(const ora_t *o, int32_t *out) {
    for (int64_t v = 0; v < o->n; v++) {
        int32_t e = (o->level[v] + 1) / o->L - 1;
        out[v] = o->deg[v] == 0 ? -1 : (e > 0 ? e : 0);
    }
}

void ora_coreness(const ora_t *o, const int32_t *vs, int64_t count, double *out) {
    int64_t c = vs ? count : o->n;
    for (int64_t i = 0; i < c; i++) {
        int32_t v = vs ? vs[i] : (int32_t)i;
        if (v < 0 || v >= o->n) {
            out[i] = -1.0;
            continue;
        }
        int32_t e = (o->level[v] + 1) / o->L - 1;
        out[i] = o->deg[v] == 0 ? 0.0 : o->pow_tab[e > 0 ? e : 0];
    }
}

int64_t ora_edges(const ora_t *o, int32_t *out) {
    int64_t k = 0;
    for (int32_t u = 0; u < (int32_t)o->n; u++)
        for (int32_t j = 0; j < o->deg[u]; j++) {
            int32_t v = o->adj[u][j];
            if (u < v) {
                if (out) {
                    out[2 * k] = u;
                    out[2 * k + 1] = v;
                }
                k++;
            }
        }
    return k;
}

int ora_load_state(ora_t *o, const int32_t *edges, int64_t m, const int32_t *levels) {
    if (!o || m < 0 || (m && !edges) || !levels) return ORA_EINVAL;
    if (m && !in_range(o, edges, m)) return ORA_ERANGE;
    for (int64_t v = 0; v < o->n; v++) {
        free(o->adj[v]);
        o->adj[v] = NULL;
        o->deg[v] = o->acap[v] = 0;
        o->dl[v] = -1;
        o->qlev[v] = -1;
        o->level[v] = levels[v];
        if (levels[v] < 0 || levels[v] >= o->K) return ORA_EINVAL;
    }
    o->m = 0;
    uint64_t *keys = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
    if (!keys) return ORA_ENOMEM;
    int64_t k = canon_unique(edges, m, keys);
    int rc = adj_apply(o, keys, k, 1);
    free(keys);
    if (rc) return rc;
    for (int32_t v = 0; v < (int32_t)o->n; v++) recount(o, v);
    return ora_check(o);
}

/* ---------------------------------------------------------- exact cores */
/* Exact coreness by bucket peeling in the order of Matula-Beck: repeatedly
 * remove a vertex of minimum remaining degree; its coreness is the largest
 * minimum seen so far (Batagelj-Zaversnik O(m) bucket form). */
int ora_exact_coreness(int64_t n, const int32_t *edges, int64_t m, int32_t *core) {
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *nb = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    int32_t *d = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!off || !nb || !d || !fill) {
        free(off), free(nb), free(d), free(fill);
        return ORA_ENOMEM;
    }
    for (int64_t i = 0; i < m; i++) {
        d[edges[2 * i]]++;
        d[edges[2 * i + 1]]++;
    }
    for (int64_t v = 0; v < n; v++) off[v + 1] = off[v] + d[v];
    for (int64_t i = 0; i < m; i++) {
        int32_t a = edges[2 * i], b = edges[2 * i + 1];
        nb[off[a] + fill[a]++] = b;
        nb[off[b] + fill[b]++] = a;
    }
    int32_t md = 0;
    for (int64_t v = 0; v < n; v++) md = d[v] > md ? d[v] : md;
    int64_t *bin = (int64_t *)calloc((size_t)md + 1, sizeof(int64_t));
    int64_t *pos = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *vert = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!bin || !pos || !vert) {
        free(off), free(nb), free(d), free(fill), free(bin), free(pos), free(vert);
        return ORA_ENOMEM;
    }
    for (int64_t v = 0; v < n; v++) bin[d[v]]++;
    int64_t start = 0;
    for (int32_t x = 0; x <= md; x++) {
        int64_t c = bin[x];
        bin[x] = start;
        start += c;
    }
    for (int64_t v = 0; v < n; v++) {
        pos[v] = bin[d[v]];
        vert[pos[v]] = (int32_t)v;
        bin[d[v]]++;
    }
    for (int32_t x = md; x >= 1; x--) bin[x] = bin[x - 1];
    bin[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t v = vert[i];
        for (int64_t j = off[v]; j < off[v + 1]; j++) {
            int32_t u = nb[j];
            if (d[u] > d[v]) {
                int32_t du = d[u];
                int64_t pu = pos[u], pw = bin[du];
                int32_t w = vert[pw];
                if (u != w) {
                    pos[u] = pw;
                    vert[pu] = w;
                    pos[w] = pu;
                    vert[pw] = u;
                }
                bin[du]++;
                d[u]--;
            }
        }
    }
    for (int64_t v = 0; v < n; v++) core[v] = d[v];
    free(off), free(nb), free(d), free(fill), free(bin), free(pos), free(vert);
    return 0;
}
