/*
 * plds_oracle.h -- sequential CPU oracle of the parallel level data structure
 * (PLDS) for batch-dynamic (2+eps)-approximate k-core decomposition
 * (Liu, Shi, Yu, Dhulipala, Shun, SPAA'22, arXiv 2106.03824).
 *
 * TEST INFRASTRUCTURE ONLY.  This file and plds_oracle.c define what the GPU
 * library must compute; they are used by tests/, by the smoke check and by the
 * CPU-baseline leg of the benchmark, never by the library itself.  They share
 * no code, header, table or helper with the HIP path.
 *
 * Everything is single-threaded, plain C, with sorted neighbour arrays and
 * plain per-level lists.  Functions cite the passage of the paper they follow.
 *
 * Error codes: 0 ok, -1 invalid argument, -2 vertex id out of range (the whole
 * call is rejected and nothing changes), -3 out of memory, -5 an assertion of
 * the paper's analysis failed inside the oracle (see ora_last_assert()).
 */
#ifndef PLDS_ORACLE_H
#define PLDS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora ora_t;

/* mode 0: counter mode -- up/up* degrees kept as counters, candidate sets
 *         kept in per-level lists, following Algorithms 2-3 step by step.
 * mode 1: full-scan mode -- every level 0..K-1 is visited and every vertex is
 *         re-examined with degrees recounted from the adjacency.  Slow; used
 *         to pin mode 0 on tiny graphs.
 * levels_per_group > 0 overrides the levels per group; -1 selects the
 * experiments' PLDSOpt variant, ceil(log_{1+delta} n / 50); 0 (or any other
 * value <= 0) the default 4*ceil(log_{1+delta} n). */
ora_t *ora_create(int64_t n, double delta, double lambda, int32_t levels_per_group, int32_t mode);
/* As ora_create; coeff > 0 (at least 1) replaces the Invariant-1 coefficient
 * 2 + 3/lambda (the experiments' heuristic parameters use 1.1), jump != 0
 * moves insertion violators straight to their desire-level (PLDS
 * implementation details) instead of one level at a time. */
ora_t *ora_create_ex(int64_t n, double delta, double lambda, int32_t levels_per_group, int32_t mode, double coeff,
                     int32_t jump);
void ora_destroy(ora_t *o);

/* out[0..7] = n, m, t = ceil(log_{1+delta} n), L, G, K, mode, 0 */
void ora_info(const ora_t *o, int64_t *out);
/* host arrays of G entries each */
void ora_tables(const ora_t *o, int32_t *up_max, int32_t *dn_min, double *pow_tab);

/* Algorithm 1: all insertions (Algorithm 2), then all deletions (Algorithm 3).
 * ins/del are int32 [count][2]; either may be NULL with count 0. */
int ora_update(ora_t *o, const int32_t *ins, int64_t n_ins, const int32_t *del, int64_t n_del);

void ora_levels(const ora_t *o, int32_t *out);   /* [n] */
void ora_degrees(const ora_t *o, int32_t *out);  /* [n] */
/* coreness estimate; vs == NULL means all n vertices (count ignored) */
void ora_coreness(const ora_t *o, const int32_t *vs, int64_t count, double *out);
/* exponent i of the estimate (1+delta)^i, -1 for an isolated vertex */
void ora_estimate_exponent(const ora_t *o, int32_t *out);

/* full check of Invariants 1 and 2, deg=0 => level 0, 0 <= level < K, and
 * (mode 0) counters equal to recounted degrees.  0 if all hold, else <0. */
int ora_check(const ora_t *o);
int ora_last_assert(const ora_t *o);

/* per-call statistics, 16 int64 (layout documented in plds_oracle.c) */
void ora_stats(const ora_t *o, int64_t *out);

/* current edge set, canonical (u<v), sorted; returns m.  out may be NULL. */
int64_t ora_edges(const ora_t *o, int32_t *out);
/* replace the state by (edges, levels); edges must be unique canonical-able
 * pairs.  Returns ora_check() of the loaded state. */
int ora_load_state(ora_t *o, const int32_t *edges, int64_t m, const int32_t *levels);

/* exact coreness by bucket peeling (Matula-Beck / Batagelj-Zaversnik) */
int ora_exact_coreness(int64_t n, const int32_t *edges, int64_t m, int32_t *core);

#ifdef __cplusplus
}
#endif
#endif
