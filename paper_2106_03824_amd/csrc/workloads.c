/*
 * workloads.c -- seeded synthetic graph and batch generators.
 *
 * These produce inputs only: they hold none of the PLDS arithmetic and are
 * shared by the GPU library's tests/benchmark and by the CPU oracle's tests.
 *
 * Random numbers are counter based: draw(seed, stream, i) is the i-th output
 * of a SplitMix64 sequence (Steele, Lea, Flood 2014) started from a key
 * derived from (seed, stream), so every draw is a pure function of its index.
 *
 *   rmat      R-MAT (Chakrabarti, Zhan, Faloutsos 2004): every candidate edge
 *             picks one of four quadrants per bit with probabilities a,b,c,d;
 *             candidates are canonicalised (min,max), self-loops dropped and
 *             the first occurrence of each pair kept, in candidate order, until
 *             the requested number of unique edges exists; the vertex ids are
 *             then relabelled by a seeded random permutation.
 *   er        G(n,p) by geometric skipping (Batagelj, Brandes 2005).
 *   permute   seeded Fisher-Yates permutation of an edge list.
 *   new_pairs uniform pairs u != v absent from a given edge set and distinct.
 *   sample    uniform sample without replacement from an edge list.
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(mix64(seed + GOLDEN) ^ (stream * 0xd1342543de82ef95ULL + 0x2545f4914f6cdd1dULL));
}
/* i-th SplitMix64 output from state `key` */
static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GOLDEN); }
static inline double unit53(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }
/* uniform integer in [0, bound) by the multiply-high map */
static inline uint64_t below(uint64_t r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

/* ------------------------------------------------------------ hash set */
typedef struct {
    uint64_t *slot;
    uint64_t mask;
} hset_t;
#define HEMPTY 0xffffffffffffffffULL

static int hset_init(hset_t *h, int64_t expected) {
    uint64_t cap = 16;
    while (cap < (uint64_t)(expected * 2 + 16)) cap <<= 1;
    h->slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!h->slot) return -1;
    memset(h->slot, 0xff, cap * sizeof(uint64_t));
    h->mask = cap - 1;
    return 0;
}
/* returns 1 if newly inserted, 0 if present */
static int hset_add(hset_t *h, uint64_t k) {
    uint64_t i = mix64(k) & h->mask;
    for (;;) {
        if (h->slot[i] == HEMPTY) {
            h->slot[i] = k;
            return 1;
        }
        if (h->slot[i] == k) return 0;
        i = (i + 1) & h->mask;
    }
}
static int hset_has(const hset_t *h, uint64_t k) {
    uint64_t i = mix64(k) & h->mask;
    for (;;) {
        if (h->slot[i] == HEMPTY) return 0;
        if (h->slot[i] == k) return 1;
        i = (i + 1) & h->mask;
    }
}
static inline uint64_t ekey(int32_t u, int32_t v) {
    uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
    return (a << 32) | b;
}

/* ------------------------------------------------------------ generators */
/* Seeded permutation of [0, n) (Fisher-Yates, draws from `stream`). */
int wl_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm) {
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

/* Candidate i of an R-MAT stream: `scale` quadrant choices, one draw each. */
static inline void rmat_cand(uint64_t key, int32_t scale, uint64_t i, double a, double ab, double abc,
                             int32_t *uo, int32_t *vo) {
    int32_t u = 0, v = 0;
    for (int32_t j = 0; j < scale; j++) {
        double r = unit53(draw(key, i * (uint64_t)scale + (uint64_t)j));
        int32_t ub = r >= ab, vb = (r >= a && r < ab) || r >= abc;
        u = (u << 1) | ub;
        v = (v << 1) | vb;
    }
    *uo = u;
    *vo = v;
}

static void relabel_edges(int64_t n, int64_t m, uint64_t seed, int32_t *out);

/* Reference form: one candidate after the other, a set of the pairs seen. */
int64_t wl_rmat_seq(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, int32_t relabel,
                    int32_t *out) {
    int64_t n = (int64_t)1 << scale;
    if (scale < 1 || scale > 30 || m < 0 || m > n * (n - 1) / 2) return -1;
    hset_t h;
    if (hset_init(&h, m)) return -1;
    uint64_t key = stream_key(seed, 1);
    double ab = a + b, abc = a + b + c;
    int64_t got = 0, cand = 0;
    while (got < m) {
        int32_t u, v;
        rmat_cand(key, scale, (uint64_t)cand, a, ab, abc, &u, &v);
        cand++;
        if (u == v) continue;
        if (!hset_add(&h, ekey(u, v))) continue;
        out[2 * got] = u;
        out[2 * got + 1] = v;
        got++;
    }
    free(h.slot);
    if (relabel) relabel_edges(n, m, seed, out);
    return cand;
}

/* ---- the same stream, generated by threads.  The edges kept are the first
 * m distinct pairs in candidate order, exactly as above: a shared table maps
 * every pair seen to the least candidate index that drew it; once the
 * candidates processed hold m distinct pairs, the m smallest such indices
 * are the kept candidates, and they are written out in index order. */
static int wl_threads(void) {
    const char *e = getenv("WL_THREADS");
    if (!e) e = getenv("OMP_NUM_THREADS");
    long t = e ? strtol(e, NULL, 10) : sysconf(_SC_NPROCESSORS_ONLN);
    if (t < 1) t = 1;
    if (t > 64) t = 64;
    return (int)t;
}

typedef struct {
    _Atomic uint64_t *key;  /* HEMPTY or the pair */
    _Atomic uint32_t *first; /* least candidate index of the pair */
    uint64_t cap;
    _Atomic int64_t distinct;
    _Atomic int32_t full;
} ftab_t;

typedef struct {
    ftab_t *t;
    uint64_t ckey, lo, hi;
    int32_t scale;
    double a, ab, abc;
    /* output pass */
    _Atomic uint64_t *bits;
    int64_t m, base;
    int32_t *out;
} rjob_t;

static void *rmat_scan_worker(void *arg) {
    rjob_t *j = (rjob_t *)arg;
    ftab_t *t = j->t;
    int64_t added = 0;
    for (uint64_t i = j->lo; i < j->hi && !atomic_load_explicit(&t->full, memory_order_relaxed); i++) {
        int32_t u, v;
        rmat_cand(j->ckey, j->scale, i, j->a, j->ab, j->abc, &u, &v);
        if (u == v) continue;
        uint64_t k = ekey(u, v);
        uint64_t s = (uint64_t)(((unsigned __int128)mix64(k) * t->cap) >> 64);
        for (uint64_t probe = 0;; probe++) {
            if (probe == t->cap) {
                atomic_store(&t->full, 1);
                break;
            }
            uint64_t cur = atomic_load_explicit(&t->key[s], memory_order_relaxed);
            if (cur == HEMPTY) {
                uint64_t expect = HEMPTY;
                if (atomic_compare_exchange_strong(&t->key[s], &expect, k)) {
                    added++;
                    cur = k;
                } else {
                    cur = expect;
                }
            }
            if (cur == k) {
                uint32_t f = atomic_load_explicit(&t->first[s], memory_order_relaxed);
                while ((uint32_t)i < f &&
                       !atomic_compare_exchange_weak(&t->first[s], &f, (uint32_t)i)) {
                }
                break;
            }
            s = s + 1 == t->cap ? 0 : s + 1;
        }
    }
    atomic_fetch_add(&t->distinct, added);
    return NULL;
}

static void *rmat_mark_worker(void *arg) {
    rjob_t *j = (rjob_t *)arg;
    ftab_t *t = j->t;
    for (uint64_t s = j->lo; s < j->hi; s++) {
        if (atomic_load_explicit(&t->key[s], memory_order_relaxed) == HEMPTY) continue;
        uint32_t f = atomic_load_explicit(&t->first[s], memory_order_relaxed);
        atomic_fetch_or_explicit(&j->bits[f >> 6], 1ull << (f & 63), memory_order_relaxed);
    }
    return NULL;
}

static void *rmat_emit_worker(void *arg) {
    rjob_t *j = (rjob_t *)arg;
    int64_t pos = j->base;
    for (uint64_t w = j->lo; w < j->hi && pos < j->m; w++) {
        uint64_t word = atomic_load_explicit(&j->bits[w], memory_order_relaxed);
        while (word && pos < j->m) {
            uint64_t i = (w << 6) + (uint64_t)__builtin_ctzll(word);
            word &= word - 1;
            int32_t u, v;
            rmat_cand(j->ckey, j->scale, i, j->a, j->ab, j->abc, &u, &v);
            j->out[2 * pos] = u;
            j->out[2 * pos + 1] = v;
            pos++;
        }
    }
    return NULL;
}

static void run_jobs(rjob_t *jobs, int nt, void *(*fn)(void *)) {
    pthread_t th[64];
    for (int i = 1; i < nt; i++)
        if (pthread_create(&th[i], NULL, fn, &jobs[i])) {
            fn(&jobs[i]);
            th[i] = 0;
        }
    fn(&jobs[0]);
    for (int i = 1; i < nt; i++)
        if (th[i]) pthread_join(th[i], NULL);
}

/* R-MAT with `m` unique undirected edges on 2^scale vertices.  out: [m][2].
 * Returns the number of candidates drawn, or -1.  Threads: WL_THREADS, else
 * OMP_NUM_THREADS, else the online processors; the result does not depend on
 * the thread count. */
int64_t wl_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, int32_t relabel,
                int32_t *out) {
    int64_t n = (int64_t)1 << scale;
    if (scale < 1 || scale > 30 || m < 0 || m > n * (n - 1) / 2) return -1;
    int nt = wl_threads();
    if (nt == 1 || m < (1 << 16)) return wl_rmat_seq(scale, m, a, b, c, seed, relabel, out);
    ftab_t t;
    t.cap = (uint64_t)(m * 5 / 2) + 1024;
    t.key = (_Atomic uint64_t *)malloc(t.cap * sizeof(uint64_t));
    t.first = (_Atomic uint32_t *)malloc(t.cap * sizeof(uint32_t));
    if (!t.key || !t.first) {
        free((void *)t.key);
        free((void *)t.first);
        return wl_rmat_seq(scale, m, a, b, c, seed, relabel, out);
    }
    memset((void *)t.key, 0xff, t.cap * sizeof(uint64_t));
    memset((void *)t.first, 0xff, t.cap * sizeof(uint32_t));
    atomic_init(&t.distinct, 0);
    atomic_init(&t.full, 0);
    rjob_t jobs[64];
    rjob_t proto = {0};
    proto.t = &t;
    proto.ckey = stream_key(seed, 1);
    proto.scale = scale;
    proto.a = a;
    proto.ab = a + b;
    proto.abc = a + b + c;
    proto.m = m;
    proto.out = out;
    uint64_t C = 0;
    int ok = 1;
    while (atomic_load(&t.distinct) < m) {
        int64_t need = m - atomic_load(&t.distinct);
        uint64_t step = (uint64_t)(need + need / 2) + 4096;
        if (C + step >= (uint64_t)UINT32_MAX ||
            (uint64_t)atomic_load(&t.distinct) + step > t.cap * 17 / 20) {
            ok = 0;    /* index or table limit: take the reference path */
            break;
        }
        for (int i = 0; i < nt; i++) {
            jobs[i] = proto;
            jobs[i].lo = C + step * (uint64_t)i / (uint64_t)nt;
            jobs[i].hi = C + step * (uint64_t)(i + 1) / (uint64_t)nt;
        }
        run_jobs(jobs, nt, rmat_scan_worker);
        if (atomic_load(&t.full)) {
            ok = 0;
            break;
        }
        C += step;
    }
    int64_t cand = -1;
    if (ok) {
        uint64_t nw = (C + 63) / 64;
        _Atomic uint64_t *bits = (_Atomic uint64_t *)calloc(nw, sizeof(uint64_t));
        int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
        if (!bits || !cnt) {
            ok = 0;
        } else {
            for (int i = 0; i < nt; i++) {
                jobs[i] = proto;
                jobs[i].bits = bits;
                jobs[i].lo = t.cap * (uint64_t)i / (uint64_t)nt;
                jobs[i].hi = t.cap * (uint64_t)(i + 1) / (uint64_t)nt;
            }
            run_jobs(jobs, nt, rmat_mark_worker);
            /* word ranges per thread and their starting output positions */
            for (int i = 0; i < nt; i++) {
                uint64_t lo = nw * (uint64_t)i / (uint64_t)nt, hi = nw * (uint64_t)(i + 1) / (uint64_t)nt;
                int64_t k = 0;
                for (uint64_t w = lo; w < hi; w++) k += __builtin_popcountll(atomic_load(&bits[w]));
                cnt[i + 1] = cnt[i] + k;
                jobs[i] = proto;
                jobs[i].bits = bits;
                jobs[i].lo = lo;
                jobs[i].hi = hi;
            }
            for (int i = 0; i < nt; i++) jobs[i].base = cnt[i];
            run_jobs(jobs, nt, rmat_emit_worker);
            /* candidates drawn by the reference form: index of the m-th kept one, plus one */
            int64_t seen = 0;
            for (uint64_t w = 0; w < nw && cand < 0; w++) {
                uint64_t word = atomic_load(&bits[w]);
                int64_t pc = __builtin_popcountll(word);
                if (seen + pc < m) {
                    seen += pc;
                    continue;
                }
                while (word) {
                    uint64_t i = (w << 6) + (uint64_t)__builtin_ctzll(word);
                    word &= word - 1;
                    if (++seen == m) {
                        cand = (int64_t)i + 1;
                        break;
                    }
                }
            }
        }
        free((void *)bits);
        free(cnt);
    }
    free((void *)t.key);
    free((void *)t.first);
    if (!ok) return wl_rmat_seq(scale, m, a, b, c, seed, relabel, out);
    if (relabel) relabel_edges(n, m, seed, out);
    return cand;
}

static void relabel_edges(int64_t n, int64_t m, uint64_t seed, int32_t *out) {
    int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!perm) return;
    wl_permutation(n, seed, 2, perm);
    for (int64_t i = 0; i < 2 * m; i++) out[i] = perm[out[i]];
    free(perm);
}

/* G(n,p) by geometric skipping over the pairs (v,w), w < v.  Writes at most
 * cap edges; returns the number of edges of the graph (may exceed cap: call
 * again with a larger buffer), or -1. */
int64_t wl_er(int64_t n, double p, uint64_t seed, int32_t *out, int64_t cap) {
    if (n < 2 || !(p > 0) || p >= 1) return -1;
    uint64_t key = stream_key(seed, 3);
    double lq = log(1.0 - p);
    int64_t v = 1, w = -1, k = 0;
    uint64_t i = 0;
    while (v < n) {
        double r = unit53(draw(key, i++));
        w += 1 + (int64_t)floor(log(1.0 - r) / lq);
        while (w >= v && v < n) {
            w -= v;
            v++;
        }
        if (v < n) {
            if (k < cap) {
                out[2 * k] = (int32_t)v;
                out[2 * k + 1] = (int32_t)w;
            }
            k++;
        }
    }
    return k;
}

/* Seeded permutation of an edge list in place. */
int wl_permute_edges(int32_t *edges, int64_t m, uint64_t seed, uint64_t stream) {
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = m - 1; i > 0; i--) {
        int64_t j = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t0 = edges[2 * i], t1 = edges[2 * i + 1];
        edges[2 * i] = edges[2 * j];
        edges[2 * i + 1] = edges[2 * j + 1];
        edges[2 * j] = t0;
        edges[2 * j + 1] = t1;
    }
    return 0;
}

/* `count` distinct uniform pairs u != v of [0,n) absent from `edges`. */
int wl_new_pairs(int64_t n, const int32_t *edges, int64_t m, int64_t count, uint64_t seed, uint64_t stream,
                 int32_t *out) {
    if (n < 2 || count < 0 || count > n * (n - 1) / 2 - m) return -1;
    hset_t h;
    if (hset_init(&h, m + count)) return -1;
    for (int64_t i = 0; i < m; i++) hset_add(&h, ekey(edges[2 * i], edges[2 * i + 1]));
    uint64_t key = stream_key(seed, stream);
    int64_t got = 0;
    uint64_t i = 0;
    while (got < count) {
        int32_t u = (int32_t)below(draw(key, i), (uint64_t)n);
        int32_t v = (int32_t)below(draw(key, i + 1), (uint64_t)n);
        i += 2;
        if (u == v || !hset_add(&h, ekey(u, v))) continue;
        out[2 * got] = u;
        out[2 * got + 1] = v;
        got++;
    }
    free(h.slot);
    return 0;
}

/* `count` edges drawn uniformly without replacement from `edges`
 * (partial Fisher-Yates over an index array). */
int wl_sample_edges(const int32_t *edges, int64_t m, int64_t count, uint64_t seed, uint64_t stream,
                    int32_t *out) {
    if (count < 0 || count > m) return -1;
    int64_t *idx = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!idx) return -1;
    for (int64_t i = 0; i < m; i++) idx[i] = i;
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < count; i++) {
        int64_t j = i + (int64_t)below(draw(key, (uint64_t)i), (uint64_t)(m - i));
        int64_t t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
        out[2 * i] = edges[2 * idx[i]];
        out[2 * i + 1] = edges[2 * idx[i] + 1];
    }
    free(idx);
    return 0;
}

/* 1 if (u,v) in the edge set given as a list (helper for test filtering). */
int wl_filter_present(const int32_t *edges, int64_t m, const int32_t *query, int64_t q, uint8_t *present) {
    hset_t h;
    if (hset_init(&h, m)) return -1;
    for (int64_t i = 0; i < m; i++) hset_add(&h, ekey(edges[2 * i], edges[2 * i + 1]));
    for (int64_t i = 0; i < q; i++) present[i] = (uint8_t)hset_has(&h, ekey(query[2 * i], query[2 * i + 1]));
    free(h.slot);
    return 0;
}

/* uniform draws for Python-side seeded choices: out[i] = draw(seed,stream,i) */
int wl_draws(uint64_t seed, uint64_t stream, int64_t count, uint64_t *out) {
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < count; i++) out[i] = draw(key, (uint64_t)i);
    return 0;
}
