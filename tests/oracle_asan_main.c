/* Exercises every entry point of the C oracle (oracle/plds_oracle.c) on
 * random tiny streams, so that the oracle can be built with AddressSanitizer
 * and UndefinedBehaviorSanitizer and checked for memory errors
 * (tests/test_oracle_asan.py).  Inputs come from a plain 64-bit LCG; the
 * program holds none of the method's arithmetic. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/plds_oracle.h"

static uint64_t s = 88172645463325252ull;
static uint32_t rnd(uint32_t k) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)((s >> 33) % (k ? k : 1));
}

static int fail(const char *what, int line) {
    fprintf(stderr, "oracle driver: %s failed at line %d\n", what, line);
    return 1;
}
#define REQ(x)                                   \
    do {                                         \
        if (!(x)) return fail(#x, __LINE__);     \
    } while (0)

int main(void) {
    const int32_t ns[] = {1, 2, 7, 40, 300};
    const int32_t lpgs[] = {0, 3, -1};
    for (int ni = 0; ni < 5; ni++)
        for (int li = 0; li < 3; li++)
            for (int mode = 0; mode < 2; mode++) {
                int32_t n = ns[ni];
                ora_t *o = ora_create(n, mode ? 1.0 : 0.4, 3.0, lpgs[li], mode);
                REQ(o);
                int64_t info[8];
                ora_info(o, info);
                int32_t G = (int32_t)info[4];
                int32_t *up = malloc(sizeof(int32_t) * G), *dn = malloc(sizeof(int32_t) * G);
                double *pw = malloc(sizeof(double) * G);
                ora_tables(o, up, dn, pw);
                int32_t *lv = malloc(sizeof(int32_t) * n), *dg = malloc(sizeof(int32_t) * n);
                double *est = malloc(sizeof(double) * n);
                int32_t *ex = malloc(sizeof(int32_t) * n), *core = malloc(sizeof(int32_t) * n);
                for (int it = 0; it < 8; it++) {
                    int64_t ki = rnd(4 * n + 2), kd = rnd(2 * n + 2);
                    int32_t *ins = malloc(sizeof(int32_t) * 2 * (ki + 1)), *del = malloc(sizeof(int32_t) * 2 * (kd + 1));
                    for (int64_t i = 0; i < 2 * ki; i++) ins[i] = (int32_t)rnd(n);   /* self-loops and duplicates too */
                    int64_t m = ora_edges(o, NULL);
                    int32_t *cur = malloc(sizeof(int32_t) * 2 * (m + 1));
                    ora_edges(o, cur);
                    for (int64_t i = 0; i < kd; i++) {
                        if (m && rnd(4)) {
                            int64_t j = rnd((uint32_t)m);
                            del[2 * i] = cur[2 * j], del[2 * i + 1] = cur[2 * j + 1];
                        } else {
                            del[2 * i] = (int32_t)rnd(n), del[2 * i + 1] = (int32_t)rnd(n);
                        }
                    }
                    REQ(ora_update(o, ki ? ins : NULL, ki, kd ? del : NULL, kd) == 0);
                    REQ(ora_check(o) == 0);
                    ora_levels(o, lv);
                    ora_degrees(o, dg);
                    ora_coreness(o, NULL, 0, est);
                    ora_estimate_exponent(o, ex);
                    int32_t q[3] = {0, n - 1, n / 2};
                    double qo[3];
                    ora_coreness(o, q, 3, qo);
                    int64_t st[16];
                    ora_stats(o, st);
                    m = ora_edges(o, NULL);
                    int32_t *e = malloc(sizeof(int32_t) * 2 * (m + 1));
                    REQ(ora_edges(o, e) == m);
                    REQ(ora_exact_coreness(n, e, m, core) == 0);
                    ora_t *o2 = ora_create(n, mode ? 1.0 : 0.4, 3.0, lpgs[li], 0);
                    REQ(o2 && ora_load_state(o2, e, m, lv) == 0);
                    ora_destroy(o2);
                    /* an out-of-range id rejects the call */
                    int32_t bad[2] = {0, n};
                    REQ(ora_update(o, bad, 1, NULL, 0) == -2);
                    free(e), free(cur), free(ins), free(del);
                }
                free(up), free(dn), free(pw), free(lv), free(dg), free(est), free(ex), free(core);
                ora_destroy(o);
            }
    REQ(ora_create(0, 0.4, 3.0, 0, 0) == NULL);
    REQ(ora_create(10, -1.0, 3.0, 0, 0) == NULL);
    printf("oracle driver ok\n");
    return 0;
}
