"""Oracle of the static approximate k-core decomposition (the static section,
Algorithm 6).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may use it.

Plain numpy, one synchronous peeling round at a time, in Algorithm 6's order
and notation, read as follows (the prose, the listing and the worked example
of the section disagree; this reading reproduces the worked example):

* C[v] starts at deg(v); a vertex with C >= 1 sits in bucket
  b(C) = ceil(log_{1+eps} C), the least b >= 0 with (1+eps)^b >= C, the
  powers formed by repeated double multiplication; vertices without edges
  get estimate 0 and are never bucketed;
* an outer iteration takes the smallest bucket as its threshold index t and
  peels that bucket; after each peel the alive neighbours v of the peeled
  set I lose r_v (their neighbours in I): C[v] = max(C[v] - r_v,
  ceil((1+eps)^(t-1))), and their bucket becomes max(b(C[v]), t);
* the outer iteration peels the next smallest bucket in turn while it is
  within the threshold ((1+eps)^next <= (2+eps)(1+eps)^t) and fewer than
  ceil(log_{1+delta} n) peels were made in it (delta = 2/eps);
* a vertex peeled from bucket b gets the estimate (1+eps)^b (the worked
  example's estimates 2 and 4 for buckets 1 and 2 at eps = 1).

Pins (tests/test_oracle_static.py): the worked example, closed forms, the
approximation bound, and hand-derived graphs on which the peel cap, the
clamp of new buckets to t and the `<=` of the continuation test each change
an estimate.  The floor ceil((1+eps)^(t-1)) is kept as the listing states
it, but it never changes a bucket under this reading: a threshold t is
always the bucket of some integer count C0 (a smallest bucket, and buckets
are b(C) or earlier thresholds), so ceil((1+eps)^(t-1)) <= C0 <= (1+eps)^t
and a count at or below the floor is clamped to t anyway.  That step alone
is parity unpinned: no input can show it.
"""
import numpy as np


def powers(base, upto):
    """[base^0, base^1, ...] by repeated double multiplication, until >= upto."""
    p = [1.0]
    while p[-1] < upto:
        p.append(p[-1] * base)
    return np.array(p, dtype=np.float64)


def rounds_cap(n, delta):
    """ceil(log_{1+delta} n): the least r >= 0 with (1+delta)^r >= n."""
    x, r = 1.0, 0
    while x < n:
        x *= 1.0 + delta
        r += 1
    return r


def static_approx_kcore(n, edges, eps, return_trace=False):
    """Estimates (float64 [n]) of Algorithm 6 with bucket base 1+eps."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    e = np.unique(np.sort(e, axis=1), axis=0)
    a, b = e[:, 0], e[:, 1]
    deg = np.bincount(np.concatenate([a, b]), minlength=n).astype(np.int64)
    pw = powers(1.0 + eps, max(int(deg.max()) if n else 1, 1) + 1)
    R = rounds_cap(n, 2.0 / eps)

    def bucket(c):
        return np.searchsorted(pw, c.astype(np.float64), side="left")

    C = deg.copy()
    alive = deg > 0
    est = np.zeros(n, dtype=np.float64)
    B = np.zeros(n, dtype=np.int64)
    B[alive] = bucket(C[alive])
    trace = []
    while alive.any():
        t = int(B[alive].min())
        bp, peels = t, 0
        while True:
            I = alive & (B == bp)
            est[I] = pw[bp]
            alive &= ~I
            trace.append((t, bp, int(I.sum())))
            # r_v: neighbours of v in I, for the alive v
            r = np.bincount(b[I[a] & alive[b]], minlength=n) + np.bincount(a[I[b] & alive[a]], minlength=n)
            hit = r > 0
            floor = int(np.ceil(pw[t - 1])) if t >= 1 else 1
            C[hit] = np.maximum(C[hit] - r[hit], floor)
            B[hit] = np.maximum(bucket(C[hit]), t)
            peels += 1
            if not alive.any():
                break
            nb = int(B[alive].min())
            if peels < R and pw[nb] <= (2.0 + eps) * pw[t]:
                bp = nb
            else:
                break
    return (est, trace) if return_trace else est
