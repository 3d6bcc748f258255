"""Pins of the static approximate k-core oracle (oracle/static_kcore.py,
Algorithm 6 of the static section).

Expected values come from the section's worked example (its figure is missing;
the graph is rebuilt from the text), hand-derived closed forms (paths,
cliques, stars) and the (2+eps)(1+eps) approximation bound against the exact
coreness by the k-core definition (brute force on tiny graphs) and by
bucket peeling (RMAT graphs).
"""
import random

import numpy as np
import pytest

import oracle as O
from brute_plds import kcore_by_definition
from oracle.static_kcore import rounds_cap, static_approx_kcore
from paper_2106_03824_amd import workloads as W


def test_worked_example():
    """eps = delta = 1: v, w, a, b have degree 2 (bucket ceil(log2 2) = 1),
    u, x, y, z degree >= 3 (bucket 2) and keep degree >= 3 once v, w, a, b
    are gone; bucket 1 is peeled first with estimate 2, then bucket 2 with 4.
    Rebuilt graph: a K4 on u, x, y, z (0..3) and the paths u-v-w-x, y-a-b-z."""
    E = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (4, 5), (6, 7), (4, 0), (5, 1), (6, 2), (7, 3)]
    est, trace = static_approx_kcore(8, E, 1.0, return_trace=True)
    assert est.tolist() == [4.0] * 4 + [2.0] * 4
    assert [bp for _, bp, _ in trace] == [1, 2]
    # eps = 1 gives delta = 2 and ceil(log_3 8) = 2 peels per threshold
    assert rounds_cap(8, 2.0) == 2


@pytest.mark.parametrize("s,eps,want", [(5, 1.0, 4.0), (6, 1.0, 8.0), (9, 1.0, 8.0), (10, 0.5, 1.5 ** 6)])
def test_clique(s, eps, want):
    """K_s: every vertex has degree s-1, all sit in bucket ceil(log_{1+eps}(s-1))
    and are peeled together with estimate (1+eps)^bucket."""
    E = [(i, j) for i in range(s) for j in range(i + 1, s)]
    est = static_approx_kcore(s + 2, E, eps)
    assert est[:s].tolist() == [want] * s and est[s:].tolist() == [0.0, 0.0]


@pytest.mark.parametrize("n", [2, 3, 7, 40])
def test_path_is_exact(n):
    """A path: the ends are in bucket 0 and peeled first; each round leaves new
    ends of induced degree <= 1, clamped to bucket 0; every estimate is 1."""
    E = [(i, i + 1) for i in range(n - 1)]
    assert static_approx_kcore(n, E, 1.0).tolist() == [1.0] * n


def test_star():
    """Star with d leaves: leaves (bucket 0) go first with estimate 1; the
    centre's C drops to max(0, ceil((1+eps)^-1)) = 1, bucket 0, estimate 1."""
    d = 20
    E = [(0, i) for i in range(1, d + 1)]
    assert static_approx_kcore(d + 1, E, 0.5).tolist() == [1.0] * (d + 1)


@pytest.mark.parametrize("seed", range(30))
def test_bound_tiny_brute(seed):
    rng = random.Random(seed)
    n = rng.choice([5, 8, 12])
    p = rng.choice([0.2, 0.4, 0.7])
    eps = rng.choice([0.25, 0.5, 1.0, 2.0])
    E = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    est = static_approx_kcore(n, E, eps)
    core = np.array(kcore_by_definition(n, E))
    nz = core > 0
    assert ((est == 0) == (core == 0)).all()
    c = (2 + eps) * (1 + eps)
    assert (est[nz] <= c * core[nz] * (1 + 1e-12)).all() and (core[nz] <= c * est[nz] * (1 + 1e-12)).all()


@pytest.mark.parametrize("scale,ef,seed", [(10, 8, 1), (12, 16, 2)])
@pytest.mark.parametrize("eps", [0.1, 0.5, 1.0, 2.0])
def test_bound_rmat(scale, ef, seed, eps):
    """(2+eps)(1+eps) = 2+eps' approximation, both ways."""
    n = 2 ** scale
    e = W.rmat(scale, ef * n, seed=seed)
    core = O.exact_coreness(n, e)
    est = static_approx_kcore(n, e, eps)
    nz = core > 0
    assert ((est == 0) == (core == 0)).all()
    r = np.maximum(est[nz] / core[nz], core[nz] / est[nz])
    assert r.max() <= (2 + eps) * (1 + eps) * (1 + 1e-12)


# ---- rules of the listing that the pins above do not exercise: each case
# below was derived by hand from Algorithm 6 under the reading above, and
# the docstring gives what the estimates would be without the rule.

def test_peel_cap_and_clamp_to_threshold():
    """eps = 1 (buckets ceil(log2 C); a continuation needs the next bucket
    within 3 * 2^t, i.e. at most t + 1), n = 6 so ceil(log_3 6) = 2 peels per
    threshold.  p=0, h=1, s=2, u1=3, u2=4, w=5; edges p-h, s-u1, s-u2,
    u1-w, u2-w, u1-h, u2-h, w-h; degrees 1,4,2,3,3,3, buckets 0,2,1,2,2,2.
    Threshold 0: peel {p} (estimate 1; h: C 3, bucket 2), then bucket 1 {s}
    (estimate 2; u1, u2: C 2, bucket 1).  Two peels: the cap ends the
    threshold.  Threshold 1: peel {u1, u2} (estimate 2); w and h lose two
    each: C = max(1, ceil(2^0)) = 1, bucket max(0, t=1) = 1; peel {w, h}
    with estimate 2.
    Without the cap the first threshold would go on and w, h would get
    bucket max(0, 0) = 0, estimate 1; without the clamp they would get
    bucket 0 under threshold 1, estimate 1 as well."""
    E = [(0, 1), (2, 3), (2, 4), (3, 5), (4, 5), (3, 1), (4, 1), (5, 1)]
    est, trace = static_approx_kcore(6, E, 1.0, return_trace=True)
    assert rounds_cap(6, 2.0) == 2
    assert est.tolist() == [1.0, 2.0, 2.0, 2.0, 2.0, 2.0]
    assert trace == [(0, 0, 1), (0, 1, 1), (1, 1, 2), (1, 1, 2)]


def test_clamp_to_threshold():
    """eps = 1, n = 8 (2 peels per threshold): a triangle a, b, v (0, 1, 2),
    an edge v-c and a K5 on c, d, e, f, g (3..7).  No vertex has degree 1,
    so the first threshold is bucket 1 (a, b).  Peeling {a, b} drops v's C
    to max(3 - 2, 1) = 1, bucket max(0, 1) = 1: v is peeled next in the same
    threshold with estimate 2; c's C goes to 4 (bucket 2).  The cap ends the
    threshold; threshold 2 peels the K5, estimate 4.  Without the clamp v
    would sit in bucket 0 and get estimate 1."""
    E = [(0, 1), (1, 2), (0, 2), (2, 3)] + [(a, b) for a in range(3, 8) for b in range(a + 1, 8)]
    est, trace = static_approx_kcore(8, E, 1.0, return_trace=True)
    assert est.tolist() == [2.0, 2.0, 2.0, 4.0, 4.0, 4.0, 4.0, 4.0]
    assert trace == [(1, 1, 2), (1, 1, 1), (2, 2, 5)]


EPS_GOLDEN = 0.6180339887498949   # (1+eps)^2 == 2+eps exactly in double arithmetic


def test_continuation_test_is_at_most():
    """At eps = 0.6180339887498949 the double powers give (1+eps)^2 == 2+eps
    exactly, so from threshold 0 the continuation test (1+eps)^next <=
    (2+eps)(1+eps)^t admits bucket 2 with equality.  No integer count has
    bucket 1 (it would need 1 < C <= 1.618); C = 2 has bucket 2, C = 3 and 4
    bucket 3.  n = 5 gives ceil(log_{4.236} 5) = 2 peels per threshold.
    p=0, h=1, s1=2, s2=3, w=4; edges p-h, s1-w, s2-w, s1-h, s2-h, w-h.
    Threshold 0: peel {p} (estimate 1; h: C 3, bucket 3); bucket 2 {s1, s2}
    passes with equality and is peeled in the same threshold (estimate
    (1+eps)^2); w and h drop to C = max(1, 1) = 1, bucket 0.  The cap ends
    the threshold; threshold 0 again peels {w, h} with estimate 1.
    With a strict test the first threshold would stop after {p}; threshold
    2 would peel {s1, s2}, floor w and h at ceil(1+eps) = 2 (bucket 2) and
    give them (1+eps)^2 as well."""
    pw = [1.0, 1.0 + EPS_GOLDEN]
    pw.append(pw[1] * (1.0 + EPS_GOLDEN))
    assert pw[2] == 2.0 + EPS_GOLDEN
    E = [(0, 1), (2, 4), (3, 4), (2, 1), (3, 1), (4, 1)]
    est, trace = static_approx_kcore(5, E, EPS_GOLDEN, return_trace=True)
    assert rounds_cap(5, 2.0 / EPS_GOLDEN) == 2
    assert est.tolist() == [1.0, 1.0, pw[2], pw[2], 1.0]
    assert trace == [(0, 0, 1), (0, 2, 2), (0, 0, 2)]


@pytest.mark.parametrize("eps", [0.05, 0.1, 0.25, 0.5, 1.0, 2.0, EPS_GOLDEN])
def test_floor_never_raises_a_bucket_above_the_threshold(eps):
    """The mathematical fact that makes the floor ceil((1+eps)^(t-1)) inert
    under this reading: a threshold t is always the bucket of some integer
    count C0 >= 1 (thresholds are smallest buckets, and buckets are b(C) or
    earlier thresholds), and then ceil((1+eps)^(t-1)) <= C0 <= (1+eps)^t, so
    the floor's own bucket is at most t and the clamp to t decides alone."""
    from oracle.static_kcore import powers
    pw = powers(1.0 + eps, 5000.0)
    for c0 in range(1, 5000):
        t = int(np.searchsorted(pw, float(c0), side="left"))
        if t >= 1:
            floor = int(np.ceil(pw[t - 1]))
            assert np.searchsorted(pw, float(floor), side="left") <= t
