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
