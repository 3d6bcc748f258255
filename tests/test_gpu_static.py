"""GPU parity of the static approximate k-core (Algorithm 6) against the oracle
(oracle/static_kcore.py): estimates are powers of 1+eps from the same
repeated-multiplication table, compared bit for bit."""
import random
import sys

import numpy as np
import pytest

import oracle.static_kcore as SKO
from paper_2106_03824_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = None


def lib():
    global P
    if P is None:
        from paper_2106_03824_amd import plds as _P
        _P.lib()
        P = _P
    return P


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def same(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.int64), np.asarray(b, np.float64).view(np.int64))


def test_worked_example():
    say("static worked example")
    E = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (4, 5), (6, 7), (4, 0), (5, 1), (6, 2), (7, 3)]
    g = lib().PLDS(8)
    assert g.insert(E) == 0
    est = g.static_kcore(1.0).cpu().numpy()
    assert est.tolist() == [4.0] * 4 + [2.0] * 4
    lv = g.levels().clone()
    g.static_kcore(0.5)
    assert torch.equal(lv, g.levels())           # the dynamic state is untouched


@pytest.mark.parametrize("seed", range(10))
def test_random_small(seed):
    rng = random.Random(seed)
    n = rng.choice([5, 20, 64, 300])
    p = rng.choice([0.05, 0.2, 0.5])
    eps = rng.choice([0.1, 0.25, 0.5, 1.0, 2.0])
    say("static small", seed, n, p, eps)
    E = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    g = lib().PLDS(n)
    if E:
        assert g.insert(E) == 0
    assert same(g.static_kcore(eps).cpu().numpy(), SKO.static_approx_kcore(n, E, eps))


@pytest.mark.parametrize("scale,ef,seed", [(12, 8, 1), (14, 16, 2), (16, 16, 3)])
@pytest.mark.parametrize("eps", [0.1, 0.5, 2.0])
def test_rmat(scale, ef, seed, eps):
    n = 2 ** scale
    say("static rmat", scale, ef, seed, eps)
    e = W.rmat(scale, ef * n, seed=seed)
    g = lib().PLDS(n)
    assert g.insert(e) == 0
    assert same(g.static_kcore(eps).cpu().numpy(), SKO.static_approx_kcore(n, e, eps))


def test_after_updates_and_errors():
    n = 2 ** 12
    e = W.rmat(12, 8 * n, seed=4)
    say("static after updates")
    g = lib().PLDS(n)
    assert g.insert(e) == 0
    assert g.delete(W.sample_edges(e, len(e) // 3, 5)) == 0
    cur, _ = g.dump()
    assert same(g.static_kcore(1.0).cpu().numpy(), SKO.static_approx_kcore(n, cur.cpu().numpy(), 1.0))
    say("static errors")
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    for bad in (0.0, -1.0, float("nan"), 1e-4):
        with pytest.raises(lib().PLDSError):
            lib().plds_static_kcore(g.h, bad, out)
    m = lib().MultiPLDS([10, 20])
    with pytest.raises(lib().PLDSError):
        lib().plds_static_kcore(m.h, 1.0, torch.empty(30, dtype=torch.float64, device="cuda"))
    say("static empty graph")
    z = lib().PLDS(100)
    assert (z.static_kcore(1.0).cpu().numpy() == 0).all()


@pytest.mark.parametrize("name,n,E,eps", [
    ("peel cap and clamp", 6, [(0, 1), (2, 3), (2, 4), (3, 5), (4, 5), (3, 1), (4, 1), (5, 1)], 1.0),
    ("clamp", 8, [(0, 1), (1, 2), (0, 2), (2, 3)] + [(a, b) for a in range(3, 8) for b in range(a + 1, 8)], 1.0),
    ("continuation at equality", 5, [(0, 1), (2, 4), (3, 4), (2, 1), (3, 1), (4, 1)], 0.6180339887498949),
])
def test_rule_pins(name, n, E, eps):
    """The hand-derived graphs that pin the peel cap, the clamp to the
    threshold and the continuation test's equality case (see
    tests/test_oracle_static.py), on the GPU."""
    say("static rule pin", name)
    g = lib().PLDS(n)
    assert g.insert(E) == 0
    assert same(g.static_kcore(eps).cpu().numpy(), SKO.static_approx_kcore(n, E, eps))
