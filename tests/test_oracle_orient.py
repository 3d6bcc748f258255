"""Pins of the orientation and densest-subgraph oracle (oracle/orient.py).

Expected values come from hand-worked examples, from Algorithm 5's flip
conditions carried out literally over the moved vertices' edges (an
independent procedure), from the out-degree bound of the orientation
corollary and from brute-force densest subgraphs of tiny graphs.
"""
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle as O
import oracle.orient as OR
from paper_2106_03824_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_orient_rule_by_hand():
    """Lower level to higher level; equal levels from the smaller id."""
    levels = [0, 1, 1, 3, 5, 2]
    edges = [(1, 0), (2, 1), (3, 2), (0, 3), (4, 5), (5, 4), (2, 5)]
    want = [(0, 1), (1, 2), (2, 3), (0, 3), (5, 4), (5, 4), (2, 5)]
    assert OR.orient(levels, edges).tolist() == [list(p) for p in want]


def test_flip_example_by_hand():
    """Path 0-1-2, all at level 0 (edges 0->1, 1->2); vertex 1 moves to
    level 1: 0->1 stays, 1->2 becomes 2->1, so F = {(1, 2)} as before."""
    e = [(0, 1), (1, 2)]
    f = OR.flips([0, 0, 0], [0, 1, 0], e, e)
    assert f.tolist() == [[1, 2]]
    # an edge inserted by the call is not a flip; a deleted one is not either
    f = OR.flips([0, 0, 0, 0], [0, 1, 0, 0], [(0, 1), (1, 2)], [(0, 1), (1, 3)])
    assert f.tolist() == []


def test_oriented_updates_example():
    """J: insertion {2,3} after the call (levels 0 -> 2 for vertex 2: 3->2
    since level(3)=1 < 2), deletion {0,2} before it (0->2, equal levels)."""
    ji, jd = OR.oriented_updates([0, 0, 0, 1], [0, 0, 2, 1], [(2, 3)], [(0, 2)])
    assert ji.tolist() == [[3, 2]] and jd.tolist() == [[0, 2]]


def test_applied_updates_batch_semantics():
    before = [(0, 1), (1, 2)]
    a_ins, a_del = OR.applied_updates(before, [(1, 0), (3, 2), (2, 3), (4, 4)], [(2, 1), (5, 6), (3, 2)])
    assert a_ins.tolist() == [[2, 3]]
    assert a_del.tolist() == [[1, 2], [2, 3]]


def _algorithm5(H, levels_after, moved, adj):
    """Algorithm 5's first loop, literally: for every edge searched by a
    vertex that moved, with key (u, v), u < v, and stored value H (0: u->v,
    1: v->u), report it (as stored) when the levels after the batch call for
    the other direction."""
    F = set()
    for x in moved:
        for y in adj[x]:
            u, v = min(x, y), max(x, y)
            if (u, v) not in H:
                continue                      # inserted by this batch: no stored orientation
            lu, lv = levels_after[u], levels_after[v]
            if H[(u, v)] == 0 and (lu > lv or (lu == lv and v < u)):
                F.add((u, v))
            elif H[(u, v)] == 1 and (lv > lu or (lu == lv and u < v)):
                F.add((v, u))
    return sorted(F)


@pytest.mark.parametrize("seed", range(25))
def test_flips_equal_algorithm5_procedure(seed):
    rng = random.Random(seed)
    n = rng.choice([6, 10, 16, 30])
    o = O.Oracle(n, 0.4, 3.0, rng.choice([0, 2, 3]))
    H = {}
    for it in range(8):
        lv0, e0 = o.levels(), o.edges()
        ins = [(rng.randrange(n), rng.randrange(n)) for _ in range(rng.randrange(0, 3 * n))]
        cur = e0.tolist()
        dele = rng.sample(cur, rng.randrange(0, len(cur) + 1)) if cur and it % 2 else []
        assert o.update(ins or None, dele or None) == 0
        lv1, e1 = o.levels(), o.edges()
        moved = [x for x in range(n) if lv0[x] != lv1[x]]
        adj = {x: [] for x in range(n)}
        for a, b in e1.tolist():
            adj[a].append(b)
            adj[b].append(a)
        # edges deleted by the call are not searched any more; H keeps the survivors
        live = OR.canonical_set(e1)
        Hs = {k: h for k, h in H.items() if k in live}
        want = _algorithm5(Hs, lv1, moved, adj)
        got = [tuple(p) for p in OR.flips(lv0, lv1, e0, e1).tolist()]
        assert got == want, (seed, it)
        # the stored orientation after the batch
        H = {(min(a, b), max(a, b)): (0 if t == min(a, b) else 1)
             for (a, b), (t, h) in zip(e1.tolist(), OR.orient(lv1, e1).tolist())}


@pytest.mark.parametrize("scale,ef,seed", [(8, 8, 1), (10, 8, 2), (10, 16, 3)])
def test_out_degree_bound(scale, ef, seed):
    """Orientation corollary: a vertex's out-neighbours are at its level or
    above, so its out-degree is at most up(v), which Invariant 1 keeps at
    most the cap of its group."""
    n = 2 ** scale
    e = W.rmat(scale, ef * n, seed=seed)
    o = O.Oracle(n, 0.4, 3.0)
    for c in np.array_split(W.permute_edges(e, seed), 3):
        assert o.insert(c) == 0
    assert o.delete(W.sample_edges(e, len(e) // 4, seed + 9)) == 0
    lv, cur = o.levels(), o.edges()
    up_max, _, _ = o.tables()
    L = o.info()["L"]
    outd = OR.out_degrees(n, lv, cur)
    up = np.zeros(n, dtype=np.int64)
    for a, b in cur.tolist():
        up[a] += lv[b] >= lv[a]
        up[b] += lv[a] >= lv[b]
    assert (outd <= up).all()
    assert (outd <= np.asarray(up_max)[lv // L]).all()
    # the reverse orientation breaks the bound on these skewed graphs
    rev = np.bincount(OR.orient(lv, cur)[:, 1], minlength=n)
    assert (rev > np.asarray(up_max)[lv // L]).any()


def _densest_brute(n, edges):
    best = 0.0
    es = [tuple(p) for p in edges]
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            s = set(S)
            m = sum(1 for a, b in es if a in s and b in s)
            best = max(best, m / k)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_densest_value_bound(seed):
    """Densest-subgraph corollary: with degeneracy d, d/2 <= rho* <= d, and
    every estimate is within c = (2+3/lambda)(1+delta) of the coreness, so
    rho*/c <= max estimate <= 2c rho*."""
    rng = random.Random(100 + seed)
    n = rng.choice([6, 8, 9])
    p = rng.choice([0.3, 0.5, 0.8])
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    o = O.Oracle(n, 0.4, 3.0)
    assert o.insert(edges or None) == 0
    rho = _densest_brute(n, edges)
    val = OR.densest_subgraph_value(o.coreness())
    c = GOLD["parameter_recipe"]["bound_delta0.4_lambda3"]
    if not edges:
        assert val == 0.0
        return
    assert rho / c <= val * (1 + 1e-12)
    assert val <= 2 * c * rho * (1 + 1e-12)
