"""Pins of the oracle's two options of the PLDSOpt row: the heuristic
Invariant-1 coefficient (experiments section: 2 + 3/lambda replaced by 1.1)
and the implementation's insertion procedure (PLDS implementation details:
vertices that move up go straight to their desire-level).

Expected values are derived by hand from Algorithms 1-3 under these readings
(docstrings), or come from the independent exact-arithmetic Python PLDS of
tests/brute_plds.py, which takes the desire-level literally from its
definition by trying every level; the counter and full-scan modes of the C
oracle must also agree with each other."""
import math
import random
from fractions import Fraction

import pytest

import oracle as O
from brute_plds import BrutePLDS, exact_params
from paper_2106_03824_amd import workloads as W


def clique(s, off=0):
    return [(off + a, off + b) for a in range(s) for b in range(a + 1, s)]


def test_coefficient_tables_exact():
    """up_max[g] = floor(1.1 (1+delta)^g) with 1.1 as the rational 11/10 and
    (1+delta)^g = 7^g / 5^g; dn_min unchanged."""
    o = O.Oracle(2 ** 20, 0.4, 3.0, coeff=1.1)
    up, dn, _ = o.tables()
    for g in range(o.G):
        assert up[g] == math.floor(Fraction(11, 10) * Fraction(7, 5) ** g)
        assert dn[g] == math.ceil(Fraction(7, 5) ** g)
    # the first caps: 1, 1, 2, 3, 4, 5, 8 -- below the floor in groups 1 and 5
    assert list(up[:7]) == [1, 1, 2, 3, 4, 5, 8] and list(dn[:7]) == [1, 2, 2, 3, 4, 6, 8]


def test_coefficient_below_one_rejected():
    with pytest.raises(ValueError):
        O.Oracle(10, 0.4, 3.0, coeff=0.9)


def test_coefficient_path():
    """c = 1.1, n = 5 (L = 4 * 5 = 20, levels 0..19 in group 0, cap 1).
    Path 0-1-2-3-4: at level 0 the inner vertices 1, 2, 3 have up = 2 > 1 and
    move to 1 together; there 1 and 3 count one up-neighbour (2), 2 counts
    two (1, 3) and moves to 2, where it counts none.  Levels 0,1,2,1,0 (with
    2 + 3/lambda = 3 nothing moves)."""
    o = O.Oracle(5, 0.4, 3.0, coeff=1.1)
    assert o.insert([(0, 1), (1, 2), (2, 3), (3, 4)]) == 0
    assert o.levels().tolist() == [0, 1, 2, 1, 0]
    assert o.stats()["sweeps_ins"] == 2 and o.stats()["moves_up"] == 4
    assert o.check() == 0


def test_coefficient_clique():
    """c = 1.1, K4 on n = 4 (t = 5, L = 20): every vertex has up = 3 and the
    four climb together to the first group with floor(1.1 * 1.4^g) >= 3,
    g = 3 (caps 1, 1, 2, 3): level 60."""
    o = O.Oracle(4, 0.4, 3.0, coeff=1.1)
    assert o.insert(clique(4)) == 0
    assert o.levels().tolist() == [60] * 4 and o.check() == 0


def test_jump_single_vertex():
    """Standard coefficient, n = 8 (t = 7, L = 28; caps 3, 4, 5, ... per group).
    A K5 on 1..5 climbs to level 28 (the first level of group 1, cap 4).
    Then vertex 0 joins all five.  Level by level (Algorithm 2) it would
    climb 0 -> 29 in 29 sweeps; its desire-level is the first level above 0
    where up(0) <= cap: 29 (at 1..28 all five count, cap 3 or 4; at 29
    none), with up*(0) = 5 >= 2 there: one round.  The K5 then has up 5 > 4
    at 28 and moves to 29 (vertex 0 is their only neighbour above 28); at 29
    all six violate and climb together one level per round (each mover's
    other neighbours are co-movers still at the round's level) to 56, the
    first level of group 2 (cap 5): 1 + 1 + 27 rounds, 1 + 5 + 27 * 6
    moves."""
    o = O.Oracle(8, 0.4, 3.0, jump=True)
    assert o.insert(clique(5, 1)) == 0
    assert o.levels().tolist() == [0] + [28] * 5 + [0, 0]   # 6 and 7 stay isolated
    assert o.insert([(0, v) for v in range(1, 6)]) == 0
    assert o.levels().tolist() == [56] * 6 + [0, 0]
    st = o.stats()
    assert st["sweeps_ins"] == 29 and st["moves_up"] == 1 + 5 + 27 * 6
    assert o.check() == 0


def rand_batch(rng, n, k):
    return [(rng.randrange(n), rng.randrange(n)) for _ in range(k)]


@pytest.mark.parametrize("seed", range(30))
def test_options_equal_python_brute(seed):
    """The counter-mode C oracle with the coefficient and/or the jump equals
    the literal Python PLDS with the same options, batch by batch."""
    rng = random.Random(7000 + seed)
    n = rng.randrange(4, 13)
    coeff = [None, 1.1, 1.5][seed % 3]
    jump = seed % 2 == 0 or coeff is None
    delta, lam = rng.choice([(Fraction(2, 5), 3), (Fraction(1), 3), (Fraction(4, 5), 12)])
    Lg = rng.choice([0, 2, 3])
    o = O.Oracle(n, float(delta), float(lam), Lg, coeff=coeff or 0.0, jump=jump)
    br = BrutePLDS(n, delta, lam, Lg, coeff=coeff, jump=jump)
    for _ in range(5):
        ins = rand_batch(rng, n, rng.randrange(0, 3 * n))
        dele = rand_batch(rng, n, rng.randrange(0, n))
        cur = o.edges().tolist()
        if cur and rng.random() < 0.7:
            dele += rng.sample(cur, rng.randrange(1, len(cur) + 1))
        assert o.update(ins, dele) == 0, o.last_assert()
        br.update(ins, dele)
        assert list(o.levels()) == br.level
        assert o.check() == 0 and br.invariants_hold()
        st = o.stats()
        assert (st["sweeps_ins"], st["sweeps_del"]) == (br.sweeps_ins, br.sweeps_del)


@pytest.mark.parametrize("seed", range(30))
def test_options_counter_equals_scan(seed):
    rng = random.Random(8000 + seed)
    n = rng.randrange(8, 50)
    coeff = [0.0, 1.1][seed % 2]
    Lg = rng.choice([0, 2, 3, -1])
    a = O.Oracle(n, 0.4, 3.0, Lg, mode=0, coeff=coeff, jump=True)
    b = O.Oracle(n, 0.4, 3.0, Lg, mode=1, coeff=coeff, jump=True)
    for _ in range(6):
        ins = rand_batch(rng, n, rng.randrange(0, 4 * n))
        cur = a.edges().tolist()
        dele = rng.sample(cur, rng.randrange(0, len(cur) + 1)) if cur else []
        assert a.update(ins, dele) == 0 and b.update(ins, dele) == 0
        assert (a.levels() == b.levels()).all()
        sa, sb = a.stats(), b.stats()
        for k in ("sweeps_ins", "sweeps_del", "moves_up", "moves_down", "applied_ins", "applied_del"):
            assert sa[k] == sb[k], k
        assert a.check() == 0


@pytest.mark.parametrize("scale", [10, 12])
def test_jump_keeps_invariants_and_bound_on_rmat(scale):
    """The jump keeps both invariants after every batch, hence the 4.2
    approximation bound (Lemma decomp-bound) against exact peeling, and
    needs no more rounds than Algorithm 2 has sweeps."""
    n = 2 ** scale
    e = W.permute_edges(W.rmat(scale, 8 * n, seed=4), 4401)
    j = O.Oracle(n, 0.4, 3.0, jump=True)
    a = O.Oracle(n, 0.4, 3.0)
    for c in (e[: len(e) // 2], e[len(e) // 2:]):
        assert j.insert(c) == 0 and a.insert(c) == 0
        assert j.check() == 0
        assert j.stats()["sweeps_ins"] <= a.stats()["sweeps_ins"]
    d = W.sample_edges(e, len(e) // 3, 4402)
    assert j.delete(d) == 0 and j.check() == 0
    cur = j.edges()
    core = O.exact_coreness(n, cur)
    est = j.coreness()
    nz = core > 0
    r = [max(x / k, k / x) for x, k in zip(est[nz], core[nz])]
    assert max(r) <= 4.2 * (1 + 1e-12)
