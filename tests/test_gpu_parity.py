"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Levels, coreness estimates and the per-batch sweep/move counts are integer
or table-gathered results and must agree bit for bit.  Every case prints its
name before touching the GPU.
"""
import math
import random
import sys

import numpy as np
import pytest

import oracle as O
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


STAT_KEYS = (("applied_ins", "applied_ins"), ("applied_del", "applied_del"), ("sweeps_ins", "sweeps_ins"),
             ("sweeps_del", "sweeps_del"), ("moves_up", "moves_up"), ("moves_down", "moves_down"),
             ("viol_ins0", "viol_ins0"), ("viol_del0", "viol_del0"))


class Pair:
    """A GPU handle and an oracle fed the same batches."""

    def __init__(self, n, delta=0.4, lam=3.0, L=0, sweep_mode=1, direct=False):
        """sweep_mode 0: one cooperative launch; 1: step kernels (prebuilt
        graphs) with climbing steps for large groups; 2: without climbing
        steps; 3: climbing steps for groups of any size.  direct: step
        kernels launched one by one instead of from the step graphs (what
        kernel timing selects): True or "ins" for the insertion steps (the
        preparation kernel timed), "del" for the deletion steps (the
        deletion scan timed)."""
        self.g = lib().PLDS(n, delta, lam, L)
        lib().plds_set_sweep_mode(self.g.h, sweep_mode)
        if direct:
            lib().plds_set_timing(self.g.h, "del_scan" if direct == "del" else "ins_prep")
        self.o = O.Oracle(n, delta, lam, L)
        self.n = n

    def step(self, ins=None, dele=None, check_state=True):
        rg = self.g.update(ins, dele, check=False)
        ro = self.o.update(ins, dele)
        assert rg == ro == 0, (rg, ro)
        self.compare(check_state)

    def compare(self, check_state=True):
        lg = self.g.levels().cpu().numpy()
        lo = self.o.levels()
        bad = np.flatnonzero(lg != lo)
        assert bad.size == 0, f"{bad.size} levels differ, first {bad[:5]}: gpu {lg[bad[:5]]} oracle {lo[bad[:5]]}"
        cg = self.g.coreness().cpu().numpy()
        co = self.o.coreness()
        assert np.array_equal(cg.view(np.int64), co.view(np.int64))
        sg, so = self.g.stats(), self.o.stats()
        for kg, ko in STAT_KEYS:
            assert sg[kg] == so[ko], (kg, sg[kg], so[ko])
        assert (self.g.degrees().cpu().numpy() == self.o.degrees()).all()
        if check_state:
            assert self.g.check() == 0


def test_thresholds_match_oracle():
    for n, d, l, L in [(2 ** 12, 0.4, 3.0, 0), (2 ** 20, 0.4, 3.0, 0), (2 ** 24, 0.4, 3.0, 0), (1000, 1.0, 3.0, 3),
                       (5000, 0.2, 6.0, 0), (1, 0.4, 3.0, 0), (2 ** 20, 0.4, 3.0, -1), (10 ** 6, 0.1, 3.0, -1)]:
        say("thresholds", n, d, l, L)
        g = lib().PLDS(n, d, l, L)
        o = O.Oracle(n, d, l, L)
        assert (g.t, g.L, g.G, g.K) == (o.t, o.L, o.G, o.K)
        up, dn, pw = g.thresholds()
        ou, od, opw = o.tables()
        assert up == list(ou) and dn == list(od)
        assert np.array_equal(np.array(pw).view(np.int64), opw.view(np.int64))
        g.close()


def test_worked_examples():
    say("insertion example")
    p = Pair(8, 0.4, 3.0, 3)
    u, v, w, x, y, z, a, b = range(8)
    edges = [(x, v), (x, y), (x, z), (x, b), (w, y), (w, z), (w, a), (u, a)]
    levels = [2, 3, 2, 3, 3, 3, 2, 3]
    assert p.g.load(edges, levels) == 0 and p.o.load_state(edges, levels) == 0
    p.step(ins=[(u, v), (u, x), (x, w)])
    lv = p.g.levels().cpu().numpy()
    assert lv[w] == 3 and lv[x] == 4
    say("deletion example")
    p = Pair(7, 1.0, 3.0, 3)
    x, y, z, w, q, s, t = range(7)
    edges = [(x, y), (x, z), (y, z), (y, w), (w, q), (y, s), (y, t), (s, t)]
    levels = [4, 5, 5, 1, 0, 1, 1]
    assert p.g.load(edges, levels) == 0 and p.o.load_state(edges, levels) == 0
    p.step(dele=[(x, z), (y, w)])
    lv = p.g.levels().cpu().numpy()
    assert (lv[x], lv[z], lv[y]) == (3, 3, 4)
    assert p.g.coreness(torch.tensor([y], dtype=torch.int32, device="cuda")).item() == 1.0


@pytest.mark.parametrize("s", [4, 10, 30])
def test_clique_and_star(s):
    say("clique/star", s)
    p = Pair(64)
    e = [(i, j) for i in range(s) for j in range(i + 1, s)] + [(40, 40 + k) for k in range(1, 20)]
    p.step(ins=e)
    p.step(dele=e[: len(e) // 2])
    p.step(dele=e)
    assert (p.g.levels().cpu().numpy() == 0).all()


def test_batch_semantics():
    say("batch semantics")
    p = Pair(10)
    p.step(ins=[(1, 2), (2, 1), (1, 2), (3, 3), (4, 5)])
    assert p.g.stats()["applied_ins"] == 2
    p.step(ins=[(2, 1)])
    p.step(dele=[(6, 7), (7, 7)])
    p.step(ins=[(6, 7)], dele=[(7, 6), (1, 2)])
    e, _ = p.g.dump()
    assert sorted(map(tuple, e.cpu().numpy().tolist())) == [(4, 5)]
    p.step(ins=np.zeros((0, 2), np.int32), dele=np.zeros((0, 2), np.int32))


def test_out_of_range_rejected_state_unchanged():
    say("out of range")
    g = lib().PLDS(10)
    assert g.insert([(i, j) for i in range(6) for j in range(i + 1, 6)]) == 0
    lv = g.levels().cpu().numpy().copy()
    assert g.update(ins=[(0, 9)], dele=[(0, 10)], check=False) == lib().PLDS_ERANGE
    assert g.update(ins=[(-1, 2)], check=False) == lib().PLDS_ERANGE
    assert (g.levels().cpu().numpy() == lv).all() and g.info()["m"] == 15
    assert g.check() == 0
    out = g.coreness(torch.tensor([3, 11], dtype=torch.int32, device="cuda")).cpu().numpy()
    assert out[1] == -1.0
    assert lib().plds_sync(g.h) == lib().PLDS_ERANGE
    assert lib().plds_sync(g.h) == 0


@pytest.mark.parametrize("seed", range(12))
def test_random_small(seed):
    rng = random.Random(seed)
    n = rng.choice([8, 20, 64, 200])
    L = rng.choice([0, 0, 2, 3, -1])
    delta, lam = rng.choice([(0.4, 3.0), (1.0, 3.0), (0.2, 6.0)])
    say("random small", seed, n, L, delta, lam)
    p = Pair(n, delta, lam, L, sweep_mode=seed % 4, direct={1: "ins", 3: "del"}.get(seed % 5, False))
    for it in range(6):
        ins = [(rng.randrange(n), rng.randrange(n)) for _ in range(rng.randrange(0, 4 * n))]
        cur = p.o.edges().tolist()
        dele = rng.sample(cur, rng.randrange(0, len(cur) + 1)) if cur and it % 2 else []
        p.step(ins=ins or None, dele=dele or None)


def test_rmat_tiny_config():
    """RMAT n=2^12 with 32,768 unique edges (seed 1), one insertion batch of
    10^4 new uniform pairs, one deletion batch of 10^4 sampled edges."""
    n = 2 ** 12
    e = W.rmat(12, 32768, seed=1)
    say("rmat tiny: build")
    p = Pair(n)
    p.step(ins=e)
    say("rmat tiny: insert 1e4")
    ins = W.new_pairs(n, e, 10 ** 4, 1001)
    p.step(ins=ins)
    say("rmat tiny: delete 1e4")
    cur = p.o.edges()
    dele = W.sample_edges(cur, 10 ** 4, 1002)
    p.step(dele=dele)
    say("rmat tiny: mixed")
    cur = p.o.edges()
    p.step(ins=W.new_pairs(n, cur, 5000, 1003), dele=W.sample_edges(cur, 5000, 1004))


@pytest.mark.parametrize("mode,direct", [(0, False), (1, False), (1, True), (1, "del"), (2, False), (3, False),
                                         (3, True)])
def test_rmat_multi_batch(mode, direct):
    """RMAT scale 14, edge factor 16, built in 4 insertion batches, then mixed
    and deletion batches, each compared with the oracle; every way of running
    the insertion level loop (one cooperative launch; kernels per part with
    or without climbing steps, replayed from a graph or launched one by one)."""
    n = 2 ** 14
    e = W.permute_edges(W.rmat(14, 16 * n, seed=3), 2001)
    p = Pair(n, sweep_mode=mode, direct=direct)
    for i, c in enumerate(np.array_split(e, 4)):
        say("rmat14 build", i)
        p.step(ins=c)
    cur = p.o.edges()
    say("rmat14 mixed")
    p.step(ins=W.new_pairs(n, cur, 20000, 2002), dele=W.sample_edges(cur, 20000, 2003))
    say("rmat14 delete")
    p.step(dele=W.sample_edges(p.o.edges(), 50000, 2004))


@pytest.mark.parametrize("mode", [1, 3])
def test_rmat_multi_batch_pldsopt(mode):
    """The RMAT scale-14 stream of test_rmat_multi_batch with the PLDSOpt
    level structure (ceil(log_{1+delta} n / 50) levels per group)."""
    n = 2 ** 14
    e = W.permute_edges(W.rmat(14, 16 * n, seed=3), 2001)
    p = Pair(n, L=lib().PLDS_LPG_OPT, sweep_mode=mode)
    assert p.g.L == p.o.L == 1
    for i, c in enumerate(np.array_split(e, 4)):
        say("rmat14 pldsopt build", i)
        p.step(ins=c)
    cur = p.o.edges()
    say("rmat14 pldsopt mixed")
    p.step(ins=W.new_pairs(n, cur, 20000, 2002), dele=W.sample_edges(cur, 20000, 2003))
    say("rmat14 pldsopt delete")
    p.step(dele=W.sample_edges(p.o.edges(), 50000, 2004))


def test_er_graph():
    n = 3000
    e = W.er(n, 12.0 / (n - 1), seed=9)
    say("er", n, len(e))
    p = Pair(n)
    p.step(ins=e)
    p.step(dele=W.sample_edges(e, len(e) // 2, 10))


def test_load_dump_roundtrip_and_determinism():
    n = 2 ** 12
    e = W.rmat(12, 20000, seed=4)
    say("dump/load")
    a = lib().PLDS(n)
    assert a.insert(e) == 0
    ed, lv = a.dump()
    b = lib().PLDS(n)
    assert b.load(ed, lv) == 0
    ins = W.new_pairs(n, e, 3000, 11)
    assert a.insert(ins) == 0 and b.insert(ins) == 0
    assert torch.equal(a.levels(), b.levels())
    o = O.Oracle(n)
    assert o.load_state(ed.cpu().numpy(), lv.cpu().numpy()) == 0
    assert o.insert(ins) == 0
    assert (o.levels() == a.levels().cpu().numpy()).all()
    say("determinism")
    c = lib().PLDS(n)
    assert c.insert(e) == 0 and c.insert(ins) == 0
    assert torch.equal(a.levels(), c.levels())


def test_load_state_rejects_bad_levels():
    say("load rejects")
    g = lib().PLDS(8, 0.4, 3.0, 3)
    star = [(0, i) for i in range(1, 6)]
    assert g.load(star, [0] * 8, check=False) == lib().PLDS_ESTATE     # centre up 5 > 3
    assert g.load([(0, 1)], [0, 0, 0, 0, 0, 0, 0, 0], check=False) == 0
    assert g.check() == 0
