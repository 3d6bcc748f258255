"""Batched form: one multi-graph handle holding independent graphs of uneven
size (each with its own levels per group and thresholds) must put every
graph through exactly the states it goes through alone -- compared with a
plain handle per graph and with the CPU oracle per graph, after every batch.
"""
import random
import sys

import numpy as np
import pytest

import oracle as O
from paper_2106_03824_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def make_graphs(k, seed, nmin_log=6, nmax_log=12):
    rng = random.Random(seed)
    gs = []
    for i in range(k):
        if i % 2 == 0:
            n = int(round(2 ** rng.uniform(nmin_log, nmax_log)))
            e = W.er(n, rng.uniform(4, 32) / max(n - 1, 1), seed=seed * 1000 + i)
        else:
            sc = rng.randint(nmin_log, nmax_log)
            n = 2 ** sc
            e = W.rmat(sc, min(8 * n, n * (n - 1) // 4), seed=seed * 1000 + i)
        gs.append((n, e))
    return gs


def run_case(k, seed, rounds, with_oracle, mode=None):
    from paper_2106_03824_amd import plds as P
    rng = random.Random(seed + 7)
    gs = make_graphs(k, seed)
    ns = [n for n, _ in gs]
    say("multi", k, "graphs, n from", min(ns), "to", max(ns), "sweep mode", mode)
    mg = P.MultiPLDS(ns)
    singles = [P.PLDS(n) for n in ns]
    if mode is not None:
        P.plds_set_sweep_mode(mg.h, mode)
    oras = [O.Oracle(n) for n in ns] if with_oracle else None
    assert len(set(gi["L"] for gi in mg.graphs)) > 1     # graphs really differ in levels per group
    cur = [e for _, e in gs]

    def compare(tag):
        lv = mg.levels()
        cg = mg.coreness()
        for g in range(k):
            a = mg.graph_levels(g, lv).cpu().numpy()
            b = singles[g].levels().cpu().numpy()
            assert np.array_equal(a, b), f"{tag}: graph {g} differs from its own handle"
            ca = cg[mg.base[g]:mg.base[g] + ns[g]].cpu().numpy()
            assert np.array_equal(ca.view(np.int64), singles[g].coreness().cpu().numpy().view(np.int64))
            if oras:
                assert np.array_equal(a, oras[g].levels()), f"{tag}: graph {g} differs from the oracle"
        assert mg.check() == 0

    # build: one insertion batch per graph in one call
    say("multi build")
    mg.update_multi(ins=cur)
    for g in range(k):
        singles[g].insert(cur[g])
        if oras:
            assert oras[g].insert(cur[g]) == 0
    compare("build")
    for r in range(rounds):
        ins, dele = [], []
        for g in range(k):
            what = rng.choice(["ins", "del", "mix", "none"])
            n = ns[g]
            a = W.new_pairs(n, cur[g], rng.randint(1, max(2, n)), seed * 100 + 10 * r + g) \
                if what in ("ins", "mix") else None
            d = W.sample_edges(cur[g], rng.randint(1, max(1, len(cur[g]) // 3)), seed * 100 + 10 * r + g + 5) \
                if what in ("del", "mix") and len(cur[g]) else None
            ins.append(a)
            dele.append(d)
        say("multi round", r)
        mg.update_multi(ins=ins, dele=dele)
        for g in range(k):
            singles[g].update(ins[g], dele[g])
            if oras:
                assert oras[g].update(ins[g], dele[g]) == 0
            e = cur[g]
            if dele[g] is not None:
                kd = set(map(tuple, np.sort(dele[g], axis=1).tolist()))
                e = np.array([x for x in np.sort(e, axis=1).tolist() if tuple(x) not in kd],
                             dtype=np.int32).reshape(-1, 2)
            if ins[g] is not None:
                e = np.concatenate([e, ins[g]])
            cur[g] = e
        compare(f"round {r}")
    for s_ in singles:
        s_.close()
    mg.close()


def test_multi_small_against_singles_and_oracle():
    run_case(6, 1, 3, True)


def test_multi_many_graphs_against_singles():
    run_case(24, 2, 2, False)


@pytest.mark.parametrize("mode", [2, 3])
def test_multi_climbing_and_plain_steps(mode):
    """Mode 3 lets groups of any size climb (so the climbing steps run with
    members of graphs that differ in levels per group and caps, landing on
    group boundaries of some graphs and not others); mode 2 runs every step
    as a plain step.  Both against the graphs' own plain handles and the
    oracle."""
    run_case(8, 5, 3, True, mode=mode)


def test_multi_range_is_per_graph():
    from paper_2106_03824_amd import plds as P
    say("multi range")
    mg = P.MultiPLDS([10, 20])
    assert mg.update_multi(ins=[[(0, 1), (2, 3)], [(0, 19)]]) == 0
    lv = mg.levels().cpu().numpy().copy()
    # vertex 12 exists in the handle (graph 1's range) but not in graph 0
    rc = mg.update_multi(ins=[[(0, 12)], None], check=False)
    assert rc == P.PLDS_ERANGE
    assert (mg.levels().cpu().numpy() == lv).all() and mg.info()["m"] == 3
    assert mg.update_multi(ins=None, dele=[None, [(0, 19)]]) == 0
    assert mg.info()["m"] == 2
    assert mg.check() == 0


def test_reset_graph_reuses_a_slot():
    """plds_reset_graph empties a graph slot and gives it a new n (at most
    its capacity): the new graph then goes through the states of a plain
    handle of its own n (compared with the oracle after every batch), the
    other graphs are untouched, and per-graph applied counts are reported."""
    from paper_2106_03824_amd import plds as P
    cap = 4096
    mg = P.MultiPLDS([cap, cap, cap])
    e0 = W.rmat(12, 8 * cap, seed=61)
    e2 = W.rmat(11, 8 * 2048, seed=62)
    say("reset graph: fill slots 0 and 2")
    assert mg.update_multi([e0, None, None]) == 0
    assert mg.update_multi([None, None, e2]) == 0
    ai, ad = P.plds_graph_applied(mg.h, 3)
    assert ai == [0, 0, len(np.unique(np.sort(e2, axis=1), axis=0))] and ad == [0, 0, 0]
    lv2 = mg.graph_levels(2).cpu().numpy().copy()
    o0 = O.Oracle(cap)
    assert o0.insert(e0) == 0
    assert np.array_equal(mg.graph_levels(0).cpu().numpy(), o0.levels())
    m_before = mg.info()["m"]
    for n_new, seed in ((1000, 63), (3000, 64)):      # slot 0 reused twice, with other sizes
        say("reset graph: slot 0 to n", n_new)
        mg.reset_graph(0, n_new)
        assert mg.graphs[0]["n"] == n_new and mg.graphs[0]["L"] == O.Oracle(n_new).L
        assert mg.info()["m"] == m_before - o0.m
        assert (mg.graph_levels(0).cpu().numpy() == 0).all()
        o0 = O.Oracle(n_new)
        e = W.er(n_new, 12.0 / n_new, seed=seed)
        for ins, dele in ((e, None), (W.new_pairs(n_new, e, 2000, seed + 1), W.sample_edges(e, 1500, seed + 2))):
            assert mg.update_multi([ins, None, None], [dele, None, None] if dele is not None else None) == 0
            assert o0.update(ins, dele) == 0
            assert np.array_equal(mg.graph_levels(0).cpu().numpy(), o0.levels())
            assert np.array_equal(mg.degrees().cpu().numpy()[:n_new], o0.degrees())
            s = o0.stats()
            ai, ad = P.plds_graph_applied(mg.h, 3)
            assert (ai[0], ad[0]) == (s["applied_ins"], s["applied_del"]) and ai[1:] == [0, 0] and ad[1:] == [0, 0]
        m_before = mg.info()["m"]
        assert np.array_equal(mg.graph_levels(2).cpu().numpy(), lv2)
        # ids of the old, larger graph are now out of range
        bad = np.array([[0, n_new]], dtype=np.int32)
        assert mg.update_multi([bad, None, None], check=False) == P.PLDS_ERANGE
    assert mg.check() == 0
    with pytest.raises(P.PLDSError):
        mg.reset_graph(1, cap + 1)
    mg.close()
