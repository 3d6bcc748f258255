"""GPU parity of the PLDSOpt row's options against the oracle: the heuristic
Invariant-1 coefficient (1.1 in place of 2 + 3/lambda) and the upward
desire-level jump of the implementation's insertion procedure, alone and
together, with the PLDSOpt level structure too.  Levels, estimates, degrees
and the per-batch sweep/move/violator counts must agree bit for bit after
every batch."""
import random
import sys

import numpy as np
import pytest

import oracle as O
from paper_2106_03824_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up", "moves_down", "viol_ins0",
        "viol_del0")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _P():
    from paper_2106_03824_amd import plds as P
    P.lib()
    return P


class OptPair:
    def __init__(self, n, delta=0.4, lam=3.0, L=0, coeff=0.0, jump=False, timed=False):
        P = _P()
        self.g = P.PLDS(n, delta, lam, L, up_coeff=coeff, up_jump=jump)
        if timed:
            P.plds_set_timing(self.g.h, "jmp_scan" if jump else "ins_prep")
        self.o = O.Oracle(n, delta, lam, L, coeff=coeff, jump=jump)

    def step(self, ins=None, dele=None):
        rg = self.g.update(ins, dele, check=False)
        ro = self.o.update(ins, dele)
        assert rg == ro == 0, (rg, ro, self.o.last_assert())
        lg, lo = self.g.levels().cpu().numpy(), self.o.levels()
        bad = np.flatnonzero(lg != lo)
        assert bad.size == 0, f"{bad.size} levels differ, first {bad[:5]}: gpu {lg[bad[:5]]} oracle {lo[bad[:5]]}"
        assert np.array_equal(self.g.coreness().cpu().numpy().view(np.int64), self.o.coreness().view(np.int64))
        assert np.array_equal(self.g.degrees().cpu().numpy(), self.o.degrees())
        sg, so = self.g.stats(), self.o.stats()
        for k in KEYS:
            assert sg[k] == so[k], (k, sg[k], so[k])
        assert self.g.check() == 0


def test_tables_with_coefficient():
    P = _P()
    g = P.PLDS(2 ** 20, 0.4, 3.0, up_coeff=1.1)
    o = O.Oracle(2 ** 20, 0.4, 3.0, coeff=1.1)
    up, dn, pw = g.thresholds()
    ou, od, op = o.tables()
    assert np.array_equal(np.asarray(up), np.asarray(ou)) and np.array_equal(np.asarray(dn), np.asarray(od))
    g.close()


def test_coefficient_below_one_rejected():
    P = _P()
    with pytest.raises(P.PLDSError):
        P.PLDS(100, 0.4, 3.0, up_coeff=0.5)


def test_hand_cases():
    say("options: hand cases")
    p = OptPair(5, coeff=1.1)
    p.step(ins=[(0, 1), (1, 2), (2, 3), (3, 4)])
    assert p.g.levels().cpu().tolist() == [0, 1, 2, 1, 0]
    p = OptPair(8, jump=True)
    p.step(ins=[(a, b) for a in range(1, 6) for b in range(a + 1, 6)])
    p.step(ins=[(0, v) for v in range(1, 6)])
    assert p.g.levels().cpu().tolist() == [56] * 6 + [0, 0]
    assert p.g.stats()["sweeps_ins"] == 29


@pytest.mark.parametrize("seed", range(16))
def test_random_small(seed):
    rng = random.Random(500 + seed)
    n = rng.choice([8, 20, 64, 200])
    L = rng.choice([0, 0, 2, 3, -1])
    coeff = [0.0, 1.1, 1.5, 1.1][seed % 4]
    jump = seed % 2 == 1 or coeff == 0.0
    delta, lam = rng.choice([(0.4, 3.0), (1.0, 3.0), (0.2, 6.0)])
    say("options small", seed, n, L, coeff, jump, delta, lam)
    p = OptPair(n, delta, lam, L, coeff, jump, timed=seed % 5 == 0)
    for it in range(6):
        ins = [(rng.randrange(n), rng.randrange(n)) for _ in range(rng.randrange(0, 4 * n))]
        cur = p.o.edges().tolist()
        dele = rng.sample(cur, rng.randrange(0, len(cur) + 1)) if cur and it % 2 else []
        p.step(ins=ins or None, dele=dele or None)


@pytest.mark.parametrize("coeff,jump,L", [(0.0, True, 0), (1.1, False, 0), (1.1, True, 0), (0.0, True, -1),
                                          (1.1, True, -1)])
def test_rmat_stream(coeff, jump, L):
    """RMAT scale 14, edge factor 16 (hubs with slabs far above a wavefront's
    512 registers), built in 4 batches, then mixed and deletion batches."""
    n = 2 ** 14
    e = W.permute_edges(W.rmat(14, 16 * n, seed=3), 2001)
    p = OptPair(n, L=L, coeff=coeff, jump=jump)
    for i, c in enumerate(np.array_split(e, 4)):
        say("options rmat14 build", coeff, jump, L, i)
        p.step(ins=c)
    cur = p.o.edges()
    say("options rmat14 mixed")
    p.step(ins=W.new_pairs(n, cur, 20000, 2002), dele=W.sample_edges(cur, 20000, 2003))
    say("options rmat14 delete")
    p.step(dele=W.sample_edges(p.o.edges(), 50000, 2004))
