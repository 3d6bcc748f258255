"""GPU parity of the orientation outputs (Algorithm 5) and the densest-subgraph
value against the oracle (oracle/orient.py on the oracle's levels, which equal
the library's bit for bit).  Sets of edges are compared sorted."""
import random
import sys

import numpy as np
import pytest

import oracle as O
import oracle.orient as OR
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


def srt(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    return a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a


class Tracked:
    """A GPU handle with orientation tracking and an oracle, fed the same calls."""

    def __init__(self, n, delta=0.4, lam=3.0, L=0, sweep_mode=1):
        self.g = lib().PLDS(n, delta, lam, L)
        lib().plds_set_sweep_mode(self.g.h, sweep_mode)
        self.g.track_orientation(True)
        self.o = O.Oracle(n, delta, lam, L)
        self.n = n

    def step(self, ins=None, dele=None):
        lv0, e0 = self.o.levels(), self.o.edges()
        assert self.g.update(ins, dele, check=False) == 0
        assert self.o.update(ins, dele) == 0
        lv1, e1 = self.o.levels(), self.o.edges()
        assert (self.g.levels().cpu().numpy() == lv1).all()
        f = self.g.flips().cpu().numpy()
        want_f = OR.flips(lv0, lv1, e0, e1)
        assert np.array_equal(srt(f), srt(want_f)), (len(f), len(want_f))
        a_ins, a_del = OR.applied_updates(e0, ins, dele)
        ji, jd = self.g.oriented_updates()
        wi, wd = OR.oriented_updates(lv0, lv1, a_ins, a_del)
        assert np.array_equal(srt(ji.cpu().numpy()), srt(wi))
        assert np.array_equal(srt(jd.cpu().numpy()), srt(wd))
        return len(want_f)


def test_orient_rule_matches_oracle():
    n = 2 ** 12
    e = W.rmat(12, 8 * n, seed=5)
    say("orient rmat12")
    g = lib().PLDS(n)
    o = O.Oracle(n)
    assert g.insert(e) == 0 and o.insert(e) == 0
    lv = o.levels()
    assert (g.levels().cpu().numpy() == lv).all()
    rng = np.random.default_rng(7)
    pairs = rng.integers(0, n, size=(50000, 2), dtype=np.int32)
    same = np.flatnonzero(lv[pairs[:, 0]] == lv[pairs[:, 1]])
    assert same.size > 0                        # ties by id are exercised
    pairs = np.concatenate([pairs, e[:20000]])
    got = g.orient(pairs).cpu().numpy()
    assert np.array_equal(got, OR.orient(lv, pairs))
    say("orient out of range")
    bad = g.orient([(0, 1), (2, n)]).cpu().numpy()
    assert bad[1].tolist() == [-1, -1] and bad[0].tolist() == OR.orient(lv, [(0, 1)])[0].tolist()
    assert lib().plds_sync(g.h) == lib().PLDS_ERANGE


@pytest.mark.parametrize("seed", range(8))
def test_flips_random_small(seed):
    rng = random.Random(seed)
    n = rng.choice([8, 20, 64, 200])
    L = rng.choice([0, 2, 3])
    say("flips small", seed, n, L)
    t = Tracked(n, 0.4, 3.0, L, sweep_mode=seed % 4)
    for it in range(6):
        ins = [(rng.randrange(n), rng.randrange(n)) for _ in range(rng.randrange(0, 4 * n))]
        cur = t.o.edges().tolist()
        dele = rng.sample(cur, rng.randrange(0, len(cur) + 1)) if cur and it % 2 else []
        t.step(ins or None, dele or None)


def test_flips_rmat14_stream():
    n = 2 ** 14
    e = W.permute_edges(W.rmat(14, 16 * n, seed=3), 2001)
    t = Tracked(n)
    total = 0
    for i, c in enumerate(np.array_split(e, 4)):
        say("flips rmat14 build", i)
        total += t.step(ins=c)
    cur = t.o.edges()
    say("flips rmat14 mixed")
    total += t.step(ins=W.new_pairs(n, cur, 20000, 2002), dele=W.sample_edges(cur, 20000, 2003))
    say("flips rmat14 delete")
    total += t.step(dele=W.sample_edges(t.o.edges(), 50000, 2004))
    assert total > 0


@pytest.mark.parametrize("sweep_mode", [1, 2])
def test_flips_every_slab_class(sweep_mode):
    """Moved vertices of every slab size the edge scan sorts apart: slabs of
    8 and 16 slots, up to 2048, and hubs of several thousand slots whose
    slabs are cut into chunks over all wavefronts."""
    n = 2 ** 13
    rng = np.random.default_rng(11)
    hubs = [0, 1, 2]
    e = [(h, v) for h in hubs for v in range(3, n) if rng.random() < 0.8]           # ~6500 each
    e += [(v, int(x)) for v in range(3, 40) for x in rng.integers(40, n, size=300)]  # mid slabs
    e += [(int(a), int(b)) for a, b in rng.integers(40, n, size=(4 * n, 2))]         # small slabs
    say("flips slab classes", sweep_mode, len(e))
    t = Tracked(n, 0.4, 3.0, 0, sweep_mode=sweep_mode)
    total = 0
    for i, c in enumerate(np.array_split(np.array(e, dtype=np.int32), 3)):
        total += t.step(ins=c)
    # a dense block on the hubs and some mid vertices lifts them
    blk = list(range(0, 60))
    total += t.step(ins=[(a, b) for a in blk for b in blk if a < b])
    cur = t.o.edges()
    total += t.step(dele=W.sample_edges(cur, len(cur) // 2, 12))
    assert total > 0


def test_flips_cap_empty_call_and_errors():
    n = 2 ** 10
    e = W.rmat(10, 8 * n, seed=8)
    say("flips cap/errors")
    g = lib().PLDS(n)
    assert g.insert(e[: len(e) // 2]) == 0
    with pytest.raises(lib().PLDSError):          # tracking off during the last call
        lib().plds_flips(g.h, None)
    g.track_orientation(True)
    with pytest.raises(lib().PLDSError):          # no call since tracking started
        lib().plds_flips(g.h, None)
    assert g.insert(e[len(e) // 2:]) == 0
    k = lib().plds_flips(g.h, None)
    assert k > 1
    full = g.flips().cpu().numpy()
    part = torch.full((k // 2, 2), -7, dtype=torch.int32, device="cuda")
    assert lib().plds_flips(g.h, part) == k
    got = {tuple(x) for x in part.cpu().numpy().tolist()}
    assert got <= {tuple(x) for x in full.tolist()} and len(got) == k // 2
    say("empty call")
    assert lib().plds_update(g.h, None, None) == 0
    assert lib().plds_flips(g.h, None) == 0
    assert lib().plds_oriented_updates(g.h, None, None) == (0, 0)
    ed, lv = g.dump()
    assert g.load(ed, lv) == 0
    with pytest.raises(lib().PLDSError):          # a loaded state has no last call
        lib().plds_flips(g.h, None)


def test_densest_value_matches_oracle():
    for scale, ef, seed in [(10, 8, 1), (12, 16, 2)]:
        n = 2 ** scale
        say("densest", scale, ef, seed)
        e = W.rmat(scale, ef * n, seed=seed)
        g = lib().PLDS(n)
        o = O.Oracle(n)
        assert g.densest_value() == 0.0
        assert g.insert(e) == 0 and o.insert(e) == 0
        want = OR.densest_subgraph_value(o.coreness())
        assert np.float64(g.densest_value()).view(np.int64) == np.float64(want).view(np.int64)
        d = W.sample_edges(e, len(e) // 2, seed)
        assert g.delete(d) == 0 and o.delete(d) == 0
        want = OR.densest_subgraph_value(o.coreness())
        assert np.float64(g.densest_value()).view(np.int64) == np.float64(want).view(np.int64)


def test_densest_value_per_graph_of_multi_handle():
    ns = [300, 2 ** 11, 50]
    say("densest multi", ns)
    m = lib().MultiPLDS(ns)
    rng = np.random.default_rng(3)
    lists = [W.er(ns[0], 0.05, seed=1), W.rmat(11, 8 * ns[1], seed=2), np.zeros((0, 2), np.int32)]
    devs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() if len(x) else None for x in lists]
    assert lib().plds_update_multi(m.h, devs, None) == 0
    for gi, (nn, ed) in enumerate(zip(ns, lists)):
        o = O.Oracle(nn)
        if len(ed):
            assert o.insert(ed) == 0
        want = OR.densest_subgraph_value(o.coreness())
        assert np.float64(m.densest_value(gi)).view(np.int64) == np.float64(want).view(np.int64)
    del rng
