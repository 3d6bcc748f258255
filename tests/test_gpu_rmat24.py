"""RMAT scale 24 (2^24 vertices, 16*2^24 unique edges), the large streamed
workload of the benchmark, run through the C ABI exactly as bench.py
--workload stream times it: the whole graph inserted as 10^6-edge batches
in a seeded random permutation, then two deletion batches of 10^6 sampled
edges and one mixed batch, then one deletion batch of every edge of the
2,000 largest hubs (random deletions leave every vertex within its floor at
this size, so this batch is the one that runs the deletion pass).

Bit-exact parity: the stream's first batches (as many as the stored oracle
trace tests/golden/rmat24_oracle_trace.json holds, written by
make_rmat24_oracle.py from the oracle alone, at one to five minutes of
oracle time per batch) must leave levels with the same SHA-256 as the
oracle's, with the same applied, sweep, move and violator counts.

The oracle would take days for the whole stream, so beyond the trace parity
is by properties that hold for every correct run, checked on the CPU from
the generated edge lists (never from edges the library reports):

  * Invariant 1 (up(v) <= floor((2+3/lambda)(1+delta)^g)) and Invariant 2
    (up*(v) >= ceil((1+delta)^g) at level > 0) at every vertex, with up and
    up* counted from the edge list and the GPU levels, and the tables from
    the oracle's exact rational arithmetic;
  * isolated vertices sit at level 0;
  * the coreness estimate of every vertex equals the estimate map applied to
    its level, and lies within the factor (2+3/lambda)(1+delta) = 4.2 of the
    exact coreness from the oracle's bucket peeling (Lemma decomp-bound).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCALE, B = 24, 10 ** 6
TRACE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat24_oracle_trace.json")


def digest(levels):
    return hashlib.sha256(np.ascontiguousarray(levels, dtype=np.int32).tobytes()).hexdigest()[:32]


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def keys(e):
    a = np.minimum(e[:, 0], e[:, 1]).astype(np.int64)
    b = np.maximum(e[:, 0], e[:, 1]).astype(np.int64)
    return (a << 32) | b


def check_invariants(n, e, lv, up_max, dn_min, L):
    a, b = e[:, 0], e[:, 1]
    la, lb = lv[a], lv[b]
    deg = np.bincount(a, minlength=n) + np.bincount(b, minlength=n)
    up = np.bincount(a, weights=lb >= la, minlength=n) + np.bincount(b, weights=la >= lb, minlength=n)
    ups = np.bincount(a, weights=lb >= la - 1, minlength=n) + np.bincount(b, weights=la >= lb - 1, minlength=n)
    g1 = lv // L
    g2 = np.maximum(lv - 1, 0) // L
    assert (up <= up_max[g1]).all(), "Invariant 1 fails"
    assert ((lv == 0) | (ups >= dn_min[g2])).all(), "Invariant 2 fails"
    assert ((deg > 0) | (lv == 0)).all(), "an isolated vertex above level 0"
    return deg


@pytest.mark.timeout(1200)
def test_rmat24_stream_properties():
    from paper_2106_03824_amd import plds as P
    from paper_2106_03824_amd import workloads as W
    n, m0 = 2 ** SCALE, 16 * 2 ** SCALE
    t = time.perf_counter()
    e = W.rmat(SCALE, m0, seed=1)
    say(f"rmat24 generated in {time.perf_counter() - t:.0f}s")
    perm = W.permute_edges(e, 1000 * 3 + 1)
    dels = W.sample_edges(e, 2 * B + B // 2, 1000 * 3 + 100)
    mix_ins = W.new_pairs(n, e, B - B // 2, 1000 * 3 + 101)
    o = O.Oracle(n, 0.4, 3.0)
    up_max, dn_min, pow_tab = (np.asarray(x) for x in o.tables())
    L = o.L
    del o
    g = P.PLDS(n, 0.4, 3.0, 0, 2 * m0)
    assert g.L == L
    dev = torch.device("cuda", 0)
    perm_d = torch.from_numpy(perm).to(dev)
    del perm
    trace = json.load(open(TRACE))["batches"] if os.path.exists(TRACE) else []
    say(f"rmat24 oracle trace: {len(trace)} batches")
    for i in range(0, m0, B):
        bi = i // B
        if i % (64 * B) == 0:
            say("rmat24 build batch", bi)
        assert P.plds_batch_insert(g.h, perm_d[i:i + B]) == 0
        if bi < len(trace):
            ref, s = trace[bi], g.stats()
            assert ref["kind"] == f"stream{bi}"
            assert digest(g.levels().cpu().numpy()) == ref["sha"], f"levels differ from the oracle after batch {bi}"
            for k in ("applied_ins", "sweeps_ins", "moves_up", "viol_ins0"):
                assert s[k] == ref[k], (bi, k, s[k], ref[k])
    assert len(trace) >= 25
    del perm_d
    say("rmat24 build done: invariants")
    check_invariants(n, e, g.levels().cpu().numpy(), up_max, dn_min, L)
    dd = torch.from_numpy(dels).to(dev)
    say("rmat24 deletions")
    assert P.plds_update(g.h, None, dd[:B]) == 0
    assert P.plds_update(g.h, None, dd[B:2 * B]) == 0
    say("rmat24 mixed")
    assert P.plds_update(g.h, torch.from_numpy(mix_ins).to(dev), dd[2 * B:]) == 0
    kept = ~np.isin(keys(e), keys(dels), assume_unique=True)
    cur = np.concatenate([e[kept], mix_ins])
    del e, kept
    # random deletions barely move anyone at this size; every edge of the
    # 2,000 largest hubs, deleted in one batch, makes the deletion pass work
    deg0 = np.bincount(cur[:, 0], minlength=n) + np.bincount(cur[:, 1], minlength=n)
    hub = np.zeros(n, dtype=bool)
    hub[np.argsort(deg0, kind="stable")[-2000:]] = True
    inc = hub[cur[:, 0]] | hub[cur[:, 1]]
    say(f"rmat24 hub deletions: {int(inc.sum())} edges")
    assert P.plds_update(g.h, None, torch.from_numpy(np.ascontiguousarray(cur[inc])).to(dev)) == 0
    s = g.stats()
    assert s["applied_del"] == int(inc.sum()) and s["sweeps_del"] > 0 and s["moves_down"] > 0, s
    say(f"rmat24 hub deletions: {s['sweeps_del']} sweeps, {s['moves_down']} moves down")
    cur = cur[~inc]
    assert g.info()["m"] == cur.shape[0]
    lv = g.levels().cpu().numpy()
    say("rmat24 final invariants")
    deg = check_invariants(n, cur, lv, up_max, dn_min, L)
    est = g.coreness().cpu().numpy()
    expect = np.where(deg > 0, pow_tab[np.maximum((lv + 1) // L - 1, 0)], 0.0)
    assert np.array_equal(est.view(np.int64), expect.view(np.int64))
    say("rmat24 exact coreness")
    k = O.exact_coreness(n, cur)
    pos = k > 0
    assert ((est > 0) == pos).all()
    ratio = np.maximum(est[pos] / k[pos], k[pos] / est[pos])
    assert ratio.max() <= 4.2 * (1 + 1e-12), ratio.max()
    say(f"rmat24 max ratio {ratio.max():.3f}, mean {ratio.mean():.3f}")
