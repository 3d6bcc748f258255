"""Serving loop with continuous batching: requests of many graphs arriving as
a Poisson stream are served in fused multi-graph calls (the updates of all
graphs of a shard with work in one plds_update_multi, their queries in one
plds_coreness), and must give exactly the results of serving each request
alone with a plain handle per graph (serve_alone), and those of the CPU
oracle replaying each graph's requests in order (levels at retirement and
every coreness query)."""
import copy
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


def make_trace(ngraphs, nreq, seed, rate, scales=(8, 12), ef=8, size_exp=(1, 3.3), query=100):
    from paper_2106_03824_amd.serve import Request
    rng = random.Random(seed)
    reqs, t, rid = [], 0.0, 0
    graphs = {}
    for g in range(ngraphs):
        sc = rng.randint(*scales)
        n = 2 ** sc
        e = W.rmat(sc, ef * n, seed=seed * 100 + g)
        graphs[g] = (n, e)
        reqs.append(Request(rid, g, "admit", t, (n, e)))
        rid += 1
    last = {g: 0.0 for g in graphs}
    for i in range(nreq):
        t += rng.expovariate(rate)
        g = rng.randrange(ngraphs)
        n, e = graphs[g]
        if rng.random() < 0.5:
            size = int(round(10 ** rng.uniform(*size_exp)))
            if rng.random() < 0.7:
                r = np.random.default_rng(seed * 7919 + i)
                ins = r.integers(0, n, size=(size, 2), dtype=np.int32)
                reqs.append(Request(rid, g, "update", t, (ins, None)))
            else:
                reqs.append(Request(rid, g, "update", t, (None, W.sample_edges(e, min(size, len(e)), seed + i))))
        else:
            r = np.random.default_rng(seed * 104729 + i)
            reqs.append(Request(rid, g, "query", t, r.integers(0, n, size=query, dtype=np.int32)))
        rid += 1
        last[g] = t
    for g in graphs:
        t += 1e-4
        reqs.append(Request(rid, g, "retire", t))
        rid += 1
    return reqs


def oracle_replay(reqs):
    out = {}
    oras = {}
    for r in sorted(reqs, key=lambda r: r.rid):
        if r.kind == "admit":
            n, e = r.payload
            oras[r.graph] = O.Oracle(n)
            assert oras[r.graph].insert(e) == 0
        elif r.kind == "update":
            ins, dele = r.payload
            assert oras[r.graph].update(ins, dele) == 0
        elif r.kind == "query":
            out[r.rid] = oras[r.graph].coreness()[r.payload]
        else:
            out[r.rid] = oras[r.graph].levels()
    return out


def results(reqs):
    out = {}
    for r in reqs:
        assert r.error is None, (r.kind, r.error)
        if r.kind == "query":
            out[r.rid] = r.result
        elif r.kind == "retire":
            out[r.rid] = r.result["levels"]
    return out


def same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.dtype == y.dtype and np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                                     y.view(np.int64) if y.dtype == np.float64 else y), k


def test_serving_mix_equals_alone_equals_oracle():
    from paper_2106_03824_amd.serve import replay, serve_alone
    reqs = make_trace(10, 120, 5, rate=4000.0)
    alone = copy.deepcopy(reqs)
    say("serve: fused, shards of 4 slots, Poisson arrivals")
    replay(reqs, budget_bytes=64 << 30, slots=4, arrival=True)
    say("serve: alone, a plain handle per graph")
    serve_alone(alone)
    say("serve: oracle replay")
    ref = oracle_replay(reqs)
    same(results(reqs), results(alone))
    same(results(reqs), ref)
    for a, b in zip(sorted(reqs, key=lambda r: r.rid), sorted(alone, key=lambda r: r.rid)):
        if a.kind == "update":
            assert a.result == b.result, (a.rid, a.result, b.result)
    # requests of different graphs were served by one fused call
    assert max(r.fused for r in reqs) > 1
    spans = sorted((r.start, r.done, r.graph) for r in reqs)
    assert any(b[0] < a[1] and b[2] != a[2] for a, b in zip(spans, spans[1:]))


def test_serving_benchmark_mix_against_oracle():
    """The serving benchmark's graph shape and request mix (R-MAT with edge
    factor 16, update batches of log-uniform size from 10^2, 70% insertions,
    coreness queries of 10^3 vertices) at scales 12..13 and batches up to
    10^4 (the oracle builds a scale-14 graph in one batch in about 11 s, a
    scale-16 one in minutes): fused serving equals the oracle's replay."""
    from paper_2106_03824_amd.serve import replay
    reqs = make_trace(4, 40, 11, rate=2000.0, scales=(12, 13), ef=16, size_exp=(2, 4), query=1000)
    say("serve: benchmark mix, fused")
    replay(reqs, budget_bytes=64 << 30, slots=4, arrival=False)
    say("serve: benchmark mix, oracle replay")
    same(results(reqs), oracle_replay(reqs))
    assert max(r.fused for r in reqs) > 1


def test_serving_admission_waits_for_budget():
    """With room for about two graphs at a time, admissions queue behind
    retirements and results are unchanged."""
    from paper_2106_03824_amd.serve import footprint_bytes, replay, serve_alone
    reqs = make_trace(5, 30, 9, rate=4000.0)
    alone = copy.deepcopy(reqs)
    biggest = max(footprint_bytes(r.payload[0], len(r.payload[1])) for r in reqs if r.kind == "admit")
    say("serve: small budget")
    replay(reqs, budget_bytes=2 * biggest, slots=2, arrival=True)
    serve_alone(alone)
    same(results(reqs), results(alone))


def test_failed_admission_drains():
    """A graph whose shard cannot be created (the library's ENOMEM, forced by
    failing its first allocation) fails its admission; its later requests
    fail at once with that error, the loop drains, and the other graph is
    served as alone."""
    from paper_2106_03824_amd import plds as P
    from paper_2106_03824_amd import serve as S
    say("serve: failed admission")
    n = 2 ** 10
    e = W.rmat(10, 8 * n, seed=5)
    bad_n = 5000          # a size class of its own, so its admission needs a new shard
    srv = S.Server(budget_bytes=1 << 40, slots=2)
    reqs = [S.Request(0, "a", "admit", 0.0, (n, e)), S.Request(1, "bad", "admit", 0.0, (bad_n, e[:10])),
            S.Request(2, "bad", "update", 0.0, (e[:5], None)),
            S.Request(3, "bad", "query", 0.0, np.arange(5, dtype=np.int32)),
            S.Request(4, "a", "query", 0.0, np.arange(50, dtype=np.int32)), S.Request(5, "bad", "retire", 0.0),
            S.Request(6, "a", "retire", 0.0)]
    try:
        srv.submit(reqs[0])
        P.plds_inject_alloc_failure(0)       # this thread creates the shards
        srv.submit(reqs[1])
        P.plds_inject_alloc_failure(-1)
        for r in reqs[2:]:
            srv.submit(r)
        srv.drain()
        assert srv.used == 0 and not srv.where
    finally:
        P.plds_inject_alloc_failure(-1)
        srv.close()
    assert isinstance(reqs[1].error, P.PLDSError)
    for r in reqs[2:4] + [reqs[5]]:
        assert r.error is not None and "not admitted" in str(r.error)
    assert reqs[0].error is None and reqs[4].error is None and reqs[6].error is None
    o = O.Oracle(n, 0.4, 3.0)
    assert o.update(e, None) == 0
    assert np.array_equal(reqs[4].result.view(np.int64), o.coreness(np.arange(50, dtype=np.int32)).view(np.int64))
    assert np.array_equal(reqs[6].result["levels"], o.levels())
