"""Launch schedules (plds_set_launch) change how a batch runs, never what it
computes: under every schedule the levels after insertion, deletion and
mixed batches equal the oracle's; out-of-range schedules are rejected; the
schedule search (autotune.tune) keeps the state and the levels."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2106_03824_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCHEDULES = [
    {},
    {"scan_blocks": 64, "graph_steps": 2, "dl_blocks": 64, "del_scan_blocks": 64},
    {"scan_blocks": 2048, "graph_steps": 64, "dl_blocks": 4096, "del_scan_blocks": 8192},
    {"scan_blocks": 300, "graph_steps": 6, "dl_blocks": 700, "del_scan_blocks": 1500},
]


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def stream(n, seed):
    e = W.rmat(12, 8 * n, seed=seed)
    ins = W.new_pairs(n, e, 6000, seed + 1)
    dele = W.sample_edges(e, 9000, seed + 2)
    cur = np.concatenate([e, ins])      # some of these are gone by then: absent edges are skipped
    mix_i = W.new_pairs(n, cur, 3000, seed + 3)
    mix_d = W.sample_edges(cur, 4000, seed + 4)
    return e, [(ins, None), (None, dele), (mix_i, mix_d)]


@pytest.mark.parametrize("jump", [False, True])
def test_every_schedule_matches_the_oracle(jump):
    from paper_2106_03824_amd import plds as P
    n = 2 ** 12
    e, batches = stream(n, 61)
    o = O.Oracle(n, jump=jump, coeff=1.1 if jump else 0.0)
    assert o.update(e, None) == 0
    want = []
    for ins, dele in batches:
        assert o.update(ins, dele) == 0
        want.append(o.levels().copy())
    for cfg in SCHEDULES:
        say("schedule", cfg, "jump", jump)
        g = P.PLDS(n, up_jump=jump, up_coeff=1.1 if jump else 0.0)
        P.plds_set_launch(g.h, **cfg)
        got = P.plds_get_launch(g.h)
        assert all(v > 0 for v in got.values())
        for f, v in cfg.items():
            assert got[f] == v
        assert g.update(e, None) == 0
        for (ins, dele), w in zip(batches, want):
            assert g.update(ins, dele) == 0
            assert np.array_equal(g.levels().cpu().numpy(), w), f"schedule {cfg} differs from the oracle"
        assert g.check() == 0


def test_out_of_range_schedules_are_rejected():
    from paper_2106_03824_amd import plds as P
    g = P.PLDS(1024)
    before = P.plds_get_launch(g.h)
    for bad in ({"scan_blocks": 63}, {"scan_blocks": 2049}, {"graph_steps": 3}, {"graph_steps": 66},
                {"graph_steps": 1}, {"dl_blocks": 5000}, {"del_scan_blocks": 32}, {"scan_blocks": -1}):
        with pytest.raises(P.PLDSError):
            P.plds_set_launch(g.h, **bad)
        assert P.plds_get_launch(g.h) == before
    c = P.plds_launch_t()
    c.reserved[2] = 1
    assert P.lib().plds_set_launch(g.h, c) == P.PLDS_EINVAL
    assert P.plds_get_launch(g.h) == before
    # defaults come back with zeros
    P.plds_set_launch(g.h, scan_blocks=512, graph_steps=4)
    P.plds_set_launch(g.h)
    assert P.plds_get_launch(g.h) == before


def test_rebuild_keeps_the_schedule():
    from paper_2106_03824_amd import plds as P
    n = 2 ** 10
    g = P.PLDS(n)
    assert g.update(W.rmat(10, 4 * n, seed=5), None) == 0
    P.plds_set_launch(g.h, scan_blocks=320, graph_steps=10, dl_blocks=128, del_scan_blocks=96)
    want = P.plds_get_launch(g.h)
    r = g.rebuild(n)
    assert P.plds_get_launch(r.h) == want


def test_search_keeps_state_and_levels():
    from paper_2106_03824_amd import autotune as AT
    from paper_2106_03824_amd import plds as P
    ns = [700, 2 ** 11, 3000, 2 ** 10]
    mg = P.MultiPLDS(ns)
    es = [W.er(ns[0], 10 / ns[0], seed=1), W.rmat(11, 8 * ns[1], seed=2), W.er(ns[2], 6 / ns[2], seed=3),
          W.rmat(10, 8 * ns[3], seed=4)]
    mg.update_multi(ins=[torch.from_numpy(x).cuda() for x in es])
    lv0 = mg.levels().clone()
    ins = [torch.from_numpy(W.new_pairs(n, x, 2000, 10 + i)).cuda() for i, (n, x) in enumerate(zip(ns, es))]
    dele = [torch.from_numpy(W.sample_edges(x, 1500, 20 + i)).cuda() for i, x in enumerate(es)]
    space = {"scan_blocks": (128, 2048), "graph_steps": (4, 32), "dl_blocks": (256,), "del_scan_blocks": (512,)}
    best, rec = AT.tune(mg, lambda: P.plds_update_multi(mg.h, ins, dele), torch, space=space, reps=1, passes=1)
    assert torch.equal(mg.levels(), lv0)          # the post-build state is back
    assert P.plds_get_launch(mg.h) == best
    assert len(rec["trials"]) >= 4 and rec["best"]["ms"] <= rec["default"]["ms"]
    # the schedule found computes what the default computes
    P.plds_update_multi(mg.h, ins, dele)
    lv_best = mg.levels().clone()
    ref = P.MultiPLDS(ns)
    ref.update_multi(ins=[torch.from_numpy(x).cuda() for x in es])
    P.plds_update_multi(ref.h, ins, dele)
    assert torch.equal(ref.levels(), lv_best)
