"""Host logic that needs no GPU: the serving loop's scheduling (which head
requests a shard pass takes, admission by free slots and HBM budget, the
release of a retired graph, the draining of a graph whose admission
failed) and the launch-schedule search (coordinate descent, the check that
no schedule changes a result, the record).  The library is replaced by
small fakes; nothing here launches a kernel."""
import types

import numpy as np
import pytest

from paper_2106_03824_amd import autotune as AT
from paper_2106_03824_amd import plds as P
from paper_2106_03824_amd import serve as S


# ---------------------------------------------------------------- serving
def fake_shard(cls, slots):
    return types.SimpleNamespace(cls=cls, slots=slots, free=list(range(slots)), graph_of={})


def server(budget=1 << 40, fuse=True):
    srv = S.Server(budget, slots=4, fuse=fuse)
    srv.shards = []
    return srv


def req(rid, g, kind, arrival, payload=None):
    return S.Request(rid, g, kind, arrival, payload)


def admit(rid, g, n=1000, m=10, arrival=0.0):
    return req(rid, g, "admit", arrival, (n, np.zeros((m, 2), dtype=np.int32)))


def test_size_class():
    assert S.size_class(1) == 1024 and S.size_class(1024) == 1024 and S.size_class(1025) == 2048
    assert S.size_class(3000, smallest=8) == 4096


def test_collect_takes_one_head_per_graph_oldest_first():
    srv = server()
    sh = fake_shard(1024, 4)
    srv.shards.append(sh)
    for g in range(3):
        srv.where[g] = (sh, g)
        sh.free.remove(g)
    srv.queues[0].extend([req(1, 0, "update", 3.0), req(2, 0, "query", 4.0)])
    srv.queues[1].append(req(3, 1, "query", 1.0))
    srv.queues[2].append(req(4, 2, "update", 2.0))
    srv.busy.add(2)                                   # graph 2 has a call in flight
    got = srv._collect(sh)
    assert [r.rid for r in got] == [3, 1]             # by arrival; graph 0 once; graph 2 skipped
    assert srv.busy == {0, 1, 2} and srv.inflight == 2
    assert [r.rid for r in srv.queues[0]] == [2]


def test_collect_without_fusing_takes_one_request():
    srv = server(fuse=False)
    sh = fake_shard(1024, 4)
    for g in range(2):
        srv.where[g] = (sh, g)
        srv.queues[g].append(req(10 + g, g, "query", float(g)))
    assert [r.rid for r in srv._collect(sh)] == [10]


def test_admissions_fill_free_slots_in_order():
    srv = server()
    sh = fake_shard(1024, 2)
    for i in range(3):
        srv.queues[i].append(admit(i, i, arrival=float(i)))
    got = srv._collect(sh)
    assert [r.rid for r in got] == [0, 1]             # two free slots
    assert srv.where[0] == (sh, 0) and srv.where[1] == (sh, 1) and sh.free == []
    assert srv.used == S.footprint_bytes(1000, 10) * 2
    assert [r.rid for r in srv.queues[2]] == [2]      # waits for a slot
    # an admission of another size class is not this shard's
    srv.queues[3].append(admit(3, 3, n=5000))
    sh2 = fake_shard(1024, 2)
    assert all(r.rid != 3 for r in srv._collect(sh2))


def test_admission_waits_for_budget():
    f = S.footprint_bytes(1000, 10)
    srv = server(budget=f + f // 2)
    sh = fake_shard(1024, 4)
    srv.queues[0].append(admit(0, 0))
    srv.queues[1].append(admit(1, 1, arrival=1.0))
    assert [r.rid for r in srv._collect(sh)] == [0]  # the second does not fit the budget
    srv.busy.clear()
    assert srv._collect(sh) == []
    srv._release(0)                                   # retiring graph 0 frees its slot and footprint
    assert srv.used == 0 and 0 in sh.free
    assert [r.rid for r in srv._collect(sh)] == [1]


def test_lone_admission_larger_than_the_budget_still_runs():
    srv = server(budget=1)
    sh = fake_shard(1024, 2)
    srv.queues[0].append(admit(0, 0))
    assert [r.rid for r in srv._collect(sh)] == [0]  # nothing resident: it may use the whole device


def test_failed_admission_fails_the_graphs_requests():
    srv = server()
    srv.queues[5].extend([req(1, 5, "update", 1.0), req(2, 5, "query", 2.0)])
    err = RuntimeError("no memory")
    srv._fail_graph(5, err)
    assert not srv.queues[5] and srv.failed[5] is err
    later = req(3, 5, "query", 3.0)
    srv.submit(later)
    assert later.error is not None and later.done is not None


# ---------------------------------------------------------------- search
class FakeTorch:
    """The few torch calls the search makes, on numpy arrays."""

    class cuda:
        @staticmethod
        def synchronize():
            pass

        @staticmethod
        def current_device():
            return 0

        @staticmethod
        def get_device_properties(i):
            return types.SimpleNamespace(name="fake")

    int32 = np.int32

    @staticmethod
    def empty(shape, dtype=None, device=None):
        return np.zeros(shape, dtype=np.int32)

    @staticmethod
    def equal(a, b):
        return bool(np.array_equal(a, b))


@pytest.fixture
def fake_lib(monkeypatch):
    """A handle whose run time depends on the schedule (fastest at
    scan_blocks 512, graph_steps 32) and whose levels can be made to depend
    on it."""
    st = {"cfg": {}, "loads": 0, "bad": None}
    defaults = {"scan_blocks": 1280, "graph_steps": 16, "dl_blocks": 1024, "del_scan_blocks": 2048}

    def set_launch(h, **cfg):
        st["cfg"] = {k: v for k, v in cfg.items() if v}

    def get_launch(h):
        return {**defaults, **st["cfg"]}

    def load_state(h, e, lv):
        st["loads"] += 1

    def levels(h, out):
        out[:] = 7
        if st["bad"] and get_launch(h)["graph_steps"] == st["bad"]:
            out[0] = 8

    monkeypatch.setattr(P, "plds_info", lambda h: {"m": 5, "n": 4})
    monkeypatch.setattr(P, "plds_dump_state", lambda h, e, lv: 5)
    monkeypatch.setattr(P, "plds_set_launch", set_launch)
    monkeypatch.setattr(P, "plds_get_launch", get_launch)
    monkeypatch.setattr(P, "plds_load_state", load_state)
    monkeypatch.setattr(P, "plds_levels", levels)
    clock = {"t": 0.0}

    def run():
        c = get_launch(None)
        clock["t"] += 1e-3 * (1 + abs(c["scan_blocks"] - 512) / 512 + abs(c["graph_steps"] - 32) / 32)

    monkeypatch.setattr(AT.time, "perf_counter", lambda: clock["t"])
    return st, run


def test_search_descends_to_the_fastest_schedule(fake_lib, tmp_path):
    st, run = fake_lib
    space = {"scan_blocks": (256, 512, 1024), "graph_steps": (8, 32), "dl_blocks": (1024,), "del_scan_blocks": (2048,)}
    path = tmp_path / "rec.json"
    best, rec = AT.tune(object(), run, FakeTorch, space=space, reps=2, passes=3, path=str(path))
    assert best["scan_blocks"] == 512 and best["graph_steps"] == 32
    assert rec["default"]["schedule"]["scan_blocks"] == 1280
    assert rec["best"]["ms"] < rec["default"]["ms"]
    keys = [tuple(t["schedule"].values()) for t in rec["trials"]]
    assert len(keys) == len(set(keys))                # every schedule timed once
    assert all(len(t["runs_ms"]) == 2 for t in rec["trials"])
    assert st["cfg"]["scan_blocks"] == 512          # the handle keeps the winner
    assert st["loads"] == 3 * len(rec["trials"]) + 1  # restored before every run, and at the end
    assert path.exists()


def test_search_rejects_a_schedule_that_changes_results(fake_lib):
    st, run = fake_lib
    st["bad"] = 8
    space = {"scan_blocks": (), "graph_steps": (8, 32), "dl_blocks": (), "del_scan_blocks": ()}
    with pytest.raises(RuntimeError, match="changed the levels"):
        AT.tune(object(), run, FakeTorch, space=space, reps=1)
