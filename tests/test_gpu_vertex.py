"""Vertex updates on the GPU against the oracle (oracle/vertex.py): vertex
deletion as the batch of its edges' deletions, vertex insertion past n and
renumbering as a rebuild."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.vertex as OV
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


def same_state(g, o):
    assert (g.levels().cpu().numpy() == o.levels()).all()
    assert np.array_equal(g.coreness().cpu().numpy().view(np.int64), o.coreness().view(np.int64))
    assert (g.degrees().cpu().numpy() == o.degrees()).all()
    assert g.check() == 0


def test_delete_vertices_matches_oracle():
    n = 2 ** 12
    e = W.rmat(12, 16 * n, seed=6)
    say("delete vertices rmat12")
    g, o = lib().PLDS(n), O.Oracle(n)
    assert g.insert(e) == 0 and o.insert(e) == 0
    deg = o.degrees()
    rng = np.random.default_rng(1)
    vs = np.concatenate([[int(deg.argmax())], rng.integers(0, n, 60), [5, 5]]).astype(np.int32)
    assert g.delete_vertices(vs) == 0
    assert OV.delete_vertices(o, vs) == 0
    same_state(g, o)
    s, so = g.stats(), o.stats()
    for k in ("applied_del", "sweeps_del", "moves_down"):
        assert s[k] == so[k], k
    lv = g.levels().cpu().numpy()
    assert (g.degrees().cpu().numpy()[vs] == 0).all() and (lv[vs] == 0).all()
    say("delete vertices: none, isolated, out of range")
    assert g.delete_vertices([]) == 0
    assert g.delete_vertices(vs[:3]) == 0             # already isolated
    same_state(g, o)
    assert g.delete_vertices([1, n], check=False) == lib().PLDS_ERANGE
    same_state(g, o)


def test_delete_vertices_every_slab_class_and_long_list():
    """Deleted vertices of every slab size (hubs of several thousand slots,
    mid-size slabs, slabs of 8 and 16), and a list longer than n with
    repeats (gathered a wavefront per listed vertex)."""
    n = 2 ** 13
    rng = np.random.default_rng(21)
    e = [(h, v) for h in (0, 1) for v in range(2, n) if rng.random() < 0.8]
    e += [(v, int(x)) for v in range(2, 30) for x in rng.integers(30, n, size=300)]
    e += [(int(a), int(b)) for a, b in rng.integers(30, n, size=(4 * n, 2))]
    e = np.array(e, dtype=np.int32)
    say("delete vertices: slab classes")
    g, o = lib().PLDS(n), O.Oracle(n)
    assert g.insert(e) == 0 and o.insert(e) == 0
    vs = np.concatenate([[0, 1], np.arange(2, 12), rng.integers(30, n, 400)]).astype(np.int32)
    assert g.delete_vertices(vs) == 0
    assert OV.delete_vertices(o, vs) == 0
    same_state(g, o)
    say("delete vertices: a list longer than n")
    vs2 = rng.integers(0, n, 3 * n).astype(np.int32)
    assert g.delete_vertices(vs2) == 0
    assert OV.delete_vertices(o, vs2) == 0
    same_state(g, o)
    assert g.stats()["applied_del"] == o.stats()["applied_del"]


def test_rebuild_grows_and_keeps_ids():
    n = 3000
    e = W.er(n, 10.0 / n, seed=2)
    say("rebuild grow")
    g, o = lib().PLDS(n), O.Oracle(n)
    assert g.insert(e) == 0 and o.insert(e) == 0
    g2 = g.rebuild(2 * n)
    o2, rc = OV.rebuild(o, 2 * n)
    assert rc == 0 and (g2.n, g2.L, g2.K) == (o2.n, o2.L, o2.K)
    same_state(g2, o2)
    same_state(g, o)                                  # the old handle is unchanged
    say("rebuild grow: edges of new vertices")
    rng = np.random.default_rng(3)
    ins = np.stack([rng.integers(n, 2 * n, 5000), rng.integers(0, 2 * n, 5000)], axis=1).astype(np.int32)
    assert g2.insert(ins) == 0 and o2.insert(ins) == 0
    same_state(g2, o2)
    g2.close()


@pytest.mark.parametrize("lpg", [0, -1, 3])
def test_rebuild_renumbers(lpg):
    n = 2 ** 11
    e = W.rmat(11, 8 * n, seed=7)
    say("rebuild renumber", lpg)
    g, o = lib().PLDS(n, levels_per_group=lpg), O.Oracle(n, 0.4, 3.0, lpg)
    assert g.insert(e) == 0 and o.insert(e) == 0
    vs = np.arange(0, n, 3, dtype=np.int32)
    assert g.delete_vertices(vs) == 0 and OV.delete_vertices(o, vs) == 0
    deg = o.degrees()
    keep = deg > 0
    relabel = np.full(n, -1, dtype=np.int32)
    relabel[keep] = np.arange(int(keep.sum()), dtype=np.int32)
    relabel[7] = -1                                   # also drop a vertex that has edges
    n2 = int(keep.sum())
    g2 = g.rebuild(n2, relabel)
    o2, rc = OV.rebuild(o, n2, relabel, lpg)
    assert rc == 0
    same_state(g2, o2)
    say("rebuild errors")
    with pytest.raises(lib().PLDSError):
        g.rebuild(n - 1)                               # shrinking without a renumbering
    bad = relabel.copy()
    bad[keep.argmax()] = n2                            # a new id out of range
    with pytest.raises(lib().PLDSError):
        g.rebuild(n2, bad)
    m = lib().MultiPLDS([10, 20])
    with pytest.raises(lib().PLDSError):
        lib().plds_rebuild(m.h, 40)
    g2.close()
