"""The seeded input generators (host code shared by the oracle side and the
GPU side; no PLDS arithmetic)."""
import os

import numpy as np
import pytest

from paper_2106_03824_amd import workloads as W


@pytest.mark.parametrize("scale,m,threads", [(12, 70000, 4), (14, 2 ** 18, 8), (15, 3 * 2 ** 17, 3),
                                             (16, 2 ** 20, 16)])
def test_threaded_rmat_equals_sequential(scale, m, threads, monkeypatch):
    """The threaded R-MAT keeps exactly the first m distinct pairs in candidate
    order, like the one-candidate-at-a-time form, for any thread count."""
    monkeypatch.setenv("WL_THREADS", str(threads))
    L = W._lib()
    a = np.empty((m, 2), np.int32)
    b = np.empty((m, 2), np.int32)
    ra = L.wl_rmat(scale, m, 0.57, 0.19, 0.19, 7, 1, a.ctypes.data_as(W._I32P))
    rb = L.wl_rmat_seq(scale, m, 0.57, 0.19, 0.19, 7, 1, b.ctypes.data_as(W._I32P))
    assert ra == rb > m
    assert np.array_equal(a, b)


def test_rmat_edges_are_unique_canonical_pairs():
    e = W.rmat(13, 50000, seed=3)
    assert e.shape == (50000, 2)
    assert (e[:, 0] != e[:, 1]).all() and e.min() >= 0 and e.max() < 2 ** 13
    k = np.minimum(e[:, 0], e[:, 1]).astype(np.int64) << 32 | np.maximum(e[:, 0], e[:, 1])
    assert np.unique(k).size == k.size


def test_batched_graphs_recipe():
    """The batched form's workload: seeded (two calls agree), graph sizes and
    batch sizes in the stated ranges, insertions are new pairs, deletions are
    present edges without repeats, clamped to m."""
    def keys(e):
        e = np.asarray(e, dtype=np.int64)
        return (np.minimum(e[:, 0], e[:, 1]) << 32) | np.maximum(e[:, 0], e[:, 1])

    a = W.batched_graphs(12)
    b = W.batched_graphs(12)
    for (n, e, (kind, x)), (n2, e2, (kind2, x2)) in zip(a, b):
        assert n == n2 and kind == kind2 and np.array_equal(e, e2) and np.array_equal(x, x2)
    for i, (n, e, (kind, x)) in enumerate(a):
        assert 2 ** 10 - 1 <= n <= 2 ** 16 + 1
        if i % 2 == 1:
            assert n & (n - 1) == 0 and len(e) == 8 * n          # R-MAT, edge factor 8
        ke = keys(e)
        assert len(np.unique(ke)) == len(ke) and (e[:, 0] != e[:, 1]).all()
        kx = keys(x)
        assert len(np.unique(kx)) == len(kx)
        if kind == "ins":
            assert 10 ** 3 <= len(x) <= 5 * 10 ** 4 and not np.isin(kx, ke).any()
        else:
            assert len(x) <= min(5 * 10 ** 4, len(e)) and np.isin(kx, ke).all()
