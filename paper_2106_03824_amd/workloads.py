"""Seeded synthetic inputs: R-MAT and G(n,p) graphs and update batches.

This module produces inputs only; it holds none of the PLDS arithmetic.  Both
the GPU library's tests and benchmark and the CPU oracle's tests draw their
graphs and batches from here, through ``csrc/workloads.c``.

Seeds: a graph uses seed 1 by default; batch stream ``j`` of workload ``c``
uses seed ``1000*c + j``.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "workloads.c")
LIB = os.path.join(HERE, "libplds_workloads.so")
_LIB = None
_I32P = ctypes.POINTER(ctypes.c_int32)
_U8P = ctypes.POINTER(ctypes.c_uint8)
_U64P = ctypes.POINTER(ctypes.c_uint64)


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-Wall", "-fPIC", "-shared", "-pthread", SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _lib():
    global _LIB
    if _LIB is None:
        L = ctypes.CDLL(build(force=False))
        L.wl_rmat.restype = ctypes.c_int64
        L.wl_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_uint64, ctypes.c_int32, _I32P]
        L.wl_rmat_seq.restype = ctypes.c_int64
        L.wl_rmat_seq.argtypes = L.wl_rmat.argtypes
        L.wl_er.restype = ctypes.c_int64
        L.wl_er.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, _I32P, ctypes.c_int64]
        L.wl_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, _I32P]
        L.wl_permute_edges.argtypes = [_I32P, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
        L.wl_new_pairs.argtypes = [ctypes.c_int64, _I32P, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_uint64, _I32P]
        L.wl_sample_edges.argtypes = [_I32P, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, _I32P]
        L.wl_filter_present.argtypes = [_I32P, ctypes.c_int64, _I32P, ctypes.c_int64, _U8P]
        L.wl_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, _U64P]
        _LIB = L
    return _LIB


def _e(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 2))


def rmat(scale, m, a=0.57, b=0.19, c=0.19, seed=1, relabel=True):
    """``m`` unique undirected R-MAT edges on ``2**scale`` vertices, int32 [m,2]."""
    out = np.empty((int(m), 2), dtype=np.int32)
    r = _lib().wl_rmat(int(scale), int(m), float(a), float(b), float(c), int(seed), int(bool(relabel)),
                       out.ctypes.data_as(_I32P))
    if r < 0:
        raise ValueError("rmat: bad arguments")
    return out


def er(n, p, seed=1):
    """G(n,p) edge list, int32 [m,2] (pairs (v,w) with w < v)."""
    cap = int(n * (n - 1) / 2 * p * 1.2 + 64)
    while True:
        out = np.empty((cap, 2), dtype=np.int32)
        k = _lib().wl_er(int(n), float(p), int(seed), out.ctypes.data_as(_I32P), cap)
        if k < 0:
            raise ValueError("er: bad arguments")
        if k <= cap:
            return out[:k].copy()
        cap = int(k)


def permutation(n, seed, stream=0):
    out = np.empty(int(n), dtype=np.int32)
    _lib().wl_permutation(int(n), int(seed), int(stream), out.ctypes.data_as(_I32P))
    return out


def permute_edges(edges, seed, stream=0):
    e = _e(edges).copy()
    _lib().wl_permute_edges(e.ctypes.data_as(_I32P), e.shape[0], int(seed), int(stream))
    return e


def new_pairs(n, edges, count, seed, stream=0):
    """``count`` distinct uniform pairs u != v absent from ``edges``."""
    e = _e(edges)
    out = np.empty((int(count), 2), dtype=np.int32)
    rc = _lib().wl_new_pairs(int(n), e.ctypes.data_as(_I32P), e.shape[0], int(count), int(seed), int(stream),
                             out.ctypes.data_as(_I32P))
    if rc:
        raise ValueError("new_pairs: bad arguments")
    return out


def sample_edges(edges, count, seed, stream=0):
    """``count`` edges of ``edges`` drawn uniformly without replacement."""
    e = _e(edges)
    out = np.empty((int(count), 2), dtype=np.int32)
    rc = _lib().wl_sample_edges(e.ctypes.data_as(_I32P), e.shape[0], int(count), int(seed), int(stream),
                                out.ctypes.data_as(_I32P))
    if rc:
        raise ValueError("sample_edges: bad arguments")
    return out


def present(edges, query):
    """Boolean mask: which undirected pairs of ``query`` occur in ``edges``."""
    e, q = _e(edges), _e(query)
    out = np.zeros(q.shape[0], dtype=np.uint8)
    _lib().wl_filter_present(e.ctypes.data_as(_I32P), e.shape[0], q.ctypes.data_as(_I32P), q.shape[0],
                             out.ctypes.data_as(_U8P))
    return out.astype(bool)


def draws(seed, stream, count):
    """Raw 64-bit counter-based draws, for seeded choices made in Python."""
    out = np.empty(int(count), dtype=np.uint64)
    _lib().wl_draws(int(seed), int(stream), int(count), out.ctypes.data_as(_U64P))
    return out


def uniforms(seed, stream, count):
    return (draws(seed, stream, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ------------------------------------------------------------ update streams
def _keys(e):
    e = np.asarray(e, dtype=np.int64).reshape(-1, 2)
    a, b = np.minimum(e[:, 0], e[:, 1]), np.maximum(e[:, 0], e[:, 1])
    return (a << 32) | b


def _unkeys(k):
    return np.stack([(k >> 32).astype(np.int32), (k & 0xffffffff).astype(np.int32)], axis=1)


class RmatStream:
    """An R-MAT graph built by insertion batches, followed by update batches.

    The graph: ``m`` unique edges on ``2**scale`` vertices (a=0.57, b=0.19,
    c=0.19, seed ``seed``), inserted as ``build_batches`` batches of a seeded
    random permutation (seed ``1000*cfg + 1``).  Update batch ``j`` uses seed
    ``1000*cfg + 100 + j``: insertions are new uniform pairs absent from the
    current graph, deletions are current edges sampled uniformly without
    replacement, mixed batches are half of each.  The current edge set is
    tracked here so every batch is a pure function of (cfg, seed, j).
    """

    def __init__(self, scale, m, seed=1, build_batches=16, cfg=2):
        self.n = 2 ** scale
        self.cfg = cfg
        e = rmat(scale, m, seed=seed)
        perm = permute_edges(e, 1000 * cfg + 1)
        self.build = np.array_split(perm, build_batches)
        self.cur = np.sort(_keys(e))
        self.j = 0

    def edges(self):
        return _unkeys(self.cur)

    def _seed(self):
        s = 1000 * self.cfg + 100 + self.j
        self.j += 1
        return s

    def insert_batch(self, count):
        ins = new_pairs(self.n, self.edges(), count, self._seed())
        self.cur = np.sort(np.concatenate([self.cur, _keys(ins)]))
        return ins

    def delete_batch(self, count):
        dele = sample_edges(self.edges(), count, self._seed())
        self.cur = np.setdiff1d(self.cur, _keys(dele), assume_unique=True)
        return dele

    def mixed_batch(self, count):
        half = count // 2
        ins = new_pairs(self.n, self.edges(), count - half, self._seed())
        dele = sample_edges(self.edges(), half, self._seed())
        cur = np.setdiff1d(self.cur, _keys(dele), assume_unique=True)
        self.cur = np.sort(np.concatenate([cur, _keys(ins)]))
        return ins, dele


def batched_graphs(k, seed=4000):
    """The batched form's workload: k graphs of uneven size, alternately
    Erdos-Renyi G(n, p) (n log-uniform in [2^10, 2^16], mean degree uniform
    in [4, 32]) and R-MAT (scale uniform in [10, 16], edge factor 8), each
    with one measured batch: insertions of new pairs or deletions of present
    edges (probability 1/2 each), size uniform in [10^3, 5*10^4], deletions
    clamped to m.  Returns [(n, edges, (kind, batch))]; graph i draws with
    seed + i, its batch with seed + 500 + i."""
    import random
    rng = random.Random(seed)
    graphs = []
    for i in range(k):
        if i % 2 == 0:
            n = int(round(2 ** rng.uniform(10, 16)))
            e = er(n, rng.uniform(4, 32) / (n - 1), seed=seed + i)
        else:
            sc = rng.randint(10, 16)
            n = 2 ** sc
            e = rmat(sc, 8 * n, seed=seed + i)
        size = rng.randint(10 ** 3, 5 * 10 ** 4)
        if rng.random() < 0.5:
            b = ("ins", new_pairs(n, e, size, seed + 500 + i))
        else:
            b = ("del", sample_edges(e, min(size, len(e)), seed + 500 + i))
        graphs.append((n, e, b))
    return graphs
