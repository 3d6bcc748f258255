"""CPU oracle of the parallel level data structure (PLDS).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It wraps ``plds_oracle.c`` (plain sequential C, no code shared with
the GPU library) through ctypes.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)

ORA_OK, ORA_EINVAL, ORA_ERANGE, ORA_ENOMEM, ORA_ESTATE = 0, -1, -2, -3, -5

STAT_NAMES = (
    "applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up", "moves_down",
    "dl_calcs", "scan_up_deg", "scan_up_U", "scan_dl_deg", "scan_down_deg", "top_level",
    "viol_ins0", "viol_del0", "r14", "r15",
)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
        L.ora_create_ex.restype = ctypes.c_void_p
        L.ora_create_ex.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_int32]
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_info.argtypes = [ctypes.c_void_p, _I64P]
        L.ora_tables.argtypes = [ctypes.c_void_p, _I32P, _I32P, _F64P]
        L.ora_update.argtypes = [ctypes.c_void_p, _I32P, ctypes.c_int64, _I32P, ctypes.c_int64]
        L.ora_levels.argtypes = [ctypes.c_void_p, _I32P]
        L.ora_degrees.argtypes = [ctypes.c_void_p, _I32P]
        L.ora_coreness.argtypes = [ctypes.c_void_p, _I32P, ctypes.c_int64, _F64P]
        L.ora_estimate_exponent.argtypes = [ctypes.c_void_p, _I32P]
        L.ora_check.argtypes = [ctypes.c_void_p]
        L.ora_last_assert.argtypes = [ctypes.c_void_p]
        L.ora_stats.argtypes = [ctypes.c_void_p, _I64P]
        L.ora_edges.restype = ctypes.c_int64
        L.ora_edges.argtypes = [ctypes.c_void_p, _I32P]
        L.ora_load_state.argtypes = [ctypes.c_void_p, _I32P, ctypes.c_int64, _I32P]
        L.ora_exact_coreness.argtypes = [ctypes.c_int64, _I32P, ctypes.c_int64, _I32P]
        _LIB = L
    return _LIB


def _edges(e):
    if e is None:
        return np.zeros((0, 2), dtype=np.int32)
    a = np.ascontiguousarray(np.asarray(e, dtype=np.int32).reshape(-1, 2))
    return a


def _p(a, t):
    return a.ctypes.data_as(t)


class Oracle:
    """Sequential PLDS.  mode 0 keeps counters (Algorithms 2-3 as printed),
    mode 1 rescans every vertex at every level (slow cross-check).  coeff > 0
    (at least 1) replaces the Invariant-1 coefficient 2 + 3/lambda (the
    experiments' heuristic parameters use 1.1); jump=True moves insertion
    violators straight to their desire-level (the implementation's
    procedure) instead of one level at a time."""

    def __init__(self, n, delta=0.4, lam=3.0, levels_per_group=0, mode=0, coeff=0.0, jump=False):
        self._destroy = lib().ora_destroy        # bound now: module globals may be gone at exit
        self._h = lib().ora_create_ex(int(n), float(delta), float(lam), int(levels_per_group), int(mode),
                                      float(coeff), int(bool(jump)))
        if not self._h:
            raise ValueError("ora_create rejected its arguments")
        info = self.info()
        self.n, self.t, self.L, self.G, self.K = info["n"], info["t"], info["L"], info["G"], info["K"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def info(self):
        out = np.zeros(8, dtype=np.int64)
        lib().ora_info(self._h, _p(out, _I64P))
        return dict(zip(("n", "m", "t", "L", "G", "K", "mode"), (int(x) for x in out[:7])))

    @property
    def m(self):
        return self.info()["m"]

    def tables(self):
        G = self.G
        up = np.zeros(G, dtype=np.int32)
        dn = np.zeros(G, dtype=np.int32)
        pw = np.zeros(G, dtype=np.float64)
        lib().ora_tables(self._h, _p(up, _I32P), _p(dn, _I32P), _p(pw, _F64P))
        return up, dn, pw

    def update(self, ins=None, dele=None):
        a, b = _edges(ins), _edges(dele)
        return lib().ora_update(self._h, _p(a, _I32P), a.shape[0], _p(b, _I32P), b.shape[0])

    def insert(self, e):
        return self.update(ins=e)

    def delete(self, e):
        return self.update(dele=e)

    def levels(self):
        out = np.zeros(self.n, dtype=np.int32)
        lib().ora_levels(self._h, _p(out, _I32P))
        return out

    def degrees(self):
        out = np.zeros(self.n, dtype=np.int32)
        lib().ora_degrees(self._h, _p(out, _I32P))
        return out

    def coreness(self, vs=None):
        if vs is None:
            out = np.zeros(self.n, dtype=np.float64)
            lib().ora_coreness(self._h, None, 0, _p(out, _F64P))
            return out
        v = np.ascontiguousarray(np.asarray(vs, dtype=np.int32))
        out = np.zeros(v.shape[0], dtype=np.float64)
        lib().ora_coreness(self._h, _p(v, _I32P), v.shape[0], _p(out, _F64P))
        return out

    def exponents(self):
        out = np.zeros(self.n, dtype=np.int32)
        lib().ora_estimate_exponent(self._h, _p(out, _I32P))
        return out

    def check(self):
        return lib().ora_check(self._h)

    def last_assert(self):
        return lib().ora_last_assert(self._h)

    def stats(self):
        out = np.zeros(16, dtype=np.int64)
        lib().ora_stats(self._h, _p(out, _I64P))
        return dict(zip(STAT_NAMES, (int(x) for x in out)))

    def edges(self):
        m = lib().ora_edges(self._h, None)
        out = np.zeros((m, 2), dtype=np.int32)
        lib().ora_edges(self._h, _p(out, _I32P))
        return out

    def load_state(self, edges, levels):
        e = _edges(edges)
        lv = np.ascontiguousarray(np.asarray(levels, dtype=np.int32))
        return lib().ora_load_state(self._h, _p(e, _I32P), e.shape[0], _p(lv, _I32P))


def exact_coreness(n, edges):
    """Exact coreness of every vertex (bucket peeling)."""
    e = _edges(edges)
    out = np.zeros(int(n), dtype=np.int32)
    rc = lib().ora_exact_coreness(int(n), _p(e, _I32P), e.shape[0], _p(out, _I32P))
    if rc:
        raise MemoryError("ora_exact_coreness failed")
    return out
