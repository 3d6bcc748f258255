"""Thin ctypes binding of ``libplds.so`` (C ABI in ``include/plds.h``).

Functions carry the C names; pointers are taken from torch CUDA tensors (or
raw integer addresses) and streams from ``torch.cuda.current_stream()``.
Nothing here computes: every step of the path runs in the library's HIP
kernels.  Loading raises if the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplds.so")

PLDS_OK, PLDS_EINVAL, PLDS_ERANGE, PLDS_ENOMEM, PLDS_EHIP, PLDS_ESTATE = 0, -1, -2, -3, -4, -5
PLDS_LPG_OPT = -1   # levels per group of the PLDSOpt variant: ceil(log_{1+delta} n / 50)
PLDS_NOALLOC_MAX_N = 1 << 21   # largest handle of plds_static_kcore_noalloc (include/plds.h)


def lib_max_noalloc_n():
    return PLDS_NOALLOC_MAX_N


class PLDSError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class plds_options_t(ctypes.Structure):
    _fields_ = [("levels_per_group", ctypes.c_int32), ("up_jump", ctypes.c_int32),
                ("edge_capacity_hint", ctypes.c_int64), ("up_coeff", ctypes.c_double),
                ("reserved", ctypes.c_int64 * 4)]


class plds_launch_t(ctypes.Structure):
    _fields_ = [("scan_blocks", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("dl_blocks", ctypes.c_int32),
                ("del_scan_blocks", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


LAUNCH_FIELDS = ("scan_blocks", "graph_steps", "dl_blocks", "del_scan_blocks")


class plds_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("t", ctypes.c_int32), ("L", ctypes.c_int32),
                ("G", ctypes.c_int32), ("K", ctypes.c_int32), ("delta", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("slab_slots", ctypes.c_int64), ("slab_used", ctypes.c_int64),
                ("ngraphs", ctypes.c_int32), ("reserved32", ctypes.c_int32)]


STAT_FIELDS = ("applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up", "moves_down", "dl_calcs",
               "slots_scanned", "top_level", "viol_ins0", "viol_del0", "host_syncs", "alg_bytes_up",
               "timed_launches", "timed_ms", "alg_bytes_peel", "alg_bytes_up_loop", "ins_steps", "ins_loop_steps",
               "ins_loop_launches")


class plds_stats_t(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in STAT_FIELDS[:-6]] + [("timed_ms", ctypes.c_double),
                                                                   ("alg_bytes_peel", ctypes.c_int64),
                                                                   ("alg_bytes_up_loop", ctypes.c_int64),
                                                                   ("ins_steps", ctypes.c_int64),
                                                                   ("ins_loop_steps", ctypes.c_int64),
                                                                   ("ins_loop_launches", ctypes.c_int64)]

TIMED_KERNELS = {"ins_scan": 1, "del_scan": 2, "dl": 3, "ins_prep": 4, "flip_scan": 5, "ins_sweep": 6, "sk_relax": 7,
                 "apply_del": 8, "del_loop": 9, "jmp_scan": 10, "ins_loop": 11}


_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2106_03824_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.plds_create.argtypes = [_I64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_VP)]
        L.plds_create_ex.argtypes = [_I64, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _I64,
                                     ctypes.POINTER(_VP)]
        L.plds_create_opts.argtypes = [_I64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(plds_options_t),
                                       ctypes.POINTER(_VP)]
        L.plds_destroy.argtypes = [_VP]
        L.plds_create_multi.argtypes = [ctypes.c_int32, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _I64,
                                        ctypes.POINTER(_VP)]
        L.plds_update_multi.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP]
        L.plds_graph_info.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(_I64), ctypes.POINTER(plds_info_t)]
        L.plds_reset_graph.argtypes = [_VP, ctypes.c_int32, _I64, _VP]
        L.plds_graph_applied.argtypes = [_VP, _VP, _VP, _VP]
        L.plds_update.argtypes = [_VP, _VP, _I64, _VP, _I64, _VP]
        L.plds_batch_insert.argtypes = [_VP, _VP, _I64, _VP]
        L.plds_batch_delete.argtypes = [_VP, _VP, _I64, _VP]
        L.plds_coreness.argtypes = [_VP, _VP, _I64, _VP, _VP]
        L.plds_levels.argtypes = [_VP, _VP, _VP]
        L.plds_degrees.argtypes = [_VP, _VP, _VP]
        L.plds_info.argtypes = [_VP, ctypes.POINTER(plds_info_t)]
        L.plds_thresholds.argtypes = [_VP, _VP, _VP, _VP]
        L.plds_stats.argtypes = [_VP, ctypes.POINTER(plds_stats_t)]
        L.plds_set_timing.argtypes = [_VP, ctypes.c_int32]
        L.plds_step_log.argtypes = [_VP, _VP, _I64, ctypes.POINTER(_I64)]
        L.plds_set_sweep_mode.argtypes = [_VP, ctypes.c_int32]
        L.plds_set_launch.argtypes = [_VP, ctypes.POINTER(plds_launch_t)]
        L.plds_get_launch.argtypes = [_VP, ctypes.POINTER(plds_launch_t)]
        L.plds_dump_state.argtypes = [_VP, _VP, _I64, ctypes.POINTER(_I64), _VP, _VP]
        L.plds_load_state.argtypes = [_VP, _VP, _I64, _VP, _VP]
        L.plds_check.argtypes = [_VP, _VP]
        L.plds_sync.argtypes = [_VP, _VP]
        L.plds_orient.argtypes = [_VP, _VP, _I64, _VP, _VP]
        L.plds_track_orientation.argtypes = [_VP, ctypes.c_int32]
        L.plds_flips.argtypes = [_VP, _VP, _I64, ctypes.POINTER(_I64), _VP]
        L.plds_oriented_updates.argtypes = [_VP, _VP, _I64, ctypes.POINTER(_I64), _VP, _I64, ctypes.POINTER(_I64),
                                            _VP]
        L.plds_densest_value.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _VP]
        L.plds_static_kcore.argtypes = [_VP, ctypes.c_double, _VP, _VP]
        L.plds_static_kcore_noalloc.argtypes = [_VP, ctypes.c_double, _VP, _VP]
        L.plds_inject_alloc_failure.argtypes = [_I64]
        L.plds_delete_vertices.argtypes = [_VP, _VP, _I64, _VP]
        L.plds_rebuild.argtypes = [_VP, _I64, _VP, ctypes.POINTER(_VP), _VP]
        L.plds_strerror.restype = ctypes.c_char_p
        L.plds_strerror.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


EXPORTS = ("plds_create", "plds_create_ex", "plds_destroy", "plds_create_multi", "plds_update_multi",
           "plds_graph_info", "plds_update", "plds_batch_insert",
           "plds_batch_delete", "plds_coreness", "plds_levels", "plds_degrees", "plds_info", "plds_thresholds",
           "plds_stats", "plds_set_timing", "plds_set_sweep_mode", "plds_step_log", "plds_dump_state", "plds_load_state", "plds_check", "plds_sync", "plds_strerror",
           "plds_orient", "plds_track_orientation", "plds_flips", "plds_oriented_updates", "plds_densest_value",
           "plds_static_kcore", "plds_static_kcore_noalloc", "plds_delete_vertices", "plds_rebuild",
           "plds_inject_alloc_failure", "plds_create_opts", "plds_reset_graph",
           "plds_graph_applied", "plds_set_launch", "plds_get_launch")


def strerror(code):
    try:
        return lib().plds_strerror(int(code)).decode()
    except ImportError:
        return str(code)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _chk(rc, where):
    if rc != PLDS_OK:
        raise PLDSError(rc, where)
    return rc


def _edges_arg(e):
    if e is None:
        return None, 0
    assert e.dtype.itemsize == 4 and e.is_cuda and e.is_contiguous() and e.dim() == 2 and e.shape[1] == 2
    return _ptr(e), int(e.shape[0])


# ---------------------------------------------------------------- C names
def plds_create(n, delta, lam):
    h = _VP()
    _chk(lib().plds_create(int(n), float(delta), float(lam), ctypes.byref(h)), "plds_create")
    return h


def plds_create_opts(n, delta, lam, levels_per_group=0, edge_capacity_hint=0, up_coeff=0.0, up_jump=False):
    o = plds_options_t()
    o.levels_per_group, o.up_jump = int(levels_per_group), int(bool(up_jump))
    o.edge_capacity_hint, o.up_coeff = int(edge_capacity_hint), float(up_coeff)
    h = _VP()
    _chk(lib().plds_create_opts(int(n), float(delta), float(lam), ctypes.byref(o), ctypes.byref(h)),
         "plds_create_opts")
    return h


def plds_create_ex(n, delta, lam, levels_per_group=0, edge_capacity_hint=0):
    h = _VP()
    _chk(lib().plds_create_ex(int(n), float(delta), float(lam), int(levels_per_group), int(edge_capacity_hint),
                              ctypes.byref(h)), "plds_create_ex")
    return h


def plds_destroy(h):
    return _chk(lib().plds_destroy(h), "plds_destroy")


def plds_create_multi(ns, delta, lam, levels_per_group=0, edge_capacity_hint=0):
    k = len(ns)
    arr = (ctypes.c_int64 * k)(*[int(x) for x in ns])
    h = _VP()
    _chk(lib().plds_create_multi(k, ctypes.addressof(arr), float(delta), float(lam), int(levels_per_group),
                                 int(edge_capacity_hint), ctypes.byref(h)), "plds_create_multi")
    return h


def plds_update_multi(h, ins=None, dele=None, stream=None, check=True):
    """ins, dele: sequences with one entry per graph (an int32 [count, 2]
    device tensor in the graph's own ids, or None), or None."""
    def arrays(lists):
        if lists is None:
            return None, None, None
        k = len(lists)
        ptrs = (ctypes.c_void_p * k)()
        cnts = (ctypes.c_int64 * k)()
        for i, e in enumerate(lists):
            p, c = _edges_arg(e)
            ptrs[i], cnts[i] = p, c
        return ptrs, cnts, (ctypes.addressof(ptrs), ctypes.addressof(cnts))
    pi, ci, ai = arrays(ins)
    pd, cd, ad = arrays(dele)
    rc = lib().plds_update_multi(h, ai[0] if ai else None, ai[1] if ai else None, ad[0] if ad else None,
                                 ad[1] if ad else None, _stream(stream))
    return _chk(rc, "plds_update_multi") if check else rc


def plds_graph_applied(h, ngraphs, stream=None):
    """(applied insertions, applied deletions) per graph of the last update call."""
    a = (ctypes.c_int64 * ngraphs)()
    b = (ctypes.c_int64 * ngraphs)()
    _chk(lib().plds_graph_applied(h, ctypes.addressof(a), ctypes.addressof(b), _stream(stream)),
         "plds_graph_applied")
    return list(a), list(b)


def plds_reset_graph(h, g, n_new, stream=None):
    return _chk(lib().plds_reset_graph(h, int(g), int(n_new), _stream(stream)), "plds_reset_graph")


def plds_graph_info(h, g):
    i = plds_info_t()
    base = _I64()
    _chk(lib().plds_graph_info(h, int(g), ctypes.byref(base), ctypes.byref(i)), "plds_graph_info")
    d = {f: getattr(i, f) for f, _ in plds_info_t._fields_}
    d["base"] = base.value
    return d


def plds_update(h, ins=None, dele=None, stream=None, check=True):
    pi, ni = _edges_arg(ins)
    pd, nd = _edges_arg(dele)
    rc = lib().plds_update(h, pi, ni, pd, nd, _stream(stream))
    return _chk(rc, "plds_update") if check else rc


def plds_batch_insert(h, edges, stream=None, check=True):
    p, c = _edges_arg(edges)
    rc = lib().plds_batch_insert(h, p, c, _stream(stream))
    return _chk(rc, "plds_batch_insert") if check else rc


def plds_batch_delete(h, edges, stream=None, check=True):
    p, c = _edges_arg(edges)
    rc = lib().plds_batch_delete(h, p, c, _stream(stream))
    return _chk(rc, "plds_batch_delete") if check else rc


def plds_coreness(h, vertices, out, stream=None):
    cnt = 0 if vertices is None else int(vertices.numel())
    return _chk(lib().plds_coreness(h, _ptr(vertices), cnt, _ptr(out), _stream(stream)), "plds_coreness")


def plds_orient(h, edges, out, stream=None):
    p, c = _edges_arg(edges)
    return _chk(lib().plds_orient(h, p, c, _ptr(out), _stream(stream)), "plds_orient")


def plds_track_orientation(h, on):
    return _chk(lib().plds_track_orientation(h, 1 if on else 0), "plds_track_orientation")


def plds_flips(h, out, stream=None):
    """Returns the number of flipped edges (rows of `out` beyond it are unset;
    only the first out.shape[0] are written)."""
    cnt = _I64()
    cap = 0 if out is None else int(out.shape[0])
    _chk(lib().plds_flips(h, _ptr(out), cap, ctypes.byref(cnt), _stream(stream)), "plds_flips")
    return cnt.value


def plds_oriented_updates(h, ins_out, del_out, stream=None):
    """Returns (applied insertions, applied deletions) of the last call."""
    ni, nd = _I64(), _I64()
    ci = 0 if ins_out is None else int(ins_out.shape[0])
    cd = 0 if del_out is None else int(del_out.shape[0])
    _chk(lib().plds_oriented_updates(h, _ptr(ins_out), ci, ctypes.byref(ni), _ptr(del_out), cd, ctypes.byref(nd),
                                     _stream(stream)), "plds_oriented_updates")
    return ni.value, nd.value


def plds_densest_value(h, graph=0, stream=None):
    out = ctypes.c_double()
    _chk(lib().plds_densest_value(h, int(graph), ctypes.byref(out), _stream(stream)), "plds_densest_value")
    return out.value


def plds_static_kcore(h, eps, out, stream=None):
    return _chk(lib().plds_static_kcore(h, float(eps), _ptr(out), _stream(stream)), "plds_static_kcore")


def plds_inject_alloc_failure(after):
    """Testing aid: the library's allocation after `after` more on this
    thread fails (after < 0: off)."""
    return _chk(lib().plds_inject_alloc_failure(int(after)), "plds_inject_alloc_failure")


def plds_static_kcore_noalloc(h, eps, out, stream=None):
    """As plds_static_kcore, with the library's fixed per-device scratch array
    instead of memory allocated on first use (n <= PLDS_NOALLOC_MAX_N)."""
    return _chk(lib().plds_static_kcore_noalloc(h, float(eps), _ptr(out), _stream(stream)),
                "plds_static_kcore_noalloc")


def plds_delete_vertices(h, vertices, stream=None, check=True):
    cnt = 0 if vertices is None else int(vertices.numel())
    rc = lib().plds_delete_vertices(h, _ptr(vertices), cnt, _stream(stream))
    return _chk(rc, "plds_delete_vertices") if check else rc


def plds_rebuild(h, new_n, relabel=None, stream=None):
    """Returns the new handle."""
    out = _VP()
    _chk(lib().plds_rebuild(h, int(new_n), _ptr(relabel), ctypes.byref(out), _stream(stream)), "plds_rebuild")
    return out.value


def plds_levels(h, out, stream=None):
    return _chk(lib().plds_levels(h, _ptr(out), _stream(stream)), "plds_levels")


def plds_degrees(h, out, stream=None):
    return _chk(lib().plds_degrees(h, _ptr(out), _stream(stream)), "plds_degrees")


def plds_info(h):
    i = plds_info_t()
    _chk(lib().plds_info(h, ctypes.byref(i)), "plds_info")
    return {f: getattr(i, f) for f, _ in plds_info_t._fields_}


def plds_thresholds(h, G):
    up = (ctypes.c_int32 * G)()
    dn = (ctypes.c_int32 * G)()
    pw = (ctypes.c_double * G)()
    _chk(lib().plds_thresholds(h, ctypes.addressof(up), ctypes.addressof(dn), ctypes.addressof(pw)),
         "plds_thresholds")
    return list(up), list(dn), list(pw)


def plds_stats(h):
    s = plds_stats_t()
    _chk(lib().plds_stats(h, ctypes.byref(s)), "plds_stats")
    return {f: getattr(s, f) for f in STAT_FIELDS}


def plds_set_sweep_mode(h, mode):
    return _chk(lib().plds_set_sweep_mode(h, int(mode)), "plds_set_sweep_mode")


def plds_set_launch(h, **fields):
    """Sets the launch schedule; fields not given (or 0) take their defaults."""
    bad = set(fields) - set(LAUNCH_FIELDS)
    if bad:
        raise TypeError(f"unknown launch fields {sorted(bad)}")
    c = plds_launch_t(**{k: int(v) for k, v in fields.items()})
    return _chk(lib().plds_set_launch(h, ctypes.byref(c)), "plds_set_launch")


def plds_get_launch(h):
    c = plds_launch_t()
    _chk(lib().plds_get_launch(h, ctypes.byref(c)), "plds_get_launch")
    return {f: getattr(c, f) for f in LAUNCH_FIELDS}


def plds_set_timing(h, kernel):
    k = int(TIMED_KERNELS.get(kernel, kernel)) if isinstance(kernel, str) else int(kernel)
    return _chk(lib().plds_set_timing(h, k), "plds_set_timing")


def plds_step_log(h, cap=100000):
    import numpy as np
    out = np.zeros((cap, 4), dtype=np.int64)
    rows = _I64()
    _chk(lib().plds_step_log(h, out.ctypes.data, cap, ctypes.byref(rows)), "plds_step_log")
    return out[:min(rows.value, cap)]


def plds_dump_state(h, edges_out, levels_out, stream=None):
    m = _I64()
    cap = 0 if edges_out is None else int(edges_out.shape[0])
    _chk(lib().plds_dump_state(h, _ptr(edges_out), cap, ctypes.byref(m), _ptr(levels_out), _stream(stream)),
         "plds_dump_state")
    return m.value


def plds_load_state(h, edges, levels, stream=None, check=True):
    p, c = _edges_arg(edges)
    rc = lib().plds_load_state(h, p, c, _ptr(levels), _stream(stream))
    return _chk(rc, "plds_load_state") if check else rc


def plds_check(h, stream=None):
    return lib().plds_check(h, _stream(stream))


def plds_sync(h, stream=None):
    return lib().plds_sync(h, _stream(stream))


# ----------------------------------------------------------- convenience
class PLDS:
    """Owning wrapper: one handle on the current device."""

    def __init__(self, n, delta=0.4, lam=3.0, levels_per_group=0, edge_capacity_hint=0, _handle=None,
                 up_coeff=0.0, up_jump=False):
        if _handle is not None:
            self.h = _handle
        elif up_coeff or up_jump:
            self.h = plds_create_opts(n, delta, lam, levels_per_group, edge_capacity_hint, up_coeff, up_jump)
        else:
            self.h = plds_create_ex(n, delta, lam, levels_per_group, edge_capacity_hint)
        info = plds_info(self.h)
        self.n, self.L, self.G, self.K, self.t = info["n"], info["L"], info["G"], info["K"], info["t"]

    def close(self):
        if getattr(self, "h", None):
            plds_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, e):
        import torch
        if e is None:
            return None
        t = torch.as_tensor(e, dtype=torch.int32).reshape(-1, 2)
        return t.to("cuda").contiguous()

    def update(self, ins=None, dele=None, check=True):
        return plds_update(self.h, self._dev(ins), self._dev(dele), check=check)

    def insert(self, e, check=True):
        return self.update(ins=e, check=check)

    def delete(self, e, check=True):
        return self.update(dele=e, check=check)

    def levels(self):
        import torch
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        plds_levels(self.h, out)
        return out

    def degrees(self):
        import torch
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        plds_degrees(self.h, out)
        return out

    def coreness(self, vertices=None):
        import torch
        cnt = self.n if vertices is None else int(vertices.numel())
        out = torch.empty(cnt, dtype=torch.float64, device="cuda")
        plds_coreness(self.h, vertices, out)
        return out

    def stats(self):
        return plds_stats(self.h)

    def info(self):
        return plds_info(self.h)

    def thresholds(self):
        return plds_thresholds(self.h, self.G)

    def check(self):
        return plds_check(self.h)

    def dump(self):
        import torch
        m = self.info()["m"]
        e = torch.empty((max(m, 1), 2), dtype=torch.int32, device="cuda")
        lv = torch.empty(self.n, dtype=torch.int32, device="cuda")
        got = plds_dump_state(self.h, e, lv)
        return e[:got], lv

    def load(self, edges, levels, check=True):
        import torch
        lv = torch.as_tensor(levels, dtype=torch.int32).to("cuda").contiguous()
        return plds_load_state(self.h, self._dev(edges), lv, check=check)

    def orient(self, edges):
        import torch
        e = self._dev(edges)
        out = torch.empty_like(e)
        plds_orient(self.h, e, out)
        return out

    def track_orientation(self, on=True):
        plds_track_orientation(self.h, on)

    def flips(self):
        """F of the last update call: device int32 [k, 2] (tail, head) as before."""
        import torch
        k = plds_flips(self.h, None)
        out = torch.empty((max(k, 1), 2), dtype=torch.int32, device="cuda")
        k2 = plds_flips(self.h, out)
        assert k2 == k
        return out[:k]

    def oriented_updates(self):
        """J of the last update call: (insertions after, deletions before)."""
        import torch
        ni, nd = plds_oriented_updates(self.h, None, None)
        a = torch.empty((max(ni, 1), 2), dtype=torch.int32, device="cuda")
        b = torch.empty((max(nd, 1), 2), dtype=torch.int32, device="cuda")
        plds_oriented_updates(self.h, a, b)
        return a[:ni], b[:nd]

    def densest_value(self, graph=0):
        return plds_densest_value(self.h, graph)

    def delete_vertices(self, vertices, check=True):
        import torch
        v = torch.as_tensor(vertices, dtype=torch.int32).reshape(-1).to("cuda").contiguous()
        return plds_delete_vertices(self.h, v, check=check)

    def rebuild(self, new_n, relabel=None):
        """A new PLDS holding this graph with new_n vertices (see plds_rebuild)."""
        import torch
        r = None if relabel is None else torch.as_tensor(relabel, dtype=torch.int32).to("cuda").contiguous()
        return PLDS(new_n, _handle=plds_rebuild(self.h, new_n, r))

    def static_kcore(self, eps):
        """Algorithm 6's estimates of the current graph: device float64 [n]."""
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        plds_static_kcore(self.h, eps, out)
        return out


class MultiPLDS(PLDS):
    """Owning wrapper of a multi-graph handle: graph g has ns[g] vertices and
    occupies global ids [base[g], base[g] + ns[g])."""

    def __init__(self, ns, delta=0.4, lam=3.0, levels_per_group=0, edge_capacity_hint=0):
        super().__init__(0, _handle=plds_create_multi(ns, delta, lam, levels_per_group, edge_capacity_hint))
        self.graphs = [plds_graph_info(self.h, g) for g in range(len(ns))]
        self.base = [gi["base"] for gi in self.graphs]
        self.ns = [gi["n"] for gi in self.graphs]

    def update_multi(self, ins=None, dele=None, check=True):
        dev = lambda lists: None if lists is None else [self._dev(e) if e is not None and len(e) else None
                                                        for e in lists]
        return plds_update_multi(self.h, dev(ins), dev(dele), check=check)

    def reset_graph(self, g, n_new, stream=None):
        """Empty graph g and give it n_new (<= its capacity) vertices."""
        plds_reset_graph(self.h, g, n_new, stream)
        self.ns[g] = int(n_new)
        self.graphs[g] = plds_graph_info(self.h, g)

    def graph_levels(self, g, levels=None):
        lv = self.levels() if levels is None else levels
        return lv[self.base[g]:self.base[g] + self.ns[g]]
