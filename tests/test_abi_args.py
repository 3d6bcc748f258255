"""Argument checks of the C ABI that come before any device work, so they
run without a GPU: every entry point rejects a NULL handle with
PLDS_EINVAL, the create calls reject bad sizes and constants (leaving *out
NULL), and every error code has its own message."""
import ctypes
import math

import pytest

from paper_2106_03824_amd import plds as P

I64 = ctypes.c_int64


@pytest.fixture(scope="module")
def L():
    try:
        return P.lib()
    except (ImportError, OSError) as e:
        pytest.skip(f"library not built: {e}")


def test_null_handle_everywhere(L):
    E = P.PLDS_EINVAL
    n = I64()
    info = P.plds_info_t()
    stats = P.plds_stats_t()
    launch = P.plds_launch_t()
    out = ctypes.c_void_p()
    calls = {
        "plds_destroy": lambda: L.plds_destroy(None),
        "plds_update": lambda: L.plds_update(None, None, 0, None, 0, None),
        "plds_update_multi": lambda: L.plds_update_multi(None, None, None, None, None, None),
        "plds_graph_applied": lambda: L.plds_graph_applied(None, None, None, None),
        "plds_reset_graph": lambda: L.plds_reset_graph(None, 0, 16, None),
        "plds_graph_info": lambda: L.plds_graph_info(None, 0, None, None),
        "plds_batch_insert": lambda: L.plds_batch_insert(None, None, 0, None),
        "plds_batch_delete": lambda: L.plds_batch_delete(None, None, 0, None),
        "plds_coreness": lambda: L.plds_coreness(None, None, 0, None, None),
        "plds_levels": lambda: L.plds_levels(None, None, None),
        "plds_degrees": lambda: L.plds_degrees(None, None, None),
        "plds_info": lambda: L.plds_info(None, ctypes.byref(info)),
        "plds_thresholds": lambda: L.plds_thresholds(None, None, None, None),
        "plds_stats": lambda: L.plds_stats(None, ctypes.byref(stats)),
        "plds_set_timing": lambda: L.plds_set_timing(None, 1),
        "plds_set_sweep_mode": lambda: L.plds_set_sweep_mode(None, 1),
        "plds_set_launch": lambda: L.plds_set_launch(None, ctypes.byref(launch)),
        "plds_get_launch": lambda: L.plds_get_launch(None, ctypes.byref(launch)),
        "plds_step_log": lambda: L.plds_step_log(None, None, 0, ctypes.byref(n)),
        "plds_dump_state": lambda: L.plds_dump_state(None, None, 0, ctypes.byref(n), None, None),
        "plds_load_state": lambda: L.plds_load_state(None, None, 0, None, None),
        "plds_check": lambda: L.plds_check(None, None),
        "plds_sync": lambda: L.plds_sync(None, None),
        "plds_orient": lambda: L.plds_orient(None, None, 0, None, None),
        "plds_track_orientation": lambda: L.plds_track_orientation(None, 1),
        "plds_flips": lambda: L.plds_flips(None, None, 0, ctypes.byref(n), None),
        "plds_oriented_updates": lambda: L.plds_oriented_updates(None, None, 0, ctypes.byref(n), None, 0,
                                                                 ctypes.byref(n), None),
        "plds_densest_value": lambda: L.plds_densest_value(None, 0, ctypes.byref(ctypes.c_double()), None),
        "plds_static_kcore": lambda: L.plds_static_kcore(None, 0.5, None, None),
        "plds_static_kcore_noalloc": lambda: L.plds_static_kcore_noalloc(None, 0.5, None, None),
        "plds_delete_vertices": lambda: L.plds_delete_vertices(None, None, 0, None),
        "plds_rebuild": lambda: L.plds_rebuild(None, 16, None, ctypes.byref(out), None),
    }
    for name, call in calls.items():
        assert call() == E, name
    assert out.value is None                      # plds_rebuild cleared *out


def test_create_rejects_bad_arguments(L):
    E = P.PLDS_EINVAL
    out = ctypes.c_void_p(1)
    for n, d, lam in [(0, 0.4, 3.0), (-1, 0.4, 3.0), (2 ** 31, 0.4, 3.0), (100, 0.0, 3.0), (100, -0.4, 3.0),
                      (100, math.nan, 3.0), (100, math.inf, 3.0), (100, 0.4, 0.0), (100, 0.4, math.nan)]:
        out.value = 1
        assert L.plds_create(n, d, lam, ctypes.byref(out)) == E, (n, d, lam)
        assert not out.value
    assert L.plds_create(100, 0.4, 3.0, None) == E
    assert L.plds_create_ex(100, 0.4, 3.0, -5, 0, ctypes.byref(out)) == E       # levels per group
    assert L.plds_create_ex(100, 0.4, 3.0, 0, -1, ctypes.byref(out)) == E       # capacity hint
    ns = (I64 * 3)(100, 0, 50)
    assert L.plds_create_multi(3, ns, 0.4, 3.0, 0, 0, ctypes.byref(out)) == E   # an empty graph
    ns = (I64 * 2)(2 ** 30, 2 ** 30)
    assert L.plds_create_multi(2, ns, 0.4, 3.0, 0, 0, ctypes.byref(out)) == E   # ids past int32
    assert L.plds_create_multi(0, ns, 0.4, 3.0, 0, 0, ctypes.byref(out)) == E
    assert L.plds_create_multi(1, None, 0.4, 3.0, 0, 0, ctypes.byref(out)) == E
    assert L.plds_create_opts(100, 0.4, 3.0, None, ctypes.byref(out)) == E
    for coeff in (0.5, 0.999, -1.0, math.inf, math.nan):
        o = P.plds_options_t(up_coeff=coeff)
        out.value = 1
        assert L.plds_create_opts(100, 0.4, 3.0, ctypes.byref(o), ctypes.byref(out)) == E, coeff
        assert not out.value


def test_error_messages(L):
    codes = [P.PLDS_OK, P.PLDS_EINVAL, P.PLDS_ERANGE, P.PLDS_ENOMEM, P.PLDS_EHIP, P.PLDS_ESTATE]
    msgs = [P.strerror(c) for c in codes]
    assert all(msgs) and len(set(msgs)) == len(msgs)
    assert P.strerror(-99)
    assert L.plds_inject_alloc_failure(-1) == P.PLDS_OK
