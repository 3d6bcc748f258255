"""The allocation-free static k-core entry point against the allocating one.

plds_static_kcore_noalloc keeps its peeling scratch in the library's fixed
per-device array.  Through the C ABI, on two calls in a row (a graph, then a
smaller one, so the second call finds the first call's contents in the
array), its estimates must equal plds_static_kcore's bit for bit; a handle
above the array's vertex limit is refused before any work.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _bits(t):
    return t.cpu().numpy().view(np.int64)


@pytest.mark.parametrize("eps", [0.5, 1.0])
def test_noalloc_equals_static_kcore_twice(eps):
    from paper_2106_03824_amd import plds as P
    from paper_2106_03824_amd import workloads as W
    for scale, seed in ((14, 5), (11, 6)):   # the second call has the smaller input
        n = 2 ** scale
        say("noalloc static k-core", scale, eps)
        g = P.PLDS(n, 0.4, 3.0)
        g.update(W.rmat(scale, 8 * n, seed=seed), None)
        ref = torch.empty(n, dtype=torch.float64, device="cuda")
        out = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
        assert P.lib().plds_static_kcore(g.h, float(eps), P._ptr(ref), None) == 0
        assert P.lib().plds_static_kcore_noalloc(g.h, float(eps), P._ptr(out), None) == 0
        assert np.array_equal(_bits(out), _bits(ref))
        assert (ref.cpu().numpy() > 0).sum() > 0
        g.close()


def test_noalloc_rejects_too_many_vertices():
    from paper_2106_03824_amd import plds as P
    n = P.lib_max_noalloc_n() + 1
    g = P.PLDS(n, 0.4, 3.0)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    assert P.lib().plds_static_kcore_noalloc(g.h, 0.5, P._ptr(out), None) == P.PLDS_EINVAL
    g.close()
