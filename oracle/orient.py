"""Oracle of the orientation and densest-subgraph outputs of the PLDS.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may use it.

Plain numpy and Python sets, written from the definitions:

* the orientation section and Algorithm 5 (LowOutDegreeOrient): every edge
  points from the endpoint at the lower level to the one at the higher level;
  on equal levels the edge with key (u, v), u < v, points u -> v.  The
  section's prose says the opposite tie-break (higher id to lower id);
  Algorithm 5's flip conditions only make sense with u -> v for equal
  levels under its key convention, and that is the reading taken here;
* Algorithm 5's outputs for a batch: F, the edges present before and after
  the batch whose orientation changed, each reported as oriented before;
  J, the batch's applied updates oriented (insertions as after the batch,
  deletions as before it);
* the densest-subgraph corollary: the largest coreness estimate is the
  structure's approximation of the densest-subgraph value.
"""
import numpy as np


def _pairs(edges):
    if edges is None:
        return np.zeros((0, 2), dtype=np.int64)
    return np.asarray(edges, dtype=np.int64).reshape(-1, 2)


def orient(levels, edges):
    """(tail, head) of every edge {u, v} under `levels` (Algorithm 5's rule):
    with u < v, u -> v when level(u) <= level(v), else v -> u.  Returns an
    int32 array [k, 2]."""
    e = _pairs(edges)
    lv = np.asarray(levels)
    u = np.minimum(e[:, 0], e[:, 1])
    v = np.maximum(e[:, 0], e[:, 1])
    fwd = lv[u] <= lv[v]
    out = np.empty((len(e), 2), dtype=np.int32)
    out[:, 0] = np.where(fwd, u, v)
    out[:, 1] = np.where(fwd, v, u)
    return out


def canonical_set(edges):
    """The undirected edges {min, max} of a pair list, self-loops dropped."""
    return {(min(a, b), max(a, b)) for a, b in _pairs(edges).tolist() if a != b}


def applied_updates(edges_before, ins, dele):
    """The applied updates of one call under the batch semantics: the
    insertions of absent pairs, then the deletions of pairs present after the
    insertions (Algorithm 1 applies all insertions first).  Both as sorted
    int32 arrays [k, 2] of (min, max)."""
    before = canonical_set(edges_before)
    a_ins = canonical_set(ins) - before
    a_del = canonical_set(dele) & (before | a_ins)

    def arr(s):
        return np.array(sorted(s), dtype=np.int32).reshape(-1, 2)
    return arr(a_ins), arr(a_del)


def flips(levels_before, levels_after, edges_before, edges_after):
    """F: the edges present both before and after a call whose orientation
    differs, each as oriented before (rows sorted)."""
    common = np.array(sorted(canonical_set(edges_before) & canonical_set(edges_after)),
                      dtype=np.int64).reshape(-1, 2)
    ob = orient(levels_before, common)
    oa = orient(levels_after, common)
    changed = (ob != oa).any(axis=1)
    f = ob[changed]
    return f[np.lexsort((f[:, 1], f[:, 0]))] if len(f) else f


def oriented_updates(levels_before, levels_after, ins_applied, del_applied):
    """J: applied insertions oriented under the levels after the call,
    applied deletions under the levels before it."""
    return orient(levels_after, ins_applied), orient(levels_before, del_applied)


def out_degrees(n, levels, edges):
    """Out-degree of every vertex under the orientation."""
    o = orient(levels, edges)
    return np.bincount(o[:, 0], minlength=n)


def densest_subgraph_value(estimates):
    """The largest coreness estimate (0 for a graph without edges)."""
    est = np.asarray(estimates, dtype=np.float64)
    return float(est.max()) if est.size else 0.0
