"""Oracle of the vertex updates (section on vertex insertions and deletions).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may use it.

A vertex deletion is the batch of edge deletions of every edge incident to
the deleted vertices (the vertex stays, without edges); a vertex insertion
past the structure's n, or a renumbering, is a rebuild: a fresh structure of
the new size that receives every edge as one insertion batch.
"""
import numpy as np

from . import Oracle


def incident_edges(edges, vertices):
    """The edges (rows of `edges`) with an end in `vertices`."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    mark = np.zeros(int(e.max()) + 1 if len(e) else 1, dtype=bool)
    vs = np.asarray(vertices, dtype=np.int64).reshape(-1)
    vs = vs[vs < len(mark)]
    mark[vs] = True
    return e[mark[e[:, 0]] | mark[e[:, 1]]].astype(np.int32)


def delete_vertices(o, vertices):
    """Deletes every edge of `vertices` from the oracle `o` as one batch."""
    return o.delete(incident_edges(o.edges(), vertices))


def rebuild(o, new_n, relabel=None, levels_per_group=0, delta=0.4, lam=3.0):
    """A fresh oracle of new_n vertices holding the graph of `o` (renumbered
    by `relabel`, -1 dropping a vertex and its edges), built by one batch."""
    e = o.edges().astype(np.int64)
    if relabel is not None:
        r = np.asarray(relabel, dtype=np.int64)
        e = np.stack([r[e[:, 0]], r[e[:, 1]]], axis=1) if len(e) else e
        e = e[(e >= 0).all(axis=1)]
    n2 = Oracle(new_n, delta, lam, levels_per_group)
    rc = n2.insert(e.astype(np.int32)) if len(e) else 0
    return n2, rc
