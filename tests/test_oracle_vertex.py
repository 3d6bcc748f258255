"""Pins of the vertex-update oracle (oracle/vertex.py) by hand-worked cases."""
import numpy as np

import oracle as O
import oracle.vertex as OV


def test_incident_edges():
    e = [(0, 1), (1, 2), (2, 3), (3, 4)]
    assert OV.incident_edges(e, [2]).tolist() == [[1, 2], [2, 3]]
    assert OV.incident_edges(e, [0, 4, 9]).tolist() == [[0, 1], [3, 4]]


def test_star_centre_deleted():
    """Deleting the centre of a star with 10 leaves (centre at level 1 since
    its up-degree 10 > 3 at delta = 0.4, lambda = 3) leaves 11 isolated
    vertices, all at level 0 with estimate 0."""
    o = O.Oracle(16)
    assert o.insert([(0, i) for i in range(1, 11)]) == 0
    assert o.levels()[0] >= 1
    assert OV.delete_vertices(o, [0]) == 0
    assert (o.levels() == 0).all() and (o.coreness() == 0).all() and o.m == 0


def test_rebuild_of_a_clique_renumbered():
    """K_5 on ids 3..7 renumbered to 0..4: the rebuilt structure holds a K_5
    on 0..4, with the same levels as a K_5 built there directly."""
    o = O.Oracle(10)
    k5 = [(a, b) for a in range(3, 8) for b in range(a + 1, 8)]
    assert o.insert(k5) == 0
    relabel = np.full(10, -1)
    relabel[3:8] = np.arange(5)
    o2, rc = OV.rebuild(o, 5, relabel)
    assert rc == 0
    d = O.Oracle(5)
    assert d.insert([(a, b) for a in range(5) for b in range(a + 1, 5)]) == 0
    assert (o2.levels() == d.levels()).all() and o2.m == 10
