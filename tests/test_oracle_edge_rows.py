"""Pins for the oracle's edge rows of the matrix (edges as visibility nodes
beside faces, Sections I and II-A; the face seen for diffraction is the face
seen for reflection, Section III-B): hand-derived closed forms on one box with
a plate in front of it, the same with a blocker between them, and two boxes
facing each other; the symmetry of edge-to-edge visibility, both directions
evaluated independently, on generated urban scenes."""
import numpy as np
import pytest

import scenegen as sg

# edges of a box from SceneBuilder.add_box (one panel per wall), in order
SW, SE, NW, NE, S_RIM, N_RIM, W_RIM, E_RIM = range(8)
SU = 16   # vertex units per metre (g = 4)


def _box_scene(extra_rects=(), second_box=False):
    b = sg.SceneBuilder(4, 3)
    b.add_box(0, 0, 10 * SU, 10 * SU, 10 * SU, 4, 0)
    if second_box:
        b.add_box(20 * SU, 0, 30 * SU, 10 * SU, 10 * SU, 4, 1)
    for v0, U, V in extra_rects:
        b.add_rect(tuple(c * SU for c in v0), tuple(c * SU for c in U), tuple(c * SU for c in V), 4)
    return b.build("boxes", 0)


PLATE = ((-5, -20, 0), (0, 0, 10), (20, 0, 0))   # y = -20, x in [-5, 15], visible side +y (towards the box)


def test_box_edges_seen_from_a_plate(oracle_mod):
    s = _box_scene([PLATE])
    assert s.edge_facets.shape[0] == 8 and s.n_facets == 6
    orc = oracle_mod.Oracle(s)
    ef, ee = oracle_mod.edge_rows(orc, s.edge_facets, s.edge_samples, s.samples_per_edge)
    # the plate's samples reach x = -2.5 and x = 12.5, so the west and east walls face
    # some of them: every corner and the south, west and east rims are seen; the north
    # rim (north wall and roof) faces none of them
    assert ef[:, 5].tolist() == [1, 1, 1, 1, 1, 0, 1, 1]
    # a convex box: its edges see none of its own facets and none of its other edges
    assert not ef[:, :5].any()
    assert not ee.any()


def test_blocker_hides_every_edge(oracle_mod):
    blocker = ((-20, -10, -1), (50, 0, 0), (0, 0, 21))
    s = _box_scene([PLATE, blocker])
    orc = oracle_mod.Oracle(s)
    ef, _ = oracle_mod.edge_rows(orc, s.edge_facets, s.edge_samples, s.samples_per_edge)
    assert not ef[:, 5].any()


def test_two_boxes_facing(oracle_mod):
    s = _box_scene(second_box=True)
    E = s.edge_facets.shape[0]
    assert E == 16
    orc = oracle_mod.Oracle(s)
    ef, ee = oracle_mod.edge_rows(orc, s.edge_facets, s.edge_samples, s.samples_per_edge)
    B = 8
    assert ee[E_RIM, B + W_RIM], "facing roof rims see each other over the gap"
    assert not ee[E_RIM, B + E_RIM], "B's east rim faces away from A"
    assert not ee[W_RIM, B + W_RIM], "A's west rim faces away from B"
    assert ee[SE, B + SW], "the south corners facing each other along y = 0"
    west_b = 5 + 2
    assert ef[E_RIM, west_b], "A's east rim sees B's west wall across the gap"
    assert not ef[W_RIM, west_b]
    assert (ee == ee.T).all() and not ee.diagonal().any()


@pytest.mark.parametrize("seed", [1, 2])
def test_symmetry_on_urban_scenes(oracle_mod, seed):
    s = sg.gen_c1(seed)
    orc = oracle_mod.Oracle(s)
    ef, ee = oracle_mod.edge_rows(orc, s.edge_facets, s.edge_samples, s.samples_per_edge)
    assert (ee == ee.T).all() and not ee.diagonal().any()
    assert 0 < ef.sum() < ef.size and 0 < ee.sum() < ee.size
    # an edge never sees its own two facets (its samples lie in both planes)
    for e, (fa, fb) in enumerate(s.edge_facets):
        assert not ef[e, fa] and (fb < 0 or not ef[e, fb])
    # subsets of rows give the same rows
    rows = np.array([3, 0, 17])
    ef2, ee2 = oracle_mod.edge_rows(orc, s.edge_facets, s.edge_samples, s.samples_per_edge, rows=rows)
    assert (ef2 == ef[rows]).all() and (ee2 == ee[rows]).all()
