"""Pins for the oracle's edge visibility (first-order diffraction, Section III-B):
closed forms on an isolated box building, a blocking plate, and the generator's
edge lists."""
import numpy as np
import pytest

import scenegen as sg


def _box_scene(extra_plate=None, tx=((0, 0, 0),)):
    # box [0, 10] x [0, 10] m, 10 m high, 4 x 4 samples (g = 4, k = 3); edges in the
    # order SW, SE, NW, NE corners, then the south, north, west and east roof rims
    g, k, n = 4, 3, 4
    su, ss = 1 << g, 1 << (g + k)
    b = sg.SceneBuilder(g, k)
    b.add_box(0, 0, 10 * su, 10 * su, 10 * su, n, 0)
    if extra_plate is not None:
        v0, U, V = extra_plate
        b.add_rect(tuple(c * su for c in v0), tuple(c * su for c in U), tuple(c * su for c in V), n)
    pts = [tuple(int(c * ss) for c in p) for p in tx]
    return b.build("box", 0, pts, pts)


def _visible(oracle_mod, s, X):
    orc = oracle_mod.Oracle(s)
    vis = oracle_mod.edge_visibility(orc, np.asarray(X, np.float32), s.edge_facets, s.edge_samples,
                                     s.samples_per_edge)
    return [set(np.nonzero(v)[0].tolist()) for v in vis]


def test_box_edges_listed(oracle_mod):
    s = _box_scene()
    assert s.edge_facets.shape == (8, 2) and s.samples_per_edge == 4
    assert s.edge_samples.shape == (32, 3)
    # every edge sample lies on both of its facets' planes
    orc = oracle_mod.Oracle(s)
    for e in range(8):
        for j in range(4):
            p = s.edge_samples[4 * e + j]
            assert orc.orient(int(s.edge_facets[e, 0]), p) == 0.0
            assert orc.orient(int(s.edge_facets[e, 1]), p) == 0.0


@pytest.mark.parametrize("X,expect", [
    ((5, -20, 5), {0, 1, 4}),               # in front of the south wall, below the roof
    ((5, 5, 30), {4, 5, 6, 7}),             # above the roof: only the rim
    ((5, -20, 20), {0, 1, 4, 5, 6, 7}),     # in front of the south wall and above the roof
    ((30, -20, 5), {0, 1, 3, 4, 7}),        # in front of the south and east walls
    ((5, 5, 10), set()),                    # on the roof plane: strictly in front of nothing
])
def test_isolated_box_closed_forms(oracle_mod, X, expect):
    """An edge is seen exactly when the point is strictly in front of one of its
    two faces; nothing else in the scene can block it."""
    s = _box_scene()
    assert _visible(oracle_mod, s, [X])[0] == expect


def test_plate_blocks_every_edge(oracle_mod):
    """A plate between the point and the building (y = -10, x in [-40, 50], z in
    [0, 50]) blocks every segment to the building's edges."""
    s = _box_scene(extra_plate=((-40, -10, 0), (90, 0, 0), (0, 0, 50)))
    assert s.edge_facets.shape[0] == 8
    assert _visible(oracle_mod, s, [(5, -20, 5)])[0] == set()
    # from 100 m up every segment crosses the plate's plane above its top (the lowest,
    # to a south-corner sample 1.25 m up, at z = 50.6): the rim and the south corners
    # come back into view
    assert _visible(oracle_mod, s, [(5, -20, 100)])[0] == {0, 1, 4, 5, 6, 7}


def test_diffraction_counts(oracle_mod):
    t = np.array([[1, 0, 1, 1], [0, 0, 0, 0]], bool)
    r = np.array([[1, 1, 0, 1], [1, 1, 1, 1]], bool)
    assert oracle_mod.diffraction_counts(t, r).tolist() == [2, 0]


def test_generated_edges_meet_two_facets(oracle_mod):
    """Every generated edge's samples lie on the planes of both of its facets
    (urban tiny scene and a large-city crop), and the two facets differ."""
    for s in (sg.gen_c1(3, n_snap=1), sg.gen_c3(3, n_snap=1, cells=6, n_buildings=8)):
        orc = oracle_mod.Oracle(s)
        S = s.samples_per_edge
        assert S > 0 and s.edge_samples.shape[0] == S * s.edge_facets.shape[0]
        for e in range(s.edge_facets.shape[0]):
            fa, fb = (int(v) for v in s.edge_facets[e])
            assert fa != fb
            for j in range(S):
                p = s.edge_samples[S * e + j]
                assert orc.orient(fa, p) == 0.0 and orc.orient(fb, p) == 0.0


def test_one_clear_sample_suffices(oracle_mod):
    """A low plate at y = -10 seen from (5, -20, 5): a segment to a sample at
    height z crosses the plate's plane at z' = (5 + z) / 2.  The corners' samples
    sit at 1.25, 3.75, 6.25 and 8.75 m (z' = 3.125 ... 6.875), the south rim's at
    10 m (z' = 7.5).  A 6 m plate leaves only each corner's top sample clear, and
    that one sample keeps the corner visible; a 7 m plate blocks all four, and
    only the rim stays in view."""
    s6 = _box_scene(extra_plate=((-40, -10, 0), (90, 0, 0), (0, 0, 6)))
    assert _visible(oracle_mod, s6, [(5, -20, 5)])[0] == {0, 1, 4}
    s7 = _box_scene(extra_plate=((-40, -10, 0), (90, 0, 0), (0, 0, 7)))
    assert _visible(oracle_mod, s7, [(5, -20, 5)])[0] == {4}
