"""Pins for the interface relations of the matrix (Section II-B, Table I: PAR
for parallel reference / aim faces, PER for perpendicular ones), on a scene
whose normals are known by construction; expected pairs derived by hand."""
import numpy as np

import scenegen as sg


def _scene():
    # normals (U x V): 0 ground +z, 1 west wall -x, 2 east wall +x, 3 south wall -y,
    # 4 roof +z, 5 vertical plate along (1, 1, 0), 6 slanted plate along (0, -1, 1)
    return sg.gen_plates([
        [[-20, -20, 0], [40, 0, 0], [0, 40, 0]],
        [[0, 0, 0], [0, 0, 8], [0, 8, 0]],
        [[10, 0, 0], [0, 8, 0], [0, 0, 8]],
        [[0, 0, 0], [8, 0, 0], [0, 0, 8]],
        [[0, 0, 8], [8, 0, 0], [0, 8, 0]],
        [[20, 0, 0], [-4, 4, 0], [0, 0, 4]],
        [[0, 20, 0], [4, 0, 0], [0, 4, 4]],
    ])


def _sym(pairs, F):
    m = np.zeros((F, F), bool)
    for i, j in pairs:
        m[i, j] = m[j, i] = True
    return m


def test_relations_by_construction(oracle_mod):
    s = _scene()
    F = s.n_facets
    M = ~np.eye(F, dtype=bool)  # every pair, to check the classification alone
    r = oracle_mod.interface_relations(s, M)
    assert (r["par"] == _sym([(0, 4), (1, 2)], F)).all()
    assert (r["per"] == _sym([(0, 1), (0, 2), (0, 3), (0, 5), (4, 1), (4, 2), (4, 3), (4, 5), (1, 3), (2, 3),
                              (6, 1), (6, 2)], F)).all()
    assert r["cls"].tolist() == [1, 0, 0, 0, 1, 0, 2]


def test_relations_follow_the_matrix(oracle_mod):
    """Only visible pairs carry a relation."""
    s = _scene()
    F = s.n_facets
    M = _sym([(1, 2), (0, 3), (5, 6)], F)
    r = oracle_mod.interface_relations(s, M)
    assert (r["par"] == _sym([(1, 2)], F)).all()
    assert (r["per"] == _sym([(0, 3)], F)).all()
    assert not (r["par"] | r["per"])[5, 6]


def test_box_walls_of_an_urban_scene(oracle_mod):
    """Every building of the tiny urban scenes is an axis-aligned box: among
    all pairs, walls relate to walls and roofs as PAR or PER only."""
    s = sg.gen_c1(1)
    F = s.n_facets
    r = oracle_mod.interface_relations(s, ~np.eye(F, dtype=bool))
    assert set(r["cls"].tolist()) <= {0, 1}
    assert (r["par"] | r["per"])[~np.eye(F, dtype=bool)].all()
    assert not (r["par"] & r["per"]).any()
