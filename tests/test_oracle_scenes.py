"""Pins for the oracle's pair and point visibility on scenes (CPU only).

Expected values come from hand-derived closed forms (tests/golden/closed_forms.json,
each entry citing Section II-B / Table I of the paper), from the symmetry of the
relation (Table I lists every relation in both directions), and from
special cases whose answer follows from the geometry alone.
"""
import json
import os

import numpy as np
import pytest

import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _golden_scenes():
    with open(GOLDEN) as fh:
        data = json.load(fh)["scenes"]
    return sorted(data.items())


@pytest.mark.parametrize("name,spec", _golden_scenes())
def test_golden_closed_forms(oracle_mod, name, spec):
    names = list(spec["facets"].keys())
    scene = sg.gen_plates([spec["facets"][n] for n in names], g=4, n=4, name=name)
    orc = oracle_mod.Oracle(scene)
    M, mism = orc.matrix(audit=True)
    assert mism == 0
    for a, b, expect, why in spec["expect"]:
        i, j = names.index(a), names.index(b)
        assert int(M[i, j]) == expect, f"{name}: {a}-{b}: {why}"
        assert int(M[j, i]) == expect, f"{name}: {b}-{a} (symmetry): {why}"


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_symmetry_audit_and_diagonal(oracle_mod, seed):
    """Both directions of every pair, computed independently, agree; M[i][i] = 0."""
    s = sg.gen_c1(seed)
    orc = oracle_mod.Oracle(s)
    M, mism = orc.matrix(audit=True)
    assert mism == 0
    assert not M.diagonal().any()
    assert (M == M.T).all()
    assert 0 < M.sum() < M.size


def test_coplanar_ground_never_visible(oracle_mod):
    s = sg.gen_c1(3)
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    ground = np.nonzero(s.facet_kind == sg.KIND_GROUND)[0]
    roofs = np.nonzero(s.facet_kind == sg.KIND_ROOF)[0]
    assert not M[np.ix_(ground, ground)].any()
    # roofs and ground all face +z: parallel planes facing one way never see each other
    assert not M[np.ix_(roofs, roofs)].any()
    assert not M[np.ix_(ground, roofs)].any()


def test_building_own_faces(oracle_mod):
    """Faces of one convex box never see each other (all corners are convex)."""
    s = sg.gen_c1(2)
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    for b in range(8):
        f = np.nonzero(s.facet_building == b)[0]
        assert len(f) == 5
        assert not M[np.ix_(f, f)].any()


def test_point_visibility_closed_forms(oracle_mod):
    # plate at z=0 facing +z, 4x4 m; a big blocker at z=5 (12x12) is added in the second scene
    plate = [[0, 0, 0], [4, 0, 0], [0, 4, 0]]
    s = sg.gen_plates([plate])
    orc = oracle_mod.Oracle(s)
    assert orc.point_visible((2, 2, 10), 0), "point in front of a lone plate sees it"
    assert orc.point_visible((100, -50, 0.5), 0), "grazing but in front"
    assert not orc.point_visible((2, 2, -10), 0), "point behind the plate"
    assert not orc.point_visible((50, 50, 0), 0), "point in the plate's plane"
    s2 = sg.gen_plates([plate, [[-4, -4, 5], [12, 0, 0], [0, 12, 0]]])
    orc2 = oracle_mod.Oracle(s2)
    assert not orc2.point_visible((2, 2, 10), 0), "a larger plate in between hides it"
    assert orc2.point_visible((40, 2, 1), 0), "a low oblique view passes under the blocker"
    assert orc2.point_visible((2, 2, 10), 1), "the blocker itself is visible from above"


def test_los_by_hand(oracle_mod):
    wall = [[0, -5, 0], [0, 10, 0], [0, 0, 10]]          # x = 0 plane, y in [-5,5], z in [0,10]
    # (-5,0,2)->(5,16,2) crosses x=0 at y=8, beside the wall; (-5,0,12)->(5,0,12) passes above it
    s = sg.gen_plates([wall])
    orc = oracle_mod.Oracle(s)
    los = orc.los(np.array([[-5, 0, 2], [-5, 0, 2], [-5, 0, 2], [-5, 0, 12]], np.float32),
                  np.array([[5, 0, 2], [5, 16, 2], [-5, 3, 2], [5, 0, 12]], np.float32))
    assert los.tolist() == [False, True, True, True]
    # a ray through the wall's exact top edge is blocked (closed triangle)
    assert not orc.los(np.array([[-5, 0, 9]], np.float32), np.array([[5, 0, 11]], np.float32))[0]


def test_c1_table_shape(oracle_mod):
    """Config-1 table: every visible facet faces the point (orientation is necessary)."""
    s = sg.gen_c1(1)
    orc = oracle_mod.Oracle(s)
    tv, rv, los = orc.txrx(s.tx, s.rx)
    assert tv.shape == (10, 42) and rv.shape == (10, 42) and los.shape == (10,)
    for n in range(10):
        for f in np.nonzero(tv[n])[0]:
            assert orc.orient(int(f), s.tx[n]) > 0
        for f in np.nonzero(rv[n])[0]:
            assert orc.orient(int(f), s.rx[n]) > 0
    # a 1.5 m receiver never sees a roof (roofs are >= 10 m high and face up)
    roofs = s.facet_kind == sg.KIND_ROOF
    assert not rv[:, roofs].any()
    # the 25 m transmitter always sees some ground
    assert tv[:, s.facet_kind == sg.KIND_GROUND].any(1).all()
