"""Pins for the oracle's angular bouncing ranges (Section II-A: two 2-D views;
Section II-B, eq. 1: the angle at an edge of the reference face between the face
and a vertex of the aim face; eq. 2: 180 degrees or more recorded as 0).

* Hand-derived closed forms on two-facet scenes: parallel walls facing each
  other and perpendicular walls in the horizontal view (the AB-EF and FG-HI
  relations of Table I), a wall and the ground in front of it in a vertical
  view (the AC-EI situation of Fig. 1(c)), both directions, and aim vertices
  behind or on the reference plane (eq. 2).
* The same ranges recomputed by an independent route on generated urban scenes
  (axis-aligned boxes): 2-D coordinates of the view plane, the ends chosen in
  those coordinates and the angle as atan2(|u x v|, u . v).
"""
import math

import numpy as np
import pytest

import scenegen as sg


def _deg(x):
    return math.degrees(x)


def _ranges(oracle_mod, rects):
    s = sg.gen_plates(rects)
    F = s.n_facets
    r = oracle_mod.angular_ranges(s, ~np.eye(F, dtype=bool))
    out = {}
    for i in range(F):
        for k in range(r["offsets"][i], r["offsets"][i + 1]):
            out[(i, int(r["cols"][k]))] = r["ranges"][k].tolist()
    return out


WALL_S = ((0, 0, 0), (0, 0, 4), (8, 0, 0))      # y = 0, x in [0, 8], z in [0, 4], visible side +y


def test_parallel_walls_facing(oracle_mod):
    north = ((0, 6, 0), (8, 0, 0), (0, 0, 4))  # y = 6, visible side -y
    r = _ranges(oracle_mod, [WALL_S, north])
    a = _deg(math.atan2(6, 8))
    for key in ((0, 1), (1, 0)):
        assert r[key] == pytest.approx([a, 90.0, a, 90.0], abs=1e-12)


def test_perpendicular_walls(oracle_mod):
    east = ((12, 2, 0), (0, 0, 4), (0, 6, 0))   # x = 12, y in [2, 8], visible side -x
    r = _ranges(oracle_mod, [WALL_S, east])
    # reference = south wall, view along +z: B = (0, 0), A = (8, 0)
    assert r[(0, 1)] == pytest.approx([_deg(math.atan2(2, 12)), _deg(math.atan2(8, 12)),
                                       180 - _deg(math.atan2(8, 4)), 180 - _deg(math.atan2(2, 4))], abs=1e-12)
    # reference = east wall: B = (12, 2), A = (12, 8)
    w = sorted([_deg(math.acos(-2 / math.sqrt(148))), _deg(math.acos(-2 / math.sqrt(20)))])
    m = sorted([_deg(math.acos(8 / math.sqrt(208))), _deg(math.acos(8 / math.sqrt(80)))])
    assert r[(1, 0)] == pytest.approx(w + m, abs=1e-12)


def test_eq2_behind_and_on_the_reference_plane(oracle_mod):
    straddle = ((12, -2, 0), (0, 0, 4), (0, 6, 0))   # y in [-2, 4]: one end behind y = 0
    r = _ranges(oracle_mod, [WALL_S, straddle])
    assert r[(0, 1)] == pytest.approx([0.0, _deg(math.atan2(4, 12)), 0.0, 135.0], abs=1e-12)
    on_plane = ((12, 0, 0), (0, 0, 4), (0, 6, 0))    # y in [0, 6]: one end on y = 0
    r = _ranges(oracle_mod, [WALL_S, on_plane])
    assert r[(0, 1)] == pytest.approx([0.0, _deg(math.atan2(6, 12)), 0.0, 180 - _deg(math.atan2(6, 4))], abs=1e-12)
    assert r[(0, 1)][0] == 0.0 and r[(0, 1)][2] == 0.0


def test_wall_and_ground_vertical_view(oracle_mod):
    ground = ((-4, 2, 0), (16, 0, 0), (0, 10, 0))    # z = 0, y in [2, 12], visible side +z
    r = _ranges(oracle_mod, [WALL_S, ground])
    # wall as reference, view along +x (the yz-plane): B = top (y 0, z 4), A = bottom (0, 0)
    assert r[(0, 1)] == pytest.approx([_deg(math.atan2(2, 4)), _deg(math.atan2(12, 4)), 90.0, 90.0], abs=1e-12)
    # ground as reference: B = (y 2, z 0), A = (12, 0); the wall's foot lies on the ground plane (eq. 2)
    assert r[(1, 0)] == pytest.approx([0.0, 180 - _deg(math.atan2(4, 2)), 0.0, _deg(math.atan2(4, 12))],
                                      abs=1e-12)


def test_view_direction_cases(oracle_mod):
    vd = oracle_mod.view_direction
    assert vd((0, 5, 0), (0, -5, 0)) == (0, 0, 1)        # parallel vertical: horizontal view
    assert vd((0, 5, 0), (-3, 0, 0)) == (0, 0, 15)       # perpendicular vertical: horizontal view
    assert vd((0, 5, 0), (0, 0, 2)) == (10, 0, 0)        # wall and ground: vertical view along x
    assert vd((0, 0, 2), (0, 5, 0)) == (10, 0, 0)        # the same view from the other side
    assert vd((0, 0, 2), (0, 0, -2)) == (1, 0, 0)        # parallel horizontal
    assert vd((0, 1, 1), (0, -1, -1)) == (1, 0, 0)       # parallel slanted: horizontal line in the plane


def _independent(scene, M):
    """Axis-aligned scenes only: every view is along a coordinate axis."""
    su = 1 << scene.g
    V = np.rint(np.asarray(scene.vertices, np.float64) * su).astype(np.int64)
    verts = [[] for _ in range(scene.n_facets)]
    for t, f in enumerate(scene.tri_facet):
        verts[int(f)].extend(V[scene.tri_vertices[t]].tolist())
    nrm = []
    for f in range(scene.n_facets):
        a, b, c = verts[f][0], verts[f][1], verts[f][2]
        nrm.append(np.cross(np.subtract(b, a), np.subtract(c, a)))
    axes = {2: (0, 1), 0: (1, 2), 1: (2, 0)}          # right-handed 2-D axes looking along z, x, y
    out = []
    for i in range(scene.n_facets):
        for j in np.nonzero(M[i])[0]:
            ni, nj = nrm[i], nrm[j]
            c = np.cross(ni, nj)
            ax = int(np.nonzero(c)[0][0]) if c.any() else (2 if ni[2] == 0 else 0)
            p, q = axes[ax]
            n2 = np.array([ni[p], ni[q]], float)
            t_i = np.array([-ni[q], ni[p]], float)
            t_j = np.array([-nj[q], nj[p]], float)
            P = lambda v: np.array([v[p], v[q]], float)
            vi = [P(v) for v in verts[i]]
            vj = [P(v) for v in verts[j]]
            A = min(vi, key=lambda x: t_i @ x)
            B = max(vi, key=lambda x: t_i @ x)
            E = min(vj, key=lambda x: t_j @ x)
            Fv = max(vj, key=lambda x: t_j @ x)

            def ang(at, other, X):
                if n2 @ (X - at) <= 0:
                    return 0.0
                u, v = other - at, X - at
                return math.degrees(math.atan2(abs(u[0] * v[1] - u[1] * v[0]), u @ v))

            out.append(sorted([ang(B, A, E), ang(B, A, Fv)]) + sorted([ang(A, B, E), ang(A, B, Fv)]))
    return np.asarray(out, float).reshape(-1, 4)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_independent_route_on_urban_scenes(oracle_mod, seed):
    s = sg.gen_c1(seed)
    M, _ = oracle_mod.Oracle(s).matrix()
    r = oracle_mod.angular_ranges(s, M)
    assert int(r["offsets"][-1]) == int(M.sum())
    exp = _independent(s, M)
    assert exp.shape == r["ranges"].shape
    np.testing.assert_allclose(r["ranges"], exp, rtol=0, atol=1e-9)
    assert ((r["ranges"] >= 0) & (r["ranges"] < 180)).all()
    # the visible pairs of box buildings and the ground are parallel or perpendicular:
    # their angles stay within the open range the visible side allows
    assert (r["ranges"][:, 1] > 0).all() and (r["ranges"][:, 3] > 0).all()
