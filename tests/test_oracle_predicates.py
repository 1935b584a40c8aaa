"""Pins for the oracle's geometric predicates (CPU only).

The segment/triangle predicate follows the division-free Moller-Trumbore test
with a closed triangle and an open segment; orientation is the sign of a
triple product (Section II-B, eq. 2: only the front side of a face is visible).
These tests pin them against textbook special cases and against an exact
128-bit integer evaluation on the dyadic grids the scenes use.
"""
import numpy as np
import pytest

import scenegen as sg

A, B, C = (0, 0, 0), (4, 0, 0), (0, 4, 0)     # triangle in the plane z = 0


@pytest.mark.parametrize("p,q,hit,why", [
    ((1, 1, 1), (1, 1, -1), True, "crosses the interior"),
    ((1, 1, -1), (1, 1, 1), True, "same segment reversed (det < 0 branch)"),
    ((1, 1, 1), (1, 1, 0), False, "ends on the triangle: open segment"),
    ((1, 1, 0), (1, 1, -3), False, "starts on the triangle: open segment"),
    ((1, 1, 3), (1, 1, 1), False, "stops short of the plane"),
    ((0, 1, 1), (0, 1, -1), True, "crosses edge x=0: closed triangle"),
    ((1, 0, 1), (1, 0, -1), True, "crosses edge y=0"),
    ((2, 2, 1), (2, 2, -1), True, "crosses the hypotenuse x+y=4"),
    ((0, 0, 1), (0, 0, -1), True, "crosses a vertex"),
    ((3, 3, 1), (3, 3, -1), False, "passes outside the hypotenuse"),
    ((-1, 1, 1), (-1, 1, -1), False, "passes outside edge x=0"),
    ((-1, 1, 0), (5, 1, 0), False, "lies in the triangle's plane: parallel never hits"),
    ((1, 1, 1), (2, 1, 1), False, "parallel above the plane"),
    ((-4, 1, 2), (4, 1, -2), True, "oblique crossing at (0,1,0) on the edge"),
    ((-4, 1, 2), (3.5, 1, -1.75), True, "oblique crossing inside"),
])
def test_segtri_textbook(oracle_mod, p, q, hit, why):
    assert oracle_mod.segtri(p, q, A, B, C) is hit, why
    # winding of the triangle must not matter for occlusion
    assert oracle_mod.segtri(p, q, A, C, B) is hit, why + " (other winding)"


def _grid_points(rng, n, lo, hi, unit):
    return (rng.integers(int(lo / unit), int(hi / unit), size=(n, 3)) * unit).astype(np.float32)


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_exact_audit_random_and_degenerate(oracle_mod, cfg):
    """FP64 signs equal exact 128-bit signs on each config's grids, including
    constructed degenerate cases (segments through vertices, along edges, in-plane)."""
    g, k, ext = {"c1": (4, 3, 200.0), "c2": (3, 4, 1000.0), "c3": (2, 3, 4000.0)}[cfg]
    rng = np.random.default_rng(7)
    n = 20000
    vu, su = 2.0 ** -g, 2.0 ** -(g + k)
    half = ext / 2
    a = _grid_points(rng, n, -half, half, vu)
    e1 = _grid_points(rng, n, -40, 40, vu)
    e2 = _grid_points(rng, n, -40, 40, vu)
    b, c = a + e1, a + e2
    p = _grid_points(rng, n, -half, half, su)
    q = _grid_points(rng, n, -half, half, su)
    # degenerate constructions: q mirrors p through a vertex / an edge midpoint
    m = n // 4
    q[:m] = 2 * a[:m] - p[:m]
    mid = (a[m:2 * m] + b[m:2 * m]) / 2
    q[m:2 * m] = 2 * mid - p[m:2 * m]
    # segments parallel to the triangle's plane
    q[2 * m:3 * m] = p[2 * m:3 * m] + (b[2 * m:3 * m] - a[2 * m:3 * m]) + (c[2 * m:3 * m] - a[2 * m:3 * m])
    for arr in (b, c, q):
        assert np.all(np.abs(arr) < 2 ** 23 * su)
    bad, zeros = oracle_mod.exact_audit(p, q, a, b, c, g + k)
    assert bad == 0
    assert zeros >= m // 2            # the parallel constructions give exact zeros


def test_exact_audit_detects_budget_violation(oracle_mod):
    """Planted failure: with 2^23-unit edges on a fine grid the degree-3 terms
    exceed 2^53, FP64 rounds, and the audit must report sign disagreements."""
    rng = np.random.default_rng(3)
    n = 20000
    unit = 2.0 ** -20
    a = np.zeros((n, 3), np.float32)
    e1 = (rng.integers(2 ** 21, 2 ** 22, size=(n, 3)) * unit).astype(np.float32)
    e2 = (rng.integers(2 ** 21, 2 ** 22, size=(n, 3)) * unit).astype(np.float32)
    b, c = a + e1, a + e2
    p = (rng.integers(-2 ** 22, 2 ** 22, size=(n, 3)) * unit).astype(np.float32)
    q = p + e1 + e2                      # exactly parallel: det = 0 exactly
    bad, zeros = oracle_mod.exact_audit(p, q, a, b, c, 20)
    assert zeros == n
    assert bad > 0


def test_orient_audit(oracle_mod):
    rng = np.random.default_rng(11)
    n = 20000
    for g, k, ext in ((4, 3, 200.0), (3, 4, 1000.0), (2, 3, 4000.0)):
        vu, su = 2.0 ** -g, 2.0 ** -(g + k)
        a = _grid_points(rng, n, -ext / 2, ext / 2, vu)
        b = a + _grid_points(rng, n, -40, 40, vu)
        c = a + _grid_points(rng, n, -40, 40, vu)
        x = _grid_points(rng, n, -ext / 2, ext / 2, su)
        x[: n // 3] = a[: n // 3] + (b[: n // 3] - a[: n // 3]) * 0.5  # on an edge: orient 0
        assert oracle_mod.orient_audit(x, a, b, c, g + k) == 0


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4"])
def test_config_grids_within_budget(cfg):
    """Every config keeps the predicates exact in FP64 (budget <= 53 bits)."""
    kw = {"c2": {"n_snap": 10}, "c3": {"n_snap": 10}, "c4": {}}.get(cfg, {})
    s = sg.make_config(cfg, **kw)
    assert sg.grid_budget_bits(s) <= 53
    scale = 2.0 ** (s.g + s.k)
    for arr in (s.samples, s.vertices, s.tx, s.rx):
        v = arr.astype(np.float64) * scale
        assert np.all(v == np.rint(v))
        assert np.all(np.abs(v) < 2 ** 24)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_exact_audit_edge_segments(oracle_mod, cfg):
    """The edge tables test segments from Tx/Rx positions to edge sample points,
    which lie on the boundary of the two facets' triangles.  On the generated
    scenes the FP64 signs of those segment-triangle predicates equal the exact
    128-bit signs, for random triangles and for the edge's own triangles (the
    degenerate case: the segment ends on the triangle's boundary), and so do
    the orientations of the positions against the edge's facets."""
    import scenegen as sg
    s = sg.make_config(cfg)
    rng = np.random.default_rng(5)
    n = 20000
    S = s.samples_per_edge
    E = s.edge_facets.shape[0]
    X = np.concatenate([s.tx, s.rx])[rng.integers(0, 2 * s.n_snapshots, n)]
    e = rng.integers(0, E, n)
    P = s.edge_samples[e * S + rng.integers(0, S, n)]
    tri = s.vertices[s.tri_vertices]                     # T x 3 x 3
    t = rng.integers(0, tri.shape[0], n)
    # half of the sample uses a triangle of one of the edge's two facets
    own = np.zeros(n, np.int64)
    first = np.searchsorted(s.tri_facet, np.arange(s.n_facets))
    f = s.edge_facets[e, rng.integers(0, 2, n)]
    own[:] = first[f]
    t[: n // 2] = own[: n // 2]
    bad, zeros = oracle_mod.exact_audit(X, P, tri[t, 0], tri[t, 1], tri[t, 2], s.g + s.k)
    assert bad == 0
    assert oracle_mod.orient_audit(X, tri[own, 0], tri[own, 1], tri[own, 2], s.g + s.k) == 0
    assert oracle_mod.orient_audit(P, tri[own, 0], tri[own, 1], tri[own, 2], s.g + s.k) == 0
