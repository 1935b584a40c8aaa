"""Pins for the oracle's occluder labels (CPU only).

A label of facet pair (i, j) marks every triangle group holding a triangle that
meets at least one admissible segment of the pair, excluding the triangles of i
and j themselves: the third faces that block the pair (Section II-B).  The group
of each triangle is an input, so these scenes assign groups by hand and the
expected masks follow from the geometry alone:

* a blocker between two facing plates sets exactly its group;
* two blockers stacked on the same segments set both groups (all hits, not the
  first one met);
* a blocker crossed only by segments that fail the visible-side rule (eq. 2)
  sets nothing, while one crossed by admissible segments of the same pair does;
* triangles of the pair's own facets never label it, even when (in a bent
  test facet the GPU library would reject) they cross its segments.
"""
import numpy as np

import scenegen as sg


def _groups(scene, assign):
    """Group per triangle: facet f's triangles get assign.get(f, 0) (or a per-triangle tuple)."""
    g = np.zeros(scene.n_triangles, np.int32)
    for t, f in enumerate(scene.tri_facet):
        a = assign.get(int(f), 0)
        if isinstance(a, tuple):
            a = a[t - int(np.nonzero(scene.tri_facet == f)[0][0])]
        g[t] = a
    return g


def _labels(oracle_mod, scene, pairs, assign):
    orc = oracle_mod.Oracle(scene)
    I = [p[0] for p in pairs]
    J = [p[1] for p in pairs]
    return [int(x) for x in orc.occluder_groups(I, J, _groups(scene, assign))]


PLATE_LO = ((0, 0, 0), (4, 0, 0), (0, 4, 0))      # z = 0, visible side +z
PLATE_HI = ((0, 0, 10), (0, 4, 0), (4, 0, 0))     # z = 10, visible side -z


def test_one_blocker_sets_its_group(oracle_mod):
    big = ((-4, -4, 5), (12, 0, 0), (0, 12, 0))
    s = sg.gen_plates([PLATE_LO, PLATE_HI, big])
    # both triangles of the blocker in group 7
    assert _labels(oracle_mod, s, [(0, 1), (1, 0)], {2: 7}) == [1 << 7, 1 << 7]
    # split over groups 4 and 9: the segments between the 4 x 4 sample grids cross both halves
    assert _labels(oracle_mod, s, [(0, 1)], {2: (4, 9)}) == [(1 << 4) | (1 << 9)]
    # nothing lies between a plate and the blocker itself
    assert _labels(oracle_mod, s, [(0, 2)], {2: 7}) == [0]


def test_stacked_blockers_set_both_groups(oracle_mod):
    c1 = ((-4, -4, 3), (12, 0, 0), (0, 12, 0))
    c2 = ((-4, -4, 7), (12, 0, 0), (0, 12, 0))
    s = sg.gen_plates([PLATE_LO, PLATE_HI, c1, c2])
    # every segment meets c1 first and c2 after it: labels record all hits
    assert _labels(oracle_mod, s, [(0, 1), (1, 0)], {2: 2, 3: 5}) == [(1 << 2) | (1 << 5)] * 2


def test_back_side_segments_never_label(oracle_mod):
    # B stands at x = 2 facing +x over plate A (z = 0): only A's samples with x > 2 are on
    # B's visible side.  D (x = 1.75) is crossed only by segments from A's samples with
    # x < 2; E (z = 0.5, x >= 2.25) only by the admissible ones.
    A = ((0, 0, 0), (4, 0, 0), (0, 4, 0))
    B = ((2, 0, 1), (0, 4, 0), (0, 0, 4))
    D = ((1.75, -1, 0.25), (0, 6, 0), (0, 0, 5.75))
    E = ((2.25, -1, 0.5), (1.75, 0, 0), (0, 6, 0))
    s = sg.gen_plates([A, B, D, E])
    orc = oracle_mod.Oracle(s)
    P = s.samples[s.sample_offsets[0]:s.sample_offsets[1]]
    Q = s.samples[s.sample_offsets[1]:s.sample_offsets[2]]
    # the construction: D is met by some non-admissible segment, E by some admissible one
    tri = s.vertices[s.tri_vertices].astype(np.float64)
    hit_d = any(oracle_mod.segtri(p, q, *tri[4]) or oracle_mod.segtri(p, q, *tri[5])
                for p in P for q in Q if p[0] < 2)
    assert hit_d
    assert all(orc.orient(1, p) <= 0 for p in P if p[0] < 2)
    assert _labels(oracle_mod, s, [(0, 1), (1, 0)], {2: 3, 3: 11}) == [1 << 11, 1 << 11]
    # without E the admissible segments are clear: the pair is visible and unlabelled
    s2 = sg.gen_plates([A, B, D])
    assert _labels(oracle_mod, s2, [(0, 1)], {2: 3}) == [0]
    assert oracle_mod.Oracle(s2).pair(0, 1) == 1


def test_own_facets_never_label(oracle_mod):
    # Facet 0 is bent on purpose: its first triangle lies in z = 0 (visible side +z) and a
    # second triangle spans z = 5 above it, crossing every segment to facet 1 (z = 10).
    # Facet 1 gets the same kind of extra triangle at z = 6.  Neither may label the pair.
    b = sg.SceneBuilder(4, 3)
    su = 16
    lo = [(0, 0, 0), (4 * su, 0, 0), (0, 4 * su, 0), (-8 * su, -8 * su, 5 * su), (16 * su, -8 * su, 5 * su),
          (-8 * su, 16 * su, 5 * su)]
    smp_lo = [(x, y, 0) for x in (64, 192) for y in (64, 128)]   # inside the first triangle
    b.add_mesh_facet(lo, [(0, 1, 2), (3, 4, 5)], smp_lo)
    hi = [(0, 0, 10 * su), (0, 4 * su, 10 * su), (4 * su, 0, 10 * su), (-8 * su, -8 * su, 6 * su),
          (16 * su, -8 * su, 6 * su), (-8 * su, 16 * su, 6 * su)]
    smp_hi = [(x, y, 10 * su * 8) for x in (64, 128) for y in (64, 192)]
    b.add_mesh_facet(hi, [(0, 1, 2), (3, 4, 5)], smp_hi)
    s = b.build("bent", 0)
    orc = oracle_mod.Oracle(s)
    tri = s.vertices[s.tri_vertices].astype(np.float64)
    P = s.samples[:4].astype(np.float64)
    Q = s.samples[4:].astype(np.float64)
    # the extra triangles do cross the segments, so a missing exclusion would show
    assert all(oracle_mod.segtri(p, q, *tri[1]) and oracle_mod.segtri(p, q, *tri[3]) for p in P for q in Q)
    assert _labels(oracle_mod, s, [(0, 1), (1, 0)], {0: (1, 6), 1: (2, 8)}) == [0, 0]
    # and with the exclusion the pair is visible
    assert orc.pair(0, 1) == 1
