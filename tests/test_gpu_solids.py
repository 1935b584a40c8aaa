"""Solid occluders and facet convexity: the device-side checks behind the bundle
certificates, and bit-exact parity on scenes built to break them.

The occluder grouping hint (ivm_scene_desc.facet_solid) must never change a
result: closed box buildings pass the prism check, open, gapped, overlapping or
merged groups fail it, and every matrix / table bit still equals the oracle's.
A non-convex occluder (a plate with a small hole that exactly one admissible
segment threads) must not be taken for a single-facet certificate.
"""
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ivm():
    import torch
    import paper_2501_02747_amd as ivm
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ivm.load_library()
    return ivm


G, N_SIDE, K = 2, 4, 3          # 0.25 m vertex grid, 4 x 4 samples, 1/32 m sample grid
VU, SU = 1 << G, 1 << (G + K)   # grid units per metre


def _parity(oracle_mod, ivm, s, hint="buildings"):
    """Full matrix and Tx/Rx tables against the oracle; returns (scene, stats)."""
    import torch
    fs = s.facet_building if isinstance(hint, str) else hint
    g = ivm.GpuScene.from_scene(s, solids=False, facet_solid=fs).check()
    st = ivm.new_stats()
    M = ivm.ivm_intervisibility_matrix(g, stats=st)
    tv, rv, los = ivm.ivm_txrx_visibility_table(g, torch.as_tensor(s.tx).cuda(), torch.as_tensor(s.rx).cuda())
    torch.cuda.synchronize()
    assert g.status() == 0
    orc = oracle_mod.Oracle(s)
    Mo, mism = orc.matrix(audit=True)
    assert mism == 0
    got = ivm.unpack_bits(M, s.n_facets)
    assert (got == Mo).all(), f"{int((got != Mo).sum())} matrix bits differ, first {np.argwhere(got != Mo)[:4].tolist()}"
    tvo, rvo, loso = orc.txrx(s.tx, s.rx)
    assert (ivm.unpack_bits(tv, s.n_facets) == tvo).all()
    assert (ivm.unpack_bits(rv, s.n_facets) == rvo).all()
    assert (los.cpu().numpy().astype(bool) == loso).all()
    return g, ivm.stats_dict(st), Mo


def _m(x):
    return int(round(x * VU))


def open_boxes_scene():
    """Ground plus six box groups; only A and G are closed prisms.
    A closed | B walls west+east missing (a tunnel along x) | C south+north
    panel 0 missing | D closed plus a duplicate west wall | E+F two closed boxes
    sharing one id | G closed, taller."""
    b = sg.SceneBuilder(G, K)
    b.add_rect((_m(-40), _m(-40), 0), (_m(80), 0, 0), (0, _m(80), 0), N_SIDE, sg.KIND_GROUND)
    b.add_box(_m(-10), _m(-4), _m(-2), _m(4), _m(8), N_SIDE, 0)                       # A
    b.add_box(_m(2), _m(-4), _m(10), _m(4), _m(8), N_SIDE, 1, omit=(2, 3))            # B tunnel
    b.add_box(_m(-10), _m(10), _m(-2), _m(18), _m(8), N_SIDE, 2, split_x=2, omit=(0, 2))  # C gaps
    b.add_box(_m(2), _m(10), _m(10), _m(18), _m(8), N_SIDE, 3)                        # D
    b.add_rect((_m(2), _m(10), 0), (0, 0, _m(8)), (0, _m(8), 0), N_SIDE, sg.KIND_WALL, 3)  # D duplicate west
    b.add_box(_m(-10), _m(-18), _m(-2), _m(-10), _m(8), N_SIDE, 4)                    # E
    b.add_box(_m(2), _m(-18), _m(10), _m(-10), _m(8), N_SIDE, 4)                      # F (same id)
    b.add_box(_m(14), _m(-4), _m(20), _m(4), _m(12), N_SIDE, 5)                       # G
    tx = [(-30 * SU, 0, 2 * SU), (0, 0, 20 * SU), (0, -7 * SU, 3 * SU)]
    rx = [(30 * SU, 1 * SU, 2 * SU), (12 * SU, 14 * SU, 2 * SU), (-6 * SU, 0, 30 * SU)]
    return b.build("open_boxes", 0, tx, rx)


def ring_scene():
    """Plates at z = 0 (facing up) and z = 10 m (facing down), 8 x 8 m, 4 x 4
    samples; between them at z = 5 m a 12 x 12 m plate with a 0.5 x 0.5 m
    square hole centred on (1, 1): only the segment (1,1,0)-(1,1,10) threads it."""
    b = sg.SceneBuilder(G, K)
    i = b.add_rect((0, 0, 0), (_m(8), 0, 0), (0, _m(8), 0), N_SIDE, sg.KIND_PLATE)
    j = b.add_rect((0, 0, _m(10)), (0, _m(8), 0), (_m(8), 0, 0), N_SIDE, sg.KIND_PLATE)
    z = _m(5)
    o = [(_m(-2), _m(-2)), (_m(10), _m(-2)), (_m(10), _m(10)), (_m(-2), _m(10))]
    h = [(_m(0.75), _m(0.75)), (_m(1.25), _m(0.75)), (_m(1.25), _m(1.25)), (_m(0.75), _m(1.25))]
    verts = [(x, y, z) for x, y in o] + [(x, y, z) for x, y in h]
    tris = []
    for k in range(4):
        k1 = (k + 1) % 4
        tris.append((k, k1, 4 + k1))
        tris.append((k, 4 + k1, 4 + k))
    smp = [(x * SU, y * SU, 5 * SU) for x, y in ((-1, -1), (9, -1), (9, 9), (-1, 9))]
    r = b.add_mesh_facet(verts, tris, smp, sg.KIND_PLATE)
    tx = [(1 * SU, 1 * SU, 12 * SU), (4 * SU, 4 * SU, 2 * SU)]
    rx = [(1 * SU, 1 * SU, -3 * SU), (6 * SU, 2 * SU, 7 * SU)]
    return b.build("ring", 0, tx, rx), (i, j, r)


def test_prism_check_counts(ivm):
    """Closed box and extruded-polygon buildings of every workload pass; the
    ground (hint -1) is never a solid."""
    cases = [("tiny urban", sg.gen_c1(1), 8), ("urban grid", sg.gen_c2(2), 200),
             ("large city", sg.gen_c3(3), 2000)]
    s4 = sg.gen_c4_scene(1005)
    cases.append(("batched scene", s4, int(s4.facet_building.max()) + 1))
    for name, s, n in cases:
        _log(f"[solids] prism check: {name}")
        g = ivm.GpuScene.from_scene(s).check()
        assert g.solids_verified() == n, name


def test_open_and_broken_groups_rejected(oracle_mod, ivm):
    _log("[solids] open / gapped / overlapping / merged groups")
    s = open_boxes_scene()
    g, st, Mo = _parity(oracle_mod, ivm, s)
    assert g.solids_verified() == 2          # A and G only
    # the tunnel through B is real: A's east wall sees G's west wall through it
    A_east = 1 + 3
    G_west = s.n_facets - 3
    assert Mo[A_east, G_west]


def test_hints_never_change_results(oracle_mod, ivm):
    """Random and permuted groupings on the tiny urban scenes: bits unchanged."""
    rng = np.random.default_rng(7)
    for seed in (1, 2, 3):
        _log(f"[solids] hint variants, seed={seed}")
        s = sg.gen_c1(seed)
        F = s.n_facets
        nb = int(s.facet_building.max()) + 1
        perm = rng.permutation(nb)
        permuted = np.where(s.facet_building >= 0, perm[np.maximum(s.facet_building, 0)], -1).astype(np.int32)
        g, _, _ = _parity(oracle_mod, ivm, s, hint=permuted)
        assert g.solids_verified() == nb
        noisy = rng.integers(-1, 6, F).astype(np.int32)
        _parity(oracle_mod, ivm, s, hint=noisy)
        none = np.full(F, -1, np.int32)
        g, st, _ = _parity(oracle_mod, ivm, s, hint=none)
        assert g.solids_verified() == 0 and st["solid_certified"] == 0


def test_urban_grid_solid_certificates(oracle_mod, ivm):
    """A 3 x 4 block urban grid: every block is a verified solid, the solid
    certificate decides pairs, and all bits equal the oracle's."""
    _log("[solids] small urban grid")
    s = sg.gen_c2(5, n_snap=24, nx=3, ny=4)
    g, st, _ = _parity(oracle_mod, ivm, s)
    assert g.solids_verified() == 12
    assert st["solid_certified"] > 0


def test_nonconvex_occluder_not_certified(oracle_mod, ivm):
    """The holed plate blocks 255 of the 256 admissible segments between the
    plates; it must not certify the pair (its triangles do not tile a convex
    polygon), and the pair is visible."""
    _log("[solids] holed plate")
    s, (i, j, r) = ring_scene()
    for no_tile in (0, 1):
        import torch
        g = ivm.GpuScene.from_scene(s).check()
        M = ivm.ivm_intervisibility_matrix(g, ivm.make_opts(no_tile=no_tile))
        torch.cuda.synchronize()
        m = ivm.unpack_bits(M, s.n_facets)
        assert m[i, j] and m[j, i]
    _, _, Mo = _parity(oracle_mod, ivm, s)
    assert Mo[i, j]
    assert oracle_mod.Oracle(s).segment_clear([1, 1, 0], [1, 1, 10], i, j)
    assert not oracle_mod.Oracle(s).segment_clear([3, 1, 0], [1, 1, 10], i, j)


def test_off_plane_samples(oracle_mod, ivm):
    """Samples lifted off their facet's plane disable the hull certificates for
    that facet; results still match the oracle."""
    _log("[solids] off-plane samples")
    s = sg.gen_c1(4)
    smp = s.samples.copy()
    f = 5
    a, b = s.sample_offsets[f], s.sample_offsets[f + 1]
    smp[a:b - 1, 2] += np.float32(0.5)   # all but one sample of facet 5 lifted by 0.5 m
    s.samples = smp
    _parity(oracle_mod, ivm, s)
