"""Angular bouncing ranges on the GPU (ivm_angular_ranges) against the oracle
(Section II-A views, Section II-B eq. 1 and eq. 2), for matrices the oracle
computed: the two-facet closed-form scenes of the oracle pins with every pair
set, tiny urban scenes, whole rows of the urban grid's stored full matrix,
the large city's stored oracle rows, and a random one-sided matrix.

Columns and CSR offsets must be equal.  The angles must agree to within a
tolerance derived from the arithmetic: both sides form the same three integer
terms exactly and round each once to FP64, then multiply, take a correctly
rounded square root and divide (identical results); only arccos differs, by
at most a few ulp of the result (the GPU's device-library arccos against the
host's), so rtol 1e-14 with an absolute floor of 1e-12 degrees for angles near
zero.  Zeros from eq. 2 are exact on both sides."""
import os
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu
CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c2_seed2.npz")
C3_CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c3_seed3_rows.npz")
RTOL, ATOL = 1e-14, 1e-12


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ivm():
    import torch
    import paper_2501_02747_amd as ivm
    assert torch.cuda.is_available()
    ivm.load_library()
    return ivm


def _pack(bits, W):
    N, F = bits.shape
    b = np.packbits(np.asarray(bits, np.uint8), axis=1, bitorder="little")
    out = np.zeros((N, W * 8), np.uint8)
    out[:, :b.shape[1]] = b
    return out.view(np.uint64)


def _compare(oracle_mod, ivm, s, Mo, rows=None, g=None):
    import torch
    g = g or ivm.GpuScene.from_scene(s).check()
    M = torch.as_tensor(_pack(Mo, g.W).view(np.int64)).cuda()
    off, cols, rng = ivm.ivm_angular_ranges(g, M)
    off, cols, rng = off.cpu().numpy(), cols.cpu().numpy(), rng.cpu().numpy()
    r = oracle_mod.angular_ranges(s, Mo, rows=rows)
    F = s.n_facets
    assert (np.diff(off) == np.asarray(Mo, bool).sum(1)).all()
    rows = range(F) if rows is None else rows
    worst = 0.0
    n = 0
    for i in rows:
        a, b = off[i], off[i + 1]
        oa, ob = r["offsets"][i], r["offsets"][i + 1]
        assert (cols[a:b] == r["cols"][oa:ob]).all(), i
        got, exp = rng[a:b], r["ranges"][oa:ob]
        assert not np.isnan(got).any(), i
        assert ((got == 0) == (exp == 0)).all(), i
        np.testing.assert_allclose(got, exp, rtol=RTOL, atol=ATOL)
        if len(got):
            worst = max(worst, float(np.abs(got - exp).max()))
        n += b - a
    _log(f"[angles] {s.name}: {n} pairs compared, largest difference {worst:.3g} degrees")
    return off, cols, rng


WALL_S = [[0, 0, 0], [0, 0, 4], [8, 0, 0]]


@pytest.mark.parametrize("other", [
    [[0, 6, 0], [8, 0, 0], [0, 0, 4]],      # parallel wall facing it
    [[12, 2, 0], [0, 0, 4], [0, 6, 0]],     # perpendicular wall
    [[12, -2, 0], [0, 0, 4], [0, 6, 0]],    # one end behind the reference plane (eq. 2)
    [[12, 0, 0], [0, 0, 4], [0, 6, 0]],     # one end on the reference plane (eq. 2)
    [[-4, 2, 0], [16, 0, 0], [0, 10, 0]],   # ground in front of the wall: a vertical view
])
def test_two_facet_closed_form_scenes(oracle_mod, ivm, other):
    s = sg.gen_plates([WALL_S, other])
    _compare(oracle_mod, ivm, s, ~np.eye(2, dtype=bool))


def test_plates_every_pair(oracle_mod, ivm):
    s = sg.gen_plates([
        [[-20, -20, 0], [40, 0, 0], [0, 40, 0]],
        [[0, 0, 0], [0, 0, 8], [0, 8, 0]],
        [[10, 0, 0], [0, 8, 0], [0, 0, 8]],
        [[0, 0, 0], [8, 0, 0], [0, 0, 8]],
        [[0, 0, 8], [8, 0, 0], [0, 8, 0]],
        [[20, 0, 0], [-4, 4, 0], [0, 0, 4]],
        [[-10, 5, 1], [3, 0, 3], [0, 6, 0]],
    ])
    _compare(oracle_mod, ivm, s, ~np.eye(s.n_facets, dtype=bool))


@pytest.mark.parametrize("seed", range(1, 9))
def test_tiny_urban_scenes(oracle_mod, ivm, seed):
    s = sg.gen_c1(seed)
    Mo, _ = oracle_mod.Oracle(s).matrix()
    _compare(oracle_mod, ivm, s, Mo)


@pytest.mark.skipif(not os.path.exists(CACHE), reason="full oracle cache not generated")
def test_urban_grid_rows(oracle_mod, ivm):
    """Every visible pair of the urban grid on the GPU; 120 seeded whole rows
    against the oracle."""
    s = sg.gen_c2(2)
    z = np.load(CACHE, allow_pickle=False)
    F = s.n_facets
    Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
    rows = np.sort(np.random.default_rng(5).choice(F, 120, replace=False))
    _compare(oracle_mod, ivm, s, Mo, rows=rows)


@pytest.mark.skipif(not os.path.exists(C3_CACHE), reason="large-city oracle rows not generated")
def test_large_city_rows(oracle_mod, ivm):
    """The 64 stored oracle rows of the large city (the other rows empty)."""
    s = sg.gen_c3(3)
    z = np.load(C3_CACHE, allow_pickle=False)
    F = s.n_facets
    Mo = np.zeros((F, F), bool)
    Mo[z["rows"]] = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
    _compare(oracle_mod, ivm, s, Mo, rows=z["rows"])


def test_random_one_sided_matrix(oracle_mod, ivm):
    """Any set bit is a pair to measure, whatever the matrix: a seeded random
    one-sided matrix over a batched-workload scene with a ragged row width."""
    s = sg.gen_c4_scene(1003, f_target=330, n_snap=4)
    F = s.n_facets
    assert F % 64
    Mo = np.random.default_rng(9).random((F, F)) < 0.03
    np.fill_diagonal(Mo, False)
    _compare(oracle_mod, ivm, s, Mo)


def test_capacity_and_empty(oracle_mod, ivm):
    import torch
    s = sg.gen_c1(2)
    Mo, _ = oracle_mod.Oracle(s).matrix()
    g = ivm.GpuScene.from_scene(s).check()
    M = torch.as_tensor(_pack(Mo, g.W).view(np.int64)).cuda()
    nnz = int(Mo.sum())
    off = torch.empty((s.n_facets + 1,), dtype=torch.int64, device="cuda")
    cols = torch.empty((nnz - 1,), dtype=torch.int32, device="cuda")
    rng = torch.empty((nnz - 1, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="IVM_ERR_CAPACITY"):
        ivm.ivm_angular_ranges(g, M, out=(off, cols, rng))
    assert (off.cpu().numpy() == np.concatenate([[0], np.cumsum(Mo.sum(1))])).all()
    # an empty matrix gives empty rows
    o, c, r = ivm.ivm_angular_ranges(g, torch.zeros_like(M))
    assert (o.cpu().numpy() == 0).all() and c.numel() == 0 and r.numel() == 0
