"""Edge rows of the matrix on the GPU (ivm_edge_rows) against the oracle, bit
for bit: edges as visibility nodes beside faces (Sections I and II-A), the face
seen for diffraction being the face seen for reflection (Section III-B).  Every
row of tiny urban scenes, seeded rows of the urban grid and of a batched-workload
scene, an edge whose samples leave its facets' planes (so the excluded facets
matter), FP64-only equal, and bad row ids reported."""
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
    assert torch.cuda.is_available()
    ivm.load_library()
    return ivm


def _run(ivm, g, s, rows, efac=None, esmp=None, **opts):
    import torch
    efac = s.edge_facets if efac is None else efac
    esmp = s.edge_samples if esmp is None else esmp
    ef, ee = ivm.ivm_edge_rows(g, torch.as_tensor(np.ascontiguousarray(efac, np.int32)).cuda(),
                               torch.as_tensor(np.ascontiguousarray(esmp, np.float32)).cuda(), s.samples_per_edge,
                               torch.as_tensor(np.asarray(rows, np.int32)).cuda(), ivm.make_opts(**opts))
    torch.cuda.synchronize()
    return ivm.unpack_bits(ef, s.n_facets), ivm.unpack_bits(ee, efac.shape[0])


def _check(oracle_mod, ivm, s, rows, threads=0):
    g = ivm.GpuScene.from_scene(s).check()
    ef, ee = _run(ivm, g, s, rows)
    assert g.status() == 0
    oef, oee = oracle_mod.edge_rows(oracle_mod.Oracle(s), s.edge_facets, s.edge_samples, s.samples_per_edge,
                                    rows=rows, threads=threads)
    assert (ef == oef).all(), f"edge-facet bits differ: {int((ef != oef).sum())}"
    assert (ee == oee).all(), f"edge-edge bits differ: {int((ee != oee).sum())}"
    _log(f"[edge rows] {s.name} seed {s.seed}: {len(rows)} rows, {int(oef.sum())} edge-facet and "
         f"{int(oee.sum())} edge-edge pairs visible")
    return g, ef, ee


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_tiny_urban_every_row(oracle_mod, ivm, seed):
    s = sg.gen_c1(seed)
    g, ef, ee = _check(oracle_mod, ivm, s, np.arange(s.edge_facets.shape[0]))
    assert (ee == ee.T).all() and not ee.diagonal().any()     # the definition is symmetric
    assert ef.any(1).mean() > 0.5


def test_urban_grid_seeded_rows(oracle_mod, ivm):
    s = sg.gen_c2(2)
    rows = np.sort(np.random.default_rng(7).choice(s.edge_facets.shape[0], 24, replace=False))
    _check(oracle_mod, ivm, s, rows)


def test_batched_scene_seeded_rows(oracle_mod, ivm):
    s = sg.gen_c4_scene(1005, f_target=900, n_snap=4)
    rows = np.sort(np.random.default_rng(8).choice(s.edge_facets.shape[0], 40, replace=False))
    _check(oracle_mod, ivm, s, rows)


def test_samples_off_the_planes(oracle_mod, ivm):
    """An edge whose samples sit 1/4 m in front of its facets: the exclusions of
    the definition then decide (segments can cross the edge's own facets)."""
    s = sg.gen_c1(5)
    efac = np.array(s.edge_facets, np.int32)
    esmp = np.array(s.edge_samples, np.float32).reshape(efac.shape[0], s.samples_per_edge, 3)
    V = np.asarray(s.vertices, np.float64)
    tf = np.asarray(s.tri_facet)
    moved = 0
    for e in range(0, efac.shape[0], 3):
        t = int(np.searchsorted(tf, efac[e, 0]))
        a, b, c = V[s.tri_vertices[t]]
        n = np.cross(b - a, c - a)
        if n[2] != 0:
            continue          # walls only: a horizontal step stays inside the scene's box
        k = int(np.argmax(np.abs(n)))
        esmp[e, :, k] += np.float32(0.25 * np.sign(n[k]))   # on the sample grid
        moved += 1
    assert moved >= 5
    esmp = esmp.reshape(-1, 3)
    g = ivm.GpuScene.from_scene(s).check()
    rows = np.arange(efac.shape[0])
    ef, ee = _run(ivm, g, s, rows, efac, esmp)
    assert g.status() == 0
    oef, oee = oracle_mod.edge_rows(oracle_mod.Oracle(s), efac, esmp, s.samples_per_edge, rows=rows)
    assert (ef == oef).all() and (ee == oee).all()


def test_fp64_only_and_options_equal(oracle_mod, ivm):
    s = sg.gen_c1(6)
    g = ivm.GpuScene.from_scene(s).check()
    rows = np.arange(s.edge_facets.shape[0])
    base = _run(ivm, g, s, rows)
    for opts in ({"fp64_only": True}, {"stack_depth": 2}, {"eps": float("inf")}):
        got = _run(ivm, g, s, rows, **opts)
        assert (got[0] == base[0]).all() and (got[1] == base[1]).all(), opts


def test_bad_row_reported(ivm):
    s = sg.gen_c1(1)
    g = ivm.GpuScene.from_scene(s).check()
    _run(ivm, g, s, [0, s.edge_facets.shape[0]])
    assert g.status() == ivm.IVM_ERR_INVALID_ARGUMENT
