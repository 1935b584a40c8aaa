"""Parity at the full workload sizes, in the launch configuration bench.py times.

* urban grid (2000 facets, 8x8 samples, 1000 snapshots): every bit of the
  matrix, both tables, LoS and the candidate counts against the full oracle
  result stored by tests/golden/make_oracle_cache.py (which calls only oracle/);
* large city (~20k facets, 10 000 snapshots) and the largest batched scene:
  seeded sampled pairs (half drawn uniformly, half among GPU-visible pairs so
  both outcomes are exercised), sampled Tx/Rx entries and LoS against the
  oracle computed one by one, plus symmetry / diagonal / padding properties.
"""
import os
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c2_seed2.npz")


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


def _run(ivm, s):
    import torch
    g = ivm.GpuScene.from_scene(s).check()
    M = ivm.ivm_intervisibility_matrix(g)
    tv, rv, los = ivm.ivm_txrx_visibility_table(g, torch.as_tensor(s.tx).cuda(), torch.as_tensor(s.rx).cuda())
    counts = ivm.ivm_image_tree_candidates(g, M, tv, rv, los, 2)
    torch.cuda.synchronize()
    assert g.status() == 0
    return g, M, tv, rv, los, counts


def _properties(ivm, M, F):
    m = ivm.unpack_bits(M, F)
    assert (m == m.T).all() and not m.diagonal().any()
    w = M.cpu().numpy().view(np.uint64)
    if F % 64:
        assert not (w[:, -1] >> np.uint64(F % 64)).any()
    return m


@pytest.mark.skipif(not os.path.exists(CACHE), reason="full oracle cache not generated")
def test_urban_grid_every_bit(oracle_mod, ivm):
    _log("[fullsize] urban grid vs the full oracle cache")
    s = sg.gen_c2(2)
    z = np.load(CACHE, allow_pickle=False)
    F = s.n_facets
    assert int(z["F"]) == F
    g, M, tv, rv, los, counts = _run(ivm, s)
    m = _properties(ivm, M, F)
    Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
    tvo = np.unpackbits(z["tx_vis"], axis=1)[:, :F].astype(bool)
    rvo = np.unpackbits(z["rx_vis"], axis=1)[:, :F].astype(bool)
    assert (m == Mo).all(), f"{int((m != Mo).sum())} matrix bits differ"
    assert (ivm.unpack_bits(tv, F) == tvo).all()
    assert (ivm.unpack_bits(rv, F) == rvo).all()
    assert (los.cpu().numpy().astype(bool) == z["los"]).all()
    assert (counts.cpu().numpy() == oracle_mod.candidates_matmul(Mo, tvo, rvo, z["los"], 2)).all()


def _sampled(oracle_mod, ivm, s, n_pairs, n_points, seed):
    g, M, tv, rv, los, counts = _run(ivm, s)
    F = s.n_facets
    m = _properties(ivm, M, F)
    orc = oracle_mod.Oracle(s)
    rng = np.random.default_rng(seed)
    I = rng.integers(0, F, n_pairs)
    J = rng.integers(0, F, n_pairs)
    vis = np.argwhere(np.triu(m, 1))
    pick = vis[rng.integers(0, len(vis), n_pairs)]
    I, J = np.concatenate([I, pick[:, 0]]), np.concatenate([J, pick[:, 1]])
    got = m[I, J]
    exp = orc.pairs(I, J)
    assert (got == exp).all(), f"pairs differ at {np.nonzero(got != exp)[0][:5]}"
    N = s.n_snapshots
    n_idx = rng.integers(0, N, n_points)
    f_idx = rng.integers(0, F, n_points)
    gtv, grv = ivm.unpack_bits(tv, F), ivm.unpack_bits(rv, F)
    # half of the entries among facets the GPU reports visible
    vt = np.argwhere(gtv)
    pt = vt[rng.integers(0, len(vt), n_points)]
    nn, ff = np.concatenate([n_idx, pt[:, 0]]), np.concatenate([f_idx, pt[:, 1]])
    assert (orc.point_facets(s.tx[nn], ff) == gtv[nn, ff]).all()
    vr = np.argwhere(grv)
    pr = vr[rng.integers(0, len(vr), n_points)]
    nn, ff = np.concatenate([n_idx, pr[:, 0]]), np.concatenate([f_idx, pr[:, 1]])
    assert (orc.point_facets(s.rx[nn], ff) == grv[nn, ff]).all()
    assert (orc.los(s.tx[n_idx], s.rx[n_idx]) == los.cpu().numpy().astype(bool)[n_idx]).all()
    # candidate counts follow from the tables by integer products (checked on sampled snapshots)
    Mi = m.astype(np.int64)
    c = counts.cpu().numpy()
    for n in n_idx[:20]:
        t, r = gtv[n].astype(np.int64), grv[n].astype(np.int64)
        assert c[n, 1] == int(t @ r) and c[n, 2] == int(t @ Mi @ r)


def test_large_city_sampled(oracle_mod, ivm):
    _log("[fullsize] large city, sampled")
    _sampled(oracle_mod, ivm, sg.gen_c3(3), 200, 150, 11)


def test_largest_batched_scene_sampled(oracle_mod, ivm):
    _log("[fullsize] largest batched scene, sampled")
    scenes_f = [(k, sg.gen_c4_scene(1000 + k).n_facets) for k in (0, 5, 12, 32)]
    k = max(scenes_f, key=lambda t: t[1])[0]
    _sampled(oracle_mod, ivm, sg.gen_c4_scene(1000 + k), 150, 150, 12)
