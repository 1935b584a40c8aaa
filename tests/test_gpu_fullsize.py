"""Parity at the full workload sizes, in the launch configuration bench.py times.

* urban grid (2000 facets, 8x8 samples, 1000 snapshots): every bit of the
  matrix, both tables, LoS and the candidate counts against the full oracle
  result stored by tests/golden/make_oracle_cache.py (which calls only oracle/);
* large city (19 872 facets, 10 000 snapshots): 64 seeded whole rows of the
  matrix and 200 seeded whole snapshots (both tables and LoS) against the
  oracle results stored by tests/golden/make_c3_oracle_cache.py, plus
  sampled pairs and table entries computed one by one;
* the largest batched scene: sampled pairs and table entries.
Sampled pairs are drawn half among the pairs that pass the orientation rule
(some admissible segment) and that the GPU reports blocked, half among the
GPU-visible ones, so a false result of either kind can show; table entries
likewise among facets in front of the point that the GPU reports hidden, and
among GPU-visible ones.  Symmetry, diagonal and padding are checked too.
"""
import os
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c2_seed2.npz")
C3_CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c3_seed3_rows.npz")


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


def _orient_any(s, F_idx, X):
    """For each k: some point X[k] (rows of points, [n, m, 3]) strictly in
    front of facet F_idx[k] (FP64, exact on the scene's grids)."""
    V = np.asarray(s.vertices, np.float64)
    tf = np.asarray(s.tri_facet)
    first = np.searchsorted(tf, F_idx)
    tri = np.asarray(s.tri_vertices)[first]
    a, b, c = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    n = np.cross(b - a, c - a)
    o = np.einsum("kmd,kd->km", X - a[:, None, :], n)
    return (o > 0).any(1)


def _facet_samples(s, f):
    off = np.asarray(s.sample_offsets)
    return np.asarray(s.samples, np.float64)[off[f]:off[f + 1]]


def _admissible(s, I, J):
    """Pair (i, j) has some admissible segment: a sample of j in front of i and
    a sample of i in front of j (the two conditions are independent)."""
    out = np.zeros(len(I), bool)
    for k, (i, j) in enumerate(zip(I, J)):
        if i == j:
            continue
        Si, Sj = _facet_samples(s, i), _facet_samples(s, j)
        out[k] = _orient_any(s, np.array([i]), Sj[None])[0] and _orient_any(s, np.array([j]), Si[None])[0]
    return out


def _pick(rng, cand, n):
    return cand[rng.choice(len(cand), min(n, len(cand)), replace=False)] if len(cand) else cand


def _sampled_check(oracle_mod, ivm, s, res, n_pairs, n_points, seed):
    g, M, tv, rv, los, counts = res
    F = s.n_facets
    m = _properties(ivm, M, F)
    orc = oracle_mod.Oracle(s)
    rng = np.random.default_rng(seed)
    # pairs: admissible and GPU-blocked (a false negative would show), and GPU-visible
    I, J = rng.integers(0, F, 40 * n_pairs), rng.integers(0, F, 40 * n_pairs)
    keep = (I != J) & ~m[I, J]
    I, J = I[keep], J[keep]
    adm = _admissible(s, I[:20 * n_pairs], J[:20 * n_pairs])
    blocked = _pick(rng, np.stack([I[:20 * n_pairs][adm], J[:20 * n_pairs][adm]], 1), n_pairs)
    visible = _pick(rng, np.argwhere(np.triu(m, 1)), n_pairs)
    P = np.concatenate([blocked, visible]).astype(np.int64)
    _log(f"[fullsize] {len(blocked)} admissible GPU-blocked + {len(visible)} GPU-visible pairs")
    assert len(blocked) > n_pairs // 2 and len(visible) > n_pairs // 2
    exp = orc.pairs(P[:, 0], P[:, 1])
    got = m[P[:, 0], P[:, 1]]
    assert (got == exp).all(), f"pairs differ at {P[np.nonzero(got != exp)[0][:5]].tolist()}"
    N = s.n_snapshots
    gtv, grv = ivm.unpack_bits(tv, F), ivm.unpack_bits(rv, F)
    for X, gt, side in ((s.tx, gtv, "tx"), (s.rx, grv, "rx")):
        nn, ff = rng.integers(0, N, 20 * n_points), rng.integers(0, F, 20 * n_points)
        hidden = ~gt[nn, ff]
        nn, ff = nn[hidden], ff[hidden]
        front = np.array([_orient_any(s, np.array([f]), np.asarray(X[n], np.float64)[None, None])[0]
                          for n, f in zip(nn[:8 * n_points], ff[:8 * n_points])], bool)
        hid = _pick(rng, np.stack([nn[:8 * n_points][front], ff[:8 * n_points][front]], 1), n_points)
        vis = _pick(rng, np.argwhere(gt), n_points)
        E = np.concatenate([hid, vis]).astype(np.int64)
        assert len(hid) > n_points // 2 and len(vis) > n_points // 2, side
        assert (orc.point_facets(X[E[:, 0]], E[:, 1]) == gt[E[:, 0], E[:, 1]]).all(), side
    n_idx = rng.integers(0, N, n_points)
    assert (orc.los(s.tx[n_idx], s.rx[n_idx]) == los.cpu().numpy().astype(bool)[n_idx]).all()
    # candidate counts follow from the tables by integer products (checked on sampled snapshots)
    Mi = m.astype(np.int64)
    c = counts.cpu().numpy()
    for n in n_idx[:20]:
        t, r = gtv[n].astype(np.int64), grv[n].astype(np.int64)
        assert c[n, 1] == int(t @ r) and c[n, 2] == int(t @ Mi @ r)


def _sampled(oracle_mod, ivm, s, n_pairs, n_points, seed):
    _sampled_check(oracle_mod, ivm, s, _run(ivm, s), n_pairs, n_points, seed)


@pytest.fixture(scope="module")
def large_city(ivm):
    s = sg.gen_c3(3)
    return s, _run(ivm, s)


@pytest.mark.skipif(not os.path.exists(C3_CACHE), reason="large-city oracle rows not generated")
def test_large_city_full_rows_and_snapshots(ivm, large_city):
    """64 whole rows (every column) and 200 whole snapshots (every facet from
    both ends, and LoS) bit for bit against the stored oracle results."""
    s, (g, M, tv, rv, los, counts) = large_city
    F = s.n_facets
    z = np.load(C3_CACHE, allow_pickle=False)
    assert int(z["F"]) == F
    rows, snaps = z["rows"], z["snaps"]
    _log(f"[fullsize] large city: {len(rows)} whole rows, {len(snaps)} whole snapshots")
    m = _properties(ivm, M, F)
    Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
    diff = m[rows] != Mo
    assert not diff.any(), f"{int(diff.sum())} matrix bits differ in the stored rows"
    assert Mo.any(1).sum() > len(rows) // 2       # the rows hold visible pairs to compare
    for key, t in (("tx_vis", tv), ("rx_vis", rv)):
        o = np.unpackbits(z[key], axis=1)[:, :F].astype(bool)
        gt = ivm.unpack_bits(t, F)[snaps]
        assert (gt == o).all(), f"{key}: {int((gt != o).sum())} bits differ"
    assert (los.cpu().numpy().astype(bool)[snaps] == z["los"]).all()


def test_large_city_sampled(oracle_mod, ivm, large_city):
    _log("[fullsize] large city, sampled")
    s, res = large_city
    _sampled_check(oracle_mod, ivm, s, res, 200, 150, 11)


def test_largest_batched_scene_sampled(oracle_mod, ivm):
    _log("[fullsize] largest batched scene, sampled")
    scenes_f = [(k, sg.gen_c4_scene(1000 + k).n_facets) for k in (0, 5, 12, 32)]
    k = max(scenes_f, key=lambda t: t[1])[0]
    _sampled(oracle_mod, ivm, sg.gen_c4_scene(1000 + k), 150, 150, 12)
