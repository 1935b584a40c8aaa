"""Exact image-method validation of candidate walks on the GPU
(ivm_validate_paths) against the oracle's exact rational validator
(Section III-A image method; Section IV-B: the pruned tree keeps the valid
rays).  The walk lists come from the oracle (its matrix and tables,
enumerated), and both sides judge the same walks; verdicts must be equal walk
for walk.  Closed forms: two parallel mirrors (two valid paths of every order
1-4), the 90-degree corner (2, 1, 0 paths of orders 1-3), a specular point on a
facet's edge (closed facet) and one grid step off it."""
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


def _csr(lists, K):
    """Oracle lists [n][k-1] -> (offsets int64 [N*K+1] in int32 elements, paths int32)."""
    offs, flat = [0], []
    for per in lists:
        for k in range(1, K + 1):
            for w in per[k - 1]:
                flat.extend(w)
            offs.append(len(flat))
    return np.asarray(offs, np.int64), np.asarray(flat, np.int32)


def _walks(offsets, paths, N, K):
    out = []
    for n in range(N):
        for k in range(1, K + 1):
            a, b = offsets[n * K + k - 1], offsets[n * K + k]
            for e in range(a, b, k):
                out.append((n, k, e, tuple(int(x) for x in paths[e:e + k])))
    return out


def _gpu_validate(ivm, s, lists, K, snaps=None):
    import torch
    g = ivm.GpuScene.from_scene(s).check()
    off, paths = _csr(lists, K)
    tx = s.tx if snaps is None else s.tx[snaps]
    rx = s.rx if snaps is None else s.rx[snaps]
    st = ivm.new_stats()
    valid, counts = ivm.ivm_validate_paths(g, torch.as_tensor(np.ascontiguousarray(tx)).cuda(),
                                           torch.as_tensor(np.ascontiguousarray(rx)).cuda(), K,
                                           torch.as_tensor(off).cuda(), torch.as_tensor(paths).cuda(), stats=st)
    torch.cuda.synchronize()
    return off, paths, valid.cpu().numpy(), counts.cpu().numpy(), ivm.stats_dict(st)


def _oracle_lists(oracle_mod, s, K):
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    tv, rv, los = orc.txrx(s.tx, s.rx)
    return oracle_mod.candidates_enum(M, tv, rv, los, K)[1]


def _check(oracle_mod, ivm, s, lists, K, sample=None, seed=0):
    off, paths, valid, counts, st = _gpu_validate(ivm, s, lists, K)
    walks = _walks(off, paths, len(lists), K)
    assert set(np.unique(valid)) <= {0, 1}
    for n, k, e, w in walks:
        assert (valid[e:e + k] == valid[e]).all()
    pick = range(len(walks))
    if sample is not None and len(walks) > sample:
        pick = np.sort(np.random.default_rng(seed).choice(len(walks), sample, replace=False))
    ex = oracle_mod._ExactImage(s)
    bad = []
    for idx in pick:
        n, k, e, w = walks[idx]
        exp = bool(oracle_mod.validate_paths_exact(s, s.tx[n], s.rx[n], [w], ex=ex)[0])
        if bool(valid[e]) != exp:
            bad.append((n, w, int(valid[e]), exp))
    assert not bad, f"verdicts differ: {bad[:5]}"
    # the per-(snapshot, order) counts are the verdict sums
    for n in range(len(lists)):
        for k in range(1, K + 1):
            a, b = off[n * K + k - 1], off[n * K + k]
            assert counts[n, k - 1] == int(valid[a:b:k].sum()) if b > a else counts[n, k - 1] == 0
    _log(f"[paths] {s.name}: {len(walks)} walks, {int(sum(valid[e] for _, _, e, _ in walks))} valid, "
         f"{len(pick)} checked against the oracle; {st['tri_tests']} leg tests, {st['rechecks']} exact")
    return off, paths, valid, counts


def test_parallel_mirrors_two_paths_every_order(oracle_mod, ivm):
    s = sg.gen_plates([
        [[0, -40, -40], [0, 80, 0], [0, 0, 80]],
        [[10, -40, -40], [0, 0, 80], [0, 80, 0]],
    ], tx=[[3, -2, 1]], rx=[[6, 5, -1]])
    lists = _oracle_lists(oracle_mod, s, 4)
    off, paths, valid, counts = _check(oracle_mod, ivm, s, lists, 4)
    assert counts[0].tolist() == [2, 2, 2, 2]


def test_corner_reflector(oracle_mod, ivm):
    s = sg.gen_plates([
        [[0, 0, -20], [0, 40, 0], [0, 0, 40]],
        [[0, 0, -20], [0, 0, 40], [40, 0, 0]],
    ], tx=[[5, 12, 1]], rx=[[14, 4, 0.5]])
    lists = _oracle_lists(oracle_mod, s, 3)
    off, paths, valid, counts = _check(oracle_mod, ivm, s, lists, 3)
    assert counts[0].tolist() == [2, 1, 0]
    ok = [w for _, k, e, w in _walks(off, paths, 1, 3) if valid[e]]
    assert (0, 1) in ok and (1, 0) not in ok


@pytest.mark.parametrize("y0,expect", [(0.0, 1), (1.0 / 16, 0)])
def test_specular_point_on_the_facet_edge(oracle_mod, ivm, y0, expect):
    s = sg.gen_plates([[[0, y0, -20], [0, 40, 0], [0, 0, 40]]], tx=[[5, -3, 1]], rx=[[5, 3, 1]])
    lists = [[[(0,)]]]
    off, paths, valid, counts = _check(oracle_mod, ivm, s, lists, 1)
    assert int(valid[0]) == expect


@pytest.mark.parametrize("seed", [1, 2])
def test_tiny_urban_orders_1_2(oracle_mod, ivm, seed):
    """Every candidate of orders 1 and 2 of the tiny urban scene (10 snapshots)."""
    s = sg.gen_c1(seed)
    lists = _oracle_lists(oracle_mod, s, 2)
    _check(oracle_mod, ivm, s, lists, 2)


def test_tiny_urban_orders_3_4_sampled(oracle_mod, ivm):
    s = sg.gen_c1(3, n_snap=2)
    lists = _oracle_lists(oracle_mod, s, 4)
    _check(oracle_mod, ivm, s, lists, 4, sample=2000, seed=3)


def test_urban_grid_sampled(oracle_mod, ivm):
    """Candidates of orders 1-2 of 3 urban-grid snapshots (all validated on the
    GPU); 12 of them judged by the oracle.  (On this trajectory, Rx 750 m from
    the Tx behind many buildings, no candidate is a valid specular path: the
    oracle's brute force over every walk agrees on smaller grids.)"""
    import os
    s = sg.gen_c2(2)
    cache = os.path.join(os.path.dirname(__file__), "golden", "cache", "c2_seed2.npz")
    if not os.path.exists(cache):
        pytest.skip("full oracle cache not generated")
    z = np.load(cache, allow_pickle=False)
    F = s.n_facets
    snaps = np.array([0, 499, 999])
    M = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
    tv = np.unpackbits(z["tx_vis"], axis=1)[snaps, :F].astype(bool)
    rv = np.unpackbits(z["rx_vis"], axis=1)[snaps, :F].astype(bool)
    _, lists = oracle_mod.candidates_enum(M, tv, rv, z["los"][snaps], 2)
    s.tx, s.rx = s.tx[snaps], s.rx[snaps]
    _check(oracle_mod, ivm, s, lists, 2, sample=12, seed=5)


def test_urban_grid_street_canyon(oracle_mod, ivm):
    """A small urban grid (4 x 3 blocks) with Rx placed along the streets that
    meet under the Tx (where first- and second-order specular paths exist):
    every candidate of orders 1-2, GPU against the oracle walk for walk."""
    s = sg.gen_c2(4, n_snap=4, nx=4, ny=3)
    T = s.tx[0]
    s.rx = np.array([[T[0] + 20, T[1], 1.5], [T[0] + 45, T[1] + 3, 1.5], [T[0], T[1] - 30, 1.5],
                     [T[0] - 3, T[1] + 60, 1.5]], np.float32)
    s.tx = np.repeat(s.tx[:1], 4, 0)
    lists = _oracle_lists(oracle_mod, s, 2)
    off, paths, valid, counts = _check(oracle_mod, ivm, s, lists, 2)
    assert counts[:3].sum(1).min() >= 3     # the canyon reflections exist


def test_bad_walks_rejected(ivm):
    import torch
    s = sg.gen_c1(1, n_snap=1)
    g = ivm.GpuScene.from_scene(s).check()
    tx, rx = torch.as_tensor(s.tx).cuda(), torch.as_tensor(s.rx).cuda()
    for walk in ([3, 3], [0, s.n_facets]):   # a facet twice in a row; an id out of range
        off = torch.as_tensor(np.array([0, 0, 2], np.int64)).cuda()
        paths = torch.as_tensor(np.array(walk, np.int32)).cuda()
        with pytest.raises(RuntimeError, match="IVM_ERR_INVALID_ARGUMENT"):
            ivm.ivm_validate_paths(g, tx, rx, 2, off, paths)
