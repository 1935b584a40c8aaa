"""GPU parity of the edge visibility for first-order diffraction (Section III-B)
through the C ABI: the bits of every edge seen from Tx and Rx, and the
Tx -> edge -> Rx counts, against the oracle.  Every predicate is exact on the
sample grid, so the bar is bit-for-bit equality.  Expected values come only
from oracle/."""
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


def _edges_gpu(ivm, s, tx, rx, opts=None):
    import torch
    g = ivm.GpuScene.from_scene(s).check()
    ef = torch.as_tensor(s.edge_facets).cuda()
    es = torch.as_tensor(s.edge_samples).cuda()
    te, re_, cnt = ivm.ivm_edge_visibility(g, ef, es, s.samples_per_edge, torch.as_tensor(tx).cuda(),
                                           torch.as_tensor(rx).cuda(), opts)
    torch.cuda.synchronize()
    assert g.status() == 0
    E = s.edge_facets.shape[0]
    return ivm.unpack_bits(te, E), ivm.unpack_bits(re_, E), cnt.cpu().numpy(), te, g


def _oracle_edges(oracle_mod, s, X):
    orc = oracle_mod.Oracle(s)
    return oracle_mod.edge_visibility(orc, X, s.edge_facets, s.edge_samples, s.samples_per_edge)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_c1_edges_parity(oracle_mod, ivm, seed):
    """Tiny urban scene (8 boxes, 64 edges, 4 samples each, 10 snapshots): every
    edge bit from Tx and Rx and every diffraction count equal the oracle's."""
    _log(f"[edges c1] seed={seed}")
    s = sg.gen_c1(seed)
    gt, gr, gc, te, _ = _edges_gpu(ivm, s, s.tx, s.rx)
    ot = _oracle_edges(oracle_mod, s, s.tx)
    orr = _oracle_edges(oracle_mod, s, s.rx)
    assert (gt == ot).all() and (gr == orr).all()
    assert (gc == oracle_mod.diffraction_counts(ot, orr)).all()
    E = s.edge_facets.shape[0]
    words = te.cpu().numpy().view(np.uint64)
    if E % 64:
        assert not (words[:, -1] >> np.uint64(E % 64)).any(), "padding bits must be zero"
    assert ot.any() and not ot.all()


def _box_scene(extra_plate=None, pts=((0, 0, 0),)):
    g, k, n = 4, 3, 4
    su, ss = 1 << g, 1 << (g + k)
    b = sg.SceneBuilder(g, k)
    b.add_box(0, 0, 10 * su, 10 * su, 10 * su, n, 0)
    if extra_plate is not None:
        v0, U, V = extra_plate
        b.add_rect(tuple(c * su for c in v0), tuple(c * su for c in U), tuple(c * su for c in V), n)
    P = [tuple(int(c * ss) for c in p) for p in pts]
    return b.build("box", 0, P, P)


def test_box_closed_forms_end_to_end(oracle_mod, ivm):
    """The closed forms the oracle is pinned to, computed on the GPU: an isolated
    box seen from five points, and a low plate that leaves only each corner's top
    sample clear (6 m) or none (7 m)."""
    pts = [(5, -20, 5), (5, 5, 30), (5, -20, 20), (30, -20, 5), (5, 5, 10)]
    expect = [{0, 1, 4}, {4, 5, 6, 7}, {0, 1, 4, 5, 6, 7}, {0, 1, 3, 4, 7}, set()]
    s = _box_scene(pts=pts)
    gt, gr, gc, _, _ = _edges_gpu(ivm, s, s.tx, s.rx)
    for n, e in enumerate(expect):
        assert set(np.nonzero(gt[n])[0].tolist()) == e, n
        assert gc[n] == len(e)
    for h, e in ((6, {0, 1, 4}), (7, {4})):
        s = _box_scene(extra_plate=((-40, -10, 0), (90, 0, 0), (0, 0, h)), pts=[(5, -20, 5)])
        gt, _, _, _, _ = _edges_gpu(ivm, s, s.tx, s.rx)
        assert set(np.nonzero(gt[0])[0].tolist()) == e, h


@pytest.mark.parametrize("cfg,n_check", [("c2", 3), ("c4", 3)])
def test_edges_full_size_sampled(oracle_mod, ivm, cfg, n_check):
    """Urban grid (2000 edges x 8 samples, 1000 snapshots) and one batched-workload
    scene (about 2400 edges x 4 samples): the whole trajectory on the GPU in the
    launch the bench times, with seeded sampled snapshots checked against the
    oracle bit for bit, and the FP64-only option giving the same bits."""
    import paper_2501_02747_amd as pkg
    s = sg.make_config(cfg)
    _log(f"[edges {cfg}] E={s.edge_facets.shape[0]} N={s.n_snapshots}")
    gt, gr, gc, _, _ = _edges_gpu(ivm, s, s.tx, s.rx)
    rng = np.random.default_rng(7)
    pick = np.sort(rng.choice(s.n_snapshots, n_check, replace=False))
    ot = _oracle_edges(oracle_mod, s, s.tx[pick])
    orr = _oracle_edges(oracle_mod, s, s.rx[pick])
    assert (gt[pick] == ot).all() and (gr[pick] == orr).all()
    assert (gc[pick] == oracle_mod.diffraction_counts(ot, orr)).all()
    assert (gc == (gt & gr).sum(1)).all()
    f64 = pkg.make_opts(fp64_only=True)
    gt2, gr2, _, _, _ = _edges_gpu(ivm, s, s.tx[pick], s.rx[pick], f64)
    assert (gt2 == gt[pick]).all() and (gr2 == gr[pick]).all()


def test_edge_inputs_checked(ivm):
    """An off-grid edge sample is reported as a grid error and a facet id out of
    range as an invalid argument, by the scene status; no edge is read out of
    bounds (the kernel skips bad ids)."""
    import torch
    s = sg.gen_c1(1, n_snap=2)
    tx, rx = torch.as_tensor(s.tx).cuda(), torch.as_tensor(s.rx).cuda()
    ef = torch.as_tensor(s.edge_facets).cuda()
    es = s.edge_samples.copy()
    es[3, 0] += 1.0 / 1024
    g = ivm.GpuScene.from_scene(s).check()
    ivm.ivm_edge_visibility(g, ef, torch.as_tensor(es).cuda(), s.samples_per_edge, tx, rx)
    torch.cuda.synchronize()
    assert g.status() == ivm.IVM_ERR_GRID
    bad = s.edge_facets.copy()
    bad[5, 1] = s.n_facets
    g = ivm.GpuScene.from_scene(s).check()
    ivm.ivm_edge_visibility(g, torch.as_tensor(bad).cuda(), torch.as_tensor(s.edge_samples).cuda(),
                            s.samples_per_edge, tx, rx)
    torch.cuda.synchronize()
    assert g.status() == ivm.IVM_ERR_INVALID_ARGUMENT
    # no edges: zero counts
    g = ivm.GpuScene.from_scene(s).check()
    te, re_, cnt = ivm.ivm_edge_visibility(g, torch.zeros((0, 2), dtype=torch.int32, device="cuda"),
                                           torch.zeros((0, 3), dtype=torch.float32, device="cuda"), 4, tx, rx)
    torch.cuda.synchronize()
    assert cnt.cpu().numpy().tolist() == [0, 0] and te.shape[1] == 0
