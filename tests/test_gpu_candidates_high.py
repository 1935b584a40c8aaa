"""GPU parity of the image-tree candidates of orders 3 and 4 (the iteration of
Section II-C to the orders timed in Section IV-C) against the oracle's walk
enumeration and integer products, through the C ABI.  Counts and lists are
integers: the bar is exact equality.  Inputs are seeded tables or oracle
matrices and tables of seeded scenes; no expected value comes from the GPU.
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


def _plate_row_scene(ivm, F):
    """F small plates on a line: a valid scene with exactly F facets (W = ceil(F/64))."""
    x = np.arange(F, dtype=np.float32)
    V = np.stack([np.stack([x, 0 * x, 0 * x], 1), np.stack([x + 0.5, 0 * x, 0 * x], 1),
                  np.stack([x + 0.5, 0 * x + 0.5, 0 * x], 1), np.stack([x, 0 * x + 0.5, 0 * x], 1)], 1)
    base = 4 * np.arange(F, dtype=np.int32)[:, None]
    T = np.stack([np.concatenate([base, base + 1, base + 2], 1), np.concatenate([base, base + 2, base + 3], 1)], 1)
    TF = np.repeat(np.arange(F, dtype=np.int32), 2)
    SM = np.stack([x + 0.25, 0 * x + 0.25, 0 * x], 1)
    OFF = np.arange(F + 1, dtype=np.int32)
    return ivm.GpuScene(V.reshape(-1, 3), T.reshape(-1, 3), TF, OFF, SM, 2, 2).check()


def _upload(ivm, M, tv, rv, los):
    import torch
    return (torch.as_tensor(ivm.pack_bits(M)).cuda(), torch.as_tensor(ivm.pack_bits(tv)).cuda(),
            torch.as_tensor(ivm.pack_bits(rv)).cuda(), torch.as_tensor(np.asarray(los, np.uint8)).cuda())


def _check_lists(off, paths, lists, N, K):
    off = off.cpu().numpy()
    paths = paths.cpu().numpy()
    for n in range(N):
        for k in range(1, K + 1):
            a, b = off[n * K + k - 1], off[n * K + k]
            got = [tuple(int(x) for x in paths[p:p + k]) for p in range(a, b, k)]
            assert got == lists[n][k - 1], (n, k)


@pytest.mark.parametrize("F,sym,seed", [(23, True, 0), (70, False, 1), (130, True, 2), (191, False, 3)])
def test_orders_3_4_random_tables(oracle_mod, ivm, F, sym, seed):
    """Seeded random tables, symmetric and one-sided matrices, ragged F (padding
    words), an empty and a full snapshot: counts and lexicographic lists of
    orders 1-4 equal the oracle's enumeration; max_order 3 equals the first
    columns of max_order 4."""
    import torch
    _log(f"[orders 3-4 random] F={F} sym={sym} seed={seed}")
    rng = np.random.default_rng(100 + seed)
    N = 9
    dens = min(0.3, 10.0 / F)
    M = rng.random((F, F)) < dens
    if sym:
        M = M | M.T
    np.fill_diagonal(M, False)
    tv = rng.random((N, F)) < 0.15
    rv = rng.random((N, F)) < 0.15
    tv[0] = False                 # nothing visible from Tx
    tv[1] = True                  # everything visible from both sides
    rv[1] = True
    los = rng.random(N) < 0.5
    g = _plate_row_scene(ivm, F)
    dM, dtv, drv, dlos = _upload(ivm, M, tv, rv, los)
    # (the oracle enumerates the all-visible snapshot, |F| d^3 walks, on the small F only)
    rows = [n for n in range(N) if n != 1 or F < 100]
    for K in (3, 4):
        counts, off, paths = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, K, lists=True)
        torch.cuda.synchronize()
        co = oracle_mod.candidates_matmul(M, tv, rv, los, K)
        assert (counts.cpu().numpy() == co).all(), K
        sel = np.array(rows)
        ce, L = oracle_mod.candidates_enum(M, tv[sel], rv[sel], los[sel], K)
        assert (ce == co[sel]).all()
        off_np = off.cpu().numpy()
        paths_np = paths.cpu().numpy()
        for i, n in enumerate(rows):
            for k in range(1, K + 1):
                a, b = off_np[n * K + k - 1], off_np[n * K + k]
                got = [tuple(int(x) for x in paths_np[p:p + k]) for p in range(a, b, k)]
                assert got == L[i][k - 1], (n, k)
        if K == 3:
            c3 = counts.cpu().numpy()
        else:
            assert (counts.cpu().numpy()[:, :4] == c3).all()


@pytest.mark.parametrize("seed", [1, 2])
def test_orders_3_4_oracle_tables_c1(oracle_mod, ivm, seed):
    """The oracle's own matrix and tables of the tiny urban scene (42 facets, 10
    snapshots) as inputs: counts and lists of orders 1-4 equal the oracle's
    enumeration."""
    import torch
    _log(f"[orders 3-4 c1] seed={seed}")
    s = sg.gen_c1(seed)
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    tv, rv, los = orc.txrx(s.tx, s.rx)
    g = ivm.GpuScene.from_scene(s).check()
    dM, dtv, drv, dlos = _upload(ivm, M, tv, rv, los)
    counts, off, paths = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 4, lists=True)
    torch.cuda.synchronize()
    N = s.tx.shape[0]
    ce, L = oracle_mod.candidates_enum(M, tv, rv, los, 4)
    assert (counts.cpu().numpy() == ce).all()
    _check_lists(off, paths, L, N, 4)


def test_parallel_mirrors_end_to_end(oracle_mod, ivm):
    """Two parallel mirrors with Tx and Rx between them: exactly two walks of
    every order (the closed form the oracle is pinned to), from the GPU's own
    matrix, tables and candidates."""
    import torch
    s = sg.gen_plates([
        [[0, -40, -40], [0, 80, 0], [0, 0, 80]],
        [[10, -40, -40], [0, 0, 80], [0, 80, 0]],
    ], tx=[[3, -2, 1]], rx=[[6, 5, -1]])
    g = ivm.GpuScene.from_scene(s).check()
    M = ivm.ivm_intervisibility_matrix(g)
    tv, rv, los = ivm.ivm_txrx_visibility_table(g, torch.as_tensor(s.tx).cuda(), torch.as_tensor(s.rx).cuda())
    counts, off, paths = ivm.ivm_image_tree_candidates(g, M, tv, rv, los, 4, lists=True)
    torch.cuda.synchronize()
    assert g.status() == 0
    assert counts.cpu().numpy()[0].tolist() == [1, 2, 2, 2, 2]
    _check_lists(off, paths, [[[(0,), (1,)], [(0, 1), (1, 0)], [(0, 1, 0), (1, 0, 1)],
                               [(0, 1, 0, 1), (1, 0, 1, 0)]]], 1, 4)


def test_orders_3_4_full_size(oracle_mod, ivm):
    """Counts of orders 1-4 at full size: 2000 facets x 200 snapshots (the urban
    grid's size, a dense symmetric table) and 20000 facets x 12 snapshots (the
    large city's size: an LDS of 80 KB per block), against the oracle's integer
    products."""
    import torch
    import scipy.sparse as sps
    _log("[orders 3-4 full] F=2000 N=200")
    rng = np.random.default_rng(2000)
    F, N = 2000, 200
    M = rng.random((F, F)) < 0.02
    M = M | M.T
    np.fill_diagonal(M, False)
    tv = rng.random((N, F)) < 0.03
    rv = rng.random((N, F)) < 0.03
    los = rng.random(N) < 0.3
    g = _plate_row_scene(ivm, F)
    dM, dtv, drv, dlos = _upload(ivm, M, tv, rv, los)
    counts = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 4)
    torch.cuda.synchronize()
    assert (counts.cpu().numpy() == oracle_mod.candidates_matmul(M, tv, rv, los, 4)).all()

    _log("[orders 3-4 full] F=20000 N=12")
    F, N, deg = 20000, 12, 20
    rows = np.repeat(np.arange(F), deg)
    cols = rng.integers(0, F, F * deg)
    S = sps.coo_matrix((np.ones(F * deg, np.int8), (rows, cols)), shape=(F, F)).tocsr()
    S = ((S + S.T) > 0).tolil()
    S.setdiag(0)
    S = S.tocsr()
    S.eliminate_zeros()
    Md = S.toarray().astype(bool)
    tv = rng.random((N, F)) < 0.01
    rv = rng.random((N, F)) < 0.01
    los = rng.random(N) < 0.3
    g = _plate_row_scene(ivm, F)
    dM, dtv, drv, dlos = _upload(ivm, Md, tv, rv, los)
    del Md
    for K in (3, 4):
        counts = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, K)
        torch.cuda.synchronize()
        assert (counts.cpu().numpy() == oracle_mod.candidates_matmul(S, tv, rv, los, K)).all(), K


def _pack_sparse(ivm, S, F):
    """Bit rows of a scipy sparse 0/1 matrix without a dense copy."""
    import scipy.sparse as sps
    C = sps.coo_matrix(S)
    W = (F + 63) // 64
    words = np.zeros((F, W), np.uint64)
    np.bitwise_or.at(words, (C.row, C.col >> 6), np.left_shift(np.uint64(1), (C.col & 63).astype(np.uint64)))
    return words.view(np.int64)


@pytest.mark.parametrize("F,N,seed", [(130, 2100, 4), (64, 1100, 5), (257, 2117, 6)])
def test_orders_3_4_many_slabs(oracle_mod, ivm, F, N, seed):
    """More snapshots than one slab of the products holds (small scenes keep a
    slab of 1024 snapshots): several slabs and a ragged last one, F on and off a
    word boundary; a second call and a call after a matrix call (which reuses
    the same scratch) return the same counts."""
    import torch
    _log(f"[orders 3-4 slabs] F={F} N={N} seed={seed}")
    rng = np.random.default_rng(300 + seed)
    M = rng.random((F, F)) < 0.1
    np.fill_diagonal(M, False)
    tv = rng.random((N, F)) < 0.2
    rv = rng.random((N, F)) < 0.2
    tv[N - 1] = True
    rv[N - 1] = True
    los = rng.random(N) < 0.5
    g = _plate_row_scene(ivm, F)
    dM, dtv, drv, dlos = _upload(ivm, M, tv, rv, los)
    co = oracle_mod.candidates_matmul(M, tv, rv, los, 4)
    c1 = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 4)
    c3 = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 3)
    torch.cuda.synchronize()
    assert (c1.cpu().numpy() == co).all()
    assert (c3.cpu().numpy() == co[:, :4]).all()
    ivm.ivm_intervisibility_matrix(g)
    c2 = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 4)
    torch.cuda.synchronize()
    assert (c2.cpu().numpy() == co).all()


def test_orders_3_4_large_walk_counts(oracle_mod, ivm):
    """Dense rows: u above 255 (both byte planes of the products carry) at
    F = 1000, and u above 32767 at F = 33000 (a facet every facet sees, Tx
    seeing all): counts against the oracle's integer products."""
    import torch
    import scipy.sparse as sps
    _log("[orders 3-4 large u] F=1000")
    rng = np.random.default_rng(4000)
    F, N = 1000, 70
    M = rng.random((F, F)) < 0.5
    np.fill_diagonal(M, False)
    tv = rng.random((N, F)) < 0.7
    rv = rng.random((N, F)) < 0.7
    tv[:5] = True
    los = rng.random(N) < 0.5
    g = _plate_row_scene(ivm, F)
    dM, dtv, drv, dlos = _upload(ivm, M, tv, rv, los)
    co = oracle_mod.candidates_matmul(M, tv, rv, los, 4)
    assert (co[:, :4] >= 0).all() and co[:5, 4].min() > 2 ** 32
    c = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 4)
    torch.cuda.synchronize()
    assert (c.cpu().numpy() == co).all()

    _log("[orders 3-4 large u] F=33000")
    F, N, deg, hub = 33000, 6, 3, 12345
    rows = np.concatenate([np.repeat(np.arange(F), deg), np.arange(F), np.full(40, hub)])
    cols = np.concatenate([rng.integers(0, F, F * deg), np.full(F, hub), rng.integers(0, F, 40)])
    S = sps.coo_matrix((np.ones(len(rows), np.int8), (rows, cols)), shape=(F, F)).tocsr()
    S = (S > 0).tolil()
    S.setdiag(0)
    S = S.tocsr().astype(np.int8)
    S.eliminate_zeros()
    tv = rng.random((N, F)) < 0.02
    rv = rng.random((N, F)) < 0.02
    tv[0] = True
    rv[0, hub] = True
    los = np.zeros(N, bool)
    g = _plate_row_scene(ivm, F)
    dM = torch.as_tensor(_pack_sparse(ivm, S, F)).cuda()
    dtv, drv = torch.as_tensor(ivm.pack_bits(tv)).cuda(), torch.as_tensor(ivm.pack_bits(rv)).cuda()
    dlos = torch.as_tensor(los.astype(np.uint8)).cuda()
    co = oracle_mod.candidates_matmul(S, tv, rv, los, 4)
    c = ivm.ivm_image_tree_candidates(g, dM, dtv, drv, dlos, 4)
    torch.cuda.synchronize()
    assert (c.cpu().numpy() == co).all()


def test_order_above_4_rejected(ivm):
    import torch
    g = _plate_row_scene(ivm, 10)
    lib = ivm.load_library()
    z = torch.zeros((10, 1), dtype=torch.int64, device="cuda")
    los = torch.zeros(1, dtype=torch.uint8, device="cuda")
    counts = torch.zeros((1, 6), dtype=torch.int64, device="cuda")
    st = lib.ivm_image_tree_candidates(g.handle, z.data_ptr(), 1, z.data_ptr(), z.data_ptr(), los.data_ptr(), 5,
                                       counts.data_ptr(), None, None, 0, None)
    assert st == ivm.IVM_ERR_INVALID_ARGUMENT
