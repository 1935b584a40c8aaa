"""Pins for the image-tree candidates, the Morton partition and the MLP reference (CPU only)."""
import numpy as np
import pytest
import torch

import scenegen as sg


# ---- candidates: Section III-B (Table II) and Section III-C --------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_enum_equals_matmul_random(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    F, N, K = 23, 7, 4
    M = rng.random((F, F)) < 0.3
    M = M | M.T
    np.fill_diagonal(M, False)
    tv = rng.random((N, F)) < 0.4
    rv = rng.random((N, F)) < 0.4
    los = rng.random(N) < 0.5
    c_enum, lists = oracle_mod.candidates_enum(M, tv, rv, los, K)
    c_mm = oracle_mod.candidates_matmul(M, tv, rv, los, K)
    assert (c_enum == c_mm).all()
    for n in range(N):
        for k in range(K):
            assert len(lists[n][k]) == c_enum[n, k + 1]
            assert lists[n][k] == sorted(lists[n][k])
            for w in lists[n][k]:
                assert tv[n, w[0]] and rv[n, w[-1]]
                assert all(M[w[m], w[m + 1]] for m in range(k))


@pytest.mark.parametrize("seed", [3, 4])
def test_enum_equals_matmul_one_sided(oracle_mod, seed):
    """Walks follow M[f_m][f_m+1] as given: a matrix that is not symmetric (a
    directed cycle 0 -> 1 -> 2 -> 0 among random rows) gives the same counts by
    enumeration and by products, dense and sparse; on the bare cycle with every
    facet visible from both sides there are exactly F walks of every order."""
    import scipy.sparse as sps
    rng = np.random.default_rng(seed)
    F, N, K = 19, 6, 4
    M = rng.random((F, F)) < 0.2
    np.fill_diagonal(M, False)
    assert (M != M.T).any()
    tv = rng.random((N, F)) < 0.4
    rv = rng.random((N, F)) < 0.4
    los = rng.random(N) < 0.5
    c_enum, _ = oracle_mod.candidates_enum(M, tv, rv, los, K)
    assert (c_enum == oracle_mod.candidates_matmul(M, tv, rv, los, K)).all()
    assert (c_enum == oracle_mod.candidates_matmul(sps.csr_matrix(M), tv, rv, los, K)).all()
    C = np.zeros((3, 3), bool)
    C[0, 1] = C[1, 2] = C[2, 0] = True
    one = np.ones((1, 3), bool)
    counts, lists = oracle_mod.candidates_enum(C, one, one, np.zeros(1, bool), K)
    assert counts[0].tolist() == [0, 3, 3, 3, 3]
    assert lists[0][2] == [(0, 1, 2), (1, 2, 0), (2, 0, 1)]


def _parallel_plates():
    # two large plates facing each other across x in [0, 10]; Tx and Rx between them
    return sg.gen_plates([
        [[0, -40, -40], [0, 80, 0], [0, 0, 80]],     # x = 0 facing +x
        [[10, -40, -40], [0, 0, 80], [0, 80, 0]],    # x = 10 facing -x
    ], tx=[[3, -2, 1]], rx=[[6, 5, -1]])


def test_parallel_plates_two_paths_per_order(oracle_mod):
    """Between two parallel mirrors there are exactly two specular paths of every
    order (they start on one mirror or the other), and the walks count two."""
    s = _parallel_plates()
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    tv, rv, los = orc.txrx(s.tx, s.rx)
    assert M[0, 1] and M[1, 0]
    assert tv.all() and rv.all() and los.all()
    K = 4
    counts = oracle_mod.candidates_matmul(M, tv, rv, los, K)
    assert counts[0].tolist() == [1, 2, 2, 2, 2]
    paths = oracle_mod.image_paths(s, orc, s.tx[0], s.rx[0], K)
    for k in range(1, K + 1):
        assert len([p for p in paths if len(p) == k]) == 2


def test_corner_reflector(oracle_mod):
    """A concave 90-degree corner (a wedge has 2 first-order images and one
    double image, shared by both reflection orders): two first-order paths, one
    second-order path (the line from the double image to Rx crosses only one of
    the two plates first: here y=0 at x=9.25, while it meets x=0 at y=-7.8,
    off the plate), none of third order.  The candidate walks keep both orders
    (A->B and B->A are mutually visible), so every valid path is a candidate."""
    s = sg.gen_plates([
        [[0, 0, -20], [0, 40, 0], [0, 0, 40]],       # x = 0 facing +x (y cross z)
        [[0, 0, -20], [0, 0, 40], [40, 0, 0]],       # y = 0 facing +y (z cross x)
    ], tx=[[5, 12, 1]], rx=[[14, 4, 0.5]])
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    tv, rv, los = orc.txrx(s.tx, s.rx)
    counts, lists = oracle_mod.candidates_enum(M, tv, rv, los, 3)
    paths = oracle_mod.image_paths(s, orc, s.tx[0], s.rx[0], 3)
    by_order = [[p for p in paths if len(p) == k] for k in (1, 2, 3)]
    assert [len(x) for x in by_order] == [2, 1, 0]
    assert by_order[1] == [(0, 1)]
    assert counts[0, 1] == 2 and counts[0, 2] == 2
    for k in (1, 2):
        assert set(by_order[k - 1]) <= set(lists[0][k - 1])


def test_pruning_recall_c1(oracle_mod):
    """Case study 2's claim (Section IV-B): the pruned image tree finds the same
    valid rays as brute force.  Every exact image-method path up to order 2 that
    starts and ends on sample-visible facets must be among the candidates; and
    the candidates prune the F^k brute-force sequences."""
    s = sg.gen_c1(1, n_snap=3)
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    tv, rv, los = orc.txrx(s.tx, s.rx)
    counts, lists = oracle_mod.candidates_enum(M, tv, rv, los, 2)
    total, found = 0, 0
    for n in range(3):
        paths = oracle_mod.image_paths(s, orc, s.tx[n], s.rx[n], 2)
        for p in paths:
            total += 1
            found += p in set(lists[n][len(p) - 1])
        F = s.n_facets
        assert counts[n, 2] < F * (F - 1)
    assert total > 0
    # sampling can miss a sliver of visibility (documented reading); require high recall
    assert found / total >= 0.9


# ---- Morton partition ---------------------------------------------------------

def test_morton_partition_by_hand(oracle_mod):
    """Four tiny triangles at the corners of the scene box: codes are all-zeros
    for the low corner and all-ones for the high corner; the x bit is the most
    significant of each triple."""
    def tri(x, y, z):
        return [[x, y, z], [0.0625, 0, 0], [0, 0.0625, 0]]
    s = sg.gen_plates([tri(0, 0, 0), tri(100, 0, 0), tri(0, 100, 0), tri(0, 0, 100),
                       tri(100, 100, 100)], g=4, n=4)
    order, group = oracle_mod.morton_treelets(s, n_groups=32)
    # each plate is two triangles; plate m has triangles 2m, 2m+1.  Expected order
    # by code: low corner (0) < z (0b001..) < y (0b010..) < x (0b100..) < all.
    plates_in_order = [int(t) // 2 for t in order[::2]]
    assert plates_in_order == [0, 3, 2, 1, 4]


def test_morton_groups_equal_count(oracle_mod):
    s = sg.gen_c1(1)
    order, group = oracle_mod.morton_treelets(s, 32)
    T = s.n_triangles
    sizes = np.bincount(group, minlength=32)
    assert sizes.sum() == T and sizes.max() - sizes.min() <= 1
    assert sorted(order.tolist()) == list(range(T))
    ranks = np.empty(T, np.int64)
    ranks[order] = np.arange(T)
    assert (group == (ranks * 32) // T).all()


# ---- MLP reference -------------------------------------------------------------

def test_mlp_param_count(oracle_mod):
    p = oracle_mod.mlp_init(0)
    assert sum(v.size for v in p.values()) == 40352


def test_mlp_fd_gradients(oracle_mod):
    rng = np.random.default_rng(1)
    p = oracle_mod.mlp_init(1, sizes=(24, 16, 16, 16, 32))
    X = rng.normal(size=(8, 24))
    Y = (rng.random((8, 32)) < 0.3).astype(np.float64)
    assert oracle_mod.mlp_fd_check(p, X, Y, n_probe=64) < 1e-6


def test_mlp_matches_torch_autograd(oracle_mod):
    """Forward, loss and every gradient against PyTorch's float64 autograd
    (an independent implementation of the same textbook operations)."""
    rng = np.random.default_rng(2)
    p = oracle_mod.mlp_init(2)
    X = rng.normal(size=(32, 24))
    Y = (rng.random((32, 32)) < 0.25).astype(np.float64)
    loss, g = oracle_mod.mlp_loss_grad(p, X, Y)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    h = torch.tensor(X)
    for l in range(4):
        h = h @ tp[f"W{l}"].T + tp[f"b{l}"]
        if l < 3:
            h = torch.relu(h)
    tl = torch.nn.functional.binary_cross_entropy_with_logits(h, torch.tensor(Y))
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12
    for k in p:
        assert np.allclose(tp[k].grad.numpy(), g[k], rtol=1e-10, atol=1e-14), k


def test_bce_and_adam_closed_forms(oracle_mod):
    assert abs(oracle_mod.bce_with_logits(np.zeros(4), np.ones(4)) - np.log(2)) < 1e-15
    assert oracle_mod.bce_with_logits(np.array([40.0]), np.array([1.0])) < 1e-15
    # first Adam step moves every weight by lr * sign(g) (bias-corrected m/sqrt(v) = g/|g|)
    p = {"W0": np.array([1.0, -2.0, 3.0])}
    g = {"W0": np.array([0.5, -4.0, 1e-3])}
    st = {}
    oracle_mod.adam_step(p, g, st, lr=0.01, eps=0.0)
    assert np.allclose(p["W0"], [0.99, -1.99, 2.99], atol=1e-12)


def test_exact_image_paths_closed_forms(oracle_mod):
    """The exact validator on the closed forms: two parallel mirrors give two
    paths of every order; the 90-degree corner gives 2, 1 and 0 paths of orders
    1-3 (the second-order one is 0 -> 1); the FP64 validator agrees."""
    s = _parallel_plates()
    orc = oracle_mod.Oracle(s)
    ex = oracle_mod.image_paths_exact(s, s.tx[0], s.rx[0], 4)
    assert [len([p for p in ex if len(p) == k]) for k in (1, 2, 3, 4)] == [2, 2, 2, 2]
    assert ex == oracle_mod.image_paths(s, orc, s.tx[0], s.rx[0], 4)
    s = sg.gen_plates([
        [[0, 0, -20], [0, 40, 0], [0, 0, 40]],
        [[0, 0, -20], [0, 0, 40], [40, 0, 0]],
    ], tx=[[5, 12, 1]], rx=[[14, 4, 0.5]])
    ex = oracle_mod.image_paths_exact(s, s.tx[0], s.rx[0], 3)
    assert [len([p for p in ex if len(p) == k]) for k in (1, 2, 3)] == [2, 1, 0]
    assert (0, 1) in ex


def test_exact_image_paths_closed_facet_boundary(oracle_mod):
    """Tx (5, -3, 1) and Rx (5, 3, 1) in front of the mirror x = 0: the specular
    point is (0, 0, 1).  A plate with its edge on y = 0 contains it (facets are
    closed), one that starts a grid step further (y = 1/16) does not."""
    for y0, expect in ((0.0, [(0,)]), (1.0 / 16, [])):
        s = sg.gen_plates([[[0, y0, -20], [0, 40, 0], [0, 0, 40]]], tx=[[5, -3, 1]], rx=[[5, 3, 1]])  # faces +x
        assert oracle_mod.image_paths_exact(s, s.tx[0], s.rx[0], 1) == expect, y0


@pytest.mark.parametrize("seed", [1, 2])
def test_exact_paths_recall_c1(oracle_mod, seed):
    """Case study 2's claim in exact arithmetic (Section IV-B): every exact
    image-method path of order <= 2 whose first and last facets are sample-visible
    is among the pruned candidates; the FP64 validator finds the same paths."""
    s = sg.gen_c1(seed, n_snap=3)
    orc = oracle_mod.Oracle(s)
    M, _ = orc.matrix()
    tv, rv, los = orc.txrx(s.tx, s.rx)
    _, lists = oracle_mod.candidates_enum(M, tv, rv, los, 2)
    for n in range(3):
        ex = oracle_mod.image_paths_exact(s, s.tx[n], s.rx[n], 2)
        assert ex == oracle_mod.image_paths(s, orc, s.tx[n], s.rx[n], 2)
        for p in ex:
            if tv[n, p[0]] and rv[n, p[-1]]:
                assert p in set(lists[n][len(p) - 1]), (n, p)
