"""GPU checks of the learned occluder ordering: features, hit-record labels,
network forward and gradients (FP32 and BF16-MFMA modes) against the FP64
oracle, Adam, training progress, and that the learned order never changes a
result bit."""
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


def _pairs(F, n, seed):
    rng = np.random.default_rng(seed)
    I = rng.integers(0, F, n)
    J = rng.integers(0, F, n)
    keep = I != J
    return np.minimum(I, J)[keep].astype(np.int32), np.maximum(I, J)[keep].astype(np.int32)


def test_features_match_oracle(oracle_mod, ivm):
    import torch
    for s in (sg.gen_c1(3), sg.gen_c2(4, n_snap=1, nx=4, ny=4)):
        _log(f"[features] F={s.n_facets}")
        g = ivm.GpuScene.from_scene(s).check()
        I, J = _pairs(s.n_facets, 500, 1)
        x = ivm.ivm_pair_features(g, torch.as_tensor(I).cuda(), torch.as_tensor(J).cuda()).cpu().numpy()
        xo = oracle_mod.pair_features(s, I, J)
        assert np.abs(x - xo).max() < 2e-5


def test_labels_match_oracle(oracle_mod, ivm):
    """Hit records are integer: bit-exact against the oracle's all-hit search."""
    import torch
    for s, n in ((sg.gen_c1(5), 861), (sg.gen_c2(6, n_snap=1, nx=4, ny=3), 300)):
        _log(f"[labels] F={s.n_facets}")
        g = ivm.GpuScene.from_scene(s).check()
        if n == 861:
            I, J = np.triu_indices(s.n_facets, 1)
            I, J = I.astype(np.int32), J.astype(np.int32)
        else:
            I, J = _pairs(s.n_facets, n, 2)
        lab = ivm.ivm_pair_occluder_labels(g, torch.as_tensor(I).cuda(), torch.as_tensor(J).cuda())
        lab = lab.cpu().numpy().view(np.uint32)
        _, groups = oracle_mod.morton_treelets(s, 32)
        expect = oracle_mod.Oracle(s).occluder_groups(I, J, groups)
        assert (lab == expect).all(), np.argwhere(lab != expect)[:5]
        assert (lab != 0).sum() > 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_forward_and_gradients_match_oracle(oracle_mod, ivm, precision):
    """FP32 mode against the FP64 reference; BF16 (MFMA) mode against the FP64
    reference with every product's operands rounded to BF16."""
    import torch
    _log(f"[mlp] {precision}")
    bf16 = precision == "bf16"
    rng = np.random.default_rng(3)
    p = oracle_mod.mlp_init(7)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    flat = oracle_mod.mlp_flatten(p).astype(np.float32)
    pf = oracle_mod.mlp_unflatten(flat.astype(np.float64))       # the FP32-stored parameters
    B = 200
    X = rng.normal(size=(B, 24)).astype(np.float32)
    Y = (rng.random((B, 32)) < 0.3).astype(np.float32)
    m = ivm.Model(max_batch=256, precision=ivm.IVM_MODEL_BF16 if bf16 else ivm.IVM_MODEL_FP32)
    m.set_params(flat)
    dX, dY = torch.as_tensor(X).cuda(), torch.as_tensor(Y).cuda()
    z = m.forward(dX).cpu().numpy()
    zo, _ = oracle_mod.mlp_forward(pf, X.astype(np.float64), bf16=bf16)
    tol = 2e-3 if bf16 else 1e-5
    assert np.abs(z - zo).max() <= tol * max(1.0, np.abs(zo).max())
    loss, grad = m.loss_grad(dX, dY)
    lo, go = oracle_mod.mlp_loss_grad(pf, X.astype(np.float64), Y.astype(np.float64), bf16=bf16)
    assert abs(float(loss.item()) - lo) <= (1e-3 if bf16 else 1e-5) * max(1.0, lo)
    g_gpu = grad.cpu().numpy().astype(np.float64)
    g_ref = oracle_mod.mlp_flatten(go)
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    assert rel <= (1e-2 if bf16 else 1e-4), rel
    # per layer as well, and element by element: |g - g_ref| <= rtol |g_ref| + atol rms(layer).
    # FP32 mode differs from the FP64 reference only in summation order (n terms of FP32
    # products: about n 2^-24 of the summed magnitudes), so rtol 1e-4 with a floor of 1e-4 of
    # the layer's rms.  BF16 mode rounds the same operands to BF16 on both sides, but an
    # activation that differs in its last FP32 bit can round to the neighbouring BF16 value
    # (a 2^-8 relative step) and move its terms by that much: rtol 5e-2 with a floor of 5e-2
    # of the layer's rms (elements far below the rms come from cancellation).
    rtol, afl = (5e-2, 5e-2) if bf16 else (1e-4, 1e-4)
    off = 0
    worst = 0.0
    for l in range(4):
        for key in (f"W{l}", f"b{l}"):
            n = go[key].size
            seg_g, seg_r = g_gpu[off:off + n], g_ref[off:off + n]
            assert np.linalg.norm(seg_g - seg_r) <= (2e-2 if bf16 else 2e-4) * np.linalg.norm(seg_r) + 1e-9, key
            rms = float(np.sqrt(np.mean(seg_r ** 2))) + 1e-30
            bound = rtol * np.abs(seg_r) + afl * rms
            ratio = np.abs(seg_g - seg_r) / bound
            worst = max(worst, float(ratio.max()))
            assert (ratio <= 1.0).all(), (key, int((ratio > 1).sum()), float(ratio.max()))
            off += n
    _log(f"[mlp] {precision}: largest element error / bound = {worst:.3f}")


def test_adam_step_matches_oracle(oracle_mod, ivm):
    import torch
    rng = np.random.default_rng(4)
    p = oracle_mod.mlp_init(1)
    flat = oracle_mod.mlp_flatten(p).astype(np.float32)
    X = rng.normal(size=(64, 24)).astype(np.float32)
    Y = (rng.random((64, 32)) < 0.3).astype(np.float32)
    m = ivm.Model(max_batch=64, precision=ivm.IVM_MODEL_FP32)
    m.set_params(flat)
    dX, dY = torch.as_tensor(X).cuda(), torch.as_tensor(Y).cuda()
    pf = oracle_mod.mlp_unflatten(flat.astype(np.float64))
    st = {}
    for _ in range(3):
        _, go = oracle_mod.mlp_loss_grad(pf, X.astype(np.float64), Y.astype(np.float64))
        oracle_mod.adam_step(pf, go, st, lr=1e-3)
        m.train_step(dX, dY, 1e-3)
    got = m.get_params().cpu().numpy().astype(np.float64)
    ref = oracle_mod.mlp_flatten(pf)
    assert np.abs(got - ref).max() < 1e-5


def test_training_reduces_loss(ivm):
    """Records from the GPU's own hit-record pass; BF16 training lowers the loss."""
    from paper_2501_02747_amd import train as tr
    s = sg.gen_c2(201, n_snap=1, nx=5, ny=5)
    X, Y = tr.collect_records(s, 20000, 0)
    assert len(X) > 1000
    m = ivm.Model(max_batch=1024, precision=ivm.IVM_MODEL_BF16)
    m.set_params(tr.he_uniform_init(0))
    hist = tr.train(m, X, Y, epochs=4, batch=256, lr=2e-3)
    _log(f"[train] losses {hist}")
    assert hist[-1] < hist[0]


@pytest.mark.parametrize("weights", ["trained", "random", "nan"])
def test_learned_order_keeps_every_bit(oracle_mod, ivm, weights):
    """IVM_ORDER_LEARNED with any weights (trained, random, NaN) gives the plain bits."""
    import torch
    from paper_2501_02747_amd import train as tr
    s = sg.gen_c2(2, n_snap=4, nx=5, ny=4)
    g = ivm.GpuScene.from_scene(s, learned=True).check()
    m = ivm.Model(max_batch=1024, precision=ivm.IVM_MODEL_BF16)
    params = tr.he_uniform_init(5)
    if weights == "trained":
        X, Y = tr.collect_records(s, 20000, 1)
        m.set_params(params)
        tr.train(m, X, Y, epochs=2, batch=256, lr=2e-3)
    elif weights == "nan":
        params = np.full_like(params, np.nan)
        m.set_params(params)
    else:
        m.set_params(params)
    ivm.ivm_scene_set_model(g, m)
    st_l, st_p = ivm.new_stats(), ivm.new_stats()
    Ml = ivm.ivm_intervisibility_matrix(g, ivm.make_opts(order_mode=ivm.IVM_ORDER_LEARNED), stats=st_l).clone()
    Mp = ivm.ivm_intervisibility_matrix(g, ivm.make_opts(order_mode=ivm.IVM_ORDER_PLAIN), stats=st_p).clone()
    torch.cuda.synchronize()
    assert torch.equal(Ml, Mp)
    Mo, _ = oracle_mod.Oracle(s).matrix()
    assert (ivm.unpack_bits(Ml, s.n_facets) == Mo).all()
    dl, dp = ivm.stats_dict(st_l), ivm.stats_dict(st_p)
    assert dl["flags"] == 0
    _log(f"[learned {weights}] box tests {dl['box_tests']} vs plain {dp['box_tests']}, "
         f"tests {dl['tri_tests']} vs {dp['tri_tests']}")


def test_learned_without_model_falls_back(ivm):
    import torch
    s = sg.gen_c1(2)
    g = ivm.GpuScene.from_scene(s).check()
    st = ivm.new_stats()
    M = ivm.ivm_intervisibility_matrix(g, ivm.make_opts(order_mode=ivm.IVM_ORDER_LEARNED), stats=st,
                                       allow_model_fallback=True)
    Mp = ivm.ivm_intervisibility_matrix(g)
    torch.cuda.synchronize()
    assert torch.equal(M, Mp)
    assert ivm.stats_dict(st)["flags"] & 1


def test_trained_network_gain_on_held_out_urban_grid(oracle_mod, ivm):
    """What the shipped network (trained on urban-grid seeds 200-209) gains on the
    held-out urban grid (seed 2, the benchmark scene): identical bits in every
    order, fewer box tests than the plain order (nearest treelet first), than a
    random-weight network and than Morton index order, and a ranking of the
    treelets that finds a blocking treelet first far more often than chance.
    Times of plain and learned calls are reported (the learned call includes
    the network's inference), not asserted."""
    import os
    import statistics
    import torch
    from paper_2501_02747_amd import train as tr
    cache = os.path.join(os.path.dirname(__file__), "golden", "cache", "c2_seed2.npz")
    if not os.path.exists(cache):
        pytest.skip("full oracle cache not generated")
    s = sg.gen_c2(2, n_snap=1)
    F = s.n_facets
    z = np.load(cache, allow_pickle=False)
    Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
    g = ivm.GpuScene.from_scene(s, learned=True).check()
    trained = ivm.Model(max_batch=1024, precision=ivm.IVM_MODEL_BF16)
    trained.set_params(np.load(tr.DEFAULT_WEIGHTS, allow_pickle=False))
    rand = ivm.Model(max_batch=1024, precision=ivm.IVM_MODEL_BF16)
    rand.set_params(tr.he_uniform_init(11))

    def run(order, model=None):
        ivm.ivm_scene_set_model(g, model)
        st = ivm.new_stats()
        times = []
        for k in range(4):
            st.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            M = ivm.ivm_intervisibility_matrix(g, ivm.make_opts(order_mode=order), stats=st)
            e1.record()
            torch.cuda.synchronize()
            if k:
                times.append(e0.elapsed_time(e1))
        assert (ivm.unpack_bits(M, F) == Mo).all(), order
        d = ivm.stats_dict(st)
        return d["box_tests"], d["tri_tests"], statistics.median(times)

    res = {"plain": run(ivm.IVM_ORDER_PLAIN), "index": run(ivm.IVM_ORDER_INDEX),
           "learned": run(ivm.IVM_ORDER_LEARNED, trained), "random-weights": run(ivm.IVM_ORDER_LEARNED, rand)}
    ivm.ivm_scene_set_model(g, None)
    for k, (b, t, ms) in res.items():
        _log(f"[gain] {k:15s} box tests {b:12d}  triangle tests {t:11d}  matrix {ms:7.3f} ms")
    lb = res["learned"][0]
    assert lb < 0.98 * res["plain"][0]
    assert lb < res["random-weights"][0] and lb < res["index"][0]
    # ranking quality on held-out hit records: the top-scored treelet holds a
    # blocker (all-hit labels, pinned against the oracle) for how many pairs
    rng = np.random.default_rng(21)
    I, J = rng.integers(0, F, 60000), rng.integers(0, F, 60000)
    keep = I != J
    I, J = np.minimum(I, J)[keep].astype(np.int32), np.maximum(I, J)[keep].astype(np.int32)
    dI, dJ = torch.as_tensor(I).cuda(), torch.as_tensor(J).cuda()
    lab = ivm.ivm_pair_occluder_labels(g, dI, dJ).cpu().numpy().view(np.uint32)
    hit = lab != 0
    X = ivm.ivm_pair_features(g, dI[torch.as_tensor(hit).cuda()], dJ[torch.as_tensor(hit).cuda()])
    lab = lab[hit]
    bits = (lab[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1

    def p_at_1(model):
        out = []
        for c0 in range(0, X.shape[0], 1024):
            out.append(model.forward(X[c0:c0 + 1024]).cpu().numpy())
        sc = np.nan_to_num(np.concatenate(out), nan=-np.inf)
        top = np.argmax(sc, 1)
        return float(bits[np.arange(len(top)), top].mean())

    p_tr, p_rand = p_at_1(trained), p_at_1(rand)
    chance = float(bits.mean())
    _log(f"[gain] {len(lab)} held-out hit records: top treelet holds a blocker for {p_tr:.3f} (trained), "
         f"{p_rand:.3f} (random weights), {chance:.3f} (a random treelet)")
    assert p_tr > p_rand + 0.2 and p_tr > 2 * chance
