"""Visibility ranges and coherence times on the GPU (ivm_visibility_ranges)
against the oracle, on tables that come from the oracle or from a seeded
generator: creation / suppression counts and range starts bit-exact, FP64
distances and times within 1e-12 relative (both sides sum the same steps in the
same order; only the square root's last bit may differ)."""
import math
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


def _pack(bits, W):
    """bool [N, F] -> uint64 [N, W], column 64 w + j in bit j of word w."""
    N, F = bits.shape
    b = np.packbits(np.asarray(bits, np.uint8), axis=1, bitorder="little")
    out = np.zeros((N, W * 8), np.uint8)
    out[:, :b.shape[1]] = b
    return out.view(np.uint64)


def _compare(oracle_mod, ivm, g, tv, rv, los, tx, rx, dt):
    import torch
    W = g.W
    d = lambda a: torch.as_tensor(a).cuda()
    ev, st, tc, dist, mean = ivm.ivm_visibility_ranges(
        g, d(_pack(tv, W).view(np.int64)), d(_pack(rv, W).view(np.int64)), d(np.asarray(los, np.uint8)),
        d(np.asarray(tx, np.float32)), d(np.asarray(rx, np.float32)), dt)
    torch.cuda.synchronize()
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, dt)
    assert (ev.cpu().numpy() == r["events"]).all()
    assert st.cpu().numpy().tolist() == r["starts"].tolist()
    gtc, otc = tc.cpu().numpy(), r["tc"]
    assert (np.isinf(gtc) == np.isinf(otc)).all()
    fin = ~np.isinf(otc)
    np.testing.assert_allclose(gtc[fin], otc[fin], rtol=1e-12, atol=0)
    np.testing.assert_allclose(dist.cpu().numpy(), r["dist"], rtol=1e-12, atol=0)
    if math.isinf(r["mean"]):
        assert math.isinf(mean)
    else:
        assert mean == pytest.approx(r["mean"], rel=1e-12)
    exact = np.array_equal(gtc[fin], otc[fin]) and np.array_equal(dist.cpu().numpy(), r["dist"])
    _log(f"[ranges] N={len(tv)} L={len(r['starts'])} FP64 outputs bit-identical: {exact}")
    return r


def _scene(ivm, F):
    """Any built scene with F facets gives the row width W the call reads."""
    s = sg.gen_c4_scene(1001, f_target=F, n_snap=4) if F > 64 else sg.gen_c1(1)
    return ivm.GpuScene.from_scene(s).check(), s.n_facets


@pytest.mark.parametrize("N,p_flip,moving", [(1, 0.0, "both"), (2, 0.5, "rx"), (57, 0.02, "both"),
                                             (700, 0.002, "rx"), (300, 0.0, "none"), (400, 0.3, "tx")])
def test_seeded_tables(oracle_mod, ivm, N, p_flip, moving):
    _log(f"[ranges] seeded N={N} flip={p_flip} moving={moving}")
    g, F = _scene(ivm, 600)
    rng = np.random.default_rng(N)
    tv = np.zeros((N, F), bool)
    rv = np.zeros((N, F), bool)
    tv[0] = rng.random(F) < 0.1
    rv[0] = rng.random(F) < 0.1
    los = np.zeros(N, bool)
    los[0] = True
    for n in range(1, N):  # sparse flips, some snapshots unchanged
        tv[n] = tv[n - 1] ^ (rng.random(F) < p_flip * 0.01)
        rv[n] = rv[n - 1] ^ (rng.random(F) < p_flip * 0.01)
        los[n] = los[n - 1] ^ (rng.random() < p_flip * 0.1)
    step = rng.normal(0, 1.0, (N, 3)).astype(np.float32) * np.float32(0.25)
    tx = np.cumsum(step, 0).astype(np.float32) if moving in ("both", "tx") else np.tile(np.float32([5, 5, 30]), (N, 1))
    rx = np.cumsum(step[::-1], 0).astype(np.float32) if moving in ("both", "rx") else np.zeros((N, 3), np.float32)
    _compare(oracle_mod, ivm, g, tv, rv, los, tx, rx, 0.01)


def test_change_at_the_last_snapshot(oracle_mod, ivm):
    g, F = _scene(ivm, 40)
    N = 12
    tv = np.zeros((N, F), bool)
    rv = np.zeros((N, F), bool)
    rv[N - 1, 3] = True
    tx = np.zeros((N, 3), np.float32)
    rx = np.zeros((N, 3), np.float32)
    rx[:, 1] = np.arange(N, dtype=np.float32)
    r = _compare(oracle_mod, ivm, g, tv, rv, np.zeros(N, bool), tx, rx, 0.02)
    assert r["starts"].tolist() == [0, N - 1]


def test_oracle_tables_of_tiny_urban_scenes(oracle_mod, ivm):
    """Tables computed by the oracle for c1 scenes (10 snapshots each)."""
    for seed in (1, 2, 3):
        _log(f"[ranges] tiny urban seed={seed}")
        s = sg.gen_c1(seed)
        g = ivm.GpuScene.from_scene(s).check()
        tvo, rvo, loso = oracle_mod.Oracle(s).txrx(s.tx, s.rx)
        _compare(oracle_mod, ivm, g, tvo, rvo, loso, s.tx, s.rx, 0.01)


@pytest.mark.skipif(not os.path.exists(CACHE), reason="full oracle cache not generated")
def test_urban_grid_trajectory(oracle_mod, ivm):
    """The urban-grid trajectory (1000 snapshots 10 ms apart) with the tables
    of the stored full oracle result."""
    _log("[ranges] urban grid from the oracle cache")
    s = sg.gen_c2(2)
    z = np.load(CACHE, allow_pickle=False)
    F = s.n_facets
    tvo = np.unpackbits(z["tx_vis"], axis=1)[:, :F].astype(bool)
    rvo = np.unpackbits(z["rx_vis"], axis=1)[:, :F].astype(bool)
    g = ivm.GpuScene.from_scene(s).check()
    r = _compare(oracle_mod, ivm, g, tvo, rvo, z["los"], s.tx, s.rx, 0.01)
    assert len(r["starts"]) > 1
