"""The allocation-free ranges call (ivm_visibility_ranges_noalloc) against the
workspace call it mirrors (ivm_visibility_ranges) and the oracle: two calls in
a row on one GPU, the second on a shorter trajectory, so the second runs over
the scratch the first left behind.  Counts and range starts bit-exact, FP64
distances and times identical to the workspace call (same kernels, same
order) and within 1e-12 relative of the oracle."""
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pack(bits, W):
    N, F = bits.shape
    b = np.packbits(np.asarray(bits, np.uint8), axis=1, bitorder="little")
    out = np.zeros((N, W * 8), np.uint8)
    out[:, :b.shape[1]] = b
    return out.view(np.uint64)


def _tables(F, N, seed):
    rng = np.random.default_rng(seed)
    tv = np.zeros((N, F), bool)
    rv = np.zeros((N, F), bool)
    tv[0] = rng.random(F) < 0.1
    rv[0] = rng.random(F) < 0.1
    los = np.zeros(N, bool)
    for n in range(1, N):
        tv[n] = tv[n - 1] ^ (rng.random(F) < 0.0004)
        rv[n] = rv[n - 1] ^ (rng.random(F) < 0.0004)
        los[n] = los[n - 1] ^ (rng.random() < 0.01)
    step = rng.normal(0, 1.0, (N, 3)).astype(np.float32) * np.float32(0.25)
    tx = np.cumsum(step, 0).astype(np.float32)
    rx = np.cumsum(step[::-1], 0).astype(np.float32)
    return tv, rv, los, tx, rx


def test_noalloc_matches_workspace_call_twice(oracle_mod):
    import torch
    import paper_2501_02747_amd as ivm
    assert torch.cuda.is_available()
    s = sg.gen_c4_scene(1001, f_target=600, n_snap=4)
    g = ivm.GpuScene.from_scene(s).check()
    F, W = s.n_facets, g.W
    dev = torch.device("cuda:0")
    for call, (N, seed) in enumerate([(5000, 11), (1200, 12)]):
        _log(f"[noalloc] call {call}: N={N} F={F}")
        tv, rv, los, tx, rx = _tables(F, N, seed)
        d = lambda a: torch.as_tensor(a).to(dev)
        dtv, drv = d(_pack(tv, W).view(np.int64)), d(_pack(rv, W).view(np.int64))
        dlos, dtx, drx = d(los.astype(np.uint8)), d(tx), d(rx)
        # outputs pre-filled with garbage: every entry the call owns must be written
        ev = torch.full((N, 5), -77, dtype=torch.int32, device=dev)
        st = torch.full((N,), -77, dtype=torch.int32, device=dev)
        tc = torch.full((N,), -7.0, dtype=torch.float64, device=dev)
        dist = torch.full((N, 2), -7.0, dtype=torch.float64, device=dev)
        nr = torch.full((1,), -1, dtype=torch.int32, device=dev)
        mean = torch.full((1,), -7.0, dtype=torch.float64, device=dev)
        ivm.ivm_visibility_ranges_noalloc(g, dtv, drv, dlos, dtx, drx, 0.01, ev, st, tc, dist, nr, mean)
        ev_w, st_w, tc_w, dist_w, mean_w = ivm.ivm_visibility_ranges(g, dtv, drv, dlos, dtx, drx, 0.01)
        torch.cuda.synchronize()
        L = int(nr.item())
        assert L == st_w.numel()
        assert torch.equal(ev, ev_w)
        assert torch.equal(st[:L], st_w)
        assert torch.equal(tc[:L], tc_w)
        assert torch.equal(dist[:L], dist_w)
        assert float(mean.item()) == mean_w
        r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, 0.01)
        assert (ev.cpu().numpy() == r["events"]).all()
        assert st[:L].cpu().numpy().tolist() == r["starts"].tolist()
        otc, gtc = r["tc"], tc[:L].cpu().numpy()
        assert (np.isinf(gtc) == np.isinf(otc)).all()
        fin = ~np.isinf(otc)
        np.testing.assert_allclose(gtc[fin], otc[fin], rtol=1e-12, atol=0)
        np.testing.assert_allclose(dist[:L].cpu().numpy(), r["dist"], rtol=1e-12, atol=0)
        _log(f"[noalloc] call {call}: L={L} equal to the workspace call and the oracle")


def test_noalloc_rejects_too_long_trajectory():
    import torch
    import paper_2501_02747_amd as ivm
    s = sg.gen_c1(1)
    g = ivm.GpuScene.from_scene(s).check()
    N = ivm.IVM_RANGES_NOALLOC_MAX_SNAP + 1
    dev = torch.device("cuda:0")
    tv = torch.zeros((N, g.W), dtype=torch.int64, device=dev)
    los = torch.zeros((N,), dtype=torch.uint8, device=dev)
    x = torch.zeros((N, 3), dtype=torch.float32, device=dev)
    out = [torch.empty((N, 5), dtype=torch.int32, device=dev), torch.empty((N,), dtype=torch.int32, device=dev),
           torch.empty((N,), dtype=torch.float64, device=dev), torch.empty((N, 2), dtype=torch.float64, device=dev),
           torch.empty((1,), dtype=torch.int32, device=dev), torch.empty((1,), dtype=torch.float64, device=dev)]
    with pytest.raises(RuntimeError, match="IVM_ERR_WORKSPACE"):
        ivm.ivm_visibility_ranges_noalloc(g, tv, tv, los, x, x, 0.01, *out)
