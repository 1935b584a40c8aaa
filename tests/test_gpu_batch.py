"""Batched scenes in one captured hipGraph: every scene's matrix, tables, LoS and
candidate counts equal the single-scene calls (and the oracle on the small
scenes), on every graph replay; the batched workload at its full size against
the single-scene calls and stored oracle rows and snapshots of every scene."""
import os
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_batch_matches_single_scene_calls_on_every_replay(oracle_mod):
    import torch
    import paper_2501_02747_amd as ivm
    scenes = [sg.gen_c4_scene(1000 + k, f_target=f, n_snap=n)
              for k, (f, n) in enumerate([(520, 40), (160, 17), (900, 64), (60, 5), (700, 3), (300, 33)])]
    scenes.append(sg.gen_c1(9))
    gs = [ivm.GpuScene.from_scene(s).check() for s in scenes]
    txs = [torch.as_tensor(s.tx).cuda() for s in scenes]
    rxs = [torch.as_tensor(s.rx).cuda() for s in scenes]
    st = ivm.new_stats()
    stream = torch.cuda.Stream()
    batch = ivm.Batch(gs, txs, rxs, stats=st)
    ref = []
    for g, s, tx, rx in zip(gs, scenes, txs, rxs):
        M = ivm.ivm_intervisibility_matrix(g).clone()
        tv, rv, los = ivm.ivm_txrx_visibility_table(g, tx, rx)
        c = ivm.ivm_image_tree_candidates(g, M, tv, rv, los, 2)
        ref.append((M, tv.clone(), rv.clone(), los.clone(), c.clone()))
    torch.cuda.synchronize()
    # the two smallest scenes also against the oracle
    for k in (3, 6):
        Mo, _ = oracle_mod.Oracle(scenes[k]).matrix()
        assert (ivm.unpack_bits(ref[k][0], scenes[k].n_facets) == Mo).all()
    for rep in range(3):
        _log(f"[batch] replay {rep}")
        for k in range(len(gs)):          # eager work between replays clears every output
            for t in (batch.M[k], batch.tv[k], batch.rv[k], batch.los[k], batch.counts[k]):
                t.fill_(-1 if t.dtype != torch.uint8 else 7)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            batch.run(stream)
        stream.synchronize()
        for k, r in enumerate(ref):
            assert torch.equal(batch.M[k], r[0]), (rep, k, "M")
            assert torch.equal(batch.tv[k], r[1]), (rep, k, "tx")
            assert torch.equal(batch.rv[k], r[2]), (rep, k, "rx")
            assert torch.equal(batch.los[k], r[3]), (rep, k, "los")
            assert torch.equal(batch.counts[k], r[4]), (rep, k, "counts")
    d = ivm.stats_dict(st)
    assert d["pairs_total"] == 3 * sum(s.n_facets * (s.n_facets - 1) // 2 for s in scenes)


@pytest.mark.parametrize("exhaustive", [False, True])
def test_batch_of_many_tiny_scenes(oracle_mod, exhaustive):
    """Twelve tiny urban scenes plus a one-facet and a two-facet scene in one
    batch: scene boundaries fall inside the waves' chunks of pairs and probes,
    and every matrix still equals the single-scene call and the oracle."""
    import torch
    import paper_2501_02747_amd as ivm
    _log(f"[batch] many tiny scenes, exhaustive={exhaustive}")
    scenes = [sg.gen_c1(40 + k) for k in range(12)]
    one = sg.gen_plates([[[0, 0, 0], [4, 0, 0], [0, 4, 0]]], tx=[[1, 1, 3]], rx=[[2, 2, 7]])
    two = sg.gen_plates([[[0, 0, 0], [4, 0, 0], [0, 4, 0]], [[0, 0, 10], [0, 4, 0], [4, 0, 0]]],
                        tx=[[1, 1, 3]], rx=[[2, 2, 7]])
    scenes[4:4] = [one]
    scenes[9:9] = [two]
    gs = [ivm.GpuScene.from_scene(s).check() for s in scenes]
    txs = [torch.as_tensor(s.tx).cuda() for s in scenes]
    rxs = [torch.as_tensor(s.rx).cuda() for s in scenes]
    opts = ivm.make_opts(exhaustive=exhaustive)
    batch = ivm.Batch(gs, txs, rxs, opts=opts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.run(stream)
    stream.synchronize()
    for k, (g, s) in enumerate(zip(gs, scenes)):
        M = ivm.ivm_intervisibility_matrix(g, opts)
        torch.cuda.synchronize()
        assert torch.equal(batch.M[k], M), k
        Mo, _ = oracle_mod.Oracle(s).matrix()
        assert (ivm.unpack_bits(batch.M[k], s.n_facets) == Mo).all(), k


C4_CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c4_rows.npz")


@pytest.mark.skipif(not os.path.exists(C4_CACHE), reason="batched-workload oracle rows not generated")
def test_batched_workload_full_size(oracle_mod):
    """The batched workload at its real size (64 scenes of 636-4856 facets,
    seeds 1000-1063, 64 077 snapshots) in one captured graph, in the launch
    configuration of the batched bench (the autotuned knobs of the calibration scene):
    every scene's matrix, tables, LoS and candidate counts equal the single-scene
    calls, and two whole seeded rows and two whole seeded snapshots of every
    scene equal the stored oracle results (tests/golden/make_c4_oracle_cache.py)."""
    import torch
    import paper_2501_02747_amd as ivm
    from paper_2501_02747_amd.autotune import KNOBS, autotune_matrix, opts_from
    _log("[batch] generating the 64 batched scenes")
    scenes = sg.gen_c4(1000, 64)
    z = np.load(C4_CACHE, allow_pickle=False)
    F = np.array([s.n_facets for s in scenes])
    assert F.max() >= 4000 and len(scenes) == 64
    gs = [ivm.GpuScene.from_scene(s).check() for s in scenes]
    txs = [torch.as_tensor(s.tx).cuda() for s in scenes]
    rxs = [torch.as_tensor(s.rx).cuda() for s in scenes]
    calib = int(np.argsort(F)[len(F) // 2])
    tune = autotune_matrix(gs[calib], repeats=1, cache_path=None)
    _log("[batch] autotuned: " + ", ".join(f"{k} {tune[k]}" for k in KNOBS))
    opts = opts_from(tune)
    batch = ivm.Batch(gs, txs, rxs, opts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.run(stream)
    stream.synchronize()
    _log("[batch] graph run done; comparing with single-scene calls and the oracle rows")
    for k, (g, s) in enumerate(zip(gs, scenes)):
        M = ivm.ivm_intervisibility_matrix(g)
        tv, rv, los = ivm.ivm_txrx_visibility_table(g, txs[k], rxs[k])
        c = ivm.ivm_image_tree_candidates(g, M, tv, rv, los, 2)
        torch.cuda.synchronize()
        assert torch.equal(batch.M[k], M), (k, "M")
        assert torch.equal(batch.tv[k], tv) and torch.equal(batch.rv[k], rv), (k, "tables")
        assert torch.equal(batch.los[k], los) and torch.equal(batch.counts[k], c), (k, "los / counts")
        tag = f"{k:02d}"
        n = s.n_facets
        assert int(z[f"F_{tag}"]) == n
        m = ivm.unpack_bits(batch.M[k], n)
        assert (m == m.T).all() and not m.diagonal().any(), k
        rows, snaps = z[f"rows_{tag}"], z[f"snaps_{tag}"]
        Mo = np.unpackbits(z[f"M_{tag}"], axis=1)[:, :n].astype(bool)
        assert (m[rows] == Mo).all(), (k, "rows", int((m[rows] != Mo).sum()))
        for key, t in (("tx", batch.tv[k]), ("rx", batch.rv[k])):
            o = np.unpackbits(z[f"{key}_{tag}"], axis=1)[:, :n].astype(bool)
            assert (ivm.unpack_bits(t, n)[snaps] == o).all(), (k, key)
        assert (batch.los[k].cpu().numpy().astype(bool)[snaps] == z[f"los_{tag}"]).all(), (k, "los")
    _log(f"[batch] 64 scenes equal ({int(F.sum())} facets)")
