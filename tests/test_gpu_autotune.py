"""The launch-knob autotuner (waves per CU, stack depth, near-field tile
capacity and treelet limit, pair-to-wave chunk): every point it times must
return the bits of the first, the tuned options give the oracle's matrix, and
the cache key names the architecture, the scene's size bucket and the loaded
library's hash (a rebuilt kernel is tuned anew)."""
import json
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_autotune_keeps_bits_and_caches_by_library(oracle_mod, tmp_path):
    import torch
    import paper_2501_02747_amd as ivm
    from paper_2501_02747_amd import autotune
    s = sg.gen_c4_scene(1007, f_target=700, n_snap=4)
    g = ivm.GpuScene.from_scene(s).check()
    cache = str(tmp_path / "tune.json")
    knobs = {"waves_per_cu": (8, 16, 32), "stack_depth": (12, 24), "tile_cap": (16, 64), "tile_treelets": (2, 6, 10),
             "pair_chunk": (0, 1, 8, 64)}
    t = autotune.autotune_matrix(g, repeats=2, cache_path=cache, knobs=knobs)
    _log("[autotune] " + ", ".join(f"{k} {t[k]}" for k in autotune.KNOBS) +
         f"; {t['points']} points, {t['default_ms']:.3f} -> {t['ms']:.3f} ms")
    assert not t["cached"] and t["points"] >= 1 + sum(len(v) - 1 for v in knobs.values())
    assert t["ms"] <= t["default_ms"]
    assert f"lib{autotune.library_hash()}" in t["bucket"] and "gfx950" in t["bucket"]
    again = autotune.autotune_matrix(g, repeats=2, cache_path=cache, knobs=knobs)
    assert again["cached"] and {k: again[k] for k in autotune.KNOBS} == {k: t[k] for k in autotune.KNOBS}
    assert json.load(open(cache))[t["bucket"]]["points"] == t["points"]
    M = ivm.ivm_intervisibility_matrix(g, autotune.opts_from(t))
    torch.cuda.synchronize()
    Mo, _ = oracle_mod.Oracle(s).matrix()
    assert (ivm.unpack_bits(M, s.n_facets) == Mo).all()


@pytest.mark.parametrize("point", [
    {"tile_cap": 1, "tile_treelets": 32}, {"tile_cap": 8, "tile_treelets": 1}, {"pair_chunk": 1},
    {"pair_chunk": 256}, {"pair_chunk": 7, "tile_cap": 33, "waves_per_cu": 5, "stack_depth": 3}])
def test_extreme_knob_values_keep_bits(oracle_mod, point):
    """Tiles that overflow at once or are gathered for every bundle, one pair per
    wave or very long chunks: the matrix of the tiny urban scenes is unchanged."""
    import torch
    import paper_2501_02747_amd as ivm
    for seed in (3, 4):
        s = sg.gen_c1(seed)
        g = ivm.GpuScene.from_scene(s).check()
        M = ivm.ivm_intervisibility_matrix(g, ivm.make_opts(**point))
        torch.cuda.synchronize()
        Mo, _ = oracle_mod.Oracle(s).matrix()
        assert (ivm.unpack_bits(M, s.n_facets) == Mo).all(), (seed, point)
