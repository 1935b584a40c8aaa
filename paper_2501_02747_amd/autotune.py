"""Launch-parameter search for the traversal kernels.

Knobs of the matrix call (none of them changes a result bit):
  waves_per_cu   persistent grid size (waves per compute unit)
  stack_depth    traversal stack entries per lane (overflow scans a subtree)
  tile_cap       near-field tile capacity (triangles gathered for a bundle)
  tile_treelets  largest number of treelets a bundle box may meet for a tile
  pair_chunk     pair-to-wave mapping: consecutive undecided pairs a wave takes
                 from the queue at a time (0 = chosen from the load)
  xcd_parts      the pair queues and table items split into one range per XCD
                 (8) or a single range (1, the default)

The search is coordinate descent: starting from the defaults, each knob in
turn is swept over its values with the others fixed, and the fastest value is
kept; the sweep repeats until a pass changes nothing (at most `passes`).  Each
point is timed with HIP events on the calibration scene, and every point must
return the bits of the first (a point that changes a bit raises).  A winner
other than the defaults is then timed again against them, alternating, and
kept only if it is still faster (single timings of a few milliseconds vary by
a few per cent, as much as most knobs gain).  Results are
cached as JSON under a key made of the GPU architecture, a size bucket of the
scene and the SHA-256 of the loaded library, so a rebuilt kernel is tuned anew.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import statistics
from typing import Dict, List, Optional, Sequence, Tuple

from . import LIB_PATH, GpuScene, ivm_intervisibility_matrix, make_opts

KNOBS: Dict[str, Tuple[int, ...]] = {
    "waves_per_cu": (8, 12, 16, 24, 32),
    "stack_depth": (12, 16, 20, 24),
    "tile_cap": (16, 32, 64),
    "tile_treelets": (2, 4, 6, 10),
    "pair_chunk": (0, 2, 4, 8, 16, 32, 64),
    "xcd_parts": (1, 8),
}
DEFAULTS = {"waves_per_cu": 24, "stack_depth": 24, "tile_cap": 64, "tile_treelets": 2, "pair_chunk": 0, "xcd_parts": 1}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ivm_autotune.json")


def library_hash(path: str = LIB_PATH) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def size_bucket(scene: GpuScene) -> str:
    """Arch + powers of two of the facet and triangle counts + samples per facet."""
    import torch
    arch = torch.cuda.get_device_properties(scene.device).gcnArchName.split(":")[0]
    spf = max(1, round(scene.S / max(scene.F, 1)))
    return f"{arch}/F{2 ** math.ceil(math.log2(max(scene.F, 2)))}/T{2 ** math.ceil(math.log2(max(scene.T, 2)))}/S{spf}"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune_matrix(scene: GpuScene, repeats: int = 3, cache_path: Optional[str] = DEFAULT_CACHE,
                    knobs: Optional[Dict[str, Sequence[int]]] = None, passes: int = 2,
                    force: bool = False, rebuild: bool = False, confirm: int = 3) -> dict:
    """Best knob values for ivm_intervisibility_matrix on this scene (see the module doc).
    With rebuild=True the scene is rebuilt before every timed call (as in a
    pipeline step that builds and then queries), so caches start as they would."""
    import torch
    key = f"{size_bucket(scene)}/lib{library_hash()}"
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        return dict(cache[key], cached=True)
    knobs = dict(knobs or KNOBS)
    out = torch.empty((scene.F, scene.W), dtype=torch.int64, device=scene.device)
    ref = None
    timed: Dict[Tuple[Tuple[str, int], ...], float] = {}
    table: List[dict] = []

    def measure(point: Dict[str, int], again: bool = False) -> float:
        nonlocal ref
        tkey = tuple(sorted(point.items()))
        if tkey in timed and not again:
            return timed[tkey]
        opts = make_opts(**point)
        ivm_intervisibility_matrix(scene, opts, out=out)            # warm-up
        times = []
        for _ in range(repeats):
            if rebuild:
                scene.rebuild()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ivm_intervisibility_matrix(scene, opts, out=out)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        if ref is None:
            ref = out.clone()
        elif not torch.equal(ref, out):
            raise RuntimeError(f"launch parameters {point} changed the result")
        ms = statistics.median(times)
        if again:
            return ms
        timed[tkey] = ms
        table.append(dict(point, ms=ms))
        return ms

    best = dict(DEFAULTS)  # knobs not swept keep their defaults
    best_ms = measure(best)
    for _ in range(passes):
        changed = False
        for name, values in knobs.items():
            for v in values:
                if v == best[name]:
                    continue
                ms = measure(dict(best, **{name: v}))
                if ms < best_ms:
                    best, best_ms, changed = dict(best, **{name: v}), ms, True
        if not changed:
            break
    default_ms = table[0]["ms"]
    if best != DEFAULTS and confirm > 0:
        tb, td = [], []
        for _ in range(confirm):
            td.append(measure(dict(DEFAULTS), again=True))
            tb.append(measure(best, again=True))
        best_ms, default_ms = statistics.median(tb), statistics.median(td)
        if best_ms >= default_ms:
            best, best_ms = dict(DEFAULTS), default_ms
    res = dict(best, ms=best_ms, default_ms=default_ms, points=len(table), table=table, bucket=key)
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return dict(res, cached=False)


def opts_from(tune: dict, **extra):
    """ivm_matrix_opts with the tuned knob values (plus any other make_opts arguments)."""
    return make_opts(**{k: tune[k] for k in KNOBS if k in tune}, **extra)
