"""Launch-parameter search for the traversal kernels.

A grid search over the persistent grid size (waves per CU) and the traversal
stack depth, timed on a calibration scene with HIP events; every point must
return the same matrix bits as the first (the parameters never change a
result).  Results are cached as JSON keyed by GPU architecture and a size
bucket of the scene, so later runs on similar scenes reuse them.
"""
from __future__ import annotations

import json
import math
import os
import statistics
from typing import Dict, List, Optional, Tuple

from . import GpuScene, ivm_intervisibility_matrix, make_opts

WAVES_PER_CU = (8, 12, 16, 24, 32)
STACK_DEPTHS = (12, 16, 20, 24)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ivm_autotune.json")


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
                    grid: Optional[List[Tuple[int, int]]] = None, force: bool = False) -> dict:
    """Best (waves_per_cu, stack_depth) for ivm_intervisibility_matrix on this scene."""
    import torch
    key = size_bucket(scene)
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        return dict(cache[key], cached=True)
    grid = grid or [(w, s) for w in WAVES_PER_CU for s in STACK_DEPTHS]
    ref = None
    table = []
    for wpc, depth in grid:
        opts = make_opts(waves_per_cu=wpc, stack_depth=depth)
        out = torch.empty((scene.F, scene.W), dtype=torch.int64, device=scene.device)
        ivm_intervisibility_matrix(scene, opts, out=out)           # warm-up
        times = []
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ivm_intervisibility_matrix(scene, opts, out=out)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        if ref is None:
            ref = out.clone()
        elif not torch.equal(ref, out):
            raise RuntimeError(f"launch parameters {wpc}, {depth} changed the result")
        table.append({"waves_per_cu": wpc, "stack_depth": depth, "ms": statistics.median(times)})
    best = min(table, key=lambda r: r["ms"])
    res = {"waves_per_cu": best["waves_per_cu"], "stack_depth": best["stack_depth"], "ms": best["ms"],
           "table": table, "bucket": key}
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return dict(res, cached=False)
