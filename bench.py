#!/usr/bin/env python3
"""Benchmark of the inter-visibility hot path on one MI355X.

One step = one pass of the whole path over the workload: build the scene
(validation + Morton LBVH), the facet-pair inter-visibility matrix, the Tx/Rx
visibility table for every snapshot, and image-tree candidate counts up to
order 2.  Inputs are resident in HBM before timing starts.

Prints one JSON line for the large-city workload (4 x 4 km, 19 872 facets,
10 000 snapshots: the largest single-GPU configuration), with the urban-grid
workload (2000 facets, 1000 snapshots) as a nested block.  value = facet-pair
queries/s = F(F-1)/2 unordered pairs decided per second of
ivm_intervisibility_matrix GPU time (median over steps); txrx_ms_per_snapshot =
(table + candidates) GPU time / snapshots.

    python bench.py [--steps K] [--warmup W] [--config c3] [--order plain]
"""
import argparse
import json
import os
import platform
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 non-packed FP32 lane-ops/s
# (one FMA = one lane-op; 78.6 TFLOP/s counting an FMA as two).  FP64 vector
# operations issue at the same one per lane per clock on MI355X.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic work per counted unit (VALU lane-ops): a segment/box slab test 14
# (three slabs: six products, six min/max, the entry/exit compare), a
# segment/triangle test ~43 (Moller-Trumbore 33 + filter 10).  These two are the
# useful FP32 work the roofline fraction counts.  Reported beside it, not in it:
# an FP64 recheck ~35 and one face-plane step of an exact solid test ~25 FP64
# lane-ops (two plane values, the interval update with an exact product compare).
OPS_BOX, OPS_TRI, OPS_RECHECK, OPS_SOLID_PLANE = 14, 43, 35, 25


PROFILES = {"c2": os.path.join(ROOT, "profiles", "k_pairs_urban_grid_c2.txt"),
            "c3": os.path.join(ROOT, "profiles", "k_pairs_large_city_c3.txt")}


def profiled_counters(config: str) -> dict:
    """Per-launch counter figures of the pair and point kernels from the committed
    rocprofv3 summary of this workload, while the traversal source still has the
    SHA-256 recorded there (else nothing): HBM bytes of one matrix call's pair
    kernels (two probe rounds and the pair kernel) and of the point kernel
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration the summary
    states), and L2 bandwidth (TCC requests x 128 B / average kernel time)."""
    import hashlib
    import re
    path = PROFILES.get(config)
    if not path or not os.path.exists(path):
        return {}
    text = open(path).read()
    m = re.search(r"sha256: ([0-9a-f]{64})", text)
    src = os.path.join(ROOT, "paper_2501_02747_amd", "csrc", "traverse.hip")
    if not m or hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(1):
        return {}
    out = {}
    hbm = {}
    for name in ("k_pairs<false>", "k_probe_pairs<false>", "k_points<false>"):
        r = re.search(re.escape(name) + r"\s+fetch\s+([0-9.]+) MiB\s+write\s+([0-9.]+) MiB", text)
        if r:
            hbm[name] = (float(r.group(1)) + float(r.group(2))) * 2 ** 20
    if "k_pairs<false>" in hbm and "k_probe_pairs<false>" in hbm:
        out["pairs_hbm_bytes"] = int(hbm["k_pairs<false>"] + 2 * hbm["k_probe_pairs<false>"])
    if "k_points<false>" in hbm:
        out["points_hbm_bytes"] = int(hbm["k_points<false>"])
    for name, key in (("k_pairs<false>", "pairs"), ("k_points<false>", "points")):
        r = re.search(re.escape(name) + r"\s+l2\s+([0-9.]+) GB/s", text)
        if r:
            out[f"{key}_l2_gbs"] = float(r.group(1))
    r = re.search(r"counters k_pairs<false>: (.*)", text)
    if r:
        out["pairs_counters"] = r.group(1).strip()
    return out


def lane_ops(st: dict) -> int:
    """Useful FP32 VALU lane-ops: box slab tests and triangle tests."""
    return st["box_tests"] * OPS_BOX + st["tri_tests"] * OPS_TRI


def fp64_lane_ops(st: dict) -> int:
    """FP64 lane-ops of rechecks and exact solid tests (reported separately)."""
    return st["rechecks"] * OPS_RECHECK + st["solid_planes"] * OPS_SOLID_PLANE


WORKLOADS = {
    "c1": "tiny urban 200x200 m, 8 boxes, 42 facets / 84 tris, 4x4 samples, 10 snapshots",
    "c2": "urban grid 1x1 km, 200 boxes on a Manhattan grid, 2000 facets / 4000 tris, 8x8 samples, "
          "1000 snapshots (Rx 120 km/h every 10 ms, Tx fixed at 30 m)",
    "c3": "large city 4x4 km, 2000 convex 4-8-gon extrusions, ~20k facets / ~44k tris, 4x4 samples, "
          "10000 snapshots (two vehicles 5-20 m/s)",
    "c4": "64 config-1-style scenes (500-5000 facets), 4x4 samples, one graph-captured batch",
}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-nested", action="store_true", help="skip the nested urban-grid block of the c3 run")
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--snapshots", type=int, default=None)
    ap.add_argument("--order", default="plain", choices=["plain", "index", "reversed", "learned"])
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--exhaustive", action="store_true",
                    help="ablation: every admissible segment searched on its own (no probes, caches or certificates)")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--stack", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch knobs on the workload before timing (always done for the nested urban grid)")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the second-order (plain vs learned) pass")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates profiler byte counters)")
    return ap.parse_args()


def cpu_baseline(scene, seconds, seed=0):
    """The FP64 oracle on a bounded, seeded sample of the same workload: uniformly
    drawn unordered facet pairs (queries/s) and a few whole snapshots (ms/snapshot)."""
    import oracle
    orc = oracle.Oracle(scene)
    rng = np.random.default_rng(seed)
    F = scene.n_facets
    cores = oracle.num_threads()
    n_pairs, t_pairs = 0, 0.0
    while t_pairs < 0.75 * seconds:
        I = rng.integers(0, F, 512)
        J = rng.integers(0, F, 512)
        keep = I != J
        I, J = I[keep], J[keep]
        t0 = time.perf_counter()
        orc.pairs(I, J)
        t_pairs += time.perf_counter() - t0
        n_pairs += len(I)
    # whole snapshots while they are cheap (small scenes); on large scenes one
    # snapshot's table over a seeded subset of the facets from both ends, scaled
    # to all F facets
    n_snap, t_snap = 0, 0.0
    idx = rng.permutation(scene.n_snapshots)
    snap_note = ""
    if F <= 4000:
        while t_snap < 0.25 * seconds and n_snap < len(idx):
            k = idx[n_snap:n_snap + 1]
            t0 = time.perf_counter()
            tv, rv, los = orc.txrx(scene.tx[k], scene.rx[k])
            oracle.candidates_matmul(np.zeros((F, F), bool), tv, rv, los, 1)
            t_snap += time.perf_counter() - t0
            n_snap += 1
        snap_note = f"Tx/Rx table for {n_snap} whole snapshots"
    else:
        n = idx[0]
        sub = np.sort(rng.choice(F, F // 16, replace=False))
        t0 = time.perf_counter()
        orc.point_facets(np.repeat(scene.tx[n:n + 1], len(sub), 0), sub)
        orc.point_facets(np.repeat(scene.rx[n:n + 1], len(sub), 0), sub)
        orc.los(scene.tx[n:n + 1], scene.rx[n:n + 1])
        t_snap = (time.perf_counter() - t0) * F / len(sub)
        n_snap = 1
        snap_note = f"Tx/Rx table of one snapshot over {len(sub)} of the {F} facets, scaled to all of them"
    # the same oracle on one host thread, on a smaller sample (a tenth of the time); the
    # oracle's thread setting persists, so it is put back afterwards
    n_one, t_one = 0, 0.0
    while t_one < 0.1 * seconds:
        I = rng.integers(0, F, 64)
        J = rng.integers(0, F, 64)
        keep = I != J
        I, J = I[keep], J[keep]
        t0 = time.perf_counter()
        orc.pairs(I, J, threads=1)
        t_one += time.perf_counter() - t0
        n_one += len(I)
    if F >= 2:
        orc.pairs(np.zeros(1, np.int64), np.ones(1, np.int64), threads=cores)
    return {"value": n_pairs / t_pairs, "unit": "facet-pair queries/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n_pairs} uniformly drawn facet pairs of the same scene ({t_pairs:.1f} s); "
                      f"{snap_note}: {1e3 * t_snap / max(n_snap, 1):.1f} ms/snapshot (table only)",
            "ms_per_snapshot": 1e3 * t_snap / max(n_snap, 1),
            "value_1core": n_one / t_one, "sample_1core": f"{n_one} facet pairs on one thread ({t_one:.1f} s)"}


def cpu_model() -> str:
    """The host CPU's model name (as the kernel reports it), else the machine type."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def verify(ivm, scene, M, tv, rv, los, counts):
    """Compare with the oracle: the full cached result if one exists for this exact
    workload, else seeded sampled pairs and snapshot entries computed now."""
    import oracle
    F = scene.n_facets
    gm = ivm.unpack_bits(M, F)
    gtv, grv = ivm.unpack_bits(tv, F), ivm.unpack_bits(rv, F)
    glos = los.cpu().numpy().astype(bool)
    cache = os.path.join(ROOT, "tests", "golden", "cache", f"{scene.name}_seed{scene.seed}.npz")
    if os.path.exists(cache) and scene.n_snapshots == 1000:
        z = np.load(cache)
        Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
        tvo = np.unpackbits(z["tx_vis"], axis=1)[:, :F].astype(bool)
        rvo = np.unpackbits(z["rx_vis"], axis=1)[:, :F].astype(bool)
        co = oracle.candidates_matmul(Mo, tvo, rvo, z["los"], 2)
        ok = bool((gm == Mo).all() and (gtv == tvo).all() and (grv == rvo).all() and (glos == z["los"]).all()
                  and (counts.cpu().numpy() == co).all())
        return {"mode": "full oracle cache", "ok": ok}
    mode, ok = "", True
    rows_cache = os.path.join(ROOT, "tests", "golden", "cache", f"{scene.name}_seed{scene.seed}_rows.npz")
    if os.path.exists(rows_cache):
        z = np.load(rows_cache, allow_pickle=False)
        if int(z["F"]) == F and int(z["snaps"].max()) < scene.n_snapshots:
            rows, snaps = z["rows"], z["snaps"]
            ok &= bool((gm[rows] == np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)).all())
            ok &= bool((gtv[snaps] == np.unpackbits(z["tx_vis"], axis=1)[:, :F].astype(bool)).all())
            ok &= bool((grv[snaps] == np.unpackbits(z["rx_vis"], axis=1)[:, :F].astype(bool)).all())
            ok &= bool((glos[snaps] == z["los"]).all())
            mode = f"{len(rows)} whole rows and {len(snaps)} whole snapshots from the stored oracle results; "
    orc = oracle.Oracle(scene)
    rng = np.random.default_rng(1)
    I = rng.integers(0, F, 300)
    J = rng.integers(0, F, 300)
    # bias half the sample toward visible GPU pairs so both outcomes are checked
    vis = np.argwhere(np.triu(gm, 1))
    if len(vis):
        pick = vis[rng.integers(0, len(vis), 150)]
        I = np.concatenate([I, pick[:, 0]])
        J = np.concatenate([J, pick[:, 1]])
    ok &= bool((orc.pairs(I, J) == gm[I, J]).all())
    N = scene.n_snapshots
    n_idx = rng.integers(0, N, 200)
    f_idx = rng.integers(0, F, 200)
    ok &= bool((orc.point_facets(scene.tx[n_idx], f_idx) == gtv[n_idx, f_idx]).all())
    ok &= bool((orc.point_facets(scene.rx[n_idx], f_idx) == grv[n_idx, f_idx]).all())
    ok &= bool((orc.los(scene.tx[n_idx], scene.rx[n_idx]) == glos[n_idx]).all())
    ok &= bool((gm == gm.T).all() and not gm.diagonal().any())
    return {"mode": mode + f"sampled: {len(I)} pairs, 200 Tx + 200 Rx entries, 200 LoS", "ok": ok}


def run_batched(args, ivm, torch, sg):
    """The batched workload: 64 config-1-style scenes of 500-5000 facets in one
    graph-captured run; launch parameters from the autotuner on a calibration scene."""
    from paper_2501_02747_amd.autotune import KNOBS, autotune_matrix, opts_from

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    scenes = sg.gen_c4(1000, 64)
    F = np.array([s.n_facets for s in scenes])
    N = np.array([s.n_snapshots for s in scenes])
    progress(f"c4: 64 scenes, F {F.min()}..{F.max()} (sum {F.sum()}), snapshots {N.sum()}")
    gs = [ivm.GpuScene.from_scene(s).check() for s in scenes]
    txs = [torch.as_tensor(s.tx).cuda() for s in scenes]
    rxs = [torch.as_tensor(s.rx).cuda() for s in scenes]
    calib = int(np.argsort(F)[len(F) // 2])
    tune = autotune_matrix(gs[calib], repeats=1, cache_path=None, rebuild=True)
    progress(f"autotuned on scene {calib} (F={F[calib]}) over {tune['points']} points: "
             + ", ".join(f"{k} {tune[k]}" for k in KNOBS) + f" ({tune['default_ms']:.2f} -> {tune['ms']:.2f} ms)")
    opts = opts_from(tune)
    st = ivm.new_stats()
    batch = ivm.Batch(gs, txs, rxs, opts, stats=st)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            batch.run(stream)
        stream.synchronize()
        st.zero_()
        times = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.run(stream)
            e1.record(stream)
            times.append((e0, e1))
        stream.synchronize()
        wall = time.perf_counter() - t0
    ms = statistics.median(e0.elapsed_time(e1) for e0, e1 in times)
    progress(f"timed {args.steps} graph runs: {ms:.2f} ms each")
    n_pairs = int((F * (F - 1) // 2).sum())
    sd = {k: v // args.steps for k, v in ivm.stats_dict(st).items()}
    ops = lane_ops(sd)
    ach = ops / (ms / 1e3) / 1e12
    out = {
        "metric": "facet-pair vis queries/s + Tx/Rx table ms/snapshot, learned vs plain, bit-exact",
        "value": n_pairs / (ms / 1e3), "unit": "facet-pair queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 recheck)",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": "c4: 64 config-1-style scenes, 500-5000 facets, 4x4 samples, 100-2000 snapshots "
                               "each, one graph-captured run", "facets": int(F.sum()), "snapshots": int(N.sum()),
                   "pairs": n_pairs, "parallelism": "single GPU"},
        "txrx_ms_per_snapshot": ms / float(N.sum()),
        "note": "queries/s and ms/snapshot are both whole-graph time (matrices, tables and candidates together)",
        "autotune": dict({k: tune[k] for k in KNOBS}, ms=tune["ms"], default_ms=tune["default_ms"],
                         points=tune["points"], calibration_scene=calib),
        "stats_per_run": sd,
        "roofline": {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                     "frac": ach / VALU_PEAK_TOPS, "traffic": None, "kernel": "whole graph (k_probe_pairs + k_pairs + k_points)"},
    }
    if not args.no_verify:
        import oracle
        progress("verifying sampled pairs of three scenes against the oracle")
        ok = True
        for k in (0, calib, int(np.argmax(F))):
            s = scenes[k]
            gm = ivm.unpack_bits(batch.M[k], s.n_facets)
            rng = np.random.default_rng(k)
            I = rng.integers(0, s.n_facets, 150)
            J = rng.integers(0, s.n_facets, 150)
            vis = np.argwhere(np.triu(gm, 1))
            pick = vis[rng.integers(0, len(vis), 50)] if len(vis) else np.zeros((0, 2), int)
            I, J = np.concatenate([I, pick[:, 0]]), np.concatenate([J, pick[:, 1]])
            ok &= bool((oracle.Oracle(s).pairs(I, J) == gm[I, J]).all())
        mode = "sampled: 200 pairs in each of 3 scenes"
        rcache = os.path.join(ROOT, "tests", "golden", "cache", "c4_rows.npz")
        if os.path.exists(rcache):
            z = np.load(rcache, allow_pickle=False)
            for k, s in enumerate(scenes):
                tag, n = f"{k:02d}", s.n_facets
                rows, snaps = z[f"rows_{tag}"], z[f"snaps_{tag}"]
                ok &= bool((ivm.unpack_bits(batch.M[k], n)[rows] ==
                            np.unpackbits(z[f"M_{tag}"], axis=1)[:, :n].astype(bool)).all())
                for key, t in (("tx", batch.tv[k]), ("rx", batch.rv[k])):
                    ok &= bool((ivm.unpack_bits(t, n)[snaps] ==
                                np.unpackbits(z[f"{key}_{tag}"], axis=1)[:, :n].astype(bool)).all())
                ok &= bool((batch.los[k].cpu().numpy().astype(bool)[snaps] == z[f"los_{tag}"]).all())
            mode = "2 whole rows and 2 whole snapshots of every scene from the stored oracle results; " + mode
        out["verified"] = {"mode": mode, "ok": ok}
    if not args.no_cpu_baseline:
        progress("timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(scenes[calib], args.cpu_baseline_seconds)
        out["cpu_baseline"]["host"] = cpu_model()
        out["cpu_baseline"]["nproc"] = os.cpu_count()
    print(json.dumps(out), flush=True)


def main():
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}): the inter-visibility "
              "path runs on a single MI355X; a run over several GPUs is not supported.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2501_02747_amd as ivm
    import scenegen as sg

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    if args.config == "c4":
        return run_batched(args, ivm, torch, sg)
    out = run_single(args, ivm, torch, sg, args.config)
    if args.config == "c3" and not args.no_nested and args.snapshots is None and args.seed is None:
        nested = run_single(args, ivm, torch, sg, "c2", headline=False)
        out["urban_grid_c2"] = {k: nested[k] for k in (
            "value", "unit", "ms_per_step", "txrx_ms_per_snapshot", "phase_ms_median", "kernel_ms", "config",
            "roofline", "roofline_points", "compare_order", "verified", "ranges", "relations", "candidates_order4",
            "edges", "autotune", "angles", "edge_rows", "paths") if k in nested}
    print(json.dumps(out), flush=True)


def run_single(args, ivm, torch, sg, config: str, headline: bool = True) -> dict:
    """One single-scene workload: timed steps, the other traversal order, the calls
    beside the hot path, verification and (for the headline line) the CPU baseline."""
    kw = {}
    if args.snapshots is not None:
        kw["n_snap"] = args.snapshots
    scene = sg.make_config(config, args.seed, **kw)
    F, N = scene.n_facets, scene.n_snapshots
    order = {"plain": ivm.IVM_ORDER_PLAIN, "index": ivm.IVM_ORDER_INDEX, "reversed": ivm.IVM_ORDER_REVERSED,
             "learned": ivm.IVM_ORDER_LEARNED}[args.order]
    weights = os.path.join(ROOT, "paper_2501_02747_amd", "models", "occluder_mlp.npy")
    have_model = os.path.exists(weights)
    g = ivm.GpuScene.from_scene(scene, learned=have_model).check()
    model = None
    if have_model:
        model = ivm.Model(max_batch=1024, precision=ivm.IVM_MODEL_BF16)
        model.set_params(np.load(weights, allow_pickle=False))
        ivm.ivm_scene_set_model(g, model)
    elif args.order == "learned":
        print("no trained occluder-ordering weights found", file=sys.stderr)
        sys.exit(1)
    tx = torch.as_tensor(scene.tx).cuda()
    rx = torch.as_tensor(scene.rx).cuda()
    M = torch.empty((F, g.W), dtype=torch.int64, device="cuda")
    tv = torch.empty((N, g.W), dtype=torch.int64, device="cuda")
    rv = torch.empty((N, g.W), dtype=torch.int64, device="cuda")
    los = torch.empty((N,), dtype=torch.uint8, device="cuda")
    counts = torch.empty((N, 3), dtype=torch.int64, device="cuda")
    st_m, st_p = ivm.new_stats(), ivm.new_stats()
    t_pairs, t_points = ivm.KernelTimer(), ivm.KernelTimer()
    # launch knobs: the autotuner's (nested urban-grid run, or --autotune), else the command line's
    from paper_2501_02747_amd.autotune import KNOBS, autotune_matrix
    tune = None
    knob = {"waves_per_cu": args.waves_per_cu, "stack_depth": args.stack}
    if (args.autotune or not headline) and not args.exhaustive:
        tune = autotune_matrix(g, repeats=3 if F <= 4000 else 1, cache_path=None, rebuild=True)
        knob = {k: tune[k] for k in KNOBS}
        print(f"[bench] {config}: autotuned over {tune['points']} points: "
              + ", ".join(f"{k} {tune[k]}" for k in KNOBS) + f" ({tune['default_ms']:.2f} -> {tune['ms']:.2f} ms)",
              file=sys.stderr, flush=True)
    om = ivm.make_opts(order_mode=order, fp64_only=args.fp64_only, timing=t_pairs, exhaustive=args.exhaustive,
                       **knob)
    # (the tuner times the matrix call: the table keeps the command line's knobs)
    op = ivm.make_opts(order_mode=order, fp64_only=args.fp64_only, timing=t_points, exhaustive=args.exhaustive,
                       waves_per_cu=args.waves_per_cu, stack_depth=args.stack)

    def step(rec):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        st_m.zero_()
        st_p.zero_()
        ev[0].record()
        g.rebuild()
        ev[1].record()
        ivm.ivm_intervisibility_matrix(g, om, out=M, stats=st_m, allow_model_fallback=False)
        ev[2].record()
        ivm.ivm_txrx_visibility_table(g, tx, rx, op, stats=st_p, out=(tv, rv, los))
        ev[3].record()
        ivm.ivm_image_tree_candidates(g, M, tv, rv, los, 2, counts=counts)
        ev[4].record()
        if rec is not None:
            rec.append((ev, t_pairs, t_points))

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        progress(f"copied {args.copy_mib} MiB (profiler calibration)")
        del src, dst
    progress(f"{config}: F={F} T={scene.n_triangles} S={scene.n_samples} N={N}; warmup {args.warmup}")
    for k in range(args.warmup):
        step(None)
        torch.cuda.synchronize()
        progress(f"warmup step {k + 1} done")
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"timed {args.steps} steps in {wall:.3f} s")
    # per-step GPU times (the kernel timers hold the last step's values; re-read per step
    # would need one timer per step, so kernel times come from the final step and a
    # check below that the matrix phase time is stable across steps)
    phases = {"build": [], "matrix": [], "txrx": [], "cand": [], "step": []}
    for ev, _, _ in recs:
        phases["build"].append(ev[0].elapsed_time(ev[1]))
        phases["matrix"].append(ev[1].elapsed_time(ev[2]))
        phases["txrx"].append(ev[2].elapsed_time(ev[3]))
        phases["cand"].append(ev[3].elapsed_time(ev[4]))
        phases["step"].append(ev[0].elapsed_time(ev[4]))
    med = {k: statistics.median(v) for k, v in phases.items()}
    pairs_kernel_ms = t_pairs.elapsed_ms()
    points_kernel_ms = t_points.elapsed_ms()
    sm, sp = ivm.stats_dict(st_m), ivm.stats_dict(st_p)
    n_pairs = F * (F - 1) // 2
    value = n_pairs / (med["matrix"] / 1e3)
    ops_pairs = lane_ops(sm)
    ops_points = lane_ops(sp)
    ach = ops_pairs / (pairs_kernel_ms / 1e3) / 1e12
    ach_p = ops_points / (points_kernel_ms / 1e3) / 1e12
    f64_pairs, f64_points = fp64_lane_ops(sm), fp64_lane_ops(sp)
    prof = profiled_counters(config)
    out = {
        "metric": "facet-pair vis queries/s + Tx/Rx table ms/snapshot, learned vs plain, bit-exact",
        "value": value,
        "unit": "facet-pair queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64_only else "f32 (f64 recheck)",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": f"{config}: {WORKLOADS[config]}", "facets": F,
                   "triangles": scene.n_triangles, "samples": scene.n_samples, "snapshots": N,
                   "seed": scene.seed, "order": args.order, "exhaustive": bool(args.exhaustive),
                   "parallelism": "single GPU"},
        "txrx_ms_per_snapshot": (med["txrx"] + med["cand"]) / N,
        "phase_ms_median": med,
        "kernel_ms": {"k_probe_pairs+k_pairs": pairs_kernel_ms, "k_points": points_kernel_ms},
        "stats_matrix": sm,
        "stats_table": sp,
        "autotune": (dict({k: tune[k] for k in KNOBS}, ms=tune["ms"], default_ms=tune["default_ms"],
                          points=tune["points"]) if tune else "not run (defaults; --autotune tunes this workload)"),
        "roofline": {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                     "frac": ach / VALU_PEAK_TOPS, "traffic": prof.get("pairs_hbm_bytes"),
                     "traffic_unit": "HBM bytes per matrix call (FETCH_SIZE + WRITE_SIZE, from profiles/)",
                     "kernel": "k_probe_pairs x2 + k_pairs (one timed region)",
                     "ops_per_launch": ops_pairs, "ops_units": "box tests x 14 + triangle tests x 43 (FP32)",
                     "fp64_ops_per_launch": f64_pairs,
                     "fp64_ops_units": "rechecks x 35 + solid face-plane steps x 25 (FP64, not in frac)",
                     "frac_incl_fp64": (ops_pairs + f64_pairs) / (pairs_kernel_ms / 1e3) / 1e12 / VALU_PEAK_TOPS,
                     "l2_gbs": prof.get("pairs_l2_gbs"), "counters": prof.get("pairs_counters")},
        "roofline_points": {"bound": "alu", "achieved": ach_p, "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                            "frac": ach_p / VALU_PEAK_TOPS, "kernel": "k_points",
                            "fp64_ops_per_launch": f64_points,
                            "frac_incl_fp64": (ops_points + f64_points) / (points_kernel_ms / 1e3) / 1e12
                            / VALU_PEAK_TOPS, "traffic": prof.get("points_hbm_bytes"),
                            "l2_gbs": prof.get("points_l2_gbs")},
    }
    # the other traversal order on the same matrix, timed the same way, bits compared
    if have_model and not args.no_compare:
        other = "plain" if args.order == "learned" else "learned"
        oo = ivm.make_opts(order_mode=ivm.IVM_ORDER_LEARNED if other == "learned" else ivm.IVM_ORDER_PLAIN,
                           fp64_only=args.fp64_only, timing=t_pairs, **knob)
        M2 = torch.empty_like(M)
        st_o = ivm.new_stats()
        times = []
        for k in range(args.warmup + args.steps):
            st_o.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ivm.ivm_intervisibility_matrix(g, oo, out=M2, stats=st_o)
            e1.record()
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(e0.elapsed_time(e1))
        so = ivm.stats_dict(st_o)
        out["compare_order"] = {
            "order": other, "matrix_ms": statistics.median(times),
            "queries_per_s": n_pairs / (statistics.median(times) / 1e3),
            "k_pairs_ms": t_pairs.elapsed_ms(), "identical_bits": bool(torch.equal(M, M2)),
            "box_tests": so["box_tests"], "tri_tests": so["tri_tests"], "segments": so["segments"],
            "certified": so["certified"], "traversed": so["traversed"], "solid_certified": so["solid_certified"],
            "solid_segments": so["solid_segments"], "solid_planes": so["solid_planes"],
            "note": "learned = network inference (in the matrix call) + learned treelet order",
        }
        progress(f"{other} order: {statistics.median(times):.2f} ms, identical bits "
                 f"{out['compare_order']['identical_bits']}")
    # visibility ranges and coherence times along the trajectory (after the table;
    # outside the step), timed the same way
    times = []
    for k in range(args.warmup + args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rr = ivm.ivm_visibility_ranges(g, tv, rv, los, tx, rx, scene.snapshot_dt, read_count=False)
        e1.record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            times.append(e0.elapsed_time(e1))
    L = int(rr[4].item())
    out["ranges"] = {"gpu_ms": statistics.median(times), "n_ranges": L, "tc_mean_s": float(rr[5].item()),
                     "snapshot_dt_s": scene.snapshot_dt}
    cache = os.path.join(ROOT, "tests", "golden", "cache", f"{scene.name}_seed{scene.seed}.npz")
    if not args.no_verify and os.path.exists(cache):
        import oracle
        z = np.load(cache, allow_pickle=False)
        tvo = np.unpackbits(z["tx_vis"], axis=1)[:, :F].astype(bool)
        rvo = np.unpackbits(z["rx_vis"], axis=1)[:, :F].astype(bool)
        t0 = time.perf_counter()
        ro = oracle.visibility_ranges(tvo, rvo, z["los"], scene.tx, scene.rx, scene.snapshot_dt)
        out["ranges"]["oracle_ms"] = 1e3 * (time.perf_counter() - t0)
        gtc = rr[2][:L].cpu().numpy()
        fin = ~np.isinf(ro["tc"])
        out["ranges"]["matches_oracle"] = bool(
            (rr[0].cpu().numpy() == ro["events"]).all() and rr[1][:L].cpu().numpy().tolist() == ro["starts"].tolist()
            and (np.isinf(gtc) == ~fin).all() and np.allclose(gtc[fin], ro["tc"][fin], rtol=1e-12, atol=0))
    progress(f"visibility ranges: {statistics.median(times):.3f} ms, L = {L}")
    # interface relations (PAR / PER) of the visible pairs of the matrix
    times = []
    for k in range(args.warmup + args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        par, per, fcls = ivm.ivm_interface_relations(g, M)
        e1.record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            times.append(e0.elapsed_time(e1))
    out["relations"] = {"gpu_ms": statistics.median(times),
                        "par_pairs": int(ivm.unpack_bits(par, F).sum()) // 2,
                        "per_pairs": int(ivm.unpack_bits(per, F).sum()) // 2}
    # angular bouncing ranges of every visible pair (Section II-B, eq. 1-2); the call
    # sizes its output with one synchronisation, so it is timed end to end
    times = []
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        aoff, acols, arng = ivm.ivm_angular_ranges(g, M)
        torch.cuda.synchronize()
        if k >= args.warmup:
            times.append(1e3 * (time.perf_counter() - t0))
    out["angles"] = {"ms": statistics.median(times), "pairs": int(acols.numel()),
                     "note": "wall time of the whole call (row counts, one read-back, angles)"}
    if not args.no_verify:
        import oracle
        rows_o, Mo_rows = None, None
        cache = os.path.join(ROOT, "tests", "golden", "cache", f"{scene.name}_seed{scene.seed}.npz")
        rcache = os.path.join(ROOT, "tests", "golden", "cache", f"{scene.name}_seed{scene.seed}_rows.npz")
        if os.path.exists(cache) and N == 1000:
            z = np.load(cache, allow_pickle=False)
            rows_o = np.sort(np.random.default_rng(3).choice(F, 16, replace=False))
            Mo_rows = np.unpackbits(z["M"], axis=1)[rows_o, :F].astype(bool)
        elif os.path.exists(rcache):
            z = np.load(rcache, allow_pickle=False)
            rows_o = z["rows"][:16]
            Mo_rows = np.unpackbits(z["M"], axis=1)[:16, :F].astype(bool)
        if rows_o is not None:
            gm_rows = ivm.unpack_bits(M, F)[rows_o]
            Mo = np.zeros((F, F), bool)
            Mo[rows_o] = Mo_rows
            t0 = time.perf_counter()
            ao = oracle.angular_ranges(scene, Mo, rows=rows_o)
            out["angles"]["oracle_ms"] = 1e3 * (time.perf_counter() - t0)
            ok = bool((gm_rows == Mo_rows).all())
            go, gc, gr = aoff.cpu().numpy(), acols.cpu().numpy(), arng.cpu().numpy()
            for r in rows_o:
                a, b, oa, ob = go[r], go[r + 1], ao["offsets"][r], ao["offsets"][r + 1]
                ok &= bool((gc[a:b] == ao["cols"][oa:ob]).all() and
                           np.allclose(gr[a:b], ao["ranges"][oa:ob], rtol=1e-14, atol=1e-12))
            out["angles"]["oracle_sample"] = f"{len(rows_o)} whole rows of the oracle's matrix"
            out["angles"]["matches_oracle"] = ok
    progress(f"angular ranges: {out['angles']['ms']:.3f} ms, {out['angles']['pairs']} pairs")
    # image-tree candidate counts of orders up to 4 (the orders timed in Section IV-C)
    # over every snapshot of the table, outside the step
    times = []
    for k in range(args.warmup + args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c4 = ivm.ivm_image_tree_candidates(g, M, tv, rv, los, 4)
        e1.record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            times.append(e0.elapsed_time(e1))
    c4np = c4.cpu().numpy()
    # orders 3-4 are integer products on the matrix cores: U = T M, V = R M^T and
    # X = U M over two byte planes of U, 4 N F^2 int8 multiply-adds on the
    # unpadded shapes, against the dense int8 MFMA peak (5.0 POP/s)
    ops = 8.0 * N * F * F
    c4_ms = statistics.median(times)
    out["candidates_order4"] = {"gpu_ms": c4_ms, "snapshots": int(c4np.shape[0]),
                                "walks_per_order": [int(x) for x in c4np[:, 1:].sum(0)],
                                "roofline": {"bound": "mfma", "dtype": "i8", "achieved": ops / (c4_ms / 1e3) / 1e12,
                                             "peak": 5000.0, "unit": "TOP/s",
                                             "frac": ops / (c4_ms / 1e3) / 5.0e15,
                                             "ops_per_call": ops}}
    if not args.no_verify and os.path.exists(cache):
        import oracle
        z = np.load(cache, allow_pickle=False)
        pick = np.arange(0, int(z["los"].shape[0]), 10) if z["los"].shape[0] == c4np.shape[0] else np.arange(0)
        if len(pick):
            Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
            tvo = np.unpackbits(z["tx_vis"], axis=1)[pick, :F].astype(bool)
            rvo = np.unpackbits(z["rx_vis"], axis=1)[pick, :F].astype(bool)
            t0 = time.perf_counter()
            co4 = oracle.candidates_matmul(Mo, tvo, rvo, z["los"][pick], 4)
            out["candidates_order4"]["oracle_ms_sample"] = 1e3 * (time.perf_counter() - t0)
            out["candidates_order4"]["oracle_sample"] = f"every 10th snapshot ({len(pick)})"
            out["candidates_order4"]["matches_oracle"] = bool((c4np[pick] == co4).all())
    progress(f"candidates up to order 4: {statistics.median(times):.3f} ms")
    # exact image-method validation of the candidate lists (orders 1-2) of the
    # first 100 snapshots (Section III-A; the walks the pruned tree keeps)
    nv = min(N, 100)
    _, voff, vpaths = ivm.ivm_image_tree_candidates(g, M, tv[:nv], rv[:nv], los[:nv], 2, lists=True)
    times = []
    for k in range(min(args.warmup, 1) + min(args.steps, 3)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vst = ivm.new_stats()
        valid, vcounts = ivm.ivm_validate_paths(g, tx[:nv], rx[:nv], 2, voff, vpaths, stats=vst)
        torch.cuda.synchronize()
        if k >= min(args.warmup, 1):
            times.append(1e3 * (time.perf_counter() - t0))
    vc = vcounts.cpu().numpy()
    vs = ivm.stats_dict(vst)
    out["paths"] = {"ms": statistics.median(times), "snapshots": nv, "walks": int(counts[:nv, 1:3].sum().item()),
                    "valid_per_order": [int(x) for x in vc.sum(0)], "leg_tests": vs["tri_tests"],
                    "exact_tests": vs["rechecks"],
                    "note": "wall time of the whole call (it synchronises once to report undecided walks)"}
    cache = os.path.join(ROOT, "tests", "golden", "cache", f"{scene.name}_seed{scene.seed}.npz")
    if not args.no_verify and os.path.exists(cache) and N == 1000:
        import oracle
        z = np.load(cache, allow_pickle=False)
        pick = np.array([0, 50, 99])
        Mo = np.unpackbits(z["M"], axis=1)[:, :F].astype(bool)
        tvo = np.unpackbits(z["tx_vis"], axis=1)[pick, :F].astype(bool)
        rvo = np.unpackbits(z["rx_vis"], axis=1)[pick, :F].astype(bool)
        _, olists = oracle.candidates_enum(Mo, tvo, rvo, z["los"][pick], 2)
        rng = np.random.default_rng(6)
        walks = [(a, w) for a, per in enumerate(olists) for k in (1, 2) for w in per[k - 1]]
        sel = [walks[q] for q in rng.choice(len(walks), min(12, len(walks)), replace=False)]
        # one snapshot entry per selected walk: list (q, order 1) then (q, order 2)
        flat_all, offs, txs, rxs, first = [], [], [], [], []
        for a, w in sel:
            txs.append(scene.tx[pick[a]])
            rxs.append(scene.rx[pick[a]])
            for k in (1, 2):
                offs.append(len(flat_all))
                if len(w) == k:
                    first.append(len(flat_all))
                    flat_all.extend(w)
        offs.append(len(flat_all))
        offs = np.asarray(offs, np.int64)
        gv, _ = ivm.ivm_validate_paths(g, torch.as_tensor(np.array(txs, np.float32)).cuda(),
                                       torch.as_tensor(np.array(rxs, np.float32)).cuda(), 2,
                                       torch.as_tensor(offs).cuda(), torch.as_tensor(np.array(flat_all, np.int32)).cuda())
        gv = gv.cpu().numpy()
        ex = oracle._ExactImage(scene)
        t0 = time.perf_counter()
        ok = True
        for q, (a, w) in enumerate(sel):
            exp = bool(oracle.validate_paths_exact(scene, scene.tx[pick[a]], scene.rx[pick[a]], [w], ex=ex)[0])
            ok &= bool(gv[first[q]]) == exp
        out["paths"]["oracle_ms_per_walk"] = 1e3 * (time.perf_counter() - t0) / len(sel)
        out["paths"]["oracle_sample"] = f"{len(sel)} walks drawn from the oracle's own candidate lists"
        out["paths"]["matches_oracle"] = ok
    progress(f"path validation: {out['paths']['ms']:.2f} ms for the walks of {nv} snapshots")
    # building edges seen from Tx and Rx and the first-order diffraction candidates
    # Tx -> edge -> Rx (Section III-B), over the first 1000 snapshots at most
    E = int(scene.edge_facets.shape[0])
    if E:
        ne = min(N, 1000)
        ef = torch.as_tensor(scene.edge_facets).cuda()
        es = torch.as_tensor(scene.edge_samples).cuda()
        times = []
        for k in range(args.warmup + args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            te, re_, dc = ivm.ivm_edge_visibility(g, ef, es, scene.samples_per_edge, tx[:ne], rx[:ne])
            e1.record()
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(e0.elapsed_time(e1))
        gte, gre = ivm.unpack_bits(te, E), ivm.unpack_bits(re_, E)
        out["edges"] = {"gpu_ms": statistics.median(times), "snapshots": ne, "edges": E,
                        "samples_per_edge": int(scene.samples_per_edge),
                        "tx_edges_mean": float(gte.sum(1).mean()), "rx_edges_mean": float(gre.sum(1).mean()),
                        "diffraction_candidates": int(dc.sum().item())}
        if not args.no_verify:
            import oracle
            orc_e = oracle.Oracle(scene)
            pick = np.array(sorted({0, ne // 2, ne - 1}))
            t0 = time.perf_counter()
            ot = oracle.edge_visibility(orc_e, scene.tx[pick], scene.edge_facets, scene.edge_samples,
                                        scene.samples_per_edge)
            orr = oracle.edge_visibility(orc_e, scene.rx[pick], scene.edge_facets, scene.edge_samples,
                                         scene.samples_per_edge)
            out["edges"]["oracle_ms_per_point"] = 1e3 * (time.perf_counter() - t0) / (2 * len(pick))
            out["edges"]["oracle_sample"] = f"snapshots {pick.tolist()}, both ends"
            out["edges"]["matches_oracle"] = bool((gte[pick] == ot).all() and (gre[pick] == orr).all() and (
                dc.cpu().numpy()[pick] == oracle.diffraction_counts(ot, orr)).all())
        progress(f"edge visibility: {statistics.median(times):.3f} ms for {ne} snapshots")
    # edge rows of the matrix (edge to facet, edge to edge) for 64 seeded edges
    if E:
        rows_e = np.sort(np.random.default_rng(4).choice(E, min(E, 64), replace=False)).astype(np.int32)
        drows = torch.as_tensor(rows_e).cuda()
        times = []
        for k in range(args.warmup + args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            erf, ere = ivm.ivm_edge_rows(g, ef, es, scene.samples_per_edge, drows)
            e1.record()
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(e0.elapsed_time(e1))
        gef, gee = ivm.unpack_bits(erf, F), ivm.unpack_bits(ere, E)
        out["edge_rows"] = {"gpu_ms": statistics.median(times), "rows": len(rows_e), "edges": E,
                            "targets_per_row": F + E, "edge_facet_visible": int(gef.sum()),
                            "edge_edge_visible": int(gee.sum())}
        if not args.no_verify:
            import oracle
            t0 = time.perf_counter()
            oef, oee = oracle.edge_rows(oracle.Oracle(scene), scene.edge_facets, scene.edge_samples,
                                        scene.samples_per_edge, rows=rows_e[:2])
            out["edge_rows"]["oracle_ms_per_row"] = 1e3 * (time.perf_counter() - t0) / 2
            out["edge_rows"]["oracle_sample"] = "the first 2 of the 64 rows"
            out["edge_rows"]["matches_oracle"] = bool((gef[:2] == oef).all() and (gee[:2] == oee).all())
        progress(f"edge rows: {statistics.median(times):.3f} ms for {len(rows_e)} rows")
    if not args.no_verify:
        progress("verifying against the oracle")
        counts_now = counts
        out["verified"] = verify(ivm, scene, M, tv, rv, los, counts_now)
    if headline and not args.no_cpu_baseline:
        progress("timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_baseline_seconds)
        out["cpu_baseline"]["host"] = cpu_model()
        out["cpu_baseline"]["nproc"] = os.cpu_count()
    return out




if __name__ == "__main__":
    main()
