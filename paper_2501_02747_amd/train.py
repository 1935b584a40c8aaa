"""Training of the occluder-ordering network on hit records produced by the GPU path.

A hit record is a facet pair with at least one blocked admissible segment; its
label is the 32-bit mask of treelets holding a blocking triangle
(ivm_pair_occluder_labels).  Features come from ivm_pair_features; training runs
the library's own forward, backward and Adam kernels (ivm_model_train_step).

    python -m paper_2501_02747_amd.train --out paper_2501_02747_amd/models/occluder_mlp.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from . import (IVM_MLP_OUTPUTS, IVM_MODEL_BF16, GpuScene, Model, ivm_pair_features, ivm_pair_occluder_labels)

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "models", "occluder_mlp.npy")


def he_uniform_init(seed: int, sizes=(24, 128, 128, 128, 32)) -> np.ndarray:
    """He-uniform weights, zero biases, flattened as W0, b0, W1, b1, ... (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(sizes) - 1):
        bound = np.sqrt(6.0 / sizes[l])
        parts.append(rng.uniform(-bound, bound, size=(sizes[l + 1], sizes[l])).ravel())
        parts.append(np.zeros(sizes[l + 1]))
    return np.concatenate(parts).astype(np.float32)


def collect_records(scene_arrays, n_pairs: int, seed: int, chunk: int = 65536):
    """Random unordered pairs of one scene -> (features [m, 24], labels [m, 32]) for
    the pairs whose label is non-zero."""
    import torch
    g = GpuScene.from_scene(scene_arrays).check()
    rng = np.random.default_rng(seed)
    F = g.F
    xs, ys = [], []
    for c0 in range(0, n_pairs, chunk):
        m = min(chunk, n_pairs - c0)
        I = rng.integers(0, F, m)
        J = rng.integers(0, F, m)
        keep = I != J
        I, J = np.minimum(I, J)[keep], np.maximum(I, J)[keep]
        dI = torch.as_tensor(I.astype(np.int32)).cuda()
        dJ = torch.as_tensor(J.astype(np.int32)).cuda()
        lab = ivm_pair_occluder_labels(g, dI, dJ)
        x = ivm_pair_features(g, dI, dJ)
        lab_np = lab.cpu().numpy().view(np.uint32)
        nz = lab_np != 0
        bits = ((lab_np[nz, None] >> np.arange(IVM_MLP_OUTPUTS, dtype=np.uint32)) & 1).astype(np.float32)
        xs.append(x.cpu().numpy()[nz])
        ys.append(bits)
    return np.concatenate(xs), np.concatenate(ys)


def train(model: Model, X: np.ndarray, Y: np.ndarray, epochs: int = 3, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Minibatch Adam over shuffled records; returns the mean loss of each epoch."""
    import torch
    rng = np.random.default_rng(seed)
    dX = torch.as_tensor(np.ascontiguousarray(X, np.float32)).cuda()
    dY = torch.as_tensor(np.ascontiguousarray(Y, np.float32)).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    history = []
    n = X.shape[0]
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n)).cuda()
        total, steps = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb, yb = dX[idx].contiguous(), dY[idx].contiguous()
            model.train_step(xb, yb, lr, loss)
            total += float(loss.item()) if steps % 50 == 0 else 0.0
            steps += 1
        # exact epoch loss on a fixed slice for the log
        m = min(n, 8 * batch)
        l_eval, _ = model.loss_grad(dX[:min(m, model.max_batch)].contiguous(), dY[:min(m, model.max_batch)].contiguous())
        history.append(float(l_eval.item()))
        if log:
            log(f"epoch {ep + 1}: loss {history[-1]:.4f} ({steps} steps)")
    return history


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--seeds", default="200-209")
    ap.add_argument("--pairs-per-scene", type=int, default=400000)
    ap.add_argument("--records", type=int, default=1000000)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--lr", type=float, default=1e-3)
    a = ap.parse_args()
    import scenegen as sg
    lo, hi = (int(v) for v in a.seeds.split("-"))
    t0 = time.time()
    Xs, Ys = [], []
    for seed in range(lo, hi + 1):
        X, Y = collect_records(sg.gen_c2(seed, n_snap=1), a.pairs_per_scene, seed)
        Xs.append(X)
        Ys.append(Y)
        print(f"[train] scene seed {seed}: {len(X)} hit records ({time.time() - t0:.1f} s)", flush=True)
    X, Y = np.concatenate(Xs)[:a.records], np.concatenate(Ys)[:a.records]
    model = Model(max_batch=8192, precision=IVM_MODEL_BF16)
    model.set_params(he_uniform_init(0))
    hist = train(model, X, Y, epochs=a.epochs, lr=a.lr, log=lambda m: print("[train]", m, flush=True))
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.save(a.out, model.get_params().cpu().numpy())
    print(f"[train] {len(X)} records, losses {hist}, wrote {a.out} ({time.time() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    sys.exit(main())
