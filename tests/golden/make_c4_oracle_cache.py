"""Write seeded full-row and full-snapshot oracle results for the batched
workload (64 config-1 style urban scenes of 636-4856 facets, seeds 1000-1063,
4 x 4 samples, 100-2000 snapshots each), so GPU parity tests of the batched run
can compare whole rows and whole snapshots of every scene bit for bit.

Per scene: 2 seeded rows of the matrix, each against every other facet, and 2
seeded snapshots (every facet seen from the Tx and from the Rx, and LoS).

Calls only the FP64 oracle (oracle/) on inputs from scenegen.  Resumable per
scene.  Output: tests/golden/cache/c4_rows.npz (keys rows_k, snaps_k, M_k,
tx_k, rx_k, los_k for scene k = 00..63, bit-packed along facets).

    python tests/golden/make_c4_oracle_cache.py [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen as sg  # noqa: E402

OUT_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cache")
OUT = os.path.join(OUT_DIR, "c4_rows.npz")
PART = os.path.join(OUT_DIR, "c4_rows_partial.npz")
FIRST_SEED, N_SCENES = 1000, 64
N_ROWS, N_SNAPS = 2, 2


def selection(k: int, F: int, N: int):
    """The seeded rows and snapshots of scene k (sorted, distinct)."""
    rng = np.random.default_rng(40000 + k)
    rows = np.sort(rng.choice(F, N_ROWS, replace=False)).astype(np.int32)
    snaps = np.sort(rng.choice(N, N_SNAPS, replace=False)).astype(np.int32)
    return rows, snaps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    os.makedirs(OUT_DIR, exist_ok=True)
    out = {}
    if os.path.exists(PART):
        z = np.load(PART, allow_pickle=False)
        out = {k: z[k] for k in z.files}
    t0 = time.time()
    for k in range(N_SCENES):
        tag = f"{k:02d}"
        if f"los_{tag}" in out:
            continue
        s = sg.gen_c4_scene(FIRST_SEED + k)
        F, N = s.n_facets, s.n_snapshots
        rows, snaps = selection(k, F, N)
        orc = oracle.Oracle(s)
        M = np.zeros((N_ROWS, F), bool)
        for r, i in enumerate(rows):
            J = np.array([j for j in range(F) if j != i], np.int32)
            M[r, J] = orc.pairs(np.full(len(J), i, np.int32), J, threads=a.threads)
        tv, rv, los = orc.txrx(s.tx[snaps], s.rx[snaps], threads=a.threads)
        out.update({f"rows_{tag}": rows, f"snaps_{tag}": snaps, f"F_{tag}": np.int32(F),
                    f"M_{tag}": np.packbits(M, axis=1), f"tx_{tag}": np.packbits(tv, axis=1),
                    f"rx_{tag}": np.packbits(rv, axis=1), f"los_{tag}": los})
        np.savez_compressed(PART, **out)
        print(f"scene {k} ({F} facets) done, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
