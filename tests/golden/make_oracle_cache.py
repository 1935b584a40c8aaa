"""Write full-size oracle results for the urban-grid workload (1 x 1 km, 2000
facets, 8 x 8 samples, seed 2) so GPU parity tests can compare every bit.

Calls only the FP64 oracle (oracle/) on inputs from scenegen.  Resumable: rows
are computed in blocks and saved as they finish.  Output:
tests/golden/cache/c2_seed2.npz with the row-packed matrix, the Tx/Rx tables
and LoS for all 1000 snapshots.

    python tests/golden/make_oracle_cache.py [--threads N]
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
OUT = os.path.join(OUT_DIR, "c2_seed2.npz")
PART = os.path.join(OUT_DIR, "c2_seed2_partial.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--block", type=int, default=40)
    a = ap.parse_args()
    os.makedirs(OUT_DIR, exist_ok=True)
    s = sg.gen_c2(2)
    orc = oracle.Oracle(s)
    F = s.n_facets
    M = np.zeros((F, F), bool)
    done = np.zeros(F, bool)
    if os.path.exists(PART):
        z = np.load(PART)
        M, done = z["M"], z["done"]
    t0 = time.time()
    for r0 in range(0, F, a.block):
        rows = [i for i in range(r0, min(F, r0 + a.block)) if not done[i]]
        if not rows:
            continue
        I = np.concatenate([np.full(F - i - 1, i) for i in rows]).astype(np.int32)
        J = np.concatenate([np.arange(i + 1, F) for i in rows]).astype(np.int32)
        r = orc.pairs(I, J, threads=a.threads)
        M[I, J] = r
        M[J, I] = r
        done[rows] = True
        np.savez_compressed(PART, M=M, done=done)
        print(f"rows {r0}..{r0 + a.block - 1} done, {time.time() - t0:.0f} s", flush=True)
    tv, rv, los = orc.txrx(s.tx, s.rx, threads=a.threads)
    np.savez_compressed(OUT, M=np.packbits(M, axis=1), tx_vis=np.packbits(tv, axis=1),
                        rx_vis=np.packbits(rv, axis=1), los=los, F=F)
    print("wrote", OUT, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
