"""Write seeded full-row and full-snapshot oracle results for the large-city
workload (4 x 4 km, 2000 convex 4-8-gon buildings, 19 872 facets, 4 x 4
samples, 10 000 snapshots of two vehicles, seed 3), so GPU parity tests can
compare whole rows and whole snapshots bit for bit.

* 64 seeded rows of the matrix, each against every other facet;
* 200 seeded snapshots: every facet seen from the Tx and from the Rx, and LoS.

Calls only the FP64 oracle (oracle/) on inputs from scenegen.  Resumable: rows
and snapshots are computed in blocks and saved as they finish.  Output:
tests/golden/cache/c3_seed3_rows.npz.

    python tests/golden/make_c3_oracle_cache.py [--threads N]
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
OUT = os.path.join(OUT_DIR, "c3_seed3_rows.npz")
PART = os.path.join(OUT_DIR, "c3_seed3_rows_partial.npz")
N_ROWS = 64
N_SNAPS = 200


def selection(F: int, N: int):
    """The seeded rows and snapshots (sorted, distinct)."""
    rng = np.random.default_rng(20250103)
    rows = np.sort(rng.choice(F, N_ROWS, replace=False)).astype(np.int32)
    snaps = np.sort(rng.choice(N, N_SNAPS, replace=False)).astype(np.int32)
    return rows, snaps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--row-block", type=int, default=4)
    ap.add_argument("--snap-block", type=int, default=5)
    a = ap.parse_args()
    os.makedirs(OUT_DIR, exist_ok=True)
    s = sg.gen_c3(3)
    F, N = s.n_facets, s.n_snapshots
    rows, snaps = selection(F, N)
    orc = oracle.Oracle(s)
    M = np.zeros((N_ROWS, F), bool)
    tv = np.zeros((N_SNAPS, F), bool)
    rv = np.zeros((N_SNAPS, F), bool)
    los = np.zeros(N_SNAPS, bool)
    row_done = np.zeros(N_ROWS, bool)
    snap_done = np.zeros(N_SNAPS, bool)
    if os.path.exists(PART):
        z = np.load(PART, allow_pickle=False)
        M, tv, rv, los, row_done, snap_done = (z[k] for k in ("M", "tx_vis", "rx_vis", "los", "row_done", "snap_done"))

    def save():
        np.savez_compressed(PART, M=M, tx_vis=tv, rx_vis=rv, los=los, row_done=row_done, snap_done=snap_done)

    t0 = time.time()
    for b0 in range(0, N_ROWS, a.row_block):
        idx = [k for k in range(b0, min(N_ROWS, b0 + a.row_block)) if not row_done[k]]
        if not idx:
            continue
        I = np.concatenate([np.full(F, rows[k]) for k in idx]).astype(np.int32)
        J = np.concatenate([np.arange(F) for _ in idx]).astype(np.int32)
        keep = I != J
        r = np.zeros(len(I), bool)
        r[keep] = orc.pairs(I[keep], J[keep], threads=a.threads)
        M[idx] = r.reshape(len(idx), F)
        row_done[idx] = True
        save()
        print(f"rows {b0}..{b0 + len(idx) - 1} done, {time.time() - t0:.0f} s", flush=True)
    for b0 in range(0, N_SNAPS, a.snap_block):
        idx = [k for k in range(b0, min(N_SNAPS, b0 + a.snap_block)) if not snap_done[k]]
        if not idx:
            continue
        n = snaps[idx]
        t, r, l = orc.txrx(s.tx[n], s.rx[n], threads=a.threads)
        tv[idx], rv[idx], los[idx] = t, r, l
        snap_done[idx] = True
        save()
        print(f"snapshots {b0}..{b0 + len(idx) - 1} done, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, rows=rows, snaps=snaps, M=np.packbits(M, axis=1), tx_vis=np.packbits(tv, axis=1),
                        rx_vis=np.packbits(rv, axis=1), los=los, F=F)
    print("wrote", OUT, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
