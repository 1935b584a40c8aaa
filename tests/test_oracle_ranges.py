"""Pins for the visibility ranges and coherence times along a trajectory
(Section III-C: visibility change nodes of a mobile Tx / Rx; Section III-D,
eq. 8: T_c,l = d_l / v_l; the smaller of the Tx-side and Rx-side values when
both move; eq. 9: the mean over the ranges).  Every expected value below is
derived by hand from those definitions."""
import math

import numpy as np
import pytest

N, F, DT = 20, 5, 0.01


def _traj(v_tx=0.0, v_rx=0.0):
    """Straight lines at constant speed along x (metres per snapshot step)."""
    tx = np.zeros((N, 3), np.float32)
    rx = np.zeros((N, 3), np.float32)
    tx[:, 0] = np.arange(N) * v_tx * DT
    rx[:, 0] = np.arange(N) * v_rx * DT
    rx[:, 2] = 1.5
    return tx, rx


def _tables():
    return np.zeros((N, F), bool), np.zeros((N, F), bool), np.zeros(N, bool)


def test_no_change_one_range(oracle_mod):
    """Constant tables, the Rx moving: one range lasting the whole trajectory."""
    tv, rv, los = _tables()
    tv[:, 1] = rv[:, 2] = True
    tx, rx = _traj(v_rx=25.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0]
    assert (r["events"] == 0).all()
    assert r["tc"][0] == pytest.approx((N - 1) * DT, rel=1e-12)
    assert r["mean"] == pytest.approx((N - 1) * DT, rel=1e-12)


def test_single_creation_splits_the_trajectory(oracle_mod):
    """Facet 3 becomes visible from the moving Rx at snapshot 7: a creation
    point, ranges [0, 7) and [7, N - 1] of 7 dt and (N - 8) dt."""
    tv, rv, los = _tables()
    rv[7:, 3] = True
    tx, rx = _traj(v_rx=30.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, 7]
    assert r["events"][7].tolist() == [0, 0, 1, 0, 0]
    assert r["events"].sum() == 1
    assert r["tc"] == pytest.approx([7 * DT, (N - 8) * DT], rel=1e-12)
    assert r["mean"] == pytest.approx((7 + N - 8) * DT / 2, rel=1e-12)


def test_two_movers_take_the_smaller_side(oracle_mod):
    """Tx-side change at 5, Rx-side change at 12: combined ranges [0,5), [5,12),
    [12, N-1]; each takes min(Tx-side range time, Rx-side range time)."""
    tv, rv, los = _tables()
    tv[5:, 0] = True           # created from the Tx at 5
    rv[:12, 4] = True          # suppressed from the Rx at 12
    tx, rx = _traj(v_tx=10.0, v_rx=20.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, 5, 12]
    assert r["events"][5].tolist() == [1, 0, 0, 0, 0]
    assert r["events"][12].tolist() == [0, 0, 0, 1, 0]
    tx_sides = [5 * DT, (N - 1 - 5) * DT]       # Tx ranges [0,5), [5,N-1]
    rx_sides = [12 * DT, (N - 1 - 12) * DT]     # Rx ranges [0,12), [12,N-1]
    want = [min(tx_sides[0], rx_sides[0]), min(tx_sides[1], rx_sides[0]), min(tx_sides[1], rx_sides[1])]
    assert r["tc"] == pytest.approx(want, rel=1e-12)
    assert r["mean"] == pytest.approx(sum(want) / 3, rel=1e-12)


def test_stationary_side_sets_no_limit(oracle_mod):
    """A fixed Tx (its visible set constant) leaves the Rx side alone to decide."""
    tv, rv, los = _tables()
    tv[:, :] = True
    rv[3:, 0] = True
    rv[11:, 1] = True
    tx, rx = _traj(v_tx=0.0, v_rx=33.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, 3, 11]
    assert r["tc"] == pytest.approx([3 * DT, 8 * DT, (N - 1 - 11) * DT], rel=1e-12)


def test_nobody_moves(oracle_mod):
    tv, rv, los = _tables()
    rv[9:, 0] = True
    tx, rx = _traj()
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, 9]
    assert all(math.isinf(t) for t in r["tc"]) and math.isinf(r["mean"])


def test_los_change_ends_both_sides(oracle_mod):
    """A LoS suppression at 6 is a change for either side; Tx-side d = 0 keeps
    the Tx out of the minimum, so the Rx durations remain."""
    tv, rv, los = _tables()
    los[:6] = True
    tx, rx = _traj(v_rx=12.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, 6]
    assert r["events"][6].tolist() == [0, 0, 0, 0, -1]
    assert r["tc"] == pytest.approx([6 * DT, (N - 7) * DT], rel=1e-12)


def test_change_at_the_last_snapshot(oracle_mod):
    """A change at N - 1 opens a range of zero duration: no coherence limit
    (d = 0), and it stays out of the mean."""
    tv, rv, los = _tables()
    rv[N - 1, 0] = True
    tx, rx = _traj(v_rx=5.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, N - 1]
    assert r["tc"][0] == pytest.approx((N - 1) * DT, rel=1e-12)
    assert math.isinf(r["tc"][1])
    assert r["mean"] == pytest.approx((N - 1) * DT, rel=1e-12)


def test_route_distance_uses_the_path_not_the_chord(oracle_mod):
    """The Rx goes 3 m along x, then 4 m along y, 1 m per step: with a change
    at snapshot 4 the Rx covers 3 + 1 = 4 m in the first range and 3 m in the
    second (the chord of the first would be sqrt(10) m); the fixed Tx covers 0."""
    n = 8
    tv = np.zeros((n, 2), bool)
    rv = np.zeros((n, 2), bool)
    los = np.zeros(n, bool)
    tx = np.zeros((n, 3), np.float32)
    rx = np.zeros((n, 3), np.float32)
    for k in range(1, n):
        rx[k] = rx[k - 1] + (np.array([1, 0, 0]) if k <= 3 else np.array([0, 1, 0]))
    rv[4:, 0] = True
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    assert r["starts"].tolist() == [0, 4]
    assert r["dist"].tolist() == [[0.0, 4.0], [0.0, 3.0]]
    assert r["tc"] == pytest.approx([4 * DT, 3 * DT], rel=1e-12)


def test_counts_against_set_differences(oracle_mod):
    """Random tables: creation / suppression counts equal the set sizes."""
    rng = np.random.default_rng(3)
    tv = rng.random((N, F)) < 0.5
    rv = rng.random((N, F)) < 0.5
    los = rng.random(N) < 0.5
    tx, rx = _traj(v_tx=3.0, v_rx=7.0)
    r = oracle_mod.visibility_ranges(tv, rv, los, tx, rx, DT)
    for n in range(1, N):
        a, b = set(np.nonzero(tv[n - 1])[0]), set(np.nonzero(tv[n])[0])
        c, d = set(np.nonzero(rv[n - 1])[0]), set(np.nonzero(rv[n])[0])
        assert r["events"][n].tolist() == [len(b - a), len(a - b), len(d - c), len(c - d),
                                           int(los[n]) - int(los[n - 1])]
    starts = [0] + [n for n in range(1, N) if a_change(tv, rv, los, n)]
    assert r["starts"].tolist() == starts


def a_change(tv, rv, los, n):
    return (tv[n] != tv[n - 1]).any() or (rv[n] != rv[n - 1]).any() or los[n] != los[n - 1]
