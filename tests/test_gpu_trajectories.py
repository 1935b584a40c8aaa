"""Tx/Rx tables along hand-made trajectories, bit for bit against the FP64 oracle.

The table kernel follows each chunk of samples from one point of a trajectory
to the next and tests first what blocked a sample at the previous point; over
a block of points it also tries one certificate for the box of those points.
These cases make that history wrong on purpose, on a 200-facet Manhattan grid
(streets at known places): points that jump between two far corners at every
snapshot, movers that cross street after street (shadow edges at every few
steps), a fixed point, a snapshot count that is not a multiple of the block and
blocks shorter than the certificate's minimum.  Positions are on the 1/128 m
grid of the scene.
"""
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ivm():
    import torch
    import paper_2501_02747_amd as ivm
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ivm.load_library()
    return ivm


@pytest.fixture(scope="module")
def grid():
    return sg.gen_c2(2, n_snap=8, nx=4, ny=5)


def _pts(a):
    a = np.asarray(a, np.float64)
    q = np.round(a * 128.0) / 128.0
    assert (q == a).all()
    return q.astype(np.float32)


def _trajectories():
    # north-south street centres x = -110, -10, 90, 190; east-west y = -85, -35, 15, 65, 115
    jump_a, jump_b = (-110.0, -85.0, 1.5), (190.0, 115.0, 1.5)
    out = {}
    n = 77
    out["jumps"] = (_pts([(90.0, 15.0, 30.0)] * n), _pts([jump_a if k % 2 == 0 else jump_b for k in range(n)]))
    n = 96
    out["crossing"] = (_pts([(-190.0 + 4.0 * k, 15.0, 20.0) for k in range(n)]),
                       _pts([(-10.0, -120.0 + 2.5 * k, 1.5) for k in range(n)]))
    n = 70
    out["fixed"] = (_pts([(-10.0, -35.0, 25.0)] * n), _pts([(90.0 - 0.25 * k, 65.0, 1.5) for k in range(n)]))
    rng = np.random.default_rng(7)
    xs = np.array([-110.0, -10.0, 90.0, 190.0])
    ys = np.array([-85.0, -35.0, 15.0, 65.0, 115.0])
    n = 5
    out["short"] = (_pts([(xs[rng.integers(4)], ys[rng.integers(5)], 12.0) for _ in range(n)]),
                    _pts([(xs[rng.integers(4)], -120.0 + 240.0 * rng.integers(0, 97) / 96.0, 1.5) for _ in range(n)]))
    return out


@pytest.mark.parametrize("name", ["jumps", "crossing", "fixed", "short"])
@pytest.mark.parametrize("fp64", [False, True])
def test_table_along_trajectory(oracle_mod, ivm, grid, name, fp64):
    import torch
    _log(f"[trajectory] {name} fp64={fp64}")
    tx, rx = _trajectories()[name]
    orc = oracle_mod.Oracle(grid)
    tvo, rvo, loso = orc.txrx(tx, rx)
    g = ivm.GpuScene.from_scene(grid).check()
    tv, rv, los = ivm.ivm_txrx_visibility_table(g, torch.as_tensor(tx).cuda(), torch.as_tensor(rx).cuda(),
                                                ivm.make_opts(fp64_only=fp64))
    torch.cuda.synchronize()
    assert g.status() == 0
    F = grid.n_facets
    assert (ivm.unpack_bits(tv, F) == tvo).all(), np.argwhere(ivm.unpack_bits(tv, F) != tvo)[:5]
    assert (ivm.unpack_bits(rv, F) == rvo).all(), np.argwhere(ivm.unpack_bits(rv, F) != rvo)[:5]
    assert (los.cpu().numpy().astype(bool) == loso).all()
    # the cases really do see something and miss something
    assert tvo.any() and rvo.any() and not tvo.all() and not rvo.all()
