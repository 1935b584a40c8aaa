"""Interface relations on the GPU (ivm_interface_relations) against the oracle,
bit for bit, for matrices the oracle computed (tiny urban scenes, the plates
scene of the oracle pins with every pair visible) and the stored full oracle
matrix of the urban grid."""
import os
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu
CACHE = os.path.join(os.path.dirname(__file__), "golden", "cache", "c2_seed2.npz")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ivm():
    import torch
    import paper_2501_02747_amd as ivm
    assert torch.cuda.is_available()
    ivm.load_library()
    return ivm


def _pack(bits, W):
    N, F = bits.shape
    b = np.packbits(np.asarray(bits, np.uint8), axis=1, bitorder="little")
    out = np.zeros((N, W * 8), np.uint8)
    out[:, :b.shape[1]] = b
    return out.view(np.uint64)


def _check(oracle_mod, ivm, s, Mo):
    import torch
    g = ivm.GpuScene.from_scene(s).check()
    M = torch.as_tensor(_pack(Mo, g.W).view(np.int64)).cuda()
    par, per, cls = ivm.ivm_interface_relations(g, M)
    torch.cuda.synchronize()
    r = oracle_mod.interface_relations(s, Mo)
    F = s.n_facets
    assert (ivm.unpack_bits(par, F) == r["par"]).all()
    assert (ivm.unpack_bits(per, F) == r["per"]).all()
    assert (cls.cpu().numpy() == r["cls"]).all()
    return r


def test_plates_every_pair(oracle_mod, ivm):
    s = sg.gen_plates([
        [[-20, -20, 0], [40, 0, 0], [0, 40, 0]],
        [[0, 0, 0], [0, 0, 8], [0, 8, 0]],
        [[10, 0, 0], [0, 8, 0], [0, 0, 8]],
        [[0, 0, 0], [8, 0, 0], [0, 0, 8]],
        [[0, 0, 8], [8, 0, 0], [0, 8, 0]],
        [[20, 0, 0], [-4, 4, 0], [0, 0, 4]],
        [[0, 20, 0], [4, 0, 0], [0, 4, 4]],
    ])
    r = _check(oracle_mod, ivm, s, ~np.eye(s.n_facets, dtype=bool))
    assert r["par"].sum() == 4 and r["per"].sum() == 24


def test_tiny_urban_scenes(oracle_mod, ivm):
    for seed in (1, 2, 3):
        _log(f"[relations] tiny urban seed={seed}")
        s = sg.gen_c1(seed)
        Mo, _ = oracle_mod.Oracle(s).matrix()
        _check(oracle_mod, ivm, s, Mo)


@pytest.mark.skipif(not os.path.exists(CACHE), reason="full oracle cache not generated")
def test_urban_grid(oracle_mod, ivm):
    _log("[relations] urban grid from the oracle cache")
    s = sg.gen_c2(2)
    z = np.load(CACHE, allow_pickle=False)
    Mo = np.unpackbits(z["M"], axis=1)[:, :s.n_facets].astype(bool)
    r = _check(oracle_mod, ivm, s, Mo)
    assert r["par"].any() and r["per"].any()
