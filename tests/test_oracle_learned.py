"""Pins for the learned-ordering parts of the oracle (CPU only): pair features on
a hand-computed scene, BF16 rounding, and the BF16-operand reference agreeing
with the plain FP64 reference when the operands are already BF16 values."""
import numpy as np

import scenegen as sg


def test_pair_features_by_hand(oracle_mod):
    # P: 4x4 plate at z=0 facing +z; Q: 4x4 plate at z=10 facing -z.
    # Vertex box [0,4]x[0,4]x[0,10]: centre (2,2,5), half-size 5.
    s = sg.gen_plates([[[0, 0, 0], [4, 0, 0], [0, 4, 0]], [[0, 0, 10], [0, 4, 0], [4, 0, 0]]])
    x = oracle_mod.pair_features(s, [0], [1])[0]
    expect = np.array([0, 0, -1, 0, 0, 1,            # centroids (2,2,0) and (2,2,10), normalised
                       0, 0, 1, 0, 0, -1,            # unit normals
                       16 / 25, 16 / 25,             # areas / s^2
                       2,                            # distance between normalised centroids
                       -0.4, -0.4, -1, 0.4, 0.4, 1,  # AABB of both facets, normalised
                       0, 0, 1])                     # direction
    assert np.allclose(x, expect, atol=1e-12)
    # swapping the pair swaps the per-facet groups and flips the direction
    y = oracle_mod.pair_features(s, [1], [0])[0]
    assert np.allclose(y[:3], x[3:6]) and np.allclose(y[21:], -x[21:])


def test_bf16_rounding_cases(oracle_mod):
    e = 2.0 ** -7                      # BF16 spacing at 1.0 (7 stored mantissa bits)
    vals = np.array([1.0, 1.0 + e / 2, 1.0 + 3 * e / 2, 1.0 + e / 2 + 2 ** -20, -2.5, 0.0, 3.0e38])
    r = oracle_mod.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie -> even
    assert r[2] == 1.0 + 2 * e         # tie -> even (odd 1+e rounds up)
    assert r[3] == 1.0 + e             # above the tie
    assert r[4] == -2.5 and r[5] == 0.0
    assert np.isfinite(r[6])


def test_bf16_reference_equals_fp64_on_bf16_operands(oracle_mod):
    """When weights and inputs are already BF16 values and the network is one
    linear layer, rounding operands changes nothing."""
    rng = np.random.default_rng(0)
    p = {"W0": oracle_mod.bf16_round(rng.normal(size=(32, 24))), "b0": rng.normal(size=32)}
    X = oracle_mod.bf16_round(rng.normal(size=(5, 24)))
    z1, _ = oracle_mod.mlp_forward(p, X, bf16=False)
    z2, _ = oracle_mod.mlp_forward(p, X, bf16=True)
    assert np.array_equal(z1, z2)


def test_flatten_layout(oracle_mod):
    p = oracle_mod.mlp_init(3)
    v = oracle_mod.mlp_flatten(p)
    assert v.size == 40352
    # W0 first (row-major 128 x 24), then b0, then W1 ...
    assert np.array_equal(v[:24], p["W0"][0]) and np.array_equal(v[3072:3200], p["b0"])
    q = oracle_mod.mlp_unflatten(v)
    assert all(np.array_equal(p[k], q[k]) for k in p)
