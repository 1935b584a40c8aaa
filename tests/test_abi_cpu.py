"""CPU-side checks of the C ABI library: it loads, exports every declared
symbol, and its host-only entry points validate arguments.  No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ivm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ivm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2501_02747_amd as ivm
    if not os.path.exists(ivm.LIB_PATH):
        ivm_build = __import__("paper_2501_02747_amd.build", fromlist=["build"])
        ivm_build.build()
    return ivm.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    import paper_2501_02747_amd as ivm
    assert sorted(ivm.EXPORTED) == names


def test_status_strings(lib):
    import paper_2501_02747_amd as ivm
    for code, name in [(0, "IVM_OK"), (-1, "IVM_ERR_INVALID_ARGUMENT"), (-2, "IVM_ERR_WORKSPACE"),
                       (-3, "IVM_ERR_GRID"), (-4, "IVM_ERR_DEGENERATE"), (-5, "IVM_ERR_HIP"),
                       (-6, "IVM_ERR_CAPACITY"), (-7, "IVM_ERR_MODEL")]:
        assert ivm.status_string(code) == name


def test_workspace_size_host_only(lib):
    import paper_2501_02747_amd as ivm
    d = ivm.ivm_scene_desc()
    d.n_vertices, d.n_triangles, d.n_facets, d.n_samples = 168, 84, 42, 672
    d.vertices = d.tri_vertices = d.tri_facet = d.sample_offsets = d.samples = 1  # never dereferenced
    d.grid_vertex_log2, d.grid_sample_log2 = 4, 7
    n = ctypes.c_size_t(0)
    assert lib.ivm_scene_workspace_size(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value > 84 * 48 + 84 * 64
    d.flags = ivm.IVM_SCENE_LEARNED
    n2 = ctypes.c_size_t(0)
    assert lib.ivm_scene_workspace_size(ctypes.byref(d), ctypes.byref(n2)) == 0
    assert n2.value >= n.value + 42 * 41 // 2 * 8 - 256   # the empty reservation still takes one 256 B slot
    # invalid descriptions are refused before any device work
    d.n_facets = -1
    assert lib.ivm_scene_workspace_size(ctypes.byref(d), ctypes.byref(n)) == ivm.IVM_ERR_INVALID_ARGUMENT
    d.n_facets, d.grid_sample_log2 = 42, 3       # sample grid coarser than vertex grid
    assert lib.ivm_scene_workspace_size(ctypes.byref(d), ctypes.byref(n)) == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_scene_workspace_size(None, ctypes.byref(n)) == ivm.IVM_ERR_INVALID_ARGUMENT


def test_null_arguments_rejected_without_gpu(lib):
    import paper_2501_02747_amd as ivm
    assert lib.ivm_intervisibility_matrix(None, None, None, None, None) == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_txrx_visibility_table(None, None, 0, None, None, None, None, None, None, None) \
        == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_image_tree_candidates(None, None, 0, None, None, None, 2, None, None, None, 0, None) \
        == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_destroy_scene(None) == ivm.IVM_ERR_INVALID_ARGUMENT
    for k in (0, 5):   # orders beyond 1..4
        assert lib.ivm_image_tree_candidates(None, None, 0, None, None, None, k, None, None, None, 0, None) \
            == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_edge_visibility(None, None, 0, 4, None, None, 0, None, None, None, None, None, None) \
        == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_interface_relations(None, None, None, None, None, None) == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_angular_ranges(None, None, None, None, None, 0, None) == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_edge_rows(None, None, 0, 4, None, None, 0, None, None, None, None) == ivm.IVM_ERR_INVALID_ARGUMENT
    for s in (0, 65):   # samples per edge beyond 1..64
        assert lib.ivm_edge_rows(None, None, 4, s, None, None, 1, None, None, None, None) \
            == ivm.IVM_ERR_INVALID_ARGUMENT
    sz = ctypes.c_size_t(0)
    assert lib.ivm_visibility_ranges_workspace_size(0, ctypes.byref(sz)) == ivm.IVM_ERR_INVALID_ARGUMENT
    assert lib.ivm_visibility_ranges_workspace_size(1000, ctypes.byref(sz)) == 0 and sz.value >= 1000 * 52
    out = ctypes.c_void_p()
    assert lib.ivm_build_scene(None, None, 0, None, ctypes.byref(out)) == ivm.IVM_ERR_INVALID_ARGUMENT
    # the allocation-free ranges call: null arguments, and a trajectory beyond its
    # fixed scratch is refused before the scene or any device memory is touched
    nul = [None] * 6
    assert lib.ivm_visibility_ranges_noalloc(None, 10, *[None] * 5, 0.01, *nul, None) \
        == ivm.IVM_ERR_INVALID_ARGUMENT
    fake = [1] * 5                                 # never dereferenced
    assert lib.ivm_visibility_ranges_noalloc(1, ivm.IVM_RANGES_NOALLOC_MAX_SNAP + 1, *fake, 0.01, *[1] * 6, None) \
        == ivm.IVM_ERR_WORKSPACE
    assert lib.ivm_visibility_ranges_noalloc(1, 10, *fake, 0.0, *[1] * 6, None) == ivm.IVM_ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("n", [1, 63, 64, 65, 130])
def test_pack_unpack_roundtrip(n):
    import paper_2501_02747_amd as ivm
    rng = np.random.default_rng(n)
    bits = rng.random((3, n)) < 0.5
    words = ivm.pack_bits(bits)
    assert words.shape == (3, (n + 63) // 64)
    assert (ivm.unpack_bits(words, n) == bits).all()
    # bit j of a row is word j >> 6, bit j & 63
    one = np.zeros((1, n), bool)
    one[0, n - 1] = True
    w = ivm.pack_bits(one).view(np.uint64)
    assert w[0, (n - 1) >> 6] == np.uint64(1) << np.uint64((n - 1) & 63)


def test_he_uniform_init_layout():
    """Host side of the training script: the flat parameter vector has the
    library's size and layout (W0, b0, W1, b1, ...), weights within the He-uniform
    bound sqrt(6 / fan_in), zero biases, and the same vector for the same seed;
    the shipped weights have the same size and are finite."""
    import paper_2501_02747_amd as ivm
    from paper_2501_02747_amd import train
    sizes = (24, 128, 128, 128, 32)
    v = train.he_uniform_init(3)
    assert v.dtype == np.float32 and v.shape == (ivm.IVM_MLP_PARAMS,)
    assert (v == train.he_uniform_init(3)).all() and not (v == train.he_uniform_init(4)).all()
    o = 0
    for l in range(len(sizes) - 1):
        n_w = sizes[l] * sizes[l + 1]
        w, b = v[o:o + n_w], v[o + n_w:o + n_w + sizes[l + 1]]
        bound = np.sqrt(6.0 / sizes[l])
        assert np.abs(w).max() <= bound and np.abs(w).max() > 0.9 * bound
        assert (b == 0).all()
        o += n_w + sizes[l + 1]
    assert o == ivm.IVM_MLP_PARAMS
    shipped = np.load(train.DEFAULT_WEIGHTS, allow_pickle=False)
    assert shipped.size == ivm.IVM_MLP_PARAMS and np.isfinite(shipped).all()
