"""Python binding of libivm (facet inter-visibility pre-processing on MI355X).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of ``libivm.so`` behind the C ABI of ``include/ivm.h``.  PyTorch supplies device
memory and the current HIP stream.  There is no CPU fallback: if the library is
missing or no GPU is present, the calls raise.

The functions below carry the names of the C entry points; ``GpuScene`` bundles
a scene handle with the device tensors it references.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libivm.so")

IVM_OK = 0
IVM_ERR_INVALID_ARGUMENT = -1
IVM_ERR_WORKSPACE = -2
IVM_ERR_GRID = -3
IVM_ERR_DEGENERATE = -4
IVM_ERR_HIP = -5
IVM_ERR_CAPACITY = -6
IVM_ERR_MODEL = -7

IVM_ORDER_PLAIN, IVM_ORDER_LEARNED, IVM_ORDER_INDEX, IVM_ORDER_REVERSED = 0, 1, 2, 3
IVM_SCENE_LEARNED = 1
IVM_MAX_STACK = 24

EXPORTED = [
    "ivm_status_string", "ivm_scene_workspace_size", "ivm_build_scene", "ivm_scene_status",
    "ivm_scene_info", "ivm_destroy_scene", "ivm_intervisibility_matrix",
    "ivm_txrx_visibility_table", "ivm_image_tree_candidates", "ivm_triangle_groups", "ivm_visibility_ranges",
    "ivm_visibility_ranges_workspace_size", "ivm_visibility_ranges_noalloc", "ivm_interface_relations",
    "ivm_edge_visibility", "ivm_edge_rows", "ivm_angular_ranges", "ivm_validate_paths",
    "ivm_model_workspace_size", "ivm_model_create", "ivm_model_destroy", "ivm_model_set_params",
    "ivm_model_get_params", "ivm_model_forward", "ivm_model_loss_grad", "ivm_model_train_step",
    "ivm_pair_features", "ivm_pair_occluder_labels", "ivm_scene_set_model",
    "ivm_batch_workspace_size", "ivm_batch_create", "ivm_batch_run", "ivm_batch_destroy",
    "ivm_scene_solids",
]

IVM_MLP_FEATURES, IVM_MLP_HIDDEN, IVM_MLP_OUTPUTS, IVM_MLP_PARAMS = 24, 128, 32, 40352
IVM_MODEL_BF16, IVM_MODEL_FP32 = 0, 1


class IvmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class ivm_scene_desc(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int32), ("n_triangles", ctypes.c_int32),
        ("n_facets", ctypes.c_int32), ("n_samples", ctypes.c_int32),
        ("vertices", ctypes.c_void_p), ("tri_vertices", ctypes.c_void_p),
        ("tri_facet", ctypes.c_void_p), ("sample_offsets", ctypes.c_void_p),
        ("samples", ctypes.c_void_p),
        ("grid_vertex_log2", ctypes.c_int32), ("grid_sample_log2", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("facet_solid", ctypes.c_void_p), ("n_solids", ctypes.c_int32),
    ]


class ivm_scene_info_t(ctypes.Structure):
    _fields_ = [
        ("n_facets", ctypes.c_int32), ("n_triangles", ctypes.c_int32),
        ("n_samples", ctypes.c_int32), ("words_per_row", ctypes.c_int32),
        ("n_treelets", ctypes.c_int32), ("max_samples_per_facet", ctypes.c_int32),
        ("n_nodes", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t),
    ]


class ivm_matrix_opts(ctypes.Structure):
    _fields_ = [
        ("order_mode", ctypes.c_int32), ("fp64_only", ctypes.c_int32),
        ("stack_depth", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
        ("eps", ctypes.c_float), ("no_tile", ctypes.c_int32),
        ("exhaustive", ctypes.c_int32),
        ("timing_events", ctypes.c_void_p),
        ("tile_cap", ctypes.c_int32), ("tile_treelets", ctypes.c_int32), ("pair_chunk", ctypes.c_int32),
        ("xcd_parts", ctypes.c_int32),
    ]


STATS_FIELDS = ["pairs_total", "pairs_candidate", "pairs_visible", "segments", "box_tests",
                "tri_tests", "rechecks", "fallbacks", "point_items", "flags", "certified",
                "subpair_runs", "tiled_pairs", "solid_certified", "traversed", "solid_segments", "solid_planes"]
STATS_WORDS = 20

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libivm.so (torch is imported first so the process has one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (brings in torch's HIP runtime before ours)
    if not os.path.exists(path):
        raise ImportError(f"libivm.so not built at {path}; run paper_2501_02747_amd/build.py")
    lib = ctypes.CDLL(path)
    P, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.ivm_status_string.restype = ctypes.c_char_p
    lib.ivm_status_string.argtypes = [i32]
    lib.ivm_scene_workspace_size.restype = i32
    lib.ivm_scene_workspace_size.argtypes = [ctypes.POINTER(ivm_scene_desc), ctypes.POINTER(sz)]
    lib.ivm_build_scene.restype = i32
    lib.ivm_build_scene.argtypes = [ctypes.POINTER(ivm_scene_desc), P, sz, P, ctypes.POINTER(P)]
    lib.ivm_scene_status.restype = i32
    lib.ivm_scene_status.argtypes = [P]
    lib.ivm_scene_info.restype = i32
    lib.ivm_scene_info.argtypes = [P, ctypes.POINTER(ivm_scene_info_t)]
    lib.ivm_scene_solids.restype = i32
    lib.ivm_scene_solids.argtypes = [P, ctypes.POINTER(i32)]
    lib.ivm_destroy_scene.restype = i32
    lib.ivm_destroy_scene.argtypes = [P]
    lib.ivm_intervisibility_matrix.restype = i32
    lib.ivm_intervisibility_matrix.argtypes = [P, ctypes.POINTER(ivm_matrix_opts), P, P, P]
    lib.ivm_txrx_visibility_table.restype = i32
    lib.ivm_txrx_visibility_table.argtypes = [P, ctypes.POINTER(ivm_matrix_opts), i32, P, P, P, P, P, P, P]
    lib.ivm_image_tree_candidates.restype = i32
    lib.ivm_image_tree_candidates.argtypes = [P, P, i32, P, P, P, i32, P, P, P, sz, P]
    lib.ivm_visibility_ranges.restype = i32
    lib.ivm_visibility_ranges.argtypes = [P, i32, P, P, P, P, P, ctypes.c_double, P, sz, P, P, P, P, P, P, P]
    lib.ivm_visibility_ranges_noalloc.restype = i32
    lib.ivm_visibility_ranges_noalloc.argtypes = [P, i32, P, P, P, P, P, ctypes.c_double, P, P, P, P, P, P, P]
    lib.ivm_interface_relations.restype = i32
    lib.ivm_interface_relations.argtypes = [P, P, P, P, P, P]
    lib.ivm_edge_rows.restype = i32
    lib.ivm_edge_rows.argtypes = [P, ctypes.POINTER(ivm_matrix_opts), i32, i32, P, P, i32, P, P, P, P]
    lib.ivm_validate_paths.restype = i32
    lib.ivm_validate_paths.argtypes = [P, i32, P, P, i32, P, P, ctypes.c_int64, P, P, P, P]
    lib.ivm_angular_ranges.restype = i32
    lib.ivm_angular_ranges.argtypes = [P, P, P, P, P, sz, P]
    lib.ivm_edge_visibility.restype = i32
    lib.ivm_edge_visibility.argtypes = [P, ctypes.POINTER(ivm_matrix_opts), i32, i32, P, P, i32, P, P, P, P, P, P]
    lib.ivm_visibility_ranges_workspace_size.restype = i32
    lib.ivm_visibility_ranges_workspace_size.argtypes = [i32, ctypes.POINTER(sz)]
    lib.ivm_triangle_groups.restype = i32
    lib.ivm_triangle_groups.argtypes = [P, P, P]
    lib.ivm_model_workspace_size.restype = i32
    lib.ivm_model_workspace_size.argtypes = [i32, ctypes.POINTER(sz)]
    lib.ivm_model_create.restype = i32
    lib.ivm_model_create.argtypes = [P, sz, i32, i32, ctypes.POINTER(P)]
    lib.ivm_model_destroy.restype = i32
    lib.ivm_model_destroy.argtypes = [P]
    for name in ("ivm_model_set_params", "ivm_model_get_params"):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [P, P, P]
    lib.ivm_model_forward.restype = i32
    lib.ivm_model_forward.argtypes = [P, i32, P, P, P]
    lib.ivm_model_loss_grad.restype = i32
    lib.ivm_model_loss_grad.argtypes = [P, i32, P, P, P, P, P]
    lib.ivm_model_train_step.restype = i32
    lib.ivm_model_train_step.argtypes = [P, i32, P, P, ctypes.c_float, P, P]
    lib.ivm_pair_features.restype = i32
    lib.ivm_pair_features.argtypes = [P, i32, P, P, P, P]
    lib.ivm_pair_occluder_labels.restype = i32
    lib.ivm_pair_occluder_labels.argtypes = [P, i32, P, P, P, P]
    lib.ivm_scene_set_model.restype = i32
    lib.ivm_scene_set_model.argtypes = [P, P]
    lib.ivm_batch_workspace_size.restype = i32
    lib.ivm_batch_workspace_size.argtypes = [i32, ctypes.POINTER(sz)]
    lib.ivm_batch_create.restype = i32
    lib.ivm_batch_create.argtypes = [i32, P, ctypes.POINTER(ivm_matrix_opts), P, P, sz, ctypes.POINTER(P)]
    lib.ivm_batch_run.restype = i32
    lib.ivm_batch_run.argtypes = [P, P]
    lib.ivm_batch_destroy.restype = i32
    lib.ivm_batch_destroy.argtypes = [P]
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load_library().ivm_status_string(status).decode()
    except Exception:
        return str(status)


def _check(status: int, where: str, ok=(IVM_OK,)):
    if status not in ok:
        raise IvmError(status, where)
    return status


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def make_opts(order_mode: int = IVM_ORDER_PLAIN, fp64_only: bool = False, stack_depth: int = 0,
              waves_per_cu: int = 0, eps: float = 0.0, timing: Optional["KernelTimer"] = None,
              no_tile: bool = False, exhaustive: bool = False, tile_cap: int = 0, tile_treelets: int = 0,
              pair_chunk: int = 0, xcd_parts: int = 0) -> ivm_matrix_opts:
    o = ivm_matrix_opts()
    o.order_mode, o.fp64_only, o.stack_depth = order_mode, int(fp64_only), stack_depth
    o.no_tile = int(no_tile)
    o.exhaustive = int(exhaustive)
    o.waves_per_cu, o.eps = waves_per_cu, eps
    o.timing_events = timing.array_ptr if timing is not None else None
    o.tile_cap, o.tile_treelets, o.pair_chunk, o.xcd_parts = tile_cap, tile_treelets, pair_chunk, xcd_parts
    return o


class KernelTimer:
    """Two HIP events (created through the HIP runtime torch has loaded) that an
    entry point records around its traversal kernel; elapsed_ms() reads them."""

    def __init__(self):
        import torch  # noqa: F401
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.events = (ctypes.c_void_p * 2)()
        for k in range(2):
            ev = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.events[k] = ev
        self.array_ptr = ctypes.cast(self.events, ctypes.c_void_p).value

    def elapsed_ms(self) -> float:
        self.hip.hipEventSynchronize(self.events[1])
        ms = ctypes.c_float(0.0)
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), self.events[0], self.events[1]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def __del__(self):
        try:
            for k in range(2):
                self.hip.hipEventDestroy(self.events[k])
        except Exception:
            pass


def new_stats(device="cuda"):
    import torch
    return torch.zeros(STATS_WORDS, dtype=torch.int64, device=device)


def stats_dict(stats) -> dict:
    v = stats.cpu().numpy().astype(np.uint64)
    return {k: int(v[i]) for i, k in enumerate(STATS_FIELDS)}


class GpuScene:
    """A scene resident in HBM with its LBVH built by ivm_build_scene.

    Takes host arrays (any object with the ``vertices``, ``tri_vertices``,
    ``tri_facet``, ``sample_offsets``, ``samples``, ``g``, ``k`` attributes,
    or explicit arrays) and copies them to the device once.  ``facet_solid``
    (optional int32[F], -1 or a group id) is the occluder grouping hint of
    ivm_scene_desc; groups are checked on the device and never change a result."""

    def __init__(self, vertices, tri_vertices, tri_facet, sample_offsets, samples, g: int, gs: int,
                 learned: bool = False, device: str = "cuda", stream=None, facet_solid=None):
        import torch
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libivm needs a HIP GPU; none is visible")
        dev = torch.device(device)
        self.vertices = torch.as_tensor(np.ascontiguousarray(vertices, np.float32)).to(dev)
        self.tri_vertices = torch.as_tensor(np.ascontiguousarray(tri_vertices, np.int32)).to(dev)
        self.tri_facet = torch.as_tensor(np.ascontiguousarray(tri_facet, np.int32)).to(dev)
        self.sample_offsets = torch.as_tensor(np.ascontiguousarray(sample_offsets, np.int32)).to(dev)
        self.samples = torch.as_tensor(np.ascontiguousarray(samples, np.float32)).to(dev)
        d = ivm_scene_desc()
        d.n_vertices = self.vertices.shape[0]
        d.n_triangles = self.tri_vertices.shape[0]
        d.n_facets = self.sample_offsets.shape[0] - 1
        d.n_samples = self.samples.shape[0]
        d.vertices, d.tri_vertices = _ptr(self.vertices), _ptr(self.tri_vertices)
        d.tri_facet, d.sample_offsets = _ptr(self.tri_facet), _ptr(self.sample_offsets)
        d.samples = _ptr(self.samples)
        d.grid_vertex_log2, d.grid_sample_log2 = g, gs
        d.flags = IVM_SCENE_LEARNED if learned else 0
        self.facet_solid = None
        if facet_solid is not None:
            fs = np.ascontiguousarray(facet_solid, np.int32)
            if fs.shape != (d.n_facets,):
                raise ValueError("facet_solid must hold one id per facet")
            self.facet_solid = torch.as_tensor(fs).to(dev)
            d.facet_solid = _ptr(self.facet_solid)
            d.n_solids = int(fs.max(initial=-1)) + 1
        self.desc = d
        nbytes = ctypes.c_size_t(0)
        _check(lib.ivm_scene_workspace_size(ctypes.byref(d), ctypes.byref(nbytes)), "ivm_scene_workspace_size")
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        base = int(self.workspace.data_ptr())
        aligned = (base + 255) & ~255
        self.handle = ctypes.c_void_p()
        _check(lib.ivm_build_scene(ctypes.byref(d), aligned, int(nbytes.value), _stream(stream),
                                   ctypes.byref(self.handle)), "ivm_build_scene")
        info = ivm_scene_info_t()
        _check(lib.ivm_scene_info(self.handle, ctypes.byref(info)), "ivm_scene_info")
        self.F, self.T, self.S, self.W = info.n_facets, info.n_triangles, info.n_samples, info.words_per_row
        self.n_treelets = info.n_treelets
        self.device = dev

    def rebuild(self, stream=None) -> "GpuScene":
        """Run ivm_build_scene again on the resident arrays and workspace (no allocation)."""
        lib = load_library()
        old = self.handle
        h = ctypes.c_void_p()
        nbytes = self.workspace.numel() - 256
        aligned = (int(self.workspace.data_ptr()) + 255) & ~255
        _check(lib.ivm_build_scene(ctypes.byref(self.desc), aligned, nbytes, _stream(stream), ctypes.byref(h)),
               "ivm_build_scene")
        self.handle = h
        if old and old.value:
            lib.ivm_destroy_scene(old)
        if getattr(self, "_model", None) is not None:   # a new handle starts without a model
            _check(lib.ivm_scene_set_model(self.handle, self._model.handle), "ivm_scene_set_model")
        return self

    @classmethod
    def from_scene(cls, sc, solids: bool = True, facet_solid=None, **kw) -> "GpuScene":
        """solids: pass the scene's building ids as the occluder grouping hint
        (an explicit facet_solid array takes precedence)."""
        fs = facet_solid
        if fs is None and solids:
            fs = getattr(sc, "facet_building", None)
        return cls(sc.vertices, sc.tri_vertices, sc.tri_facet, sc.sample_offsets, sc.samples,
                   sc.g, sc.g + sc.k, facet_solid=fs, **kw)

    def solids_verified(self) -> int:
        """Number of hint groups that passed the device-side prism check (synchronises)."""
        n = ctypes.c_int32(0)
        _check(load_library().ivm_scene_solids(self.handle, ctypes.byref(n)), "ivm_scene_solids")
        return int(n.value)

    def status(self) -> int:
        return ivm_scene_status(self)

    def check(self):
        _check(self.status(), "scene validation")
        return self

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load_library().ivm_destroy_scene(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- entry points with the C names ---------------------------------------------

def ivm_scene_status(scene: GpuScene) -> int:
    return int(load_library().ivm_scene_status(scene.handle))


def ivm_intervisibility_matrix(scene: GpuScene, opts: Optional[ivm_matrix_opts] = None, out=None, stats=None,
                               stream=None, allow_model_fallback: bool = False):
    """Returns the bit-packed matrix as an int64 tensor [F, W] (bit j of row i = word j>>6, bit j&63)."""
    import torch
    if out is None:
        out = torch.empty((scene.F, scene.W), dtype=torch.int64, device=scene.device)
    st = load_library().ivm_intervisibility_matrix(scene.handle, ctypes.byref(opts) if opts is not None else None,
                                                   _ptr(out), _ptr(stats), _stream(stream))
    _check(st, "ivm_intervisibility_matrix", ok=(IVM_OK, IVM_ERR_MODEL) if allow_model_fallback else (IVM_OK,))
    return out


def ivm_txrx_visibility_table(scene: GpuScene, tx, rx, opts: Optional[ivm_matrix_opts] = None, stats=None,
                              out=None, stream=None):
    """tx, rx: float32 device tensors [N, 3].  Returns (tx_vis [N, W] int64, rx_vis, los uint8 [N])."""
    import torch
    N = int(tx.shape[0])
    if out is None:
        out = (torch.empty((N, scene.W), dtype=torch.int64, device=scene.device),
               torch.empty((N, scene.W), dtype=torch.int64, device=scene.device),
               torch.empty((N,), dtype=torch.uint8, device=scene.device))
    tv, rv, los = out
    _check(load_library().ivm_txrx_visibility_table(
        scene.handle, ctypes.byref(opts) if opts is not None else None, N, _ptr(tx), _ptr(rx),
        _ptr(tv), _ptr(rv), _ptr(los), _ptr(stats), _stream(stream)), "ivm_txrx_visibility_table")
    return tv, rv, los


def ivm_image_tree_candidates(scene: GpuScene, M, tx_vis, rx_vis, los, max_order: int = 2, lists: bool = False,
                              paths_cap: Optional[int] = None, counts=None, stream=None):
    """Counts int64 [N, K+1]; with lists=True also (offsets int64 [N*K+1], paths int32)."""
    import torch
    N = int(tx_vis.shape[0])
    if counts is None:
        counts = torch.empty((N, max_order + 1), dtype=torch.int64, device=scene.device)
    lib = load_library()
    if not lists:
        _check(lib.ivm_image_tree_candidates(scene.handle, _ptr(M), N, _ptr(tx_vis), _ptr(rx_vis), _ptr(los),
                                             max_order, _ptr(counts), None, None, 0, _stream(stream)),
               "ivm_image_tree_candidates")
        return counts
    offsets = torch.empty((N * max_order + 1,), dtype=torch.int64, device=scene.device)
    cap = paths_cap if paths_cap is not None else 1
    paths = torch.empty((max(cap, 1),), dtype=torch.int32, device=scene.device)
    st = lib.ivm_image_tree_candidates(scene.handle, _ptr(M), N, _ptr(tx_vis), _ptr(rx_vis), _ptr(los), max_order,
                                       _ptr(counts), _ptr(offsets), _ptr(paths), cap, _stream(stream))
    if st == IVM_ERR_CAPACITY and paths_cap is None:
        need = int(offsets[-1].item())
        paths = torch.empty((max(need, 1),), dtype=torch.int32, device=scene.device)
        st = lib.ivm_image_tree_candidates(scene.handle, _ptr(M), N, _ptr(tx_vis), _ptr(rx_vis), _ptr(los),
                                           max_order, _ptr(counts), _ptr(offsets), _ptr(paths), need,
                                           _stream(stream))
    _check(st, "ivm_image_tree_candidates")
    return counts, offsets, paths


def ivm_edge_visibility(scene: GpuScene, edge_facets, edge_samples, samples_per_edge: int, tx, rx,
                        opts: Optional[ivm_matrix_opts] = None, stream=None):
    """edge_facets int32 [E, 2], edge_samples float32 [E * s, 3], tx / rx float32
    [N, 3] (device tensors).  Returns (tx_edges, rx_edges) int64 [N, ceil(E/64)]
    bit rows and the diffraction candidate counts int64 [N]."""
    import torch
    N, E = int(tx.shape[0]), int(edge_facets.shape[0])
    We = (E + 63) // 64
    te = torch.empty((N, max(We, 1)), dtype=torch.int64, device=scene.device)
    re_ = torch.empty((N, max(We, 1)), dtype=torch.int64, device=scene.device)
    cnt = torch.empty((max(N, 1),), dtype=torch.int64, device=scene.device)
    _check(load_library().ivm_edge_visibility(
        scene.handle, ctypes.byref(opts) if opts is not None else None, E, samples_per_edge, _ptr(edge_facets),
        _ptr(edge_samples), N, _ptr(tx), _ptr(rx), _ptr(te), _ptr(re_), _ptr(cnt), _stream(stream)),
        "ivm_edge_visibility")
    return te[:, :We], re_[:, :We], cnt[:N]


def ivm_edge_rows(scene: GpuScene, edge_facets, edge_samples, samples_per_edge: int, rows,
                  opts: Optional[ivm_matrix_opts] = None, stream=None):
    """Edge rows of the matrix for the edges listed in `rows` (int32 [n], device):
    (edge_facet int64 [n, W], edge_edge int64 [n, ceil(E/64)]) bit rows."""
    import torch
    n, E = int(rows.shape[0]), int(edge_facets.shape[0])
    We = (E + 63) // 64
    ef = torch.empty((max(n, 1), scene.W), dtype=torch.int64, device=scene.device)
    ee = torch.empty((max(n, 1), max(We, 1)), dtype=torch.int64, device=scene.device)
    _check(load_library().ivm_edge_rows(
        scene.handle, ctypes.byref(opts) if opts is not None else None, E, samples_per_edge, _ptr(edge_facets),
        _ptr(edge_samples), n, _ptr(rows), _ptr(ef), _ptr(ee), _stream(stream)), "ivm_edge_rows")
    return ef[:n], ee[:n, :We]


def ivm_angular_ranges(scene: GpuScene, M, out=None, stream=None):
    """Angular bouncing ranges of the set bits of M (row = reference facet,
    column = aim facet): CSR offsets int64 [F + 1], columns int32 [nnz] and
    ranges float64 [nnz, 4] = (omega_lo, omega_hi, mu_lo, mu_hi) in degrees,
    as device tensors.  Without `out` the offsets are computed first and read
    back (one synchronisation) to size the outputs; with out=(offsets, cols,
    ranges) the call writes into them (cols.numel() is the capacity)."""
    import torch
    lib = load_library()
    h, s = scene.handle, _stream(stream)
    if out is None:
        off = torch.empty((scene.F + 1,), dtype=torch.int64, device=scene.device)
        _check(lib.ivm_angular_ranges(h, _ptr(M), _ptr(off), None, None, 0, s), "ivm_angular_ranges")
        if stream is not None:
            stream.synchronize()
        nnz = int(off[-1].item())
        cols = torch.empty((max(nnz, 1),), dtype=torch.int32, device=scene.device)
        rng = torch.empty((max(nnz, 1), 4), dtype=torch.float64, device=scene.device)
        _check(lib.ivm_angular_ranges(h, _ptr(M), _ptr(off), _ptr(cols), _ptr(rng), nnz, s), "ivm_angular_ranges")
        return off, cols[:nnz], rng[:nnz]
    off, cols, rng = out
    _check(lib.ivm_angular_ranges(h, _ptr(M), _ptr(off), _ptr(cols), _ptr(rng), int(cols.numel()), s),
           "ivm_angular_ranges")
    return off, cols, rng


def ivm_validate_paths(scene: GpuScene, tx, rx, max_order: int, offsets, paths, stats=None, stream=None):
    """Exact image-method verdicts for candidate lists (offsets int64 [N*K+1] in
    int32 elements, paths int32, as ivm_image_tree_candidates writes them):
    valid uint8 [len(paths)] (each element of a walk's k-tuple carries the walk's
    verdict: 1 valid, 0 not) and the valid walks per snapshot and order int64 [N, K]."""
    import torch
    N = int(tx.shape[0])
    n_elems = int(paths.numel())
    valid = torch.empty((max(n_elems, 1),), dtype=torch.uint8, device=scene.device)
    counts = torch.empty((max(N, 1), max_order), dtype=torch.int64, device=scene.device)
    _check(load_library().ivm_validate_paths(scene.handle, N, _ptr(tx), _ptr(rx), max_order, _ptr(offsets),
                                             _ptr(paths), n_elems, _ptr(valid), _ptr(counts), _ptr(stats),
                                             _stream(stream)), "ivm_validate_paths")
    return valid[:n_elems], counts[:N]


def ivm_interface_relations(scene: GpuScene, M, stream=None):
    """(par, per) int64 [F, W] bit matrices in M's layout and the facet classes int8 [F]."""
    import torch
    par = torch.empty_like(M)
    per = torch.empty_like(M)
    cls = torch.empty((max(scene.F, 1),), dtype=torch.int8, device=scene.device)
    lib = load_library()
    _check(lib.ivm_interface_relations(scene.handle, _ptr(M), _ptr(par), _ptr(per), _ptr(cls), _stream(stream)),
           "ivm_interface_relations")
    return par, per, cls[:scene.F]


def ivm_visibility_ranges(scene: GpuScene, tx_vis, rx_vis, los, tx, rx, dt: float, stream=None,
                          read_count: bool = True):
    """Ray creation / suppression counts int32 [N, 5], visibility range starts
    int32 [L], coherence times float64 [L], route distances float64 [L, 2] and
    the mean time (a float): device tensors, L read back after a stream sync.
    With read_count=False nothing is synchronised and the full-capacity tensors
    come back with L and the mean as one-element device tensors."""
    import torch
    N = int(tx_vis.shape[0])
    dev = scene.device
    events = torch.empty((N, 5), dtype=torch.int32, device=dev)
    starts = torch.empty((N,), dtype=torch.int32, device=dev)
    tc = torch.empty((N,), dtype=torch.float64, device=dev)
    dist = torch.empty((N, 2), dtype=torch.float64, device=dev)
    nr = torch.empty((1,), dtype=torch.int32, device=dev)
    mean = torch.empty((1,), dtype=torch.float64, device=dev)
    lib = load_library()
    nbytes = ctypes.c_size_t(0)
    _check(lib.ivm_visibility_ranges_workspace_size(N, ctypes.byref(nbytes)), "ivm_visibility_ranges_workspace_size")
    ws = torch.empty((nbytes.value + 255) // 256 * 32, dtype=torch.float64, device=dev)  # 256-B aligned
    _check(lib.ivm_visibility_ranges(scene.handle, N, _ptr(tx_vis), _ptr(rx_vis), _ptr(los), _ptr(tx), _ptr(rx),
                                     float(dt), _ptr(ws), ws.numel() * 8, _ptr(events), _ptr(starts), _ptr(tc),
                                     _ptr(dist), _ptr(nr), _ptr(mean), _stream(stream)), "ivm_visibility_ranges")
    if not read_count:
        return events, starts, tc, dist, nr, mean
    if stream is not None:
        stream.synchronize()
    L = int(nr.item())
    return events, starts[:L], tc[:L], dist[:L], float(mean.item())


IVM_RANGES_NOALLOC_MAX_SNAP = 32768


def ivm_visibility_ranges_noalloc(scene: GpuScene, tx_vis, rx_vis, los, tx, rx, dt: float, events, starts, tc,
                                  dist, n_ranges, mean, stream=None):
    """The allocation-free ranges call: the outputs are caller tensors (events
    int32 [N, 5], starts int32 [N], tc float64 [N], dist float64 [N, 2],
    n_ranges int32 [1], mean float64 [1], all on the current device) and the
    library's fixed scratch replaces the workspace.  Nothing is allocated or
    synchronised here."""
    N = int(tx_vis.shape[0])
    lib = load_library()
    _check(lib.ivm_visibility_ranges_noalloc(scene.handle, N, _ptr(tx_vis), _ptr(rx_vis), _ptr(los), _ptr(tx),
                                             _ptr(rx), float(dt), _ptr(events), _ptr(starts), _ptr(tc), _ptr(dist),
                                             _ptr(n_ranges), _ptr(mean), _stream(stream)),
           "ivm_visibility_ranges_noalloc")


def ivm_triangle_groups(scene: GpuScene, stream=None):
    import torch
    out = torch.empty((max(scene.T, 1),), dtype=torch.int32, device=scene.device)
    _check(load_library().ivm_triangle_groups(scene.handle, _ptr(out), _stream(stream)), "ivm_triangle_groups")
    return out[: scene.T]


# ---- learned occluder ordering ------------------------------------------------------

class Model:
    """The occluder-ordering network (parameters, gradients, Adam state in one
    device workspace).  precision: IVM_MODEL_BF16 (MFMA) or IVM_MODEL_FP32."""

    def __init__(self, max_batch: int = 1024, precision: int = IVM_MODEL_BF16, device: str = "cuda"):
        import torch
        lib = load_library()
        nbytes = ctypes.c_size_t(0)
        _check(lib.ivm_model_workspace_size(max_batch, ctypes.byref(nbytes)), "ivm_model_workspace_size")
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
        aligned = (int(self.workspace.data_ptr()) + 255) & ~255
        self.handle = ctypes.c_void_p()
        _check(lib.ivm_model_create(aligned, int(nbytes.value), max_batch, precision, ctypes.byref(self.handle)),
               "ivm_model_create")
        self.max_batch, self.precision, self.device = max_batch, precision, torch.device(device)

    def set_params(self, params, stream=None):
        import torch
        t = torch.as_tensor(np.ascontiguousarray(params, np.float32) if isinstance(params, np.ndarray) else params,
                            dtype=torch.float32).to(self.device).contiguous()
        assert t.numel() == IVM_MLP_PARAMS
        _check(load_library().ivm_model_set_params(self.handle, _ptr(t), _stream(stream)), "ivm_model_set_params")
        torch.cuda.current_stream().synchronize()

    def get_params(self, stream=None):
        import torch
        out = torch.empty(IVM_MLP_PARAMS, dtype=torch.float32, device=self.device)
        _check(load_library().ivm_model_get_params(self.handle, _ptr(out), _stream(stream)), "ivm_model_get_params")
        return out

    def forward(self, x, stream=None):
        import torch
        n = int(x.shape[0])
        out = torch.empty((n, IVM_MLP_OUTPUTS), dtype=torch.float32, device=self.device)
        _check(load_library().ivm_model_forward(self.handle, n, _ptr(x), _ptr(out), _stream(stream)),
               "ivm_model_forward")
        return out

    def loss_grad(self, x, y, stream=None):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(IVM_MLP_PARAMS, dtype=torch.float32, device=self.device)
        _check(load_library().ivm_model_loss_grad(self.handle, int(x.shape[0]), _ptr(x), _ptr(y), _ptr(loss),
                                                  _ptr(grad), _stream(stream)), "ivm_model_loss_grad")
        return loss, grad

    def train_step(self, x, y, lr: float = 1e-3, loss=None, stream=None):
        _check(load_library().ivm_model_train_step(self.handle, int(x.shape[0]), _ptr(x), _ptr(y), float(lr),
                                                   _ptr(loss), _stream(stream)), "ivm_model_train_step")

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load_library().ivm_model_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ivm_pair_features(scene: GpuScene, I, J, stream=None):
    import torch
    n = int(I.shape[0])
    out = torch.empty((n, IVM_MLP_FEATURES), dtype=torch.float32, device=scene.device)
    _check(load_library().ivm_pair_features(scene.handle, n, _ptr(I), _ptr(J), _ptr(out), _stream(stream)),
           "ivm_pair_features")
    return out


def ivm_pair_occluder_labels(scene: GpuScene, I, J, stream=None):
    import torch
    n = int(I.shape[0])
    out = torch.empty((n,), dtype=torch.int32, device=scene.device)
    _check(load_library().ivm_pair_occluder_labels(scene.handle, n, _ptr(I), _ptr(J), _ptr(out), _stream(stream)),
           "ivm_pair_occluder_labels")
    return out


def ivm_scene_set_model(scene: GpuScene, model: Optional[Model]):
    _check(load_library().ivm_scene_set_model(scene.handle, model.handle if model is not None else None),
           "ivm_scene_set_model")
    scene._model = model


# ---- batched scenes ---------------------------------------------------------------

class ivm_batch_item(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("d_M", ctypes.c_void_p), ("n_snap", ctypes.c_int32),
                ("d_tx", ctypes.c_void_p), ("d_rx", ctypes.c_void_p), ("d_tx_vis", ctypes.c_void_p),
                ("d_rx_vis", ctypes.c_void_p), ("d_los", ctypes.c_void_p), ("d_counts", ctypes.c_void_p)]


class Batch:
    """Many scenes run together (ivm_batch_*): outputs are allocated here, one per
    scene; run() replays the captured graph on the given (non-default) stream."""

    def __init__(self, scenes, txs, rxs, opts: Optional[ivm_matrix_opts] = None, stats=None):
        import torch
        lib = load_library()
        self.scenes = list(scenes)
        self.tx = [t.contiguous() for t in txs]
        self.rx = [r.contiguous() for r in rxs]
        self.M, self.tv, self.rv, self.los, self.counts = [], [], [], [], []
        n = len(self.scenes)
        arr = (ivm_batch_item * n)()
        for k, g in enumerate(self.scenes):
            N = int(self.tx[k].shape[0])
            self.M.append(torch.zeros((g.F, g.W), dtype=torch.int64, device=g.device))
            self.tv.append(torch.zeros((N, g.W), dtype=torch.int64, device=g.device))
            self.rv.append(torch.zeros((N, g.W), dtype=torch.int64, device=g.device))
            self.los.append(torch.zeros((N,), dtype=torch.uint8, device=g.device))
            self.counts.append(torch.zeros((N, 3), dtype=torch.int64, device=g.device))
            it = arr[k]
            it.scene, it.d_M, it.n_snap = g.handle.value, _ptr(self.M[k]), N
            it.d_tx, it.d_rx = _ptr(self.tx[k]), _ptr(self.rx[k])
            it.d_tx_vis, it.d_rx_vis, it.d_los = _ptr(self.tv[k]), _ptr(self.rv[k]), _ptr(self.los[k])
            it.d_counts = _ptr(self.counts[k])
        self._items = arr
        nbytes = ctypes.c_size_t(0)
        _check(lib.ivm_batch_workspace_size(n, ctypes.byref(nbytes)), "ivm_batch_workspace_size")
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.scenes[0].device)
        aligned = (int(self.workspace.data_ptr()) + 255) & ~255
        self.stats = stats
        self.handle = ctypes.c_void_p()
        _check(lib.ivm_batch_create(n, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts) if opts else None,
                                    _ptr(stats), aligned, int(nbytes.value), ctypes.byref(self.handle)),
               "ivm_batch_create")

    def run(self, stream):
        _check(load_library().ivm_batch_run(self.handle, int(stream.cuda_stream)), "ivm_batch_run")

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load_library().ivm_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- host-side helpers (no visibility arithmetic) --------------------------------

def unpack_bits(words, n: int) -> np.ndarray:
    """[..., W] int64 words -> [..., n] bool (bit j = word j>>6, bit j&63)."""
    w = np.ascontiguousarray(words.cpu().numpy() if hasattr(words, "cpu") else words).view(np.uint64)
    b = np.unpackbits(w.view(np.uint8).reshape(*w.shape, 8), axis=-1, bitorder="little")
    return b.reshape(*w.shape[:-1], w.shape[-1] * 64)[..., :n].astype(bool)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """[..., n] bool -> [..., ceil(n/64)] int64 words."""
    bits = np.asarray(bits, bool)
    n = bits.shape[-1]
    W = (n + 63) // 64
    pad = np.zeros((*bits.shape[:-1], W * 64), bool)
    pad[..., :n] = bits
    by = np.packbits(pad.reshape(*bits.shape[:-1], W * 8, 8), axis=-1, bitorder="little")
    return by.reshape(*bits.shape[:-1], W * 8).view(np.uint64).view(np.int64).reshape(*bits.shape[:-1], W)
