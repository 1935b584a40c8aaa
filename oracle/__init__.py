"""Plain FP64 CPU oracle for the inter-visibility hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the bench's CPU
baseline may import this package; the GPU library never does, and the two share
no code.  Each function says which passage of the paper it follows.

* ``Oracle`` wraps ivm_oracle.c (plain C, FP64, OpenMP over rows): pair
  visibility (Section II-B), point-facet visibility and LoS (Section III-B,
  Table II), and 128-bit exactness audits.
* ``candidates_enum`` / ``candidates_matmul``: image-tree reflection candidates
  (Section III-B, Table II; Section III-C) computed twice, by enumerating walks
  and by integer vector-matrix products.
* ``morton_treelets``: the Morton (Z-order) partition of triangles into 32
  contiguous equal-count groups, written from its definition.
* ``image_paths`` / ``image_paths_exact``: image-method specular paths on tiny
  scenes (the image method of Section II and case study 2, Section IV-B), in
  FP64 with a tolerance and in exact rational arithmetic, used to pin that
  pruning keeps every valid path.
* ``mlp_*``: FP64 reference of the occluder-ordering network (forward, BCE,
  backward, Adam) and a finite-difference check.
* ``visibility_ranges``: ray creation and suppression points along a sampled
  trajectory, the visibility ranges between them and their coherence times
  (Section III-C; Section III-D, eqs. 8 and 9), in sequential FP64 steps.
* ``interface_relations``: the interface relation of each visible facet pair
  (parallel or perpendicular planes, Section II-B, Table I) in exact integers.
* ``edge_visibility`` / ``diffraction_counts``: building edges seen from Tx/Rx
  positions and the first-order diffraction candidates Tx -> edge -> Rx
  (Section III-B), with the same exact predicates as the face tables.
* ``edge_rows``: the edge rows of the matrix (edge to facet and edge to
  edge visibility; edges are visibility nodes beside faces, Sections I, II-A).
* ``angular_ranges``: the angular bouncing range of each visible pair (Section
  II-A: the scene seen in two 2-D views; Section II-B, eq. 1: the angle at an
  edge of the reference face between the face itself and a vertex of the aim
  face; eq. 2: angles of 180 degrees or more recorded as 0).
"""
from __future__ import annotations

import bisect
import ctypes
import os
import subprocess
from typing import Dict, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ivm_oracle.c")
_LIB = os.path.join(_HERE, "libivm_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, no FP contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.ivo_create.restype = P
        lib.ivo_create.argtypes = [i32, i32, i32, P, P, P, P, P]
        lib.ivo_free.argtypes = [P]
        lib.ivo_segtri.restype = i32
        lib.ivo_segtri.argtypes = [P, P, P, P, P]
        lib.ivo_orient.restype = ctypes.c_double
        lib.ivo_orient.argtypes = [P, i32, P]
        lib.ivo_pair.restype = i32
        lib.ivo_pair.argtypes = [P, i32, i32]
        lib.ivo_pair_directed.restype = i32
        lib.ivo_pair_directed.argtypes = [P, i32, i32]
        lib.ivo_matrix.restype = i64
        lib.ivo_matrix.argtypes = [P, P, i32, i32]
        lib.ivo_pairs.argtypes = [P, i32, P, P, P, i32]
        lib.ivo_point_visible.restype = i32
        lib.ivo_point_visible.argtypes = [P, P, i32]
        lib.ivo_txrx.argtypes = [P, i32, P, P, P, P, P, i32]
        lib.ivo_point_facets.argtypes = [P, i32, P, P, P, i32]
        lib.ivo_los.argtypes = [P, i32, P, P, P]
        lib.ivo_segment_clear.restype = i32
        lib.ivo_segment_clear.argtypes = [P, P, P, i32, i32]
        lib.ivo_pairs_occluder_groups.argtypes = [P, i32, P, P, P, P, i32]
        lib.ivo_edge_rows.restype = None
        lib.ivo_edge_rows.argtypes = [P, i32, P, P, i32, i32, P, P, P, i32]
        lib.ivo_exact_audit.restype = i64
        lib.ivo_exact_audit.argtypes = [i32, P, P, P, P, P, i32, P]
        lib.ivo_orient_audit.restype = i64
        lib.ivo_orient_audit.argtypes = [i32, P, P, P, P, i32]
        lib.ivo_num_threads.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))


class Oracle:
    """The brute-force oracle bound to one scene (arrays as produced by scenegen)."""

    def __init__(self, scene):
        self.lib = _load()
        self.scene = scene
        self._keep = [np.ascontiguousarray(scene.vertices, np.float32),
                      np.ascontiguousarray(scene.tri_vertices, np.int32),
                      np.ascontiguousarray(scene.tri_facet, np.int32),
                      np.ascontiguousarray(scene.sample_offsets, np.int32),
                      np.ascontiguousarray(scene.samples, np.float32)]
        v, tv, tf, so, sm = self._keep
        self.F, self.T, self.S = scene.n_facets, scene.n_triangles, scene.n_samples
        self.h = self.lib.ivo_create(self.F, self.T, self.S, _ptr(v), _ptr(tv), _ptr(tf), _ptr(so), _ptr(sm))

    def close(self):
        if self.h:
            self.lib.ivo_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Section II-B: facet pairs ------------------------------------------
    def pair(self, i: int, j: int) -> int:
        return int(self.lib.ivo_pair(self.h, i, j))

    def pair_directed(self, i: int, j: int) -> int:
        return int(self.lib.ivo_pair_directed(self.h, i, j))

    def matrix(self, audit: bool = False, threads: int = 0) -> Tuple[np.ndarray, int]:
        M = np.zeros((self.F, self.F), dtype=np.uint8)
        mism = self.lib.ivo_matrix(self.h, _ptr(M), 1 if audit else 0, threads)
        return M.astype(bool), int(mism)

    def pairs(self, I: Sequence[int], J: Sequence[int], threads: int = 0) -> np.ndarray:
        I = np.ascontiguousarray(I, np.int32)
        J = np.ascontiguousarray(J, np.int32)
        out = np.zeros(len(I), np.uint8)
        self.lib.ivo_pairs(self.h, len(I), _ptr(I), _ptr(J), _ptr(out), threads)
        return out.astype(bool)

    def orient(self, f: int, x) -> float:
        return float(self.lib.ivo_orient(self.h, f, _ptr(_f64(x))))

    def segment_clear(self, p, q, ex1: int = -1, ex2: int = -1) -> bool:
        return bool(self.lib.ivo_segment_clear(self.h, _ptr(_f64(p)), _ptr(_f64(q)), ex1, ex2))

    # -- Section III-B: specific points ---------------------------------------
    def point_visible(self, X, f: int) -> bool:
        return bool(self.lib.ivo_point_visible(self.h, _ptr(_f64(X)), f))

    def txrx(self, tx: np.ndarray, rx: np.ndarray, threads: int = 0):
        tx = np.ascontiguousarray(tx, np.float32)
        rx = np.ascontiguousarray(rx, np.float32)
        N = tx.shape[0]
        tv = np.zeros((N, self.F), np.uint8)
        rv = np.zeros((N, self.F), np.uint8)
        los = np.zeros(N, np.uint8)
        self.lib.ivo_txrx(self.h, N, _ptr(tx), _ptr(rx), _ptr(tv), _ptr(rv), _ptr(los), threads)
        return tv.astype(bool), rv.astype(bool), los.astype(bool)

    def point_facets(self, X: np.ndarray, f: Sequence[int], threads: int = 0) -> np.ndarray:
        X = np.ascontiguousarray(X, np.float32).reshape(-1, 3)
        f = np.ascontiguousarray(f, np.int32)
        out = np.zeros(len(f), np.uint8)
        self.lib.ivo_point_facets(self.h, len(f), _ptr(X), _ptr(f), _ptr(out), threads)
        return out.astype(bool)

    def los(self, A: np.ndarray, B: np.ndarray) -> np.ndarray:
        A = np.ascontiguousarray(A, np.float32).reshape(-1, 3)
        B = np.ascontiguousarray(B, np.float32).reshape(-1, 3)
        out = np.zeros(A.shape[0], np.uint8)
        self.lib.ivo_los(self.h, A.shape[0], _ptr(A), _ptr(B), _ptr(out))
        return out.astype(bool)

    def occluder_groups(self, I, J, group_of_tri: np.ndarray, threads: int = 0) -> np.ndarray:
        I = np.ascontiguousarray(I, np.int32)
        J = np.ascontiguousarray(J, np.int32)
        g = np.ascontiguousarray(group_of_tri, np.int32)
        out = np.zeros(len(I), np.uint32)
        self.lib.ivo_pairs_occluder_groups(self.h, len(I), _ptr(I), _ptr(J), _ptr(g), _ptr(out), threads)
        return out


def segtri(p, q, a, b, c) -> bool:
    return bool(_load().ivo_segtri(_ptr(_f64(p)), _ptr(_f64(q)), _ptr(_f64(a)), _ptr(_f64(b)), _ptr(_f64(c))))


def exact_audit(P, Q, A, B, C, grid_log2: int) -> Tuple[int, int]:
    """(number of FP64/exact disagreements, number of exactly-zero determinants)."""
    arrs = [np.ascontiguousarray(x, np.float32).reshape(-1, 3) for x in (P, Q, A, B, C)]
    zeros = np.zeros(1, np.int64)
    bad = _load().ivo_exact_audit(arrs[0].shape[0], *[_ptr(a) for a in arrs], grid_log2, _ptr(zeros))
    return int(bad), int(zeros[0])


def orient_audit(X, A, B, C, grid_log2: int) -> int:
    arrs = [np.ascontiguousarray(x, np.float32).reshape(-1, 3) for x in (X, A, B, C)]
    return int(_load().ivo_orient_audit(arrs[0].shape[0], *[_ptr(a) for a in arrs], grid_log2))


def num_threads() -> int:
    return int(_load().ivo_num_threads())


# ---------------------------------------------------------------------------
# Image-tree candidates (Section III-B, Table II: parent Tx -> reference face ->
# aim face from the matrix; Section III-C: reflections up to the order needed)
# ---------------------------------------------------------------------------

def candidates_enum(M: np.ndarray, tx_vis: np.ndarray, rx_vis: np.ndarray, los: np.ndarray,
                    K: int) -> Tuple[np.ndarray, List[List[List[Tuple[int, ...]]]]]:
    """Enumerate walks f1 -> ... -> fk (k <= K) with vis_T(f1), M[f_m][f_m+1] and
    vis_R(fk).  counts[n][0] = LoS; lists[n][k-1] are the k-tuples in
    lexicographic order."""
    M = np.asarray(M, bool)
    N, F = tx_vis.shape
    counts = np.zeros((N, K + 1), np.int64)
    lists: List[List[List[Tuple[int, ...]]]] = []
    nbrs = [list(np.nonzero(M[f])[0]) for f in range(F)]
    for n in range(N):
        counts[n, 0] = int(bool(los[n]))
        per_order: List[List[Tuple[int, ...]]] = [[] for _ in range(K)]

        def walk(prefix):
            k = len(prefix)
            if rx_vis[n, prefix[-1]]:
                per_order[k - 1].append(tuple(prefix))
            if k == K:
                return
            for f in nbrs[prefix[-1]]:
                walk(prefix + [int(f)])

        for f1 in range(F):
            if tx_vis[n, f1]:
                walk([f1])
        for k in range(K):
            per_order[k].sort()
            counts[n, k + 1] = len(per_order[k])
        lists.append(per_order)
    return counts, lists


def candidates_matmul(M: np.ndarray, tx_vis: np.ndarray, rx_vis: np.ndarray, los: np.ndarray,
                      K: int) -> np.ndarray:
    """Same counts by integer vector-matrix products: c_k = t^T M^(k-1) r.
    M may be a dense boolean array or a scipy sparse matrix (for large F; the
    product is the same integer product, taken as M^T w^T)."""
    import scipy.sparse as sps
    sparse = sps.issparse(M)
    Mi = sps.csr_matrix(M, dtype=np.int64) if sparse else np.asarray(M, np.int64)
    t = np.asarray(tx_vis, np.int64)
    r = np.asarray(rx_vis, np.int64)
    N = t.shape[0]
    counts = np.zeros((N, K + 1), np.int64)
    counts[:, 0] = np.asarray(los, np.int64)
    w = t.copy()
    for k in range(1, K + 1):
        counts[:, k] = (w * r).sum(1)
        w = np.asarray(Mi.T @ w.T).T if sparse else w @ Mi
    return counts


# ---------------------------------------------------------------------------
# Morton partition of triangles (Z-order curve, Morton 1966)
# ---------------------------------------------------------------------------

def morton_treelets(scene, n_groups: int = 32) -> Tuple[np.ndarray, np.ndarray]:
    """Sort triangles by the 30-bit Morton code of their centroid (index breaks
    ties) and cut the order into n_groups contiguous equal-count groups.

    The centroid is quantised exactly in integers: with vertex coordinates in
    grid units, c3 = a + b + c (three times the centroid) and the scene box
    [lo, hi] over all triangle vertices, q = floor((c3 - 3 lo) * 1024 / (3 (hi - lo) + 1))
    per axis, in [0, 1023].  Bits interleave as x, y, z from the top.
    Returns (order, group_of_tri): order[r] = triangle at sorted rank r; group
    of rank r = floor(r * n_groups / T)."""
    scale = 2 ** scene.g
    V = np.rint(scene.vertices.astype(np.float64) * scale).astype(np.int64)
    assert np.all(V == scene.vertices.astype(np.float64) * scale)
    tv = V[scene.tri_vertices]                      # T x 3 x 3
    lo = tv.reshape(-1, 3).min(0)
    hi = tv.reshape(-1, 3).max(0)
    c3 = tv.sum(1)
    den = 3 * (hi - lo) + 1
    q = ((c3 - 3 * lo) * 1024) // den               # floor division, non-negative
    assert q.min() >= 0 and q.max() <= 1023
    T = tv.shape[0]
    codes = np.zeros(T, np.int64)
    for bit in range(10):
        for ax, shift in ((0, 2), (1, 1), (2, 0)):
            codes |= ((q[:, ax] >> bit) & 1) << (3 * bit + shift)
    order = np.lexsort((np.arange(T), codes))
    group_of_rank = (np.arange(T) * n_groups) // max(T, 1)
    group_of_tri = np.empty(T, np.int32)
    group_of_tri[order] = group_of_rank
    return order.astype(np.int32), group_of_tri


# ---------------------------------------------------------------------------
# Image-method specular paths (for the pruning-recall pin)
# ---------------------------------------------------------------------------

def _facet_planes(scene):
    V = scene.vertices.astype(np.float64)
    F = scene.n_facets
    first = np.full(F, -1)
    for t in range(scene.n_triangles - 1, -1, -1):
        first[scene.tri_facet[t]] = t
    a = V[scene.tri_vertices[first, 0]]
    b = V[scene.tri_vertices[first, 1]]
    c = V[scene.tri_vertices[first, 2]]
    n = np.cross(b - a, c - a)
    return a, n


def _in_facet(scene, f, x, tol=1e-9):
    V = scene.vertices.astype(np.float64)
    tris = np.nonzero(scene.tri_facet == f)[0]
    for t in tris:
        a, b, c = V[scene.tri_vertices[t]]
        n = np.cross(b - a, c - a)
        nn = np.dot(n, n)
        w0 = np.dot(np.cross(b - a, x - a), n) / nn
        w1 = np.dot(np.cross(c - b, x - b), n) / nn
        w2 = np.dot(np.cross(a - c, x - c), n) / nn
        if w0 >= -tol and w1 >= -tol and w2 >= -tol:
            return True
    return False


def image_paths(scene, orc: Oracle, T, R, K: int) -> List[Tuple[int, ...]]:
    """All valid specular reflection paths T -> f1 -> ... -> fk -> R (k <= K) by the
    image method: mirror T successively in the planes of f1..fk, trace back from
    R, require each reflection point inside its facet with the segment crossing
    the plane between its ends, and every leg clear (excluding the facets at its
    ends).  Float64 with a small tolerance; for well-conditioned pins only."""
    a, n = _facet_planes(scene)
    F = scene.n_facets
    T = np.asarray(T, np.float64)
    R = np.asarray(R, np.float64)
    out = []

    def reflect(x, f):
        return x - 2.0 * np.dot(x - a[f], n[f]) / np.dot(n[f], n[f]) * n[f]

    def valid(walk):
        imgs = [T]
        for f in walk:
            imgs.append(reflect(imgs[-1], f))
        pts = [None] * len(walk)
        target = R
        for m in range(len(walk) - 1, -1, -1):
            f = walk[m]
            I = imgs[m + 1]
            da = np.dot(target - a[f], n[f])
            db = np.dot(I - a[f], n[f])
            if not (da > 1e-12 and db < -1e-12):
                return False
            s = da / (da - db)
            P = target + s * (I - target)
            if not _in_facet(scene, f, P):
                return False
            pts[m] = P
            target = P
        chain = [T] + pts + [R]
        facs = [-1] + list(walk) + [-1]
        for m in range(len(chain) - 1):
            if not orc.segment_clear(chain[m], chain[m + 1], facs[m], facs[m + 1]):
                return False
        return True

    def rec(walk):
        if walk and valid(walk):
            out.append(tuple(walk))
        if len(walk) == K:
            return
        for f in range(F):
            if walk and walk[-1] == f:
                continue
            rec(walk + [f])

    rec([])
    return sorted(out, key=lambda w: (len(w), w))


def _q3(x):
    from fractions import Fraction
    return tuple(Fraction(float(c)) for c in x)          # float32/float64 values are dyadic: exact


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _segtri_exact(p, q, a, b, c) -> bool:
    """The division-free Moller-Trumbore test of ivm_oracle.c (open segment,
    closed triangle, a segment parallel to the plane never hits) in rational
    arithmetic, for end points off the grid."""
    d, e1, e2, sv = _sub(q, p), _sub(b, a), _sub(c, a), _sub(p, a)
    h = _cross(d, e2)
    det = _dot(e1, h)
    if det == 0:
        return False
    u = _dot(sv, h)
    g = _cross(sv, e1)
    v, t = _dot(d, g), _dot(e2, g)
    if det > 0:
        return u >= 0 and v >= 0 and u + v <= det and 0 < t < det
    return u <= 0 and v <= 0 and u + v >= det and det < t < 0


class _ExactImage:
    """The exact image method on one scene (rational arithmetic, no tolerance):
    mirror T in the planes of f1..fk, trace back from R; each reflection point
    must lie in its closed facet, with the segment's end strictly in front of
    the plane and the image strictly behind, and every leg's open segment must
    miss every triangle outside the facets at its ends."""

    def __init__(self, scene):
        V = [_q3(v) for v in scene.vertices]
        tv = scene.tri_vertices
        self.tris = [(V[tv[t, 0]], V[tv[t, 1]], V[tv[t, 2]]) for t in range(tv.shape[0])]
        self.tfac = [int(f) for f in scene.tri_facet]
        self.F = scene.n_facets
        self.by_facet = [[] for _ in range(self.F)]
        for t, f in enumerate(self.tfac):
            self.by_facet[f].append(self.tris[t])
        self.plane = []
        for f in range(self.F):
            a, b, c = self.by_facet[f][0]
            self.plane.append((a, _cross(_sub(b, a), _sub(c, a))))

    def reflect(self, x, f):
        a, n = self.plane[f]
        k = 2 * _dot(_sub(x, a), n) / _dot(n, n)
        return (x[0] - k * n[0], x[1] - k * n[1], x[2] - k * n[2])

    def in_facet(self, x, f):
        for a, b, c in self.by_facet[f]:
            n = _cross(_sub(b, a), _sub(c, a))
            if (_dot(_cross(_sub(b, a), _sub(x, a)), n) >= 0 and _dot(_cross(_sub(c, b), _sub(x, b)), n) >= 0
                    and _dot(_cross(_sub(a, c), _sub(x, c)), n) >= 0):
                return True
        return False

    def clear(self, p, q, ex1, ex2):
        return not any(_segtri_exact(p, q, *self.tris[t]) for t in range(len(self.tris))
                       if self.tfac[t] not in (ex1, ex2))

    def valid(self, T, R, walk) -> bool:
        imgs = [T]
        for f in walk:
            imgs.append(self.reflect(imgs[-1], f))
        pts = [None] * len(walk)
        target = R
        for m in range(len(walk) - 1, -1, -1):
            f = walk[m]
            a, n = self.plane[f]
            I = imgs[m + 1]
            da, db = _dot(_sub(target, a), n), _dot(_sub(I, a), n)
            if not (da > 0 and db < 0):
                return False
            s_ = da / (da - db)
            P = tuple(target[i] + s_ * (I[i] - target[i]) for i in range(3))
            if not self.in_facet(P, f):
                return False
            pts[m] = P
            target = P
        chain = [T] + pts + [R]
        facs = [-1] + list(walk) + [-1]
        return all(self.clear(chain[m], chain[m + 1], facs[m], facs[m + 1]) for m in range(len(chain) - 1))


def image_paths_exact(scene, T, R, K: int) -> List[Tuple[int, ...]]:
    """Every walk f1 -> ... -> fk (k <= K, no facet twice in a row) that is a
    valid specular path from T to R by the exact image method (_ExactImage)."""
    ex = _ExactImage(scene)
    T, R = _q3(T), _q3(R)
    out = []

    def rec(walk):
        if walk and ex.valid(T, R, walk):
            out.append(tuple(walk))
        if len(walk) == K:
            return
        for f in range(ex.F):
            if not (walk and walk[-1] == f):
                rec(walk + [f])

    rec([])
    return sorted(out, key=lambda w: (len(w), w))


def validate_paths_exact(scene, T, R, walks, ex: "_ExactImage" = None) -> np.ndarray:
    """Validity of each given walk as a specular path from T to R by the exact
    image method (the same steps as image_paths_exact): bool per walk."""
    ex = ex or _ExactImage(scene)
    T, R = _q3(T), _q3(R)
    return np.array([ex.valid(T, R, [int(f) for f in w]) for w in walks], bool)


# ---------------------------------------------------------------------------
# Occluder-ordering network, FP64 reference
# ---------------------------------------------------------------------------

MLP_SIZES = (24, 128, 128, 128, 32)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def pair_features(scene, I, J) -> np.ndarray:
    """The 24 features of facet pairs (i, j), in FP64, from their definition:
    with the box of all triangle vertices (centre c0, half-size s of its largest
    axis): centroids of the two facets' samples, (x - c0) / s; unit normals of the
    first triangles; areas / s^2; distance between the normalised centroids; the
    AABB of both facets' vertices, min then max, (x - c0) / s; unit direction from
    the first centroid to the second (zero when they coincide)."""
    V = scene.vertices.astype(np.float64)
    tv = V[scene.tri_vertices]
    lo, hi = tv.reshape(-1, 3).min(0), tv.reshape(-1, 3).max(0)
    c0 = (lo + hi) / 2
    hs = float(((hi - lo) / 2).max())
    hs = hs if hs > 0 else 1.0
    F = scene.n_facets
    smp = scene.samples.astype(np.float64)
    off = scene.sample_offsets
    cent = np.array([smp[off[f]:off[f + 1]].mean(0) for f in range(F)])
    first = np.full(F, -1)
    for t in range(scene.n_triangles - 1, -1, -1):
        first[scene.tri_facet[t]] = t
    e1 = tv[:, 1] - tv[:, 0]
    e2 = tv[:, 2] - tv[:, 0]
    cr = np.cross(e1, e2)
    nrm = cr[first] / np.linalg.norm(cr[first], axis=1, keepdims=True)
    area = np.zeros(F)
    np.add.at(area, scene.tri_facet, 0.5 * np.linalg.norm(cr, axis=1))
    blo = np.full((F, 3), np.inf)
    bhi = np.full((F, 3), -np.inf)
    np.minimum.at(blo, scene.tri_facet, tv.min(1))
    np.maximum.at(bhi, scene.tri_facet, tv.max(1))
    I = np.asarray(I)
    J = np.asarray(J)
    ci, cj = (cent[I] - c0) / hs, (cent[J] - c0) / hs
    d = cj - ci
    dist = np.linalg.norm(d, axis=1)
    safe = np.where(dist > 0, dist, 1.0)
    direc = np.where(dist[:, None] > 0, d / safe[:, None], 0.0)
    return np.concatenate([ci, cj, nrm[I], nrm[J], area[I, None] / hs ** 2, area[J, None] / hs ** 2, dist[:, None],
                           (np.minimum(blo[I], blo[J]) - c0) / hs, (np.maximum(bhi[I], bhi[J]) - c0) / hs, direc], 1)


def mlp_init(seed: int = 0, sizes=MLP_SIZES) -> Dict[str, np.ndarray]:
    """Deterministic He-uniform initialisation (numpy PCG64 with the given seed)."""
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(len(sizes) - 1):
        fan_in = sizes[l]
        bound = np.sqrt(6.0 / fan_in)
        p[f"W{l}"] = rng.uniform(-bound, bound, size=(sizes[l + 1], sizes[l]))
        p[f"b{l}"] = np.zeros(sizes[l + 1])
    return p


def mlp_forward(p: Dict[str, np.ndarray], X: np.ndarray, bf16: bool = False):
    """ReLU hidden layers, linear output.  Returns (logits, activations).  With
    bf16=True both operands of every product are first rounded to BF16 (the
    arithmetic of a BF16 matrix unit with wide accumulation)."""
    r = bf16_round if bf16 else (lambda a: a)
    acts = [np.asarray(X, np.float64)]
    L = len([k for k in p if k.startswith("W")])
    h = acts[0]
    for l in range(L):
        z = r(h) @ r(p[f"W{l}"]).T + p[f"b{l}"]
        h = np.maximum(z, 0.0) if l < L - 1 else z
        acts.append(h)
    return h, acts


def bce_with_logits(z: np.ndarray, y: np.ndarray) -> float:
    """Mean over all outputs of max(z,0) - z y + log(1 + exp(-|z|))."""
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def mlp_loss_grad(p: Dict[str, np.ndarray], X: np.ndarray, Y: np.ndarray, bf16: bool = False):
    """Loss and gradients of the mean BCE-with-logits loss (operands of every
    product rounded to BF16 when bf16=True, as in mlp_forward)."""
    r = bf16_round if bf16 else (lambda a: a)
    z, acts = mlp_forward(p, X, bf16)
    loss = bce_with_logits(z, Y)
    L = len([k for k in p if k.startswith("W")])
    dz = (1.0 / (1.0 + np.exp(-z)) - Y) / z.size
    g = {}
    for l in range(L - 1, -1, -1):
        g[f"W{l}"] = r(dz).T @ r(acts[l])
        g[f"b{l}"] = dz.sum(0)
        if l > 0:
            dh = r(dz) @ r(p[f"W{l}"])
            dz = dh * (acts[l] > 0.0)
    return loss, g


def mlp_flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    """Parameters as one array: W0, b0, W1, b1, W2, b2, W3, b3 (row-major)."""
    L = len([k for k in p if k.startswith("W")])
    return np.concatenate([np.concatenate([p[f"W{l}"].ravel(), p[f"b{l}"].ravel()]) for l in range(L)])


def mlp_unflatten(v: np.ndarray, sizes=MLP_SIZES) -> Dict[str, np.ndarray]:
    p, o = {}, 0
    for l in range(len(sizes) - 1):
        n, k = sizes[l + 1], sizes[l]
        p[f"W{l}"] = np.asarray(v[o:o + n * k], np.float64).reshape(n, k)
        o += n * k
        p[f"b{l}"] = np.asarray(v[o:o + n], np.float64).copy()
        o += n
    return p


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def mlp_fd_check(p, X, Y, n_probe: int = 20, h: float = 1e-6, seed: int = 0) -> float:
    """Largest relative difference between analytic and central-difference gradients."""
    rng = np.random.default_rng(seed)
    _, g = mlp_loss_grad(p, X, Y)
    worst = 0.0
    for k in p:
        for _ in range(max(1, n_probe // len(p))):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            old = p[k][idx]
            p[k][idx] = old + h
            lp, _ = mlp_loss_grad(p, X, Y)
            p[k][idx] = old - h
            lm, _ = mlp_loss_grad(p, X, Y)
            p[k][idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k][idx]
            worst = max(worst, abs(fd - an) / max(1e-8, abs(fd) + abs(an)))
    return worst


# ---------------------------------------------------------------------------
# Visibility ranges and coherence time along a trajectory (Section III-C: the
# visibility change nodes of the inter-visibility table of a mobile Tx / Rx;
# Section III-D: eq. 8, T_c,l = d_l / v_l per visibility range, the smaller of
# the Tx-side and Rx-side values when both move, eq. 9, the mean over ranges)
# ---------------------------------------------------------------------------

def visibility_ranges(tx_vis: np.ndarray, rx_vis: np.ndarray, los: np.ndarray, tx: np.ndarray,
                      rx: np.ndarray, dt: float) -> Dict[str, object]:
    """Snapshots n = 0..N-1 at times n * dt; snapshot n's visibility holds until
    snapshot n + 1 and the last snapshot ends the trajectory.

    events[n] (n >= 1, zero for n = 0): facets that became visible from the
    Tx (ray creation), facets no longer visible from the Tx (suppression), the
    same two counts for the Rx, and the LoS change (+1 created, -1 suppressed).
    A side's range ends where its visible set or the LoS changes.  A side range
    [a, e) (the last one ends at N - 1) has route distance d = sum of the
    position steps from snapshot a to e, duration tau = (e - a) dt, velocity
    v = d / tau and coherence time d / v (eq. 8); a side that does not move in
    it (d = 0) sets no limit (+inf).  The combined ranges start at every change
    of either side; each takes the smaller coherence time of the two side
    ranges that contain it, and the mean of the finite ones is eq. 9 (+inf when
    none is finite).  dist[l] is each side's route distance over combined range
    l (from its first snapshot to the next range's, or to N - 1).  Returns
    events int32[N][5], starts int32[L], tc float64[L], dist float64[L][2],
    mean float64."""
    tv = np.asarray(tx_vis, bool)
    rv = np.asarray(rx_vis, bool)
    lo = np.asarray(los, bool)
    N = tv.shape[0]
    P = {0: np.asarray(tx, np.float64), 1: np.asarray(rx, np.float64)}
    events = np.zeros((N, 5), np.int32)
    change = np.zeros((N, 2), bool)
    for n in range(1, N):
        for s, vis in ((0, tv), (1, rv)):
            events[n, 2 * s] = int(np.sum(vis[n] & ~vis[n - 1]))
            events[n, 2 * s + 1] = int(np.sum(~vis[n] & vis[n - 1]))
        events[n, 4] = int(lo[n]) - int(lo[n - 1])
        for s in (0, 1):
            change[n, s] = events[n, 2 * s] != 0 or events[n, 2 * s + 1] != 0 or events[n, 4] != 0
    starts = [0] + [n for n in range(1, N) if change[n, 0] or change[n, 1]]
    L = len(starts)
    tc = [float('inf')] * L

    def step(s, n):  # route distance from snapshot n - 1 to snapshot n
        d = P[s][n] - P[s][n - 1]
        return float(np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]))

    def side_time(d, a, e):
        tau = (e - a) * dt
        if not d > 0.0:
            return float('inf')
        v = d / tau
        return d / v

    for s in (0, 1):
        # this side's ranges: [bounds[r], bounds[r + 1]), the last one to snapshot N - 1
        bounds = [0] + [n for n in range(1, N) if change[n, s]]
        for r, a in enumerate(bounds):
            last = r + 1 == len(bounds)
            e = N - 1 if last else bounds[r + 1]
            d = 0.0
            for n in range(a + 1, e + 1):
                d += step(s, n)
            t = side_time(d, a, e)
            hi = N if last else e  # the combined ranges starting in [a, hi) lie inside this one
            for l in range(bisect.bisect_left(starts, a), bisect.bisect_left(starts, hi)):
                tc[l] = min(tc[l], t)
    dist = np.zeros((L, 2), np.float64)
    for l in range(L):
        e = starts[l + 1] if l + 1 < L else N - 1
        for s in (0, 1):
            d = 0.0
            for n in range(starts[l] + 1, e + 1):
                d += step(s, n)
            dist[l, s] = d
    finite = [t for t in tc if t != float('inf')]
    mean = float('inf')
    if finite:
        acc = 0.0
        for t in finite:
            acc += t
        mean = acc / len(finite)
    return {"events": events, "starts": np.asarray(starts, np.int32), "tc": np.asarray(tc, np.float64),
            "dist": dist, "mean": mean}


# ---------------------------------------------------------------------------
# Interface relations of the inter-visibility matrix (Section II-B, Table I:
# reference face, aim face and whether their planes are parallel (PAR) or
# perpendicular (PER); the horizontal view holds relations between vertical
# faces, a vertical view those involving horizontal faces)
# ---------------------------------------------------------------------------

def facet_normals_int(scene) -> List[Tuple[int, int, int]]:
    """The normal (b - a) x (c - a) of each facet's first triangle in vertex-grid
    units, as exact Python integers (the plane triple of the visible-side rule)."""
    su = 1 << scene.g
    V = [[int(round(float(x) * su)) for x in v] for v in np.asarray(scene.vertices, np.float64)]
    tv = np.asarray(scene.tri_vertices)
    tf = np.asarray(scene.tri_facet)
    out = []
    for f in range(scene.n_facets):
        t = int(np.searchsorted(tf, f))
        a, b, c = (V[int(tv[t, m])] for m in range(3))
        e1 = [b[k] - a[k] for k in range(3)]
        e2 = [c[k] - a[k] for k in range(3)]
        out.append((e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]))
    return out


def interface_relations(scene, M: np.ndarray) -> Dict[str, np.ndarray]:
    """par[i, j] / per[i, j]: M[i, j] and the two facets' planes are parallel
    (normals' cross product zero) / perpendicular (dot product zero); cls[f]:
    0 vertical facet (normal z = 0), 1 horizontal (normal x = y = 0), 2 other."""
    nrm = facet_normals_int(scene)
    F = len(nrm)
    M = np.asarray(M, bool)
    par = np.zeros((F, F), bool)
    per = np.zeros((F, F), bool)
    for i in range(F):
        a = nrm[i]
        for j in range(F):
            if not M[i, j]:
                continue
            b = nrm[j]
            cross = (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])
            par[i, j] = cross == (0, 0, 0)
            per[i, j] = a[0] * b[0] + a[1] * b[1] + a[2] * b[2] == 0
    cls = np.array([0 if n[2] == 0 else (1 if n[0] == 0 and n[1] == 0 else 2) for n in nrm], np.int8)
    return {"par": par, "per": per, "cls": cls}


# ---------------------------------------------------------------------------
# Edge visibility for first-order diffraction (Section III-B: the receiver's
# diffracting edge is found the way a reflecting face is; edges are visibility
# nodes next to faces, Section I and Section II-A)
# ---------------------------------------------------------------------------

def edge_visibility(orc: "Oracle", X: np.ndarray, edge_facets: np.ndarray, edge_samples: np.ndarray,
                    s: int) -> np.ndarray:
    """bool [N][E]: edge e, where facets fa and fb meet, is visible from the
    point x iff x lies strictly on the visible side of fa or of fb (an edge is
    seen where one of its faces is) and the segment from x to one of the edge's
    s sample points meets no triangle of a facet other than fa and fb."""
    X = np.asarray(X, np.float64).reshape(-1, 3)
    E = int(edge_facets.shape[0])
    out = np.zeros((X.shape[0], E), bool)
    for n in range(X.shape[0]):
        for e in range(E):
            fa, fb = int(edge_facets[e, 0]), int(edge_facets[e, 1])
            front = orc.orient(fa, X[n]) > 0 or (fb >= 0 and orc.orient(fb, X[n]) > 0)
            if not front:
                continue
            for j in range(s):
                if orc.segment_clear(X[n], edge_samples[e * s + j], fa, fb):
                    out[n, e] = True
                    break
    return out


def edge_rows(orc: "Oracle", edge_facets: np.ndarray, edge_samples: np.ndarray, s: int, rows=None,
              threads: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """The edge rows of the matrix (edges as visibility nodes beside faces,
    Sections I and II-A; the face seen for diffraction is the face seen for
    reflection, Section III-B): for each edge e in `rows` (all by default),
    ef[k][f] for every facet and ee[k][e'] for every edge.  Nodes see each other
    when some sample p of one and q of the other have q strictly in front of one
    of the first node's facets, p in front of one of the second's, and the open
    segment (p, q) meets no triangle outside the facets of both."""
    E = int(edge_facets.shape[0])
    rows = np.arange(E, dtype=np.int32) if rows is None else np.ascontiguousarray(rows, np.int32)
    efac = np.ascontiguousarray(edge_facets, np.int32)
    esmp = np.ascontiguousarray(edge_samples, np.float32)
    ef = np.zeros((len(rows), orc.F), np.uint8)
    ee = np.zeros((len(rows), E), np.uint8)
    orc.lib.ivo_edge_rows(orc.h, E, _ptr(efac), _ptr(esmp), s, len(rows), _ptr(rows), _ptr(ef), _ptr(ee), threads)
    return ef.astype(bool), ee.astype(bool)


def diffraction_counts(tx_edges: np.ndarray, rx_edges: np.ndarray) -> np.ndarray:
    """First-order diffraction candidates Tx -> edge -> Rx per snapshot: the
    edges visible from both ends."""
    return (np.asarray(tx_edges, bool) & np.asarray(rx_edges, bool)).sum(1).astype(np.int64)


# ---------------------------------------------------------------------------
# Angular bouncing ranges (Section II-A: the 3-D scene is read in 2-D views, a
# horizontal one for vertical faces and a vertical one otherwise; Section II-B,
# eq. 1: at an edge B of the reference face the angle between BA, along the
# face, and BF, towards a vertex F of the aim face, is arccos of their
# normalised dot product; eq. 2: an angle of 180 degrees or more, measured from
# BA towards the face's visible side, is recorded as 0)
# ---------------------------------------------------------------------------

def _facet_vertices_int(scene) -> List[List[Tuple[int, int, int]]]:
    """Every vertex of each facet's triangles, in vertex-grid units (exact)."""
    su = 1 << scene.g
    V = [tuple(int(round(float(x) * su)) for x in v) for v in np.asarray(scene.vertices, np.float64)]
    out: List[List[Tuple[int, int, int]]] = [[] for _ in range(scene.n_facets)]
    for t, f in enumerate(np.asarray(scene.tri_facet)):
        for m in range(3):
            out[int(f)].append(V[int(scene.tri_vertices[t, m])])
    return out


def view_direction(ni, nj) -> Tuple[int, int, int]:
    """The direction the pair's 2-D view looks along (integers): the line where
    the two facets' planes meet, n_i x n_j; for parallel planes the vertical for
    vertical facets (the horizontal view), x for horizontal ones, else the
    horizontal direction in facet i's plane.  Its first non-zero component in
    the order z, x, y is made positive."""
    d = (ni[1] * nj[2] - ni[2] * nj[1], ni[2] * nj[0] - ni[0] * nj[2], ni[0] * nj[1] - ni[1] * nj[0])
    if d == (0, 0, 0):
        if ni[2] == 0:
            d = (0, 0, 1)
        elif ni[0] == 0 and ni[1] == 0:
            d = (1, 0, 0)
        else:
            d = (-ni[1], ni[0], 0)
    for k in (2, 0, 1):
        if d[k] != 0:
            if d[k] < 0:
                d = (-d[0], -d[1], -d[2])
            break
    return d


def angular_ranges(scene, M: np.ndarray, rows=None) -> Dict[str, np.ndarray]:
    """For every pair with M[i, j] (i the reference face, j the aim face), in
    row-major order: offsets int64 [F + 1] (CSR over the rows), cols int32 [nnz]
    and ranges float64 [nnz, 4] = (omega_lo, omega_hi, mu_lo, mu_hi) in degrees.

    The pair is seen along d = view_direction(n_i, n_j), which lies in both
    facets' planes, so each facet appears as a segment.  The reference facet's
    ends are its vertices with the smallest (A) and largest (B) value of
    (d x n_i) . v; the aim facet's ends E, F are its extreme vertices along
    d x n_j.  omega is the pair of angles at B between BA and BE, BF; mu the
    pair at A between AB and AE, AF; each pair sorted.  An angle is that of the
    two vectors projected on the view plane, arccos(u.v / (|u| |v|)) (eq. 1),
    and it is 0 when the aim vertex is not strictly on the reference facet's
    visible side, i.e. at or beyond 180 degrees from the face direction (eq. 2)."""
    import math
    nrm = facet_normals_int(scene)
    verts = _facet_vertices_int(scene)
    F = len(nrm)
    M = np.asarray(M, bool)
    offsets = np.zeros(F + 1, np.int64)
    cols: List[int] = []
    out: List[Tuple[float, float, float, float]] = []

    def dot(a, b):
        return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]

    def cross(a, b):
        return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])

    def sub(a, b):
        return (a[0] - b[0], a[1] - b[1], a[2] - b[2])

    def ends(f, t):
        vs = verts[f]
        k = [dot(t, v) for v in vs]
        return vs[int(np.argmin(k))], vs[int(np.argmax(k))]

    todo = set(range(F)) if rows is None else {int(r) for r in rows}
    for i in range(F):
        if i not in todo:
            offsets[i + 1] = len(cols)
            continue
        a_i = verts[i][0]   # a vertex of the first triangle: the plane's point
        for j in np.nonzero(M[i])[0]:
            j = int(j)
            d = view_direction(nrm[i], nrm[j])
            dd = dot(d, d)
            A, B = ends(i, cross(d, nrm[i]))
            E, Fv = ends(j, cross(d, nrm[j]))

            def angle(at, other, P):
                if dot(sub(P, a_i), nrm[i]) <= 0:      # eq. 2: not strictly on the visible side
                    return 0.0
                u, v = sub(other, at), sub(P, at)
                # projected dot products times d.d, exact in integers, then rounded once each
                uv = dd * dot(u, v) - dot(u, d) * dot(v, d)
                uu = dd * dot(u, u) - dot(u, d) ** 2
                vv = dd * dot(v, v) - dot(v, d) ** 2
                c = float(uv) / math.sqrt(float(uu) * float(vv))
                return math.degrees(math.acos(min(1.0, max(-1.0, c))))

            w = sorted((angle(B, A, E), angle(B, A, Fv)))
            m = sorted((angle(A, B, E), angle(A, B, Fv)))
            cols.append(j)
            out.append((w[0], w[1], m[0], m[1]))
        offsets[i + 1] = len(cols)
    return {"offsets": offsets, "cols": np.asarray(cols, np.int32).reshape(-1),
            "ranges": np.asarray(out, np.float64).reshape(-1, 4)}
