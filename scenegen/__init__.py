"""Seeded synthetic urban scenes: the shared input generator.

This module only produces inputs (geometry, sample points, Tx/Rx positions).
It holds none of the visibility arithmetic: no orientation, occlusion or
candidate logic lives here.  Both the FP64 oracle (``oracle/``) and the GPU
library (``paper_2501_02747_amd``) consume its arrays; neither imports the
other.

The paper's scenes exist only as figures (the scenario database of Section III-C
lists vertex points, face IDs and edge IDs per building face; case study 2 of
Section IV-B is a Manhattan-grid city of box buildings), so the generators below
stand in for them with seeded urban layouts of the same kind:

* every coordinate sits on a dyadic grid: vertices on multiples of 2^-g m,
  sample points and Tx/Rx positions on multiples of 2^-(g+k) m, where an n x n
  cell-centre sample grid needs k = log2(2n).  This keeps every coordinate, and
  every coordinate difference, exact in FP32, and keeps the degree-3 visibility
  predicates exact in FP64 (the budget is checked by ``grid_budget_bits``).
* each planar facet is a convex polygon whose vertex winding makes the first
  triangle's normal point to the facet's visible side (outside of a building,
  or up for roofs and ground).  Facets are fan-triangulated; the triangles of a
  facet are contiguous and tagged with the facet id.
* samples are the n x n cell centres of a rectangle, or of a convex roof
  polygon's bounding box restricted to points strictly inside the polygon.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014); every
draw used for geometry is an integer on the stated grid.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "SplitMix64", "Scene", "SceneBuilder", "grid_budget_bits",
    "gen_c1", "gen_c2", "gen_c3", "gen_c4_scene", "gen_c4",
    "gen_plates", "make_config",
]

_MASK = (1 << 64) - 1

KIND_GROUND, KIND_WALL, KIND_ROOF, KIND_PLATE = 0, 1, 2, 3


class SplitMix64:
    """SplitMix64 generator (Steele, Lea, Flood 2014): 64-bit state, golden-gamma increment."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on [lo, hi] (inclusive), from the top 53 bits."""
        n = hi - lo + 1
        return lo + (((self.next_u64() >> 11) * n) >> 53)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


@dataclasses.dataclass
class Scene:
    """A scene as flat arrays, ready to hand to either consumer.

    vertices       f32[V][3]   metres, multiples of 2^-g
    tri_vertices   i32[T][3]   vertex indices; triangles of a facet are contiguous
    tri_facet      i32[T]      facet id per triangle, non-decreasing
    sample_offsets i32[F+1]    CSR offsets into samples
    samples        f32[S][3]   metres, multiples of 2^-(g+k)
    tx, rx         f32[N][3]   Tx / Rx positions per snapshot (sample grid)
    snapshot_dt    seconds between consecutive snapshots of a trajectory
    edge_facets    i32[E][2]   the two facets meeting at each building edge (a
                               vertical corner or a roof rim segment)
    edge_samples   f32[E*s][3] s points per edge at (j + 1/2) / s of its length
                               (sample grid; s = samples_per_edge)
    """
    name: str
    seed: int
    g: int
    k: int
    vertices: np.ndarray
    tri_vertices: np.ndarray
    tri_facet: np.ndarray
    sample_offsets: np.ndarray
    samples: np.ndarray
    facet_kind: np.ndarray
    facet_building: np.ndarray
    tx: np.ndarray
    rx: np.ndarray
    snapshot_dt: float = 0.01
    edge_facets: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 2), np.int32))
    edge_samples: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3), np.float32))
    samples_per_edge: int = 0

    @property
    def n_facets(self) -> int:
        return int(self.sample_offsets.shape[0] - 1)

    @property
    def n_triangles(self) -> int:
        return int(self.tri_vertices.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.samples.shape[0])

    @property
    def n_snapshots(self) -> int:
        return int(self.tx.shape[0])

    def with_snapshots(self, tx: np.ndarray, rx: np.ndarray) -> "Scene":
        return dataclasses.replace(self, tx=np.ascontiguousarray(tx, np.float32),
                                   rx=np.ascontiguousarray(rx, np.float32))

    def summary(self) -> dict:
        return {"name": self.name, "seed": self.seed, "facets": self.n_facets,
                "triangles": self.n_triangles, "samples": self.n_samples,
                "snapshots": self.n_snapshots, "g": self.g, "k": self.k}


class SceneBuilder:
    """Accumulates convex planar facets in integer grid units.

    Vertex coordinates are integers in units of 2^-g m, sample coordinates
    integers in units of 2^-(g+k) m.  ``add_rect`` takes (v0, U, V) with the
    visible side along U x V.
    """

    def __init__(self, g: int, k: int):
        self.g, self.k = g, k
        self.vs = 1 << k          # sample units per vertex unit
        self.verts: List[Tuple[int, int, int]] = []
        self.tris: List[Tuple[int, int, int]] = []
        self.tri_facet: List[int] = []
        self.samples: List[Tuple[int, int, int]] = []
        self.offsets: List[int] = [0]
        self.kind: List[int] = []
        self.building: List[int] = []
        # building edges: (a, b) in vertex units and the two facets meeting there
        self.edges: List[Tuple[Tuple[int, int, int], Tuple[int, int, int], int, int]] = []

    def add_edge(self, a, b, fa: int, fb: int) -> None:
        self.edges.append((tuple(int(c) for c in a), tuple(int(c) for c in b), int(fa), int(fb)))

    @property
    def n_facets(self) -> int:
        return len(self.kind)

    def _add_facet(self, poly, samples, kind, building):
        f = self.n_facets
        base = len(self.verts)
        self.verts.extend(tuple(int(c) for c in v) for v in poly)
        for m in range(1, len(poly) - 1):
            self.tris.append((base, base + m, base + m + 1))
            self.tri_facet.append(f)
        self.samples.extend(tuple(int(c) for c in s) for s in samples)
        self.offsets.append(len(self.samples))
        self.kind.append(kind)
        self.building.append(building)
        return f

    def add_mesh_facet(self, verts, tris, samples, kind: int = KIND_PLATE, building: int = -1) -> int:
        """Facet from explicit triangles: verts (vertex units), tris (indices into
        verts, the first triangle's winding gives the visible side), samples
        (sample units).  For test scenes with non-convex facets."""
        f = self.n_facets
        base = len(self.verts)
        self.verts.extend(tuple(int(c) for c in v) for v in verts)
        for t in tris:
            self.tris.append(tuple(base + int(c) for c in t))
            self.tri_facet.append(f)
        self.samples.extend(tuple(int(c) for c in q) for q in samples)
        self.offsets.append(len(self.samples))
        self.kind.append(kind)
        self.building.append(building)
        return f

    def add_rect(self, v0, U, V, n: int, kind: int = KIND_PLATE, building: int = -1) -> int:
        """Rectangle v0, v0+U, v0+U+V, v0+V (vertex units); n x n cell-centre samples."""
        if (1 << self.k) != 2 * n:
            raise ValueError(f"n={n} samples per side needs k={int(math.log2(2 * n))}, builder has k={self.k}")
        v0, U, V = (tuple(int(c) for c in x) for x in (v0, U, V))
        poly = [v0,
                tuple(v0[i] + U[i] for i in range(3)),
                tuple(v0[i] + U[i] + V[i] for i in range(3)),
                tuple(v0[i] + V[i] for i in range(3))]
        # p_ab = v0 + (2a+1)/(2n) U + (2b+1)/(2n) V; in sample units 2^k = 2n.
        smp = []
        for a in range(n):
            for b in range(n):
                smp.append(tuple(v0[i] * 2 * n + (2 * a + 1) * U[i] + (2 * b + 1) * V[i] for i in range(3)))
        return self._add_facet(poly, smp, kind, building)

    def add_roof_polygon(self, xy_ccw: Sequence[Tuple[int, int]], z: int, n: int,
                         building: int = -1) -> int:
        """Horizontal convex polygon (CCW seen from above, vertex units) at height z."""
        poly = [(x, y, z) for (x, y) in xy_ccw]
        vs = self.vs
        xs = [p[0] for p in xy_ccw]
        ys = [p[1] for p in xy_ccw]
        x0, x1, y0, y1 = min(xs), max(xs), min(ys), max(ys)
        sv = [(x * vs, y * vs) for (x, y) in xy_ccw]
        m = len(sv)

        def strictly_inside(px, py):
            for i in range(m):
                ax, ay = sv[i]
                bx, by = sv[(i + 1) % m]
                if (bx - ax) * (py - ay) - (by - ay) * (px - ax) <= 0:
                    return False
            return True

        smp = []
        for a in range(n):
            for b in range(n):
                px = x0 * 2 * n + (2 * a + 1) * (x1 - x0)
                py = y0 * 2 * n + (2 * b + 1) * (y1 - y0)
                if strictly_inside(px, py):
                    smp.append((px, py, z * vs))
        if not smp:
            cx = round(sum(x for x, _ in sv) / m)
            cy = round(sum(y for _, y in sv) / m)
            if not strictly_inside(cx, cy):
                raise ValueError("roof polygon has no interior sample point")
            smp.append((cx, cy, z * vs))
        return self._add_facet(poly, smp, KIND_ROOF, building)

    def add_box(self, x0, y0, x1, y1, h, n, building, split_x: int = 1, omit=()) -> List[int]:
        """Axis-aligned box building: 4 walls (x-walls split into `split_x` panels) + roof.
        Facets are made in the order south panels, north panels, west, east, roof;
        positions listed in `omit` are left out (test scenes with open boxes)."""
        ids = []
        w, d = x1 - x0, y1 - y0
        if w % split_x:
            raise ValueError("panel split must land on the vertex grid")
        pw = w // split_x
        parts = []
        for s in range(split_x):   # south wall, outward -y: U=+x, V=+z
            parts.append(((x0 + s * pw, y0, 0), (pw, 0, 0), (0, 0, h), KIND_WALL))
        for s in range(split_x):   # north wall, outward +y: U=+z, V=+x
            parts.append(((x0 + s * pw, y1, 0), (0, 0, h), (pw, 0, 0), KIND_WALL))
        parts.append(((x0, y0, 0), (0, 0, h), (0, d, 0), KIND_WALL))  # west, -x
        parts.append(((x1, y0, 0), (0, d, 0), (0, 0, h), KIND_WALL))  # east, +x
        parts.append(((x0, y0, h), (w, 0, 0), (0, d, 0), KIND_ROOF))  # roof, +z
        pid = {}
        for m, (v0, U, V, kind) in enumerate(parts):
            if m not in omit:
                pid[m] = self.add_rect(v0, U, V, n, kind, building)
                ids.append(pid[m])
        # edges where two present facets meet: four vertical corners, the roof rim
        south, north = list(range(split_x)), list(range(split_x, 2 * split_x))
        west, east, roof = 2 * split_x, 2 * split_x + 1, 2 * split_x + 2

        def edge(a, b, m1, m2):
            if m1 in pid and m2 in pid:
                self.add_edge(a, b, pid[m1], pid[m2])

        edge((x0, y0, 0), (x0, y0, h), south[0], west)
        edge((x1, y0, 0), (x1, y0, h), south[-1], east)
        edge((x0, y1, 0), (x0, y1, h), north[0], west)
        edge((x1, y1, 0), (x1, y1, h), north[-1], east)
        for s in range(split_x):
            edge((x0 + s * pw, y0, h), (x0 + (s + 1) * pw, y0, h), south[s], roof)
            edge((x0 + s * pw, y1, h), (x0 + (s + 1) * pw, y1, h), north[s], roof)
        edge((x0, y0, h), (x0, y1, h), west, roof)
        edge((x1, y0, h), (x1, y1, h), east, roof)
        return ids

    def build(self, name: str, seed: int, tx_s=None, rx_s=None) -> Scene:
        """Convert to metres (exact power-of-two scaling into float32)."""
        vscale = 2.0 ** (-self.g)
        sscale = 2.0 ** (-(self.g + self.k))
        verts = np.asarray(self.verts, dtype=np.int64).reshape(-1, 3)
        smp = np.asarray(self.samples, dtype=np.int64).reshape(-1, 3)
        lim = 1 << 24
        if np.abs(verts).max(initial=0) >= lim or np.abs(smp).max(initial=0) >= lim:
            raise ValueError("coordinate does not fit FP32 exactly")
        # edge samples at (2j + 1) / (2 s) of each edge, s = 2^(k-1) (the facet sample
        # spacing along a side): integers in sample units
        s_e = self.vs // 2
        esmp = [tuple(a[i] * self.vs + (b[i] - a[i]) * (2 * j + 1) for i in range(3))
                for (a, b, _, _) in self.edges for j in range(s_e)]
        esmp = np.asarray(esmp, dtype=np.int64).reshape(-1, 3)
        if np.abs(esmp).max(initial=0) >= lim:
            raise ValueError("edge sample does not fit FP32 exactly")
        tx_s = np.zeros((0, 3), np.int64) if tx_s is None else np.asarray(tx_s, np.int64).reshape(-1, 3)
        rx_s = np.zeros((0, 3), np.int64) if rx_s is None else np.asarray(rx_s, np.int64).reshape(-1, 3)
        return Scene(
            name=name, seed=seed, g=self.g, k=self.k,
            vertices=(verts.astype(np.float64) * vscale).astype(np.float32),
            tri_vertices=np.asarray(self.tris, dtype=np.int32).reshape(-1, 3),
            tri_facet=np.asarray(self.tri_facet, dtype=np.int32),
            sample_offsets=np.asarray(self.offsets, dtype=np.int32),
            samples=(smp.astype(np.float64) * sscale).astype(np.float32),
            facet_kind=np.asarray(self.kind, dtype=np.int8),
            facet_building=np.asarray(self.building, dtype=np.int32),
            tx=(tx_s.astype(np.float64) * sscale).astype(np.float32),
            rx=(rx_s.astype(np.float64) * sscale).astype(np.float32),
            edge_facets=np.asarray([(fa, fb) for (_, _, fa, fb) in self.edges], dtype=np.int32).reshape(-1, 2),
            edge_samples=(esmp.astype(np.float64) * sscale).astype(np.float32),
            samples_per_edge=s_e if self.edges else 0,
        )


def grid_budget_bits(scene: Scene) -> float:
    """log2 of the largest integer (in the finest grid unit of each quantity)
    that an FP64 evaluation of the degree-3 segment/triangle and orientation
    predicates can produce.  <= 53 means FP64 evaluation is exact.

    D = largest absolute coordinate difference between any two points (vertices,
    samples, Tx/Rx); E = largest absolute component of a triangle edge.  In units
    of 2^-(3g+2k) m^3 the u+v-vs-det comparison is bounded by 6 D E^2 + 12 D^2 E.
    """
    pts = [scene.vertices.astype(np.float64), scene.samples.astype(np.float64)]
    if scene.tx.size:
        pts += [scene.tx.astype(np.float64), scene.rx.astype(np.float64)]
    allp = np.concatenate(pts)
    D = float((allp.max(0) - allp.min(0)).max())
    v = scene.vertices.astype(np.float64)[scene.tri_vertices]
    E = float(max(np.abs(v[:, 1] - v[:, 0]).max(), np.abs(v[:, 2] - v[:, 0]).max(),
                  np.abs(v[:, 2] - v[:, 1]).max()))
    bound = (6 * D * E * E + 12 * D * D * E) * 2.0 ** (3 * scene.g + 2 * scene.k)
    return math.log2(bound) if bound > 0 else 0.0


# ---------------------------------------------------------------------------
# Closed-form helper scenes
# ---------------------------------------------------------------------------

def gen_plates(rects, g: int = 4, n: int = 4, tx=None, rx=None, name="plates") -> Scene:
    """Scene of explicit rectangles given in metres as (v0, U, V) with visible side U x V."""
    k = int(math.log2(2 * n))
    b = SceneBuilder(g, k)
    su = 1 << g
    for v0, U, V in rects:
        conv = lambda x: tuple(_to_units(c, su) for c in x)
        b.add_rect(conv(v0), conv(U), conv(V), n, KIND_PLATE, -1)
    ss = 1 << (g + k)
    tx_s = None if tx is None else [[_to_units(c, ss) for c in p] for p in tx]
    rx_s = None if rx is None else [[_to_units(c, ss) for c in p] for p in rx]
    return b.build(name, 0, tx_s, rx_s)


def _to_units(x: float, per_m: int) -> int:
    v = x * per_m
    if v != int(v):
        raise ValueError(f"{x} is not on the 1/{per_m} m grid")
    return int(v)


# ---------------------------------------------------------------------------
# Config 1: tiny urban scene (200 x 200 m, 8 boxes, 42 facets / 84 triangles)
# ---------------------------------------------------------------------------

def _place_boxes(rng, n_boxes, lo, hi, side_lo, side_hi, gap, su):
    """Rejection-place n axis-aligned footprints (vertex units) with >= gap between them."""
    boxes = []
    tries = 0
    while len(boxes) < n_boxes:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place buildings")
        w = rng.randint(side_lo * su, side_hi * su)
        d = rng.randint(side_lo * su, side_hi * su)
        x0 = rng.randint(lo * su + 2 * su, hi * su - 2 * su - w)
        y0 = rng.randint(lo * su + 2 * su, hi * su - 2 * su - d)
        ok = True
        for (bx0, by0, bx1, by1) in boxes:
            if not (x0 + w + gap * su <= bx0 or bx1 + gap * su <= x0 or
                    y0 + d + gap * su <= by0 or by1 + gap * su <= y0):
                ok = False
                break
        if ok:
            boxes.append((x0, y0, x0 + w, y0 + d))
    return boxes


def _outside_all(x, y, boxes_m, clear):
    for (x0, y0, x1, y1) in boxes_m:
        if x0 - clear < x < x1 + clear and y0 - clear < y < y1 + clear:
            return False
    return True


def _random_free_point(rng, lo, hi, boxes_m, ss, clear=1.0):
    while True:
        x = rng.randint(int(lo * ss), int(hi * ss))
        y = rng.randint(int(lo * ss), int(hi * ss))
        if _outside_all(x / ss, y / ss, boxes_m, clear):
            return x, y


def gen_c1(seed: int = 1, n_snap: int = 10) -> Scene:
    """200 x 200 m ground (two 100 x 200 m facets), 8 box buildings with sides
    U[10,30] m and heights U[10,40] m, >= 4 m apart; 4 x 4 samples; g = 4."""
    g, n = 4, 4
    k = 3
    su, ss = 1 << g, 1 << (g + k)
    rng = SplitMix64(0xC1C1_0000_0000 + seed)
    b = SceneBuilder(g, k)
    b.add_rect((-100 * su, -100 * su, 0), (100 * su, 0, 0), (0, 200 * su, 0), n, KIND_GROUND)
    b.add_rect((0, -100 * su, 0), (100 * su, 0, 0), (0, 200 * su, 0), n, KIND_GROUND)
    boxes = _place_boxes(rng, 8, -100, 100, 10, 30, 4, su)
    for bi, (x0, y0, x1, y1) in enumerate(boxes):
        h = rng.randint(10 * su, 40 * su)
        b.add_box(x0, y0, x1, y1, h, n, bi)
    boxes_m = [tuple(c / su for c in bx) for bx in boxes]
    tx, rx = [], []
    for _ in range(n_snap):
        x, y = _random_free_point(rng, -99, 99, boxes_m, ss)
        tx.append((x, y, 25 * ss))
        x, y = _random_free_point(rng, -99, 99, boxes_m, ss)
        rx.append((x, y, int(1.5 * ss)))
    return b.build("c1", seed, tx, rx)


# ---------------------------------------------------------------------------
# Config 2: 1 x 1 km Manhattan grid, 200 buildings, 2000 facets / 4000 triangles
# ---------------------------------------------------------------------------

def gen_c2(seed: int = 2, n_snap: int = 1000, nx: int = 10, ny: int = 20) -> Scene:
    """nx x ny lattice of 100 x 50 m cells (80 x 30 m block + 20 m streets).
    Each block: 80 m walls as two 40 m panels, 30 m walls, roof (7 facets);
    each cell: 3 street ground tiles.  Heights U[10,60] m; 8 x 8 samples; g = 3.
    Rx drives 120 km/h along an east-west street centreline at 1.5 m, one snapshot
    every 10 ms; Tx is fixed 30 m above an intersection centre."""
    g, n, k = 3, 8, 4
    su, ss = 1 << g, 1 << (g + k)
    rng = SplitMix64(0xC2C2_0000_0000 + seed)
    b = SceneBuilder(g, k)
    ox, oy = -50 * nx, -25 * ny
    for cy in range(ny):
        for cx in range(nx):
            x0, y0 = (ox + 100 * cx) * su, (oy + 50 * cy) * su
            h = rng.randint(10 * su, 60 * su)
            bid = cy * nx + cx
            b.add_box(x0, y0, x0 + 80 * su, y0 + 30 * su, h, n, bid, split_x=2)
            # street tiles (ground, facing up): east strip, north strip, intersection
            b.add_rect((x0 + 80 * su, y0, 0), (20 * su, 0, 0), (0, 30 * su, 0), n, KIND_GROUND)
            b.add_rect((x0, y0 + 30 * su, 0), (80 * su, 0, 0), (0, 20 * su, 0), n, KIND_GROUND)
            b.add_rect((x0 + 80 * su, y0 + 30 * su, 0), (20 * su, 0, 0), (0, 20 * su, 0), n, KIND_GROUND)
    # Rx: 120 km/h = 1/3 m per 10 ms, snapped to the sample grid.
    row = rng.randint(0, ny - 1)
    yc = (oy + 50 * row + 40) * ss
    route = n_snap / 3.0
    span = 100 * nx - 10
    start = rng.randint(0, max(0, int(span - route) - 1))
    xs0 = (ox + 5 + start) * ss
    rx = [(xs0 + round(i * ss / 3.0), yc, int(1.5 * ss)) for i in range(n_snap)]
    tcx, tcy = rng.randint(0, nx - 1), rng.randint(0, ny - 1)
    txp = ((ox + 100 * tcx + 90) * ss, (oy + 50 * tcy + 40) * ss, 30 * ss)
    tx = [txp] * n_snap
    return b.build("c2", seed, tx, rx)


# ---------------------------------------------------------------------------
# Config 3: 4 x 4 km city of extruded convex 4..8-gons
# ---------------------------------------------------------------------------

def _convex_polygon(rng, cx, cy, k, radius_units, snap):
    """Convex k-gon at sorted random angles, vertices snapped to multiples of `snap`."""
    for _ in range(64):
        ang = sorted(rng.uniform() * 2 * math.pi for _ in range(k))
        pts = []
        for a in ang:
            x = cx + radius_units * math.cos(a)
            y = cy + radius_units * math.sin(a)
            pts.append((int(round(x / snap)) * snap, int(round(y / snap)) * snap))
        ok = len(set(pts)) == k
        if ok:
            for i in range(k):
                ax, ay = pts[i]
                bx, by = pts[(i + 1) % k]
                cx2, cy2 = pts[(i + 2) % k]
                if (bx - ax) * (cy2 - by) - (by - ay) * (cx2 - bx) <= 0:
                    ok = False
                    break
        if ok:
            return pts
    r = int(radius_units * 0.7 / snap) * snap
    return [(cx - r, cy - r), (cx + r, cy - r), (cx + r, cy + r), (cx - r, cy + r)]


def gen_c3(seed: int = 3, n_snap: int = 10000, cells: int = 50, n_buildings: int = 2000,
           max_panel: float = 25.0) -> Scene:
    """cells x cells lattice of 80 m cells; n_buildings cells (seeded) hold a
    convex k-gon (k ~ U{4..8}, radius U[10,30] m) extruded to U[10,60] m.  Walls
    are split into 1, 2 or 4 equal panels of <= 25 m (about 20k facets /
    44k triangles in total), roofs are one facet, ground is one
    80 x 80 m tile per cell.  4 x 4 samples; g = 2.  Tx and Rx are vehicles at
    1.5 m on the cell-boundary corridors, 5-20 m/s, one snapshot per 10 ms."""
    g, n, k = 2, 4, 3
    su, ss = 1 << g, 1 << (g + k)
    rng = SplitMix64(0xC3C3_0000_0000 + seed)
    b = SceneBuilder(g, k)
    half = cells * 40
    for cy in range(cells):
        for cx in range(cells):
            x0, y0 = (-half + 80 * cx) * su, (-half + 80 * cy) * su
            b.add_rect((x0, y0, 0), (80 * su, 0, 0), (0, 80 * su, 0), n, KIND_GROUND)
    idx = list(range(cells * cells))
    for i in range(len(idx) - 1, 0, -1):           # Fisher-Yates with SplitMix64
        j = rng.randint(0, i)
        idx[i], idx[j] = idx[j], idx[i]
    snap = 2 * su                                   # polygon corners on a 2 m grid
    for bid, c in enumerate(sorted(idx[:n_buildings])):
        cx, cy = c % cells, c // cells
        ccx, ccy = (-half + 80 * cx + 40) * su, (-half + 80 * cy + 40) * su
        kk = rng.randint(4, 8)
        rad = rng.randint(10 * su, 30 * su)
        poly = _convex_polygon(rng, ccx, ccy, kk, rad, snap)
        h = rng.randint(10 * su, 60 * su)
        walls, rim = [], []
        for m in range(len(poly)):
            ax, ay = poly[m]
            bx, by = poly[(m + 1) % len(poly)]
            dx, dy = bx - ax, by - ay
            L = math.hypot(dx, dy) / su
            gcd = math.gcd(abs(dx), abs(dy))
            npan = 1
            while L / npan > max_panel and gcd % (npan * 2) == 0:
                npan *= 2
            px, py = dx // npan, dy // npan
            panels = []
            for s in range(npan):
                panels.append(b.add_rect((ax + s * px, ay + s * py, 0), (px, py, 0), (0, 0, h), n, KIND_WALL, bid))
                rim.append(((ax + s * px, ay + s * py, h), (ax + (s + 1) * px, ay + (s + 1) * py, h), panels[-1]))
            walls.append(panels)
        roof = b.add_roof_polygon(poly, h, n, bid)
        # building edges: the vertical corner at each polygon vertex, the roof rim over every panel
        for m in range(len(poly)):
            ax, ay = poly[m]
            b.add_edge((ax, ay, 0), (ax, ay, h), walls[m - 1][-1], walls[m][0])
        for a, bb, f in rim:
            b.add_edge(a, bb, f, roof)
    tx = _corridor_drive(rng, cells, half, ss, n_snap)
    rx = _corridor_drive(rng, cells, half, ss, n_snap)
    return b.build("c3", seed, tx, rx)


def _corridor_drive(rng, cells, half, ss, n_snap, dt=0.01):
    """Vehicle on the cell-boundary lines at 1.5 m, constant speed U[5,20] m/s,
    random turn at every corridor crossing (never leaving the interior lines)."""
    speed = 5 + 15 * rng.uniform()
    gx, gy = rng.randint(1, cells - 1), rng.randint(1, cells - 1)
    dirs = [(1, 0), (0, 1), (-1, 0), (0, -1)]
    d = dirs[rng.randint(0, 3)]
    s_along = 0.0                 # metres travelled since the last crossing
    out = []
    for _ in range(n_snap):
        x = (-half + 80 * gx) + d[0] * s_along
        y = (-half + 80 * gy) + d[1] * s_along
        out.append((int(round(x * ss)), int(round(y * ss)), int(1.5 * ss)))
        s_along += speed * dt
        while s_along >= 80.0:
            s_along -= 80.0
            gx += d[0]
            gy += d[1]
            options = []
            for nd in dirs:
                if nd == (-d[0], -d[1]):
                    continue
                nx_, ny_ = gx + nd[0], gy + nd[1]
                if 1 <= nx_ <= cells - 1 and 1 <= ny_ <= cells - 1:
                    options.append(nd)
            d = options[rng.randint(0, len(options) - 1)]
    return out


# ---------------------------------------------------------------------------
# Config 4: 64 uneven scenes from the config-1 generator, scaled
# ---------------------------------------------------------------------------

def gen_c4_scene(seed: int, f_target: Optional[int] = None, n_snap: Optional[int] = None) -> Scene:
    """Config-1 style scene at config-1 building density (5000 m^2 per box),
    F ~ U[500, 5000], 200 x 200 m ground tiles, 4 x 4 samples, N ~ U{100..2000}
    snapshots: Tx fixed at 25 m, Rx random walk (0.5 m steps) at 1.5 m."""
    n, k = 4, 3
    rng = SplitMix64(0xC4C4_0000_0000 + seed)
    if f_target is None:
        f_target = rng.randint(500, 5000)
    if n_snap is None:
        n_snap = rng.randint(100, 2000)
    nb = max(1, f_target // 5)
    for _ in range(8):
        side = max(200, int(math.ceil(math.sqrt(nb * 5000.0) / 200.0)) * 200)
        tiles = (side // 200) ** 2
        nb_new = max(1, (f_target - tiles) // 5)
        if nb_new == nb:
            break
        nb = nb_new
    half = side // 2
    # largest vertex grid that keeps the FP64 predicates exact (checked below)
    for g in (4, 3, 2):
        D, E = float(side), 200.0
        if math.log2((6 * D * E * E + 12 * D * D * E) * 2.0 ** (3 * g + 2 * k)) <= 52:
            break
    su, ss = 1 << g, 1 << (g + k)
    b = SceneBuilder(g, k)
    for ty in range(side // 200):
        for tx_ in range(side // 200):
            b.add_rect(((-half + 200 * tx_) * su, (-half + 200 * ty) * su, 0), (200 * su, 0, 0),
                       (0, 200 * su, 0), n, KIND_GROUND)
    boxes = _place_boxes(rng, nb, -half, half, 10, 30, 4, su)
    for bi, (x0, y0, x1, y1) in enumerate(boxes):
        h = rng.randint(10 * su, 40 * su)
        b.add_box(x0, y0, x1, y1, h, n, bi)
    boxes_m = [tuple(c / su for c in bx) for bx in boxes]
    tx = [(*_random_free_point(rng, -half + 1, half - 1, boxes_m, ss), 25 * ss)] * n_snap
    x, y = _random_free_point(rng, -half + 1, half - 1, boxes_m, ss)
    rx = []
    step = ss // 2
    dirs = [(1, 0), (0, 1), (-1, 0), (0, -1)]
    for _ in range(n_snap):
        rx.append((x, y, int(1.5 * ss)))
        for _t in range(8):
            dx, dy = dirs[rng.randint(0, 3)]
            nx_, ny_ = x + dx * step, y + dy * step
            if (-half + 1) * ss <= nx_ <= (half - 1) * ss and (-half + 1) * ss <= ny_ <= (half - 1) * ss \
                    and _outside_all(nx_ / ss, ny_ / ss, boxes_m, 1.0):
                x, y = nx_, ny_
                break
    return b.build(f"c4_{seed}", seed, tx, rx)


def gen_c4(first_seed: int = 1000, n_scenes: int = 64) -> List[Scene]:
    return [gen_c4_scene(first_seed + i) for i in range(n_scenes)]


def make_config(name: str, seed: Optional[int] = None, **kw) -> Scene:
    """Named workloads: c1 tiny urban, c2 urban grid, c3 large city, c4 one batched scene."""
    if name == "c1":
        return gen_c1(1 if seed is None else seed, **kw)
    if name == "c2":
        return gen_c2(2 if seed is None else seed, **kw)
    if name == "c3":
        return gen_c3(3 if seed is None else seed, **kw)
    if name == "c4":
        return gen_c4_scene(1000 if seed is None else seed, **kw)
    raise KeyError(name)
