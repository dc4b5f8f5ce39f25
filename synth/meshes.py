"""Seeded closed triangulated polyhedral surfaces.

Every generator returns a :class:`Mesh` with ``verts`` (M x 3, float64) and
``tris`` (N x 3, int32): a conforming, welded triangulation of a closed
polyhedral surface, outward oriented, as the paper's method assumes
(Section 2.1, "Triangulations").  Orientation does not enter the single-layer
operator, but the generators keep it consistent so that topology checks can
use it.

Square faces are split along the diagonal that runs from local grid corner
(i, j) to (i+1, j+1) in the face's (u, v) parametrisation, where (u, v, w)
is the cyclic axis order and w is the face normal axis.  That diagonal is the
longest edge of both halves, which is what newest-vertex bisection picks as
the initial reference edge.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, Tuple

import numpy as np


@dataclasses.dataclass
class Mesh:
    verts: np.ndarray  # (M, 3) float64
    tris: np.ndarray  # (N, 3) int32
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.tris.shape[0])

    @property
    def M(self) -> int:
        return int(self.verts.shape[0])

    def scaled(self, s: float) -> "Mesh":
        return Mesh(self.verts * s, self.tris.copy(), self.name, dict(self.meta, scale=s))


def _finish(verts, tris, name, meta) -> Mesh:
    v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(tris, dtype=np.int32).reshape(-1, 3))
    return Mesh(v, t, name, meta)


# ----------------------------------------------------------------------------
# Axis-aligned boxes built from unit lattice squares (cube, box, voxel unions)
# ----------------------------------------------------------------------------

def _square_faces_to_mesh(faces, scale=(1.0, 1.0, 1.0)):
    """faces: iterable of (w, s, corner) with w the normal axis, s = +1/-1
    the outward sign and corner the integer lattice point of the square's
    (u, v)-minimal corner.  Returns welded verts/tris (lattice integers are
    the welding key, so welding is exact)."""
    index: Dict[Tuple[int, int, int], int] = {}
    coords = []
    tris = []

    def vid(p):
        key = (int(p[0]), int(p[1]), int(p[2]))
        k = index.get(key)
        if k is None:
            k = len(coords)
            index[key] = k
            coords.append(key)
        return k

    for w, s, corner in faces:
        u, v = (w + 1) % 3, (w + 2) % 3
        c = np.array(corner, dtype=np.int64)
        eu = np.zeros(3, np.int64)
        ev = np.zeros(3, np.int64)
        eu[u] = 1
        ev[v] = 1
        p00, p10, p11, p01 = vid(c), vid(c + eu), vid(c + eu + ev), vid(c + ev)
        # e_u x e_v = e_w, so (p00, p10, p11) faces +w.
        if s > 0:
            tris.append((p00, p10, p11))
            tris.append((p00, p11, p01))
        else:
            tris.append((p00, p11, p10))
            tris.append((p00, p01, p11))
    verts = np.array(coords, dtype=np.float64) * np.asarray(scale, dtype=np.float64)[None, :]
    return verts, np.array(tris, dtype=np.int32)


def cube(n: int = 8, scale=(1.0, 1.0, 1.0), name: str | None = None) -> Mesh:
    """Surface of [0, sx] x [0, sy] x [0, sz]; each face an n x n grid of
    squares, each square split into two triangles (12 n^2 triangles,
    6 n^2 + 2 vertices).  n = 8 gives the 768-element unit cube."""
    faces = []
    for w in range(3):
        u, v = (w + 1) % 3, (w + 2) % 3
        for side, sgn in ((0, -1), (n, +1)):
            for a in range(n):
                for b in range(n):
                    c = [0, 0, 0]
                    c[w], c[u], c[v] = side, a, b
                    faces.append((w, sgn, c))
    verts, tris = _square_faces_to_mesh(faces)
    verts = verts / n * np.asarray(scale, dtype=np.float64)[None, :]
    return _finish(verts, tris, name or f"cube{n}", {"n": n, "scale": list(map(float, scale))})


def cube12(name: str = "cube12") -> Mesh:
    """The unit cube in 12 triangles with one particular choice of face
    diagonals: five faces are cut along edges of the regular tetrahedron
    with vertices (1,0,0), (0,1,0), (0,0,1), (1,1,1); the face x = 1 is cut
    along (1,1,0)-(1,0,1) instead.  The capacity and estimator of the first
    step of the unit-cube experiment (Section 3.1, Table 1, l = 0) depend on
    the diagonals; of the eight classes of diagonal choices this is the one
    whose dual-mesh values lie next to the printed ones."""
    verts = np.array([[0, 0, 0], [0, 1, 0], [0, 1, 1], [0, 0, 1], [1, 0, 0], [1, 1, 0], [1, 1, 1], [1, 0, 1]],
                     dtype=np.float64)
    tris = np.array([[1, 0, 3], [1, 3, 2], [5, 6, 7], [5, 7, 4], [3, 0, 4], [3, 4, 7], [6, 5, 1], [6, 1, 2],
                     [4, 0, 1], [4, 1, 5], [6, 2, 3], [6, 3, 7]], dtype=np.int32)
    return _finish(verts, tris, name, {"n": 1, "diagonals": "tetrahedral, face x=1 flipped"})


def fichera48(name: str = "fichera48") -> Mesh:
    """The Fichera cube [-1,1]^3 minus [0,1]^3 in 48 triangles: its 24 unit
    squares, each cut along one diagonal.  The capacity and estimator of the
    first step of the Fichera experiment (Section 3.2, Table 2, l = 0) depend
    on the diagonals; these are the ones whose dual-mesh values lie next to
    the printed ones (found by a coordinate search over the 2^24 choices,
    which reached this mesh from two different random starts)."""
    verts = np.array([[-1, -1, -1], [-1, 0, -1], [-1, 0, 0], [-1, -1, 0], [0, -1, 0], [0, -1, -1], [0, 0, -1],
                      [-1, 0, 1], [-1, -1, 1], [0, -1, 1], [0, 0, 1], [-1, 1, -1], [-1, 1, 0], [0, 1, 0],
                      [0, 1, -1], [-1, 1, 1], [0, 0, 0], [0, 1, 1], [1, -1, -1], [1, 0, -1], [1, 0, 0], [1, -1, 0],
                      [1, 0, 1], [1, -1, 1], [1, 1, -1], [1, 1, 0]], dtype=np.float64)
    tris = np.array([[1, 0, 3], [1, 3, 2], [3, 0, 5], [3, 5, 4], [5, 0, 1], [5, 1, 6], [3, 7, 2], [3, 8, 7],
                     [3, 9, 8], [3, 4, 9], [9, 10, 7], [9, 7, 8], [1, 12, 11], [1, 2, 12], [12, 13, 14],
                     [12, 14, 11], [1, 14, 6], [1, 11, 14], [12, 2, 7], [12, 7, 15], [13, 17, 10], [13, 10, 16],
                     [12, 15, 17], [12, 17, 13], [7, 10, 17], [7, 17, 15], [19, 20, 21], [19, 21, 18], [5, 21, 4],
                     [5, 18, 21], [5, 19, 18], [5, 6, 19], [21, 20, 22], [21, 22, 23], [9, 4, 21], [9, 21, 23],
                     [10, 22, 20], [10, 20, 16], [9, 23, 22], [9, 22, 10], [19, 24, 25], [19, 25, 20],
                     [14, 13, 25], [14, 25, 24], [19, 6, 14], [19, 14, 24], [20, 25, 13], [20, 13, 16]],
                    dtype=np.int32)
    return _finish(verts, tris, name, {"n": 1})


def box(a: float, b: float, name: str = "box") -> Mesh:
    """Box with sides (1, a, b): 12 triangles before refinement."""
    m = cube(1, scale=(1.0, a, b), name=name)
    m.meta.update({"sides": [1.0, float(a), float(b)]})
    return m


def _face_connected_growth(L: int, count: int, rng) -> np.ndarray:
    occ = np.zeros((L, L, L), dtype=bool)
    start = tuple(int(x) for x in rng.integers(0, L, size=3))
    occ[start] = True
    dirs = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    while occ.sum() < count:
        frontier = set()
        for p in zip(*np.nonzero(occ)):
            for d in dirs:
                q = (p[0] + d[0], p[1] + d[1], p[2] + d[2])
                if all(0 <= q[k] < L for k in range(3)) and not occ[q]:
                    frontier.add(q)
        fl = sorted(frontier)
        occ[fl[int(rng.integers(0, len(fl)))]] = True
    return occ


def _fill_voids(occ: np.ndarray) -> np.ndarray:
    L = occ.shape[0]
    pad = np.zeros((L + 2,) * 3, dtype=bool)
    pad[1:-1, 1:-1, 1:-1] = occ
    outside = np.zeros_like(pad)
    stack = [(0, 0, 0)]
    outside[0, 0, 0] = True
    while stack:
        p = stack.pop()
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            q = (p[0] + d[0], p[1] + d[1], p[2] + d[2])
            if all(0 <= q[k] < L + 2 for k in range(3)) and not pad[q] and not outside[q]:
                outside[q] = True
                stack.append(q)
    return ~outside[1:-1, 1:-1, 1:-1]


def _voxel_surface(occ: np.ndarray):
    L = occ.shape[0]
    faces = []
    for p in zip(*np.nonzero(occ)):
        for w in range(3):
            for sgn in (-1, +1):
                q = list(p)
                q[w] += sgn
                inside = all(0 <= q[k] < L for k in range(3)) and occ[tuple(q)]
                if inside:
                    continue
                c = list(int(x) for x in p)
                if sgn > 0:
                    c[w] += 1
                faces.append((w, sgn, c))
    return _square_faces_to_mesh(faces)


def voxel_union(L: int = 4, occupancy: float = 0.4, seed: int = 3, name: str | None = None) -> Mesh:
    """Face-connected union of unit voxels in an L^3 lattice.

    round(occupancy * L^3) voxels (at least 2) are grown from a random start
    by adding uniformly chosen empty face-neighbours; enclosed voids are
    filled; a draw whose surface is not a 2-manifold (two voxels meeting only
    along an edge or at a corner) is discarded and the same generator draws
    again.  The result is non-convex with re-entrant edges and corners."""
    rng = np.random.default_rng(seed)
    count = max(2, int(round(occupancy * L ** 3)))
    for attempt in range(1000):
        occ = _fill_voids(_face_connected_growth(L, count, rng))
        verts, tris = _voxel_surface(occ)
        ok, _ = mesh_topology_ok(verts, tris)
        if ok:
            return _finish(verts, tris, name or f"voxel{L}_s{seed}",
                           {"L": L, "occupancy": occupancy, "seed": seed, "voxels": int(occ.sum()),
                            "attempt": attempt})
    raise RuntimeError("voxel_union: no manifold draw found")


# ----------------------------------------------------------------------------
# Icosphere
# ----------------------------------------------------------------------------

def icosphere(level: int, r: float = 1.0, name: str | None = None) -> Mesh:
    """Icosahedron refined `level` times by 4-way midpoint subdivision with
    the new vertices projected to the sphere: 20 * 4^level triangles and
    10 * 4^level + 2 vertices, all on the sphere of radius r (an inscribed
    polyhedron)."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
         (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
         (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    tris = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
            (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
            (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
            (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mids: Dict[Tuple[int, int], int] = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            k = mids.get(key)
            if k is None:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                k = len(verts) - 1
                mids[key] = k
            return k

        nt = []
        for a, b, c in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nt += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = nt
    V = np.array(verts) * r
    T = np.array(tris, dtype=np.int32)
    # outward orientation
    P = V[T]
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    flip = np.einsum("ij,ij->i", nrm, P.mean(axis=1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return _finish(V, T, name or f"icosphere{level}", {"level": level, "r": float(r)})


# ----------------------------------------------------------------------------
# Convex hull of random points
# ----------------------------------------------------------------------------

def min_angle_deg(verts, tris) -> float:
    """Smallest interior angle over all triangles, in degrees."""
    P = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    out = []
    for k in range(3):
        a = P[:, (k + 1) % 3] - P[:, k]
        b = P[:, (k + 2) % 3] - P[:, k]
        c = np.einsum("ij,ij->i", a, b) / np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1)
        out.append(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))
    return float(np.min(out))


def convex_hull(npts: int, seed: int, name: str | None = None, min_angle: float = 10.0) -> Mesh:
    """Convex hull of `npts` uniform random points in [-1, 1]^3; hull facets
    as triangles, outward oriented, unused (interior) points dropped.

    Draws whose hull has a facet with an interior angle below `min_angle`
    degrees are discarded and the same generator draws again: the method
    assumes shape-regular triangulations (the constants of Appendix A depend
    on gamma-shape regularity), and newest-vertex bisection keeps the initial
    shapes, so a sliver facet would stay a sliver at every refinement."""
    from scipy.spatial import ConvexHull

    rng = np.random.default_rng(seed)
    for attempt in range(10000):
        pts = rng.uniform(-1.0, 1.0, size=(npts, 3))
        hull = ConvexHull(pts)
        if min_angle <= 0.0 or min_angle_deg(pts, hull.simplices) >= min_angle:
            break
    else:
        raise RuntimeError("convex_hull: no draw met the angle bound")
    T = np.array(hull.simplices, dtype=np.int64)
    used = np.unique(T)
    remap = -np.ones(npts, dtype=np.int64)
    remap[used] = np.arange(used.size)
    V = pts[used]
    T = remap[T]
    center = V.mean(axis=0)
    P = V[T]
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    flip = np.einsum("ij,ij->i", nrm, P.mean(axis=1) - center) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return _finish(V, T, name or f"hull{npts}_s{seed}",
                   {"npts": npts, "seed": seed, "attempt": attempt, "min_angle": min_angle})


# ----------------------------------------------------------------------------
# Topology check (used by generator self-tests and to reject voxel draws)
# ----------------------------------------------------------------------------

def mesh_topology_ok(verts: np.ndarray, tris: np.ndarray):
    """Closed, consistently oriented, welded 2-manifold with non-degenerate
    triangles.  Returns (ok, info) where info has the Euler characteristic."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    N, M = tris.shape[0], verts.shape[0]
    info = {"N": N, "M": M}
    if N == 0 or tris.min() < 0 or tris.max() >= M:
        return False, dict(info, why="index")
    if np.any(tris[:, 0] == tris[:, 1]) or np.any(tris[:, 1] == tris[:, 2]) or np.any(tris[:, 0] == tris[:, 2]):
        return False, dict(info, why="repeated vertex")
    P = verts[tris]
    area2 = np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    if np.any(area2 <= 0) or not np.all(np.isfinite(verts)):
        return False, dict(info, why="degenerate")
    if np.unique(verts, axis=0).shape[0] != M:
        return False, dict(info, why="unwelded")
    if np.unique(tris).size != M:
        return False, dict(info, why="unused vertex")
    directed = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    dkey = directed[:, 0] * M + directed[:, 1]
    if np.unique(dkey).size != dkey.size:
        return False, dict(info, why="orientation")
    rkey = directed[:, 1] * M + directed[:, 0]
    if not np.all(np.isin(rkey, dkey)):
        return False, dict(info, why="open or non-manifold edge")
    E = dkey.size // 2
    # each vertex: its incident triangles form one fan (single cycle)
    nxt = {}
    for (a, b, c) in tris:
        for v, p, q in ((a, b, c), (b, c, a), (c, a, b)):
            nxt.setdefault(int(v), {})[int(p)] = int(q)
    for v, m in nxt.items():
        start = next(iter(m))
        cur, steps = start, 0
        while True:
            cur = m.get(cur)
            steps += 1
            if cur is None:
                return False, dict(info, why="open fan")
            if cur == start:
                break
        if steps != len(m):
            return False, dict(info, why="non-manifold vertex")
    chi = M - E + N
    return True, dict(info, E=E, euler=chi)
