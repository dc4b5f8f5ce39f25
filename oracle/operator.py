"""Galerkin matrix of the single-layer operator on P0(T) (test infrastructure).

V[i, j] = <V chi_j, chi_i> = (1 / 4 pi) int_{T_i} int_{T_j} 1 / |x - y| dy dx
(Appendix A, eq. "discreteform:residual", with the operator of eq.
"strongform"; matrix form as in eq. "laplace_system").  The matrix is
symmetric, so only i <= j is computed and mirrored.

Pair classes are decided from vertex indices (the mesh is conforming,
Section 2.1): 3 shared vertices = coincident, 2 = edge-adjacent,
1 = vertex-adjacent, 0 = regular.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from .quadrature import ss_rule, triangle_rule

FOUR_PI = 4.0 * math.pi


def element_geometry(verts, tris):
    """Per element: area |T| = |(P1 - P0) x (P2 - P0)| / 2, centroid
    (P0 + P1 + P2) / 3 and the squared diameter (largest squared edge
    length) of each plane triangle (Section 2.1)."""
    P = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    P0, P1, P2 = P[:, 0], P[:, 1], P[:, 2]
    area = 0.5 * np.linalg.norm(np.cross(P1 - P0, P2 - P0), axis=1)
    cen = (P0 + P1 + P2) / 3.0

    def l2(a, b):
        d = b - a
        return d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]

    diam2 = np.maximum(np.maximum(l2(P0, P1), l2(P1, P2)), l2(P2, P0))
    return {"area": area, "centroid": cen, "diam2": diam2, "diam": np.sqrt(diam2)}


def quad_points(verts, tris, n: int = 4):
    """Physical points x = P0 + s (P1 - P0) + t (P2 - P0) and weights
    W = 2 |T| w of the collapsed n x n rule on every element; sum W = |T|."""
    s, t, w = triangle_rule(n)
    P = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    P0, P1, P2 = P[:, 0], P[:, 1], P[:, 2]
    X = P0[:, None, :] + s[None, :, None] * (P1 - P0)[:, None, :] + t[None, :, None] * (P2 - P0)[:, None, :]
    area = element_geometry(verts, tris)["area"]
    W = 2.0 * area[:, None] * w[None, :]
    return X, W


def _vertex_to_elements(tris, M=None):
    tris = np.asarray(tris)
    M = int(tris.max()) + 1 if M is None else M
    v2e = [[] for _ in range(M)]
    for e, (a, b, c) in enumerate(tris.tolist()):
        v2e[a].append(e)
        v2e[b].append(e)
        v2e[c].append(e)
    return v2e


def classify_pairs(tris):
    """All touching pairs (i, j), i <= j, with their class and canonical
    vertex orders, as a list of (i, j, kind, Ti, Tj) where Ti, Tj are
    vertex-index triples in the order the singular rule uses:

    * coincident: Ti = Tj = T_i in input order;
    * edge: Ti = (A, B, C), Tj = (A, B, D), {A, B} the shared edge with
      A the lower vertex index, C and D the non-shared vertices;
    * vertex: Ti = (A, B, C), Tj = (A, D, E), A the shared vertex, the
      other vertices of each element in its cyclic input order after A.

    Sorted by (i, j)."""
    tris = np.asarray(tris)
    v2e = _vertex_to_elements(tris)
    out = []
    for i, ti in enumerate(tris.tolist()):
        nb = sorted(set(e for v in ti for e in v2e[v] if e >= i))
        si = set(ti)
        for j in nb:
            tj = tris[j].tolist()
            shared = si & set(tj)
            ns = len(shared)
            if ns == 3:
                out.append((i, j, "coincident", tuple(ti), tuple(ti)))
            elif ns == 2:
                A, B = sorted(shared)
                C = [v for v in ti if v not in shared][0]
                D = [v for v in tj if v not in shared][0]
                out.append((i, j, "edge", (A, B, C), (A, B, D)))
            elif ns == 1:
                A = next(iter(shared))
                k = ti.index(A)
                l = tj.index(A)
                out.append((i, j, "vertex", (A, ti[(k + 1) % 3], ti[(k + 2) % 3]),
                            (A, tj[(l + 1) % 3], tj[(l + 2) % 3])))
    return out


def near_pairs(verts, tris, near_factor: float):
    """Pairs (i, j), i != j, sharing no vertex, whose centroids are closer
    than near_factor * max(diam_i, diam_j).  The test is done on squares:
    |c_i - c_j|^2 < near_factor^2 * max(diam_i^2, diam_j^2), with
    |d|^2 = (dx dx + dy dy) + dz dz.  Returned sorted by (i, j), both
    orders included.  (Mixed-precision bookkeeping, no arithmetic of the
    method.)  Pinned by hand-built pairs at known distances and by a k-d
    tree search over the same definition."""
    g = element_geometry(verts, tris)
    c, d2 = g["centroid"], g["diam2"]
    tris = np.asarray(tris)
    nf2 = near_factor * near_factor
    out = []
    for i in range(len(tris)):
        dx = c[i, 0] - c[:, 0]
        dy = c[i, 1] - c[:, 1]
        dz = c[i, 2] - c[:, 2]
        r2 = dx * dx + dy * dy + dz * dz
        thr = nf2 * np.maximum(d2[i], d2)
        cand = np.nonzero(r2 < thr)[0]
        ti = set(tris[i].tolist())
        for j in cand.tolist():
            if j != i and not (ti & set(tris[j].tolist())):
                out.append((i, j))
    return out


def regular_entry(Xi, Wi, Xj, Wj):
    """(1 / 4 pi) sum_a sum_b W_a W_b / |x_a - y_b| for one pair."""
    d = Xi[:, None, :] - Xj[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=-1))
    return float(np.sum(Wi[:, None] * Wj[None, :] / r)) / FOUR_PI


def _chi(A, B, C, x):
    return A[None, :] + x[:, :1] * (B - A)[None, :] + x[:, 1:2] * (C - B)[None, :]


def singular_entry(verts, kind, Ti, Tj, n: int = 4):
    """(1 / 4 pi) (2|T_i|)(2|T_j|) sum w / |chi_i(x) - chi_j(y)| with the
    Sauter-Schwab-type rule of `kind` and canonical vertex orders Ti, Tj
    (see classify_pairs).  chi(x) = A + x1 (B - A) + x2 (C - B)."""
    V = np.asarray(verts, dtype=np.float64)
    A, B, C = V[Ti[0]], V[Ti[1]], V[Ti[2]]
    D0, D1, D2 = V[Tj[0]], V[Tj[1]], V[Tj[2]]
    X, Y, W = ss_rule(kind, n)
    x = _chi(A, B, C, X)
    y = _chi(D0, D1, D2, Y)
    d = x - y
    r = np.sqrt(np.sum(d * d, axis=1))
    ai = 0.5 * np.linalg.norm(np.cross(B - A, C - A))
    aj = 0.5 * np.linalg.norm(np.cross(D1 - D0, D2 - D0))
    return (2.0 * ai) * (2.0 * aj) * float(np.sum(W / r)) / FOUR_PI


class SSOrders:
    """Order of the singular rule of each touching pair (points per
    coordinate of the 4-D rule).  `base` for coincident pairs, `edge` and
    `vertex` for edge- and vertex-adjacent pairs (0: `base`); with
    `sliver` > 0, every touching pair with an element whose diam^2 exceeds
    `sliver_ratio` |T| takes at least `sliver` points (the rules lose
    accuracy on thin elements: at order 4 the coincident integral of a
    triangle with angles (10, 85, 85) degrees, diam^2/|T| = 11.5, is off by
    2.4e-3, at order 8 by 2.7e-5).  An int n stands for SSOrders(n)."""

    def __init__(self, base: int = 4, edge: int = 0, vertex: int = 0, sliver: int = 0, sliver_ratio: float = 0.0):
        self.base, self.edge, self.vertex = int(base), int(edge), int(vertex)
        self.sliver, self.sliver_ratio = int(sliver), float(sliver_ratio)

    @staticmethod
    def of(x) -> "SSOrders":
        return x if isinstance(x, SSOrders) else SSOrders(int(x))

    def order(self, kind: str, diam2_i: float, area_i: float, diam2_j: float, area_j: float) -> int:
        n = self.base
        if kind == "edge" and self.edge > 0:
            n = self.edge
        elif kind == "vertex" and self.vertex > 0:
            n = self.vertex
        if self.sliver > 0 and (diam2_i > self.sliver_ratio * area_i or diam2_j > self.sliver_ratio * area_j):
            n = max(n, self.sliver)
        return n


def _pair_order(orders, geo, kind, i, j) -> int:
    return orders.order(kind, geo["diam2"][i], geo["area"][i], geo["diam2"][j], geo["area"][j])


def entry(verts, tris, i: int, j: int, far_order: int = 4, ss_order=4):
    """One matrix entry V[i, j], computed on its own (used for sampled
    checks at sizes where the full matrix is too slow on the CPU)."""
    tris = np.asarray(tris)
    a, b = (i, j) if i <= j else (j, i)
    ta, tb = tris[a].tolist(), tris[b].tolist()
    shared = set(ta) & set(tb)
    if shared:
        orders = SSOrders.of(ss_order)
        geo = element_geometry(verts, tris[[a, b]])
        for (p, q, kind, Ti, Tj) in _classify_one(tris, a, b):
            n = orders.order(kind, geo["diam2"][0], geo["area"][0], geo["diam2"][-1], geo["area"][-1])
            return singular_entry(verts, kind, Ti, Tj, n)
    X, W = quad_points(verts, tris[[a, b]], far_order)
    return regular_entry(X[0], W[0], X[1], W[1])


def _classify_one(tris, i, j):
    sub = np.asarray(tris)[[i, j]] if i != j else np.asarray(tris)[[i]]
    res = classify_pairs(sub)
    for (p, q, kind, Ti, Tj) in res:
        if (i == j and p == 0 and q == 0) or (i != j and p == 0 and q == 1):
            yield (i, j, kind, Ti, Tj)


def _rows_worker(args):
    """Rows i >= j part of V for the rows of one block: V[i, i:] with the
    regular rule (the coincident entry, where r = 0, is replaced later by the
    singular rule).  Columns are taken in chunks and the three coordinates as
    separate arrays only to bound the temporaries (a row of N = 60000 would
    otherwise hold 0.4 GB); every entry is the same sum
    (1 / 4 pi) sum_a sum_b W_a W_b / |x_a - y_b| over the 16 x 16 points."""
    verts, tris, rows, far_order = args
    X, W = quad_points(verts, tris, far_order)
    Xc = [np.ascontiguousarray(X[:, :, k]) for k in range(3)]
    N = X.shape[0]
    chunk = 512
    out = []
    for i in rows:
        vals = np.empty(N - i)
        for c0 in range(i, N, chunk):
            c1 = min(N, c0 + chunk)
            dx = Xc[0][i][None, :, None] - Xc[0][c0:c1][:, None, :]
            dy = Xc[1][i][None, :, None] - Xc[1][c0:c1][:, None, :]
            dz = Xc[2][i][None, :, None] - Xc[2][c0:c1][:, None, :]
            r = np.sqrt(dx * dx + dy * dy + dz * dz)
            with np.errstate(divide="ignore", invalid="ignore"):
                vals[c0 - i:c1 - i] = np.sum((W[i][None, :, None] * W[c0:c1][:, None, :]) / r, axis=(1, 2)) / FOUR_PI
        out.append((i, vals))
    return out


def assemble_rows(verts, tris, rows, far_order: int = 4, ss_order=4):
    """Full rows V[rows, :] (dense, N columns each), regular rule everywhere
    and singular rule on touching pairs (ss_order: an int or SSOrders)."""
    tris = np.asarray(tris)
    N = len(tris)
    orders = SSOrders.of(ss_order)
    geo = element_geometry(verts, tris)
    X, W = quad_points(verts, tris, far_order)
    v2e = _vertex_to_elements(tris, np.asarray(verts).shape[0])
    out = np.empty((len(rows), N))
    for k, i in enumerate(rows):
        d = X[i][None, :, None, :] - X[:, None, :, :]
        r = np.sqrt(np.sum(d * d, axis=-1))
        with np.errstate(divide="ignore", invalid="ignore"):
            out[k] = np.sum((W[i][None, :, None] * W[:, None, :]) / r, axis=(1, 2)) / FOUR_PI
        nb = sorted(set(e for v in tris[i].tolist() for e in v2e[v]))
        for j in nb:
            a, b = (i, j) if i <= j else (j, i)
            for (_, _, kind, Ti, Tj) in _classify_one(tris, a, b):
                out[k, j] = singular_entry(verts, kind, Ti, Tj, _pair_order(orders, geo, kind, a, b))
    return out


def mirror_upper(V, block: int = 2048):
    """V[j, i] = V[i, j] for i < j, in square blocks (no index arrays of
    N^2 / 2 entries, so that N = 60000 fits next to the 28.8 GB matrix)."""
    N = V.shape[0]
    for r0 in range(0, N, block):
        r1 = min(N, r0 + block)
        D = V[r0:r1, r0:r1]
        iu = np.triu_indices(r1 - r0, 1)
        D[(iu[1], iu[0])] = D[iu]
        for c0 in range(r1, N, block):
            c1 = min(N, c0 + block)
            V[c0:c1, r0:r1] = V[r0:r1, c0:c1].T


def assemble(verts, tris, far_order: int = 4, ss_order=4, workers: int | None = None):
    """Dense FP64 Galerkin matrix V (N x N).  Regular rule on every i <= j,
    then the singular rule overwrites the touching pairs (ss_order: an int,
    or SSOrders for orders chosen per pair); mirrored."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    N = len(tris)
    V = np.zeros((N, N))
    if workers is None:
        workers = min(os.cpu_count() or 1, 16) if N > 1500 else 1
    # interleaved row blocks balance the triangular work
    blocks = [list(range(k, N, workers * 8)) for k in range(workers * 8)] if workers > 1 else [list(range(N))]
    if workers > 1:
        import multiprocessing as mp

        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            results = ex.map(_rows_worker, [(verts, tris, b, far_order) for b in blocks])
            for res in results:
                for i, vals in res:
                    V[i, i:] = vals
    else:
        for i, vals in _rows_worker((verts, tris, blocks[0], far_order)):
            V[i, i:] = vals
    orders = SSOrders.of(ss_order)
    geo = element_geometry(verts, tris)
    for (i, j, kind, Ti, Tj) in classify_pairs(tris):
        V[i, j] = singular_entry(verts, kind, Ti, Tj, _pair_order(orders, geo, kind, i, j))
    mirror_upper(V)
    return V
