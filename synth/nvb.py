"""Newest-vertex bisection (NVB) for surface triangulations.

Convention: a triangle stored as (a, b, c) has reference edge (a, b); c is
its newest vertex.  Bisecting it inserts the midpoint m of (a, b) and gives
the sons (c, a, m) and (b, c, m), whose reference edges (c, a) and (b, c)
lie opposite the newest vertex m (Fig. "nvb" of the paper).  Both sons keep
the parent's orientation.

Refinement follows Algorithm step (iv): the marked elements get their edges
marked (all three for "bisec3", the reference edge only for "bisec1"), the
marking is closed so that every element with a marked edge also has its
reference edge marked (this is what prevents hanging nodes), and each element
is then split into 2, 3 or 4 sons.  Midpoints are plain edge midpoints (the
surfaces are polyhedral).
"""

from __future__ import annotations

import numpy as np


def init_reference_edges(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Rotate every triangle cyclically (orientation kept) so that its longest
    edge is the reference edge (a, b).  Ties go to the lowest local edge."""
    tris = np.asarray(tris, dtype=np.int64)
    P = np.asarray(verts, dtype=np.float64)[tris]
    l01 = np.linalg.norm(P[:, 1] - P[:, 0], axis=1)
    l12 = np.linalg.norm(P[:, 2] - P[:, 1], axis=1)
    l20 = np.linalg.norm(P[:, 0] - P[:, 2], axis=1)
    k = np.argmax(np.stack([l01, l12, l20], axis=1), axis=1)  # first max wins
    out = tris.copy()
    r1 = k == 1
    r2 = k == 2
    out[r1] = tris[r1][:, [1, 2, 0]]
    out[r2] = tris[r2][:, [2, 0, 1]]
    return out.astype(np.int32)


def _edge_keys(tris: np.ndarray, M: int):
    a, b, c = tris[:, 0].astype(np.int64), tris[:, 1].astype(np.int64), tris[:, 2].astype(np.int64)

    def key(p, q):
        return np.minimum(p, q) * M + np.maximum(p, q)

    return key(a, b), key(b, c), key(c, a)


def refine_nvb(verts: np.ndarray, tris: np.ndarray, marked, mode: str = "bisec3"):
    """Refine the marked elements (indices or boolean mask).

    Returns (verts, tris, parent) where parent[k] is the index of the element
    of the input mesh that contains new element k.  New vertices are
    appended in increasing order of their edge key, sons are emitted in
    parent order, so the result is deterministic."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    N, M = tris.shape[0], verts.shape[0]
    mk = np.zeros(N, dtype=bool)
    mk[np.asarray(marked)] = True
    e01, e12, e20 = _edge_keys(tris, M)
    if mode == "bisec3":
        emark = np.unique(np.concatenate([e01[mk], e12[mk], e20[mk]]))
    elif mode == "bisec1":
        emark = np.unique(e01[mk])
    else:
        raise ValueError(mode)
    # closure: an element with any marked edge gets its reference edge marked
    while True:
        m12 = np.isin(e12, emark)
        m20 = np.isin(e20, emark)
        m01 = np.isin(e01, emark)
        add = ~m01 & (m12 | m20)
        if not add.any():
            break
        emark = np.unique(np.concatenate([emark, e01[add]]))
    if emark.size == 0:
        return verts.copy(), tris.astype(np.int32), np.arange(N)
    ea = emark // M
    eb = emark % M
    new_v = 0.5 * (verts[ea] + verts[eb])
    V = np.concatenate([verts, new_v], axis=0)

    def mid(keys):
        return M + np.searchsorted(emark, keys)

    a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
    r, s1, s2 = m01, m20, m12
    pieces = []  # (parent, slot, tri(n,3))
    idx = np.arange(N)
    keep = ~r
    pieces.append((idx[keep], 0, tris[keep]))
    # son 1 = (c, a, m), its reference edge (c, a) is edge e20
    t = r & ~s1
    m = mid(e01[t])
    pieces.append((idx[t], 0, np.stack([c[t], a[t], m], axis=1)))
    t = r & s1
    m = mid(e01[t])
    m1 = mid(e20[t])
    pieces.append((idx[t], 0, np.stack([m, c[t], m1], axis=1)))
    pieces.append((idx[t], 1, np.stack([a[t], m, m1], axis=1)))
    # son 2 = (b, c, m), its reference edge (b, c) is edge e12
    t = r & ~s2
    m = mid(e01[t])
    pieces.append((idx[t], 2, np.stack([b[t], c[t], m], axis=1)))
    t = r & s2
    m = mid(e01[t])
    m2 = mid(e12[t])
    pieces.append((idx[t], 2, np.stack([m, b[t], m2], axis=1)))
    pieces.append((idx[t], 3, np.stack([c[t], m, m2], axis=1)))
    par = np.concatenate([p for p, _, _ in pieces])
    slot = np.concatenate([np.full(p.size, s) for p, s, _ in pieces])
    T = np.concatenate([x.reshape(-1, 3) for _, _, x in pieces], axis=0)
    order = np.lexsort((slot, par))
    return V, T[order].astype(np.int32), par[order]


def refine_uniform(verts, tris, times: int = 1):
    """Each refinement splits every triangle into 4 (bisec3 of all)."""
    parent = np.arange(len(tris))
    for _ in range(times):
        verts, tris, p = refine_nvb(verts, tris, np.arange(len(tris)), "bisec3")
        parent = parent[p]
    return verts, tris, parent


def _diam(verts, tris):
    P = np.asarray(verts)[np.asarray(tris)]
    return np.max(np.stack([np.linalg.norm(P[:, 1] - P[:, 0], axis=1),
                            np.linalg.norm(P[:, 2] - P[:, 1], axis=1),
                            np.linalg.norm(P[:, 0] - P[:, 2], axis=1)], axis=1), axis=1)


def refine_to_size(verts, tris, target: int):
    """Uniform refinement while the result stays <= target, then bisection of
    the largest-diameter elements (ties: lower index) until N >= target."""
    tris = np.asarray(tris)
    while 4 * len(tris) <= target:
        verts, tris, _ = refine_nvb(verts, tris, np.arange(len(tris)), "bisec3")
    while len(tris) < target:
        need = target - len(tris)
        d = _diam(verts, tris)
        order = np.lexsort((np.arange(len(tris)), -d))
        k = max(1, min(len(tris), (need + 2) // 3))
        verts, tris, _ = refine_nvb(verts, tris, order[:k], "bisec1")
    return np.asarray(verts), np.asarray(tris, dtype=np.int32)
