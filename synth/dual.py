"""Barycentric refinement and the vertex-to-element incidence of a surface
triangulation (Section 2.1 of the paper, Fig. "dual_element").

Each triangle (v0, v1, v2) is split into six by joining its centre of
gravity c to its vertices and to the midpoints m01, m12, m20 of its edges.
The sons, in this order,

    (v0, m01, c), (m01, v1, c), (v1, m12, c), (m12, v2, c), (v2, m20, c), (m20, v0, c),

keep the parent's orientation.  Son 6t + s lies in the dual cell of the
parent vertex it touches: v0 for s = 0 and 5, v1 for s = 1 and 2, v2 for
s = 3 and 4.  The dual cell of a vertex is the union of the sons that touch
it, so the barycentric mesh is the coarsest common refinement of the mesh
and its dual.

Vertices of the barycentric mesh: the M input vertices, then one midpoint per
edge (edges numbered by increasing key min * M + max), then one centre of
gravity per triangle.  This is mesh topology and coordinates only; none of
the method's arithmetic (areas, integrals, operators) is here.
"""

from __future__ import annotations

import numpy as np

from .meshes import Mesh

# local parent vertex (0, 1, 2) of each of the six sons
SON_VERTEX = np.array([0, 1, 1, 2, 2, 0], dtype=np.int32)


def barycentric(verts: np.ndarray, tris: np.ndarray):
    """Returns (mesh, parent, owner): the barycentric refinement as a Mesh
    with 6 N triangles, parent[k] = k // 6 (the input triangle of son k) and
    owner[k] = the input vertex whose dual cell contains son k."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    N, M = tris.shape[0], verts.shape[0]
    a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
    keys = np.stack([np.minimum(a, b) * M + np.maximum(a, b),
                     np.minimum(b, c) * M + np.maximum(b, c),
                     np.minimum(c, a) * M + np.maximum(c, a)], axis=1)  # edges 01, 12, 20
    uk, inv = np.unique(keys.ravel(), return_inverse=True)
    E = uk.size
    mid_id = (M + inv).reshape(N, 3)
    p, q = uk // M, uk % M
    mids = 0.5 * (verts[p] + verts[q])
    cents = (verts[a] + verts[b] + verts[c]) / 3.0
    cid = M + E + np.arange(N)
    m01, m12, m20 = mid_id[:, 0], mid_id[:, 1], mid_id[:, 2]
    sons = np.stack([
        np.stack([a, m01, cid], 1), np.stack([m01, b, cid], 1),
        np.stack([b, m12, cid], 1), np.stack([m12, c, cid], 1),
        np.stack([c, m20, cid], 1), np.stack([m20, a, cid], 1),
    ], axis=1).reshape(6 * N, 3)
    bverts = np.concatenate([verts, mids, cents], axis=0)
    parent = np.repeat(np.arange(N, dtype=np.int32), 6)
    owner = tris[np.arange(6 * N) // 6, SON_VERTEX[np.arange(6 * N) % 6]].astype(np.int32)
    return Mesh(bverts, sons.astype(np.int32), name="bary"), parent, owner


def vertex_incidence(tris: np.ndarray, M: int):
    """CSR of the triangles around each vertex, in increasing triangle order:
    (ptr[M + 1], tri[3 N], corner[3 N]) with corner the local index (0, 1, 2)
    of the vertex in that triangle."""
    tris = np.asarray(tris, dtype=np.int64)
    N = tris.shape[0]
    v = tris.ravel()
    t = np.repeat(np.arange(N), 3)
    k = np.tile(np.arange(3), N)
    order = np.lexsort((t, v))
    counts = np.bincount(v, minlength=M)
    ptr = np.zeros(M + 1, dtype=np.int32)
    np.cumsum(counts, out=ptr[1:])
    return ptr, t[order].astype(np.int32), k[order].astype(np.int32)
