"""Dual-mesh Galerkin system and operator preconditioner (test
infrastructure; Section 2.1 "Triangulations", Section 2.3 "Discrete function
spaces" and "Galerkin discretization", Section 2.6 "Operator preconditioning
with the hypersingular operator", eq. "zz:T").

Plain NumPy in FP64, written from the definitions:

* the barycentric refinement, built here triangle by triangle (the GPU side
  takes it from ``synth``; tests compare the two);
* V_bary, the P0 Galerkin matrix of the single-layer operator on the
  barycentric mesh (the same ``assemble`` as the primal path);
* P, the 6N x M matrix that writes the dual-cell indicator chi_j^dual as the
  sum of the barycentric indicators it covers, V_dual = P^T V_bary P, and the
  dual load f_j = <1, chi_j^dual>;
* the surface curls of the hat functions, the matrices Q_m (m-th component
  of curl phi_j on each barycentric element), the hypersingular Galerkin
  matrix D = sum_m Q_m^T V_bary Q_m (integration by parts formula of
  Section 2.6) and D_reg = D + a a^T with a_j = <phi_j, 1>;
* the mass matrix M[i][j] = <phi_j, chi_i^dual>;
* the direct solution of V_dual x = f, the capacity (1/4pi) f^T x
  (eq. "cap:ell") and the ZZ indicators of the dual solution (eq. "zz:T").

The preconditioned GMRES of eq. "laplace_precond_discrete" has the same
solution x as V_dual x = f; the oracle solves the latter directly.
"""

from __future__ import annotations

import math

import numpy as np

from .operator import assemble, element_geometry

FOUR_PI = 4.0 * math.pi


def barycentric_mesh(verts, tris):
    """(bary verts, bary tris, parent, owner) of the barycentric refinement
    (Section 2.1, Fig. "dual_element"): each triangle (v0, v1, v2) is cut by
    its medians into six sons, in the order (v0, m01, c), (m01, v1, c),
    (v1, m12, c), (m12, v2, c), (v2, m20, c), (m20, v0, c) (c the centre of
    gravity, m the edge midpoints); son 6t + s lies in the dual cell of the
    vertex it contains (owner).  New vertices: one midpoint per edge, edges
    numbered by increasing (min, max) vertex pair, then one centre per
    triangle in triangle order."""
    verts = [tuple(map(float, p)) for p in np.asarray(verts, dtype=np.float64)]
    tris = [tuple(map(int, t)) for t in np.asarray(tris)]
    M = len(verts)
    edges = sorted({(min(a, b), max(a, b)) for t in tris for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))})
    mid = {e: M + k for k, e in enumerate(edges)}
    bverts = list(verts)
    for (a, b) in edges:
        bverts.append(tuple(0.5 * (verts[a][c] + verts[b][c]) for c in range(3)))
    sons, parent, owner = [], [], []
    for t, (v0, v1, v2) in enumerate(tris):
        c = M + len(edges) + t
        bverts.append(tuple((verts[v0][k] + verts[v1][k] + verts[v2][k]) / 3.0 for k in range(3)))
        m01, m12, m20 = mid[(min(v0, v1), max(v0, v1))], mid[(min(v1, v2), max(v1, v2))], mid[(min(v2, v0), max(v2, v0))]
        for son, own in (((v0, m01, c), v0), ((m01, v1, c), v1), ((v1, m12, c), v1), ((m12, v2, c), v2),
                         ((v2, m20, c), v2), ((m20, v0, c), v0)):
            sons.append(son)
            parent.append(t)
            owner.append(own)
    return (np.array(bverts, dtype=np.float64), np.array(sons, dtype=np.int32), np.array(parent, dtype=np.int32),
            np.array(owner, dtype=np.int32))


def prolongation(owner, M):
    """P[k][j] = 1 if barycentric element k lies in the dual cell of vertex j
    (chi_j^dual = sum_k P[k][j] chi_k^bary)."""
    P = np.zeros((len(owner), M))
    P[np.arange(len(owner)), owner] = 1.0
    return P


def dual_load(verts, tris):
    """f_j = <1, chi_j^dual> = |T_j^dual|, summed from the areas of the
    barycentric elements in the cell."""
    bv, bt, parent, owner = barycentric_mesh(verts, tris)
    area = element_geometry(bv, bt)["area"]
    f = np.zeros(np.asarray(verts).shape[0])
    np.add.at(f, owner, area)
    return f


def surface_curls(verts, tris):
    """curl_G phi_a = n x grad_G phi_a on each triangle, for its three local
    hat functions a = 0, 1, 2: array (N, 3 [a], 3 [xyz]).  The surface
    gradient is the in-plane vector g with g . (P_b - P_0) = phi_a(P_b) -
    phi_a(P_0) for b = 1, 2, found from the 2 x 2 Gram system."""
    P = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n, axis=1)[:, None]
    G = np.stack([np.stack([(e1 * e1).sum(1), (e1 * e2).sum(1)], 1),
                  np.stack([(e2 * e1).sum(1), (e2 * e2).sum(1)], 1)], 1)  # (N, 2, 2)
    out = np.zeros((P.shape[0], 3, 3))
    vals = np.eye(3)
    for a in range(3):
        rhs = np.broadcast_to(np.array([vals[a, 1] - vals[a, 0], vals[a, 2] - vals[a, 0]])[None, :, None],
                              (P.shape[0], 2, 1))
        c = np.linalg.solve(G, rhs)[:, :, 0]  # g = c0 e1 + c1 e2
        g = c[:, 0:1] * e1 + c[:, 1:2] * e2
        out[:, a, :] = np.cross(n, g)
    return out


def curl_matrices(verts, tris):
    """Q_m (m = 0, 1, 2), each 6N x M: Q_m[k][j] = (curl_G phi_j)_m on
    barycentric element k (constant on the parent triangle)."""
    tris = np.asarray(tris)
    N, M = tris.shape[0], np.asarray(verts).shape[0]
    C = surface_curls(verts, tris)
    Q = np.zeros((3, 6 * N, M))
    for t in range(N):
        for s in range(6):
            k = 6 * t + s
            for a in range(3):
                Q[:, k, tris[t, a]] += C[t, a, :]
    return Q


def hat_integrals(verts, tris):
    """a_j = <phi_j, 1>: each triangle containing vertex j contributes
    |T| / 3 (the integral of a barycentric coordinate)."""
    tris = np.asarray(tris)
    area = element_geometry(verts, tris)["area"]
    a = np.zeros(np.asarray(verts).shape[0])
    for k in range(3):
        np.add.at(a, tris[:, k], area / 3.0)
    return a


def dual_mass(verts, tris):
    """M[i][j] = <phi_j, chi_i^dual>: phi_j is affine on each barycentric
    element, so its integral there is the area times its value at the
    element's centre of gravity."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    bv, bt, parent, owner = barycentric_mesh(verts, tris)
    geo = element_geometry(bv, bt)
    area, cen = geo["area"], geo["centroid"]
    Mv = verts.shape[0]
    Mm = np.zeros((Mv, Mv))
    P = verts[tris]
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    for k in range(bt.shape[0]):
        t = parent[k]
        # barycentric coordinates of the son's centre of gravity in its parent
        d = cen[k] - P[t, 0]
        G = np.array([[e1[t] @ e1[t], e1[t] @ e2[t]], [e2[t] @ e1[t], e2[t] @ e2[t]]])
        s, u = np.linalg.solve(G, np.array([d @ e1[t], d @ e2[t]]))
        lam = np.array([1.0 - s - u, s, u])
        for a in range(3):
            Mm[owner[k], tris[t, a]] += area[k] * lam[a]
    return Mm


def assemble_dual(verts, tris, far_order: int = 4, ss_order: int = 4, workers: int | None = None):
    """(V_bary, P, bary mesh verts, bary mesh tris) for the dual system."""
    bv, bt, parent, owner = barycentric_mesh(verts, tris)
    Vb = assemble(bv, bt, far_order, ss_order, workers=workers)
    return Vb, prolongation(owner, np.asarray(verts).shape[0]), bv, bt


def hypersingular(Vb, Q):
    """D = sum_m Q_m^T V_bary Q_m (Section 2.6)."""
    return sum(Q[m].T @ Vb @ Q[m] for m in range(3))


def solve_dual(Vb, P, f):
    """x = (P^T V_bary P)^{-1} f by Cholesky, and the dual matrix."""
    import scipy.linalg

    Vd = P.T @ Vb @ P
    c, low = scipy.linalg.cho_factor(Vd)
    return scipy.linalg.cho_solve((c, low), f), Vd


def capacity_dual(x, f):
    """(1/4pi) <Phi^dual, 1> = (1/4pi) sum_j x_j |T_j^dual| (eq. "cap:ell")."""
    return math.fsum(np.asarray(x) * np.asarray(f)) / FOUR_PI


def zz_dual(verts, tris, x, h_mode: str = "diam"):
    """eta_T^2 = h_T || Phi - I Phi ||^2_{L2(T)} (eq. "zz:T"), Phi = x_j on
    the dual cell of vertex j, I Phi = sum_j x_j phi_j.  On each barycentric
    son Phi - I Phi is affine, so the three-point edge-midpoint rule
    integrates its square exactly."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    x = np.asarray(x, dtype=np.float64)
    bv, bt, parent, owner = barycentric_mesh(verts, tris)
    area = element_geometry(bv, bt)["area"]
    geo = element_geometry(verts, tris)
    P = verts[tris]
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    eta2 = np.zeros(tris.shape[0])
    for k in range(bt.shape[0]):
        t = parent[k]
        G = np.array([[e1[t] @ e1[t], e1[t] @ e2[t]], [e2[t] @ e1[t], e2[t] @ e2[t]]])
        tot = 0.0
        for q in range(3):
            pt = 0.5 * (bv[bt[k, q]] + bv[bt[k, (q + 1) % 3]])
            d = pt - P[t, 0]
            s, u = np.linalg.solve(G, np.array([d @ e1[t], d @ e2[t]]))
            lam = np.array([1.0 - s - u, s, u])
            g = x[owner[k]] - lam @ x[tris[t]]
            tot += g * g
        eta2[t] += area[k] / 3.0 * tot
    h = geo["diam"] if h_mode == "diam" else np.sqrt(geo["area"])
    return h * eta2
