"""Weighted-residual error estimator of the primal P0 Galerkin solution
(Appendix A, eq. "residual:indicator"; test infrastructure only).

    mu_l(T)^2 = diam(T) || grad_G (f - V Phi_l) ||^2_{L2(T)},   f = 1.

The residual is evaluated in the space of discontinuous piecewise linear
functions P1(T_l), as the paper's remark on the estimator's cost describes
(the P1 Galerkin operator, projected onto P0 for the system, also gives the
residual in P1): on every element the residual is replaced by its L2
projection onto the linear functions on T, whose surface gradient is a
constant vector.  The projection needs the three first moments

    m_k(T_i) = <V Phi, lambda_k>_{T_i}
             = sum_j Phi_j (1/4pi) int_{T_i} lambda_k(x) int_{T_j} 1/|x - y| dy dx,

lambda_k the barycentric coordinate of vertex k of T_i (input order), with
the same quadrature as the matrix: the collapsed 4 x 4 Gauss rule on both
triangles for pairs that share no vertex, the Sauter-Schwab-type rules for
touching pairs (sum_k m_k is then exactly the row of V Phi).

Steps, in the order of eq. "residual:indicator":
  1. moments of the residual  <1 - V Phi, lambda_k> = |T|/3 - m_k;
  2. local mass matrix  M_T[k][l] = <lambda_l, lambda_k> = |T| (1 + delta_kl) / 12,
     coefficients  c = M_T^{-1} (moments);
  3. gradient of  sum_k c_k lambda_k  in the plane of T: g = E alpha with
     E = [P1 - P0, P2 - P0] and (E^T E) alpha = (c_1 - c_0, c_2 - c_0);
  4. mu(T)^2 = diam(T) |T| |g|^2 (the gradient is constant on T).
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from .operator import SSOrders, _pair_order, classify_pairs, element_geometry, quad_points
from .quadrature import ss_rule, triangle_rule

FOUR_PI = 4.0 * math.pi


def _regular_rows(args):
    """Regular-rule moments of the rows `rows` against every column:
    R[k, j] = (1/4pi) sum_a W_a lambda_k(x_a) sum_b W_b / |x_a - y_b|, with
    the columns that share a vertex with the row set to 0 (the singular
    rules replace them)."""
    verts, tris, rows, far_order = args
    X, W = quad_points(verts, tris, far_order)
    s, t, _ = triangle_rule(far_order)
    lam = np.stack([1.0 - s - t, s, t])  # (3, Q): lambda_k at the rule's points (input vertex order)
    Xc = [np.ascontiguousarray(X[:, :, c]) for c in range(3)]
    N = X.shape[0]
    tris = np.asarray(tris)
    chunk = 512
    out = []
    for i in rows:
        R = np.empty((3, N))
        for c0 in range(0, N, chunk):
            c1 = min(N, c0 + chunk)
            dx = Xc[0][i][None, :, None] - Xc[0][c0:c1][:, None, :]
            dy = Xc[1][i][None, :, None] - Xc[1][c0:c1][:, None, :]
            dz = Xc[2][i][None, :, None] - Xc[2][c0:c1][:, None, :]
            r = np.sqrt(dx * dx + dy * dy + dz * dz)
            with np.errstate(divide="ignore", invalid="ignore"):
                sa = np.sum(W[c0:c1][:, None, :] / r, axis=2)  # (chunk, a): sum_b W_b / r_ab
                R[:, c0:c1] = (lam[:, None, :] * (W[i][None, None, :] * sa[None, :, :])).sum(axis=2) / FOUR_PI
        touch = np.any(np.isin(tris, tris[i]), axis=1)
        R[:, touch] = 0.0
        out.append((i, R))
    return out


def _bary_on(Tcanon, Tinput, P):
    """Barycentric weights of the points P (K, 2) of the reference map
    chi(x) = A + x1 (B - A) + x2 (C - B), (A, B, C) = Tcanon, as a (K, 3)
    array in the input vertex order of the element Tinput: lambda_A = 1 - x1,
    lambda_B = x1 - x2, lambda_C = x2."""
    lam_c = np.stack([1.0 - P[:, 0], P[:, 0] - P[:, 1], P[:, 1]], axis=1)
    out = np.zeros_like(lam_c)
    for c, v in enumerate(Tcanon):
        out[:, list(Tinput).index(v)] += lam_c[:, c]
    return out


def touching_moments(verts, tris, p, q, kind, Tp, Tq, ss_order: int = 4):
    """(3,) and (3,) moment vectors of one touching pair p <= q with the
    singular rule of `kind`: the moments on T_p (lambda of T_p at the rule's
    x points) and on T_q (lambda of T_q at its y points), each without the
    density factor."""
    V = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    X, Y, W = ss_rule(kind, ss_order)
    A, B, C = V[Tp[0]], V[Tp[1]], V[Tp[2]]
    D0, D1, D2 = V[Tq[0]], V[Tq[1]], V[Tq[2]]
    x = A[None, :] + X[:, :1] * (B - A)[None, :] + X[:, 1:2] * (C - B)[None, :]
    y = D0[None, :] + Y[:, :1] * (D1 - D0)[None, :] + Y[:, 1:2] * (D2 - D1)[None, :]
    r = np.sqrt(np.sum((x - y) ** 2, axis=1))
    ap = 0.5 * np.linalg.norm(np.cross(B - A, C - A))
    aq = 0.5 * np.linalg.norm(np.cross(D1 - D0, D2 - D0))
    base = (2.0 * ap) * (2.0 * aq) * W / r / FOUR_PI
    mp = _bary_on(Tp, tris[p].tolist(), X).T @ base
    mq = _bary_on(Tq, tris[q].tolist(), Y).T @ base
    return mp, mq


def p1_moments(verts, tris, sigma, far_order: int = 4, ss_order=4, workers: int | None = None):
    """m (N, 3): m[i, k] = <V Phi, lambda_k>_{T_i} for the P0 density Phi =
    sigma (see the module docstring); ss_order an int or SSOrders, as for
    the matrix."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    sigma = np.asarray(sigma, dtype=np.float64)
    N = len(tris)
    m = np.zeros((N, 3))
    if workers is None:
        workers = min(os.cpu_count() or 1, 16) if N > 1500 else 1
    blocks = [list(range(k, N, workers * 8)) for k in range(workers * 8)] if workers > 1 else [list(range(N))]
    if workers > 1:
        import multiprocessing as mp

        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            for res in ex.map(_regular_rows, [(verts, tris, b, far_order) for b in blocks]):
                for i, R in res:
                    m[i] = R @ sigma
    else:
        for i, R in _regular_rows((verts, tris, blocks[0], far_order)):
            m[i] = R @ sigma
    orders = SSOrders.of(ss_order)
    geo = element_geometry(verts, tris)
    for (p, q, kind, Tp, Tq) in classify_pairs(tris):
        mp_, mq_ = touching_moments(verts, tris, p, q, kind, Tp, Tq, _pair_order(orders, geo, kind, p, q))
        m[p] += sigma[q] * mp_
        if q != p:
            m[q] += sigma[p] * mq_
    return m


def residual_from_moments(verts, tris, m):
    """mu(T)^2 (N,) from the moments m[i, k] = <V Phi, lambda_k>_{T_i}, by
    steps 1-4 of the module docstring (f = 1)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    g = element_geometry(verts, tris)
    out = np.empty(len(tris))
    for i, (a, b, c) in enumerate(tris.tolist()):
        P0, P1, P2 = verts[a], verts[b], verts[c]
        area = g["area"][i]
        rhs = area / 3.0 - m[i]                                    # 1. <1 - V Phi, lambda_k>
        M = area / 12.0 * (np.ones((3, 3)) + np.eye(3))           # 2. local mass matrix
        coef = np.linalg.solve(M, rhs)
        E = np.stack([P1 - P0, P2 - P0], axis=1)                   # 3. gradient in the plane of T
        alpha = np.linalg.solve(E.T @ E, np.array([coef[1] - coef[0], coef[2] - coef[0]]))
        grad = E @ alpha
        out[i] = g["diam"][i] * area * float(grad @ grad)          # 4. diam(T) ||grad||^2_{L2(T)}
    return out


def residual_indicators(verts, tris, sigma, far_order: int = 4, ss_order=4, workers: int | None = None):
    """mu_l(T)^2 for every element (eq. "residual:indicator") of the P0
    density sigma; returns (mu2 (N,), m (N, 3))."""
    m = p1_moments(verts, tris, sigma, far_order, ss_order, workers)
    return residual_from_moments(verts, tris, m), m
