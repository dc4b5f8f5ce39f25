"""Solve, capacity, ZZ indicators and Doerfler marking (test infrastructure).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .operator import element_geometry

FOUR_PI = 4.0 * math.pi


def rhs(verts, tris):
    """Load vector b_i = <1, chi_i> = |T_i| (right-hand side f = 1 of the
    capacity problem, eq. "cap"; discrete load as in eq. "laplace_system")."""
    return element_geometry(verts, tris)["area"].copy()


def solve_direct(V, b, overwrite: bool = False):
    """x = V^{-1} b by a dense Cholesky factorisation (the paper notes the
    system can be solved by a dense direct method for smaller sizes,
    Section 2.5).  A failed factorisation means V is not SPD, which
    contradicts eq. "laplace_system", and raises.  overwrite=True factors V
    in place (its transpose, the same symmetric matrix in column-major
    order, so LAPACK needs no copy): for matrices of tens of GB; V is
    destroyed."""
    if overwrite:
        c = scipy.linalg.cho_factor(V.T, lower=False, overwrite_a=True, check_finite=False)
        if not np.all(np.isfinite(np.diag(c[0]))):
            raise np.linalg.LinAlgError("non-finite Cholesky factor")
    else:
        c = scipy.linalg.cho_factor(V, lower=False, check_finite=True)
    return scipy.linalg.cho_solve(c, b)


def solve_cg(V, b, rtol: float = 1e-14, max_iter: int = 20000, rows: int = 4096):
    """x with ||b - V x|| <= rtol ||b|| by conjugate gradients with diagonal
    (Jacobi) preconditioning in FP64 (V is symmetric positive definite,
    eq. "laplace_system").  For matrices of more than 2^31 entries, where the
    dense LAPACK factorisation of this environment does not apply (its
    32-bit indexing fails on them); the products V p are taken in blocks of
    `rows` rows.  Returns (x, rel_residual of the true residual, iterations).
    The capacity of x then differs from the exact solution's by at most
    ||x|| ||r|| / |b^T x| relative, to first order (4 pi (Cap* - Cap) =
    x*^T r for symmetric V)."""
    N = V.shape[0]

    def mv(p):
        y = np.empty(N)
        for r0 in range(0, N, rows):
            y[r0:r0 + rows] = V[r0:r0 + rows] @ p
        return y

    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / np.diag(V).copy()
    x = np.zeros(N)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for k in range(1, max_iter + 1):
        q = mv(p)
        pq = p @ q
        if not pq > 0.0:
            raise np.linalg.LinAlgError("p^T V p <= 0: V is not positive definite")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= 0.5 * rtol * bn:
            rt = b - mv(x)  # the true residual decides
            if np.linalg.norm(rt) <= rtol * bn:
                return x, float(np.linalg.norm(rt) / bn), k
            r = rt
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise np.linalg.LinAlgError("CG did not reach the tolerance")


def capacity(x, area):
    """Cap = (1 / 4 pi) sum_i x_i |T_i| (eq. "cap:ell"; 4 pi Cap_l = 1 . x
    in the proof of the capacity proposition), summed with math.fsum."""
    return math.fsum((np.asarray(x) * np.asarray(area)).tolist()) / FOUR_PI


def zz_indicators(verts, tris, sigma, h_mode: str = "diam"):
    """ZZ-type indicators eta(T)^2 = h_T || sigma_T - I sigma ||^2_{L2(T)}
    (eq. "zz:T", Section 2.4) for a P0 density on the primal mesh.

    The paper defines I for the dual-mesh solution, whose values sit at
    vertices.  For the primal P0 density the nodal value at a vertex z is the
    area-weighted mean of sigma over the elements containing z (summed in
    increasing element order), and I sigma is the S^1 function with these
    nodal values.  On T, sigma_T - I sigma is linear with vertex values -d_k,
    d_k = (I sigma)(z_k) - sigma_T, so with int_T lambda_k lambda_l =
    |T| (1 + delta_kl) / 12 the squared L2 norm is
    |T| / 12 * ((d1 + d2 + d3)^2 + d1^2 + d2^2 + d3^2).
    h_T = diam(T) (default, as in eq. "zz:T") or |T|^(1/2) (h_mode="area")."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    sigma = np.asarray(sigma, dtype=np.float64)
    g = element_geometry(verts, tris)
    area = g["area"]
    M = verts.shape[0]
    num = [[] for _ in range(M)]
    den = [[] for _ in range(M)]
    for e, (a, b, c) in enumerate(tris.tolist()):
        for v in (a, b, c):
            num[v].append(area[e] * sigma[e])
            den[v].append(area[e])
    nodal = np.zeros(M)
    for v in range(M):
        s_num = 0.0
        s_den = 0.0
        for p, q in zip(num[v], den[v]):
            s_num += p
            s_den += q
        nodal[v] = s_num / s_den if den[v] else 0.0
    d = nodal[tris] - sigma[:, None]
    l2 = area / 12.0 * ((d[:, 0] + d[:, 1] + d[:, 2]) ** 2 + d[:, 0] ** 2 + d[:, 1] ** 2 + d[:, 2] ** 2)
    h = g["diam"] if h_mode == "diam" else np.sqrt(area)
    return h * l2


def doerfler(eta2, theta: float):
    """Doerfler marking (eq. "doerfler"): the smallest set M with
    theta * sum_T eta_T^2 <= sum_{T in M} eta_T^2, taken greedily by
    decreasing eta^2 (ties: lower index first).  Returns the sorted
    indices."""
    eta2 = np.asarray(eta2, dtype=np.float64)
    order = sorted(range(len(eta2)), key=lambda k: (-eta2[k], k))
    total = math.fsum(eta2.tolist())
    acc = 0.0
    marked = []
    for k in order:
        marked.append(k)
        acc += eta2[k]
        if acc >= theta * total:
            break
    return np.array(sorted(marked), dtype=np.int64)


def mesh_check(verts, tris):
    """Validity of the input (Section 2.1: conforming triangulation of a
    closed surface into plane triangles).  Returns (ok, reason)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    M, N = verts.shape[0], tris.shape[0]
    if N < 4 or M < 4:
        return False, "too small"
    if not np.all(np.isfinite(verts)):
        return False, "non-finite vertex"
    if tris.min() < 0 or tris.max() >= M:
        return False, "index out of range"
    if np.any(tris[:, 0] == tris[:, 1]) or np.any(tris[:, 1] == tris[:, 2]) or np.any(tris[:, 0] == tris[:, 2]):
        return False, "repeated vertex"
    if np.any(element_geometry(verts, tris)["area"] <= 0):
        return False, "zero area"
    if np.unique(verts, axis=0).shape[0] != M:
        return False, "unwelded vertices"
    e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e[:, 0] * M + e[:, 1], return_counts=True)
    if np.any(cnt != 2):
        return False, "edge not shared by exactly two triangles"
    return True, "ok"
