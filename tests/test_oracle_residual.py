"""Pins of the oracle's weighted-residual estimator (Appendix A, eq.
"residual:indicator"; oracle/residual.py) against facts independent of it:

* the P1 projection and its gradient reproduce a linear function exactly
  (moments of u(x) = a.x + b in closed form, int_T lambda_k u =
  |T| (u_k + u_0 + u_1 + u_2) / 12);
* the first moments of far, coincident, edge- and vertex-adjacent pairs
  against a semi-analytic reference: the closed-form potential of a flat
  triangle (edge sums of log and arctan terms, itself pinned against brute
  force in test_oracle_quadrature.py) integrated against lambda_k over the
  other triangle with a high-order collapsed Gauss rule;
* the three moments of a row add up to the row of V Phi (lambda_0 + lambda_1
  + lambda_2 = 1), with V from the pinned matrix oracle;
* under uniform refinement of the unit cube the estimator and the error
  against the literature capacity decay together, their ratio constant
  (reliability, Appendix A's corollary), at the rate of uniform refinement
  (Section 3.1).
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import residual as R

from test_oracle_quadrature import _area, triangle_potential

P = lambda *a: np.array(a, dtype=np.float64)  # noqa: E731


def _moment_semi(Ti, Tj, n=80):
    """int_{T_i} lambda_k(x) (1/4pi) int_{T_j} 1/|x - y| dy dx, k = 0, 1, 2
    (lambda in the vertex order of Ti), by an n x n collapsed Gauss rule on
    T_i of the closed-form potential of T_j."""
    A, B, C = Ti
    s, t, w = oracle.triangle_rule(n)
    xs = A + s[:, None] * (B - A) + t[:, None] * (C - A)
    u = triangle_potential(*Tj, xs) / (4 * math.pi)
    W = 2 * _area(A, B, C) * w
    return np.array([np.sum(W * (1 - s - t) * u), np.sum(W * s * u), np.sum(W * t * u)])


def _pair_mesh(Ti, Tj):
    verts = np.array(list(Ti) + list(Tj))
    return verts, np.array([[0, 1, 2], [3, 4, 5]])


def test_projection_gradient_exact_on_linear_functions():
    rng = np.random.default_rng(1)
    for _ in range(20):
        verts = rng.normal(size=(3, 3))
        tris = np.array([[0, 1, 2]])
        a, b = rng.normal(size=3), rng.normal()
        u = verts @ a + b
        area = 0.5 * np.linalg.norm(np.cross(verts[1] - verts[0], verts[2] - verts[0]))
        m = (area / 12.0 * (u + u.sum()))[None, :]  # moments of u, standing in for V Phi
        n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
        n /= np.linalg.norm(n)
        at = a - (a @ n) * n
        diam = max(np.linalg.norm(verts[k] - verts[(k + 1) % 3]) for k in range(3))
        got = R.residual_from_moments(verts, tris, m)[0]
        assert abs(got - diam * area * (at @ at)) <= 1e-12 * diam * area * (a @ a)


def test_far_pair_moments_semi_analytic():
    Ti = (P(0, 0, 0), P(1, 0.1, 0), P(0.3, 0.9, 0.2))
    Tj = (P(2.5, 0.4, 1.0), P(3.2, 1.1, 0.8), P(2.7, 0.2, 1.9))
    verts, tris = _pair_mesh(Ti, Tj)
    res = dict(R._regular_rows((verts, tris, [0, 1], 10)))
    ref_i = _moment_semi(Ti, Tj)
    ref_j = _moment_semi(Tj, Ti)
    assert np.max(np.abs(res[0][:, 1] - ref_i) / ref_i) < 1e-11
    assert np.max(np.abs(res[1][:, 0] - ref_j) / ref_j) < 1e-11
    # the 4 x 4 rule of the assembly is within its quadrature error there
    res4 = dict(R._regular_rows((verts, tris, [0], 4)))
    assert np.max(np.abs(res4[0][:, 1] - ref_i) / ref_i) < 1e-5
    # the moments are not symmetric in k: a permuted lambda would be caught
    assert np.min(np.abs(ref_i[:, None] - ref_i[None, :]) + np.eye(3)) > 1e-3 * ref_i.max()


def _touch(verts, tris, order):
    pairs = [c for c in oracle.classify_pairs(tris) if c[0] == 0 and c[1] == (1 if len(tris) > 1 else 0)]
    (p, q, kind, Tp, Tq), = pairs
    return kind, R.touching_moments(verts, tris, p, q, kind, Tp, Tq, order)


def test_coincident_moments_semi_analytic():
    T = (P(0, 0, 0), P(1.3, 0.2, 0), P(0.4, 0.9, 0))
    verts, tris = np.array(T), np.array([[0, 1, 2]])
    kind, (mp, mq) = _touch(verts, tris, 14)
    assert kind == "coincident"
    ref = _moment_semi(T, T, n=240)
    assert np.max(np.abs(mp - ref) / ref) < 2e-8
    # the three moments of a scalene triangle differ
    assert np.ptp(ref) > 1e-2 * ref.max()
    # order 4 is within its quadrature error
    _, (m4, _) = _touch(verts, tris, 4)
    assert np.max(np.abs(m4 - ref) / ref) < 1e-3


@pytest.mark.parametrize("tri_j", [[0, 1, 3], [1, 0, 3], [3, 1, 0]])
def test_edge_moments_semi_analytic(tri_j):
    A, B, C, D = P(0, 0, 0), P(1, 0, 0), P(0.3, 0.8, 0), P(0.5, 0, 0.7)
    verts = np.array([A, B, C, D])
    tris = np.array([[0, 1, 2], tri_j])
    kind, (mp, mq) = _touch(verts, tris, 14)
    assert kind == "edge"
    Tj = tuple(verts[k] for k in tri_j)
    ref_p = _moment_semi((A, B, C), Tj, n=200)
    ref_q = _moment_semi(Tj, (A, B, C), n=200)
    assert np.max(np.abs(mp - ref_p) / ref_p) < 1e-8
    assert np.max(np.abs(mq - ref_q) / ref_q) < 1e-8


def test_vertex_moments_semi_analytic():
    A = P(0, 0, 0)
    B, C = P(1, 0.1, 0), P(0.6, 0.9, 0)
    ca, sa = math.cos(1.7), math.sin(1.7)
    D, E = P(-0.2, -0.9 * ca, -0.9 * sa), P(-1.0, -0.3 * ca, -0.3 * sa)
    verts = np.array([A, B, C, D, E])
    tris = np.array([[1, 2, 0], [3, 0, 4]])  # the shared vertex in different input slots
    kind, (mp, mq) = _touch(verts, tris, 14)
    assert kind == "vertex"
    ref_p = _moment_semi((B, C, A), (D, A, E), n=200)
    ref_q = _moment_semi((D, A, E), (B, C, A), n=200)
    assert np.max(np.abs(mp - ref_p) / ref_p) < 1e-8
    assert np.max(np.abs(mq - ref_q) / ref_q) < 1e-8


@pytest.mark.parametrize("name", ["cube2", "voxel"])
def test_moments_add_up_to_V_phi(name):
    m = synth.cube(2) if name == "cube2" else synth.voxel_union(3, 0.4, 21)
    V = oracle.assemble(m.verts, m.tris)
    s = np.random.default_rng(2).standard_normal(m.N)
    mom = R.p1_moments(m.verts, m.tris, s)
    ref = V @ s
    mag = np.abs(V) @ np.abs(s)
    assert np.max(np.abs(mom.sum(axis=1) - ref) / mag) < 1e-14


def test_estimator_tracks_the_capacity_error_on_the_cube():
    """Unit cube, nested uniform refinements (48, 192, 768 triangles): the
    error against the literature capacity quoted in Section 1.2,
    err_l = Cap - Cap_l, is bounded by C mu_l^2 (Appendix A's corollary:
    0 <= Cap - Cap_l <= C_cap mu_l^2) with a level-independent constant,
    and both decay at the rate of uniform refinement on the cube, about
    N^(-2/3) (Section 3.1: a factor 4^(2/3) = 2.52 per level)."""
    errs, mus = [], []
    for n in (2, 4, 8):
        m = synth.cube(n)
        V = oracle.assemble(m.verts, m.tris)
        b = oracle.rhs(m.verts, m.tris)
        x = oracle.solve_direct(V, b)
        errs.append(0.66067815409957 - oracle.capacity(x, b))
        mu2, _ = R.residual_indicators(m.verts, m.tris, x)
        mus.append(mu2.sum())
    ratio = np.array(errs) / np.array(mus)
    assert np.all(ratio > 0)
    assert ratio.max() / ratio.min() < 1.1, ratio  # observed 0.0565, 0.0573, 0.0570
    for k in range(2):
        assert 2.0 < errs[k] / errs[k + 1] < 3.0 and 2.0 < mus[k] / mus[k + 1] < 3.0, (errs, mus)
