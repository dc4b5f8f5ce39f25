"""Pins of the oracle's quadrature rules against facts independent of it:
a library Gauss-Legendre rule, exact polynomial integrals, closed-form
singular integrals of 1/|x-y| over triangles, and a semi-analytic reference
built from the closed-form potential of a flat triangle."""

import itertools
import math

import numpy as np
import pytest

import oracle

P = lambda *a: np.array(a, dtype=np.float64)  # noqa: E731


# ---------------------------------------------------------------- Gauss rules

@pytest.mark.parametrize("n", list(range(1, 21)))
def test_gauss_legendre_matches_library(n):
    x, w = oracle.gauss_legendre01(n)
    xl, wl = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, (xl + 1) / 2, rtol=0, atol=2e-15)
    assert np.allclose(w, wl / 2, rtol=0, atol=2e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9])
def test_gauss_legendre_exactness(n):
    x, w = oracle.gauss_legendre01(n)
    for k in range(2 * n):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
    # degree 2n is not integrated exactly: the rule has exactly this order
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_triangle_rule_exactness(n):
    s, t, w = oracle.triangle_rule(n)
    assert abs(w.sum() - 0.5) < 1e-15
    assert np.all(s + t <= 1 + 1e-15) and np.all(s >= 0) and np.all(t >= 0)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(w * s ** a * t ** b) - exact) < 1e-15 * max(1, 1 / exact)


def test_quad_points_weights_and_moments():
    rng = np.random.default_rng(0)
    verts = rng.normal(size=(3, 3))
    tris = np.array([[0, 1, 2]])
    X, W = oracle.quad_points(verts, tris, 4)
    area = 0.5 * np.linalg.norm(np.cross(verts[1] - verts[0], verts[2] - verts[0]))
    assert abs(W.sum() - area) < 1e-15
    # first moment: the weighted mean of the points is the centroid
    assert np.allclose((W[0][:, None] * X[0]).sum(0) / area, verts.mean(0), atol=1e-15)
    # second moments of a triangle: int x x^T = |T|/12 (sum v v^T + 9 c c^T)
    c = verts.mean(0)
    exact = area / 12.0 * (sum(np.outer(v, v) for v in verts) + 9 * np.outer(c, c))
    got = (W[0][:, None, None] * X[0][:, :, None] * X[0][:, None, :]).sum(0)
    assert np.allclose(got, exact, atol=1e-14)


# ------------------------------------------------ Sauter-Schwab-type rules

def _mom(a, b):
    # int over K = {0 <= x2 <= x1 <= 1} of x1^a x2^b
    return 1.0 / ((b + 1) * (a + b + 2))


@pytest.mark.parametrize("kind", ["coincident", "edge", "vertex"])
def test_ss_rule_is_a_decomposition_of_KxK(kind):
    X, Y, W = oracle.ss_rule(kind, 9)
    for x in (X, Y):
        assert np.all(x[:, 1] <= x[:, 0] + 1e-15) and np.all(x >= -1e-15) and np.all(x[:, 0] <= 1 + 1e-15)
    for a1, b1, a2, b2 in itertools.product(range(4), repeat=4):
        got = np.sum(W * X[:, 0] ** a1 * X[:, 1] ** b1 * Y[:, 0] ** a2 * Y[:, 1] ** b2)
        exact = _mom(a1, b1) * _mom(a2, b2)
        assert abs(got - exact) <= 1e-13 * exact, (a1, b1, a2, b2)


def _area(A, B, C):
    return 0.5 * np.linalg.norm(np.cross(B - A, C - A))


def coincident_closed_form(A, B, C):
    """int_T int_T 1/|x-y| for a flat triangle with sides a, b, c and area
    |T|: (4 |T|^2 / 3) sum_cyc (1/a) ln(((a+b)^2 - c^2) / (b^2 - (c-a)^2))."""
    a = np.linalg.norm(B - C)
    b = np.linalg.norm(C - A)
    c = np.linalg.norm(A - B)
    s = 0.0
    for x, y, z in ((a, b, c), (b, c, a), (c, a, b)):
        s += math.log(((x + y) ** 2 - z ** 2) / (y ** 2 - (z - x) ** 2)) / x
    return 4.0 * _area(A, B, C) ** 2 / 3.0 * s


def unit_square_closed_form():
    """int_Q int_Q 1/|x-y| over the unit square."""
    return 4.0 * math.log(1.0 + math.sqrt(2.0)) - 4.0 / 3.0 * (math.sqrt(2.0) - 1.0)


def _ss(verts, tris, i, j, n):
    for (p, q, kind, Ti, Tj) in oracle.classify_pairs(tris):
        if (p, q) == (i, j):
            return 4 * math.pi * oracle.singular_entry(verts, kind, Ti, Tj, n), kind
    raise AssertionError("pair not touching")


TRIANGLES = {
    "equilateral": (P(0, 0, 0), P(1, 0, 0), P(0.5, math.sqrt(3) / 2, 0)),
    "right_isosceles": (P(0, 0, 0), P(1, 0, 0), P(0, 1, 0)),
    "scalene": (P(0, 0, 0), P(1.3, 0.2, 0), P(0.4, 0.9, 0)),
    "tilted": (P(0.1, -0.2, 0.3), P(1.1, 0.5, -0.4), P(-0.3, 0.8, 0.9)),
}


@pytest.mark.parametrize("name", list(TRIANGLES))
def test_ss_coincident_closed_form(name):
    A, B, C = TRIANGLES[name]
    exact = coincident_closed_form(A, B, C)
    verts = np.array([A, B, C])
    tris = np.array([[0, 1, 2]])
    errs = [abs(_ss(verts, tris, 0, 0, n)[0] - exact) / exact for n in (2, 4, 6, 8, 14)]
    assert errs[-1] < 1e-11
    assert errs[1] < 3e-4  # the production order 4
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1))


def test_closed_form_values():
    # sanity of the closed forms themselves: equilateral side 1 -> (3/4) ln 3
    A, B, C = TRIANGLES["equilateral"]
    assert abs(coincident_closed_form(A, B, C) - 0.75 * math.log(3.0)) < 1e-14
    assert abs(unit_square_closed_form() - 2.9732095982) < 1e-10


def test_ss_edge_coplanar_square_diagonal():
    # unit square = two right-isosceles triangles sharing the diagonal:
    # I_sq = 2 I_T + 2 I_edge
    verts = np.array([P(0, 0, 0), P(1, 0, 0), P(1, 1, 0), P(0, 1, 0)])
    tris = np.array([[0, 1, 2], [0, 2, 3]])
    IT = coincident_closed_form(verts[0], verts[1], verts[2])
    exact = (unit_square_closed_form() - 2 * IT) / 2
    assert abs(exact - 0.4835389143) < 1e-10
    errs = [abs(_ss(verts, tris, 0, 1, n)[0] - exact) / exact for n in (2, 4, 6, 8, 14)]
    assert _ss(verts, tris, 0, 1, 4)[1] == "edge"
    assert errs[-1] < 1e-11 and errs[1] < 1e-4
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1))


@pytest.mark.parametrize("center_first", [True, False])
def test_ss_four_way_split_square(center_first):
    # square split by both diagonals: four triangles around the centre.
    # I_half = 2 I_self + 2 I_edge (half square = two small triangles),
    # I_sq = 4 I_self + 8 I_edge + 4 I_vertex.
    c = P(0.5, 0.5, 0)
    corners = [P(0, 0, 0), P(1, 0, 0), P(1, 1, 0), P(0, 1, 0)]
    verts = np.array([c] + corners) if center_first else np.array(corners + [c])
    ci = 0 if center_first else 4
    k = (lambda m: m + 1) if center_first else (lambda m: m)
    tris = np.array([[ci, k(m), k((m + 1) % 4)] for m in range(4)])
    Iself = coincident_closed_form(c, corners[0], corners[1])
    Ihalf = coincident_closed_form(corners[0], corners[1], corners[2])
    Iedge = (Ihalf - 2 * Iself) / 2
    Ivert = (unit_square_closed_form() - 4 * Iself - 8 * Iedge) / 4
    assert abs(Iedge - 0.146895597834) < 1e-11 and abs(Ivert - 0.094873859339) < 1e-11
    ge, ke = _ss(verts, tris, 0, 1, 14)
    gv, kv = _ss(verts, tris, 0, 2, 14)
    assert ke == "edge" and kv == "vertex"
    assert abs(ge - Iedge) / Iedge < 1e-11
    assert abs(gv - Ivert) / Ivert < 1e-11
    assert abs(_ss(verts, tris, 0, 2, 4)[0] - Ivert) / Ivert < 1e-4


def _log_ratio(R, l, R02):
    # log(R + l) computed without cancellation when l < 0 (R^2 - l^2 = R02)
    return np.where(l >= 0, np.log(R + np.abs(l)), np.log(R02 / (R + np.abs(l))))


def triangle_potential(V0, V1, V2, x):
    """int_T 1/|x - y| dy for a flat triangle T and points x (K, 3): the
    classical edge-sum formula (log terms for the in-plane part and arctan
    terms for the out-of-plane part)."""
    n = np.cross(V1 - V0, V2 - V0)
    n /= np.linalg.norm(n)
    w0 = (x - V0) @ n
    aw = np.abs(w0)
    rho = x - w0[:, None] * n[None, :]
    tot = np.zeros(len(x))
    for a, b in ((V0, V1), (V1, V2), (V2, V0)):
        l = (b - a) / np.linalg.norm(b - a)
        u = np.cross(l, n)
        lp = (b - rho) @ l
        lm = (a - rho) @ l
        t0 = (a - rho) @ u
        Rp = np.linalg.norm(x - b, axis=1)
        Rm = np.linalg.norm(x - a, axis=1)
        R02 = t0 * t0 + w0 * w0
        lg = _log_ratio(Rp, lp, R02) - _log_ratio(Rm, lm, R02)
        with np.errstate(divide="ignore", invalid="ignore"):
            at = np.arctan(t0 * lp / (R02 + aw * Rp)) - np.arctan(t0 * lm / (R02 + aw * Rm))
        tot += np.where(t0 == 0, 0.0, t0 * lg) - aw * np.nan_to_num(at)
    return tot


def semi_analytic(Ti, Tj, n=120):
    A, B, C = Ti
    s, t, w = oracle.triangle_rule(n)
    xs = A + s[:, None] * (B - A) + t[:, None] * (C - A)
    return np.sum(2 * _area(A, B, C) * w * triangle_potential(*Tj, xs))


def test_radon7_degree_five():
    """Radon's rule integrates every monomial s^i t^j of total degree <= 5
    exactly over the reference triangle (i! j! / (i + j + 2)!), has positive
    weights and interior points, and is not exact at degree 6."""
    s, t, w = oracle.radon7()
    assert s.shape == t.shape == w.shape == (7,)
    assert np.all(w > 0) and np.all(s > 0) and np.all(t > 0) and np.all(s + t < 1)
    for i in range(6):
        for j in range(6 - i):
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            assert abs(np.sum(w * s**i * t**j) - exact) <= 1e-15, (i, j)
    worst = max(abs(np.sum(w * s**i * t**(6 - i)) - math.factorial(i) * math.factorial(6 - i) / math.factorial(8))
                for i in range(7))
    assert worst > 1e-6


def test_radon7_far_pair_accuracy():
    """On triangle pairs at least 8 diameters apart the 7 x 7 product of
    Radon's rule matches a 12 x 12 collapsed Gauss reference to 1e-9."""
    rng = np.random.default_rng(3)
    s7, t7, w7 = oracle.radon7()
    s12, t12, w12 = oracle.triangle_rule(12)

    def pts(T, s, t, w):
        return T[0] + s[:, None] * (T[1] - T[0]) + t[:, None] * (T[2] - T[0]), 2 * w

    def pair(Ta, Tb, rule):
        Xa, Wa = pts(Ta, *rule)
        Xb, Wb = pts(Tb, *rule)
        r = np.linalg.norm(Xa[:, None, :] - Xb[None, :, :], axis=2)
        return np.sum(Wa[:, None] * Wb[None, :] / r)

    worst = 0.0
    for _ in range(200):
        Ta, Tb = rng.normal(size=(3, 3)), rng.normal(size=(3, 3))
        d = max(np.linalg.norm(T[i] - T[k]) for T in (Ta, Tb) for i in range(3) for k in range(i))
        Ta, Tb = Ta / d, Tb / d
        u = rng.normal(size=3)
        Tb = Tb - Tb.mean(0) + Ta.mean(0) + 8.0 * u / np.linalg.norm(u)
        ref = pair(Ta, Tb, (s12, t12, w12))
        worst = max(worst, abs(pair(Ta, Tb, (s7, t7, w7)) / ref - 1))
    assert worst <= 1e-9, worst


def test_radon7_accuracy_by_distance():
    """The distance thresholds of Radon's rule: at 32 diameters (the FP64
    far field's) its relative error against a 12 x 12 collapsed Gauss
    reference is below 2e-13 on random pairs, and it falls like d^-6
    (16 -> 32 diameters: a factor of at least 30)."""
    rng = np.random.default_rng(5)
    s7, t7, w7 = oracle.radon7()
    s12, t12, w12 = oracle.triangle_rule(12)

    def pair(Ta, Tb, s, t, w):
        Xa = Ta[0] + s[:, None] * (Ta[1] - Ta[0]) + t[:, None] * (Ta[2] - Ta[0])
        Xb = Tb[0] + s[:, None] * (Tb[1] - Tb[0]) + t[:, None] * (Tb[2] - Tb[0])
        r = np.linalg.norm(Xa[:, None, :] - Xb[None, :, :], axis=2)
        return np.sum(w[:, None] * w[None, :] / r)

    worst = {}
    for D in (16.0, 32.0):
        wmax = 0.0
        for _ in range(400):
            Ta, Tb = rng.normal(size=(3, 3)), rng.normal(size=(3, 3))
            d = max(np.linalg.norm(T[i] - T[k]) for T in (Ta, Tb) for i in range(3) for k in range(i))
            Ta, Tb = Ta / d, Tb / d
            u = rng.normal(size=3)
            Tb = Tb - Tb.mean(0) + Ta.mean(0) + D * u / np.linalg.norm(u)
            wmax = max(wmax, abs(pair(Ta, Tb, s7, t7, w7) / pair(Ta, Tb, s12, t12, w12) - 1))
        worst[D] = wmax
    assert worst[32.0] < 2e-13, worst
    assert worst[16.0] / worst[32.0] > 30, worst


def test_triangle_potential_far_point():
    A, B, D = P(0, 0, 0), P(1, 0, 0), P(0.5, 0, 0.7)
    x = P(0.2, 0.3, 1.5)[None]
    s, t, w = oracle.triangle_rule(30)
    y = A + s[:, None] * (B - A) + t[:, None] * (D - A)
    brute = np.sum(2 * _area(A, B, D) * w / np.linalg.norm(y - x, axis=1))
    assert abs(triangle_potential(A, B, D, x)[0] - brute) < 1e-13


def test_ss_edge_right_angle_semi_analytic():
    A, B, C, D = P(0, 0, 0), P(1, 0, 0), P(0.3, 0.8, 0), P(0.5, 0, 0.7)
    ref = semi_analytic((A, B, C), (A, B, D))
    assert abs(ref - 0.341248709039) < 2e-11
    verts = np.array([A, B, C, D])
    tris = np.array([[0, 1, 2], [0, 1, 3]])
    g, kind = _ss(verts, tris, 0, 1, 14)
    assert kind == "edge"
    assert abs(g - ref) / ref < 1e-10
    assert abs(_ss(verts, tris, 0, 1, 4)[0] - ref) / ref < 1e-4


@pytest.mark.parametrize("angle", [0.6, 1.7, 2.6])
def test_ss_vertex_folded_semi_analytic(angle):
    # two triangles sharing only the origin, the second rotated out of plane
    A = P(0, 0, 0)
    B, C = P(1, 0.1, 0), P(0.6, 0.9, 0)
    ca, sa = math.cos(angle), math.sin(angle)
    D, E = P(-0.2, -0.9 * ca, -0.9 * sa), P(-1.0, -0.3 * ca, -0.3 * sa)
    ref = semi_analytic((A, B, C), (A, D, E), n=160)
    verts = np.array([A, B, C, D, E])
    tris = np.array([[0, 1, 2], [0, 3, 4]])
    g, kind = _ss(verts, tris, 0, 1, 14)
    assert kind == "vertex"
    assert abs(g - ref) / ref < 1e-9


def test_ss_edge_folded_both_vertex_orders():
    # the canonical order puts the lower shared index first; the value must
    # not depend on how the input lists the vertices
    A, B, C, D = P(0, 0, 0), P(1, 0.2, 0), P(0.3, 0.8, 0.1), P(0.5, -0.6, 0.5)
    ref = semi_analytic((A, B, C), (A, B, D), n=160)
    for tris in ([[0, 1, 2], [1, 0, 3]], [[2, 0, 1], [3, 1, 0]], [[1, 2, 0], [0, 3, 1]]):
        g, kind = _ss(np.array([A, B, C, D]), np.array(tris), 0, 1, 14)
        assert kind == "edge" and abs(g - ref) / ref < 1e-9
