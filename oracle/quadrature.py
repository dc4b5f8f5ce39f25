"""Quadrature rules of the oracle (test infrastructure only).

Reference triangle conventions
------------------------------
* Regular rule: the triangle {s, t >= 0, s + t <= 1} mapped to T = (P0, P1, P2)
  by x = P0 + s (P1 - P0) + t (P2 - P0); Jacobian 2|T|.
* Singular rule: the triangle K = {0 <= x2 <= x1 <= 1} mapped by
  chi(x) = A + x1 (B - A) + x2 (C - B); Jacobian 2|T| as well.
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def gauss_legendre01(n: int):
    """n-point Gauss-Legendre rule on [0, 1], nodes ascending.

    Nodes are the roots of the Legendre polynomial P_n, found by Newton's
    method from the asymptotic guesses cos(pi (k - 1/4) / (n + 1/2)); P_n and
    P_n' come from the three-term recurrence.  Weights 2 / ((1 - x^2) P_n'^2)
    on [-1, 1], halved for [0, 1].  Pinned against numpy's leggauss and
    polynomial exactness."""
    if n < 1:
        raise ValueError("n >= 1")
    xs = np.empty(n)
    ws = np.empty(n)
    for k in range(1, n + 1):
        x = math.cos(math.pi * (k - 0.25) / (n + 0.5))
        for _ in range(100):
            p0, p1 = 1.0, x
            if n == 1:
                pn, pm = x, 1.0
            else:
                for j in range(1, n):
                    p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
                pn, pm = p1, p0
            dp = n * (x * pn - pm) / (x * x - 1.0)
            dx = pn / dp
            x -= dx
            if abs(dx) < 1e-16:
                break
        # final derivative at the converged root
        p0, p1 = 1.0, x
        for j in range(1, n):
            p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
        pn, pm = (p1, p0) if n > 1 else (x, 1.0)
        dp = n * (x * pn - pm) / (x * x - 1.0)
        xs[k - 1] = x
        ws[k - 1] = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(xs)
    return (xs[order] + 1.0) / 2.0, ws[order] / 2.0


def triangle_rule(n: int):
    """Collapsed (Duffy) tensor rule with n x n points on the reference
    triangle {s, t >= 0, s + t <= 1}: points (xi_a, xi_b (1 - xi_a)), weights
    w_a w_b (1 - xi_a), a-major order.  Weights sum to 1/2 (the reference
    area).  Exact for polynomials of total degree <= 2n - 2."""
    x, w = gauss_legendre01(n)
    s = np.repeat(x, n)
    t = np.tile(x, n) * (1.0 - s)
    wt = np.repeat(w, n) * np.tile(w, n) * (1.0 - s)
    return s, t, wt


def radon7():
    """Radon's 7-point rule of degree 5 on the reference triangle
    {s, t >= 0, s + t <= 1} (Stroud, Approximate Calculation of Multiple
    Integrals, formula T2:5-1): the centroid with weight 9/40, and two orbits
    of three points whose barycentric coordinates are (1 - 2b, b, b) in every
    order, b = (6 - sqrt(15)) / 21 with weight (155 - sqrt(15)) / 1200 and
    b = (6 + sqrt(15)) / 21 with weight (155 + sqrt(15)) / 1200; the weights
    are then scaled by the reference area 1/2.  Returns (s, t, w) with s, t the second and third barycentric
    coordinates.  Used by the mixed-precision far field on distant blocks (an
    implementation choice of quadrature order by distance, not the paper's)."""
    r = math.sqrt(15.0)
    bary = [(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0)]
    for sign in (-1.0, 1.0):
        b = (6.0 + sign * r) / 21.0
        a = 1.0 - 2.0 * b
        wo = (155.0 + sign * r) / 1200.0
        bary += [(a, b, b, wo), (b, a, b, wo), (b, b, a, wo)]
    B = np.array(bary)
    return B[:, 1].copy(), B[:, 2].copy(), 0.5 * B[:, 3]


def _grid4(n: int):
    x, w = gauss_legendre01(n)
    idx = np.array(list(itertools.product(range(n), repeat=4)))
    p = x[idx]
    ww = np.prod(w[idx], axis=1)
    return p[:, 0], p[:, 1], p[:, 2], p[:, 3], ww


def ss_rule(kind: str, n: int):
    """Sauter-Schwab-type rule for the 4-D reference integral
    int_K int_K f(x, y) dy dx with a singularity where the two
    parametrisations meet.  Returns (x (K,2), y (K,2), w (K,)) such that
    sum w f(x, y) approximates the integral, with the Jacobian of the
    regularising transformation folded into w.

    The textbook the paper cites for Galerkin BEM quadrature (Sauter and
    Schwab) treats the three touching cases; the transformations below were
    derived afresh for the conventions of this module:

    * "coincident" (same triangle, singular on x = y): the difference x - y
      is split into the 6 sectors cut out by the lines d1 = 0, d2 = 0 and
      d1 = d2; in each sector a Duffy map with Jacobian xi^3 eta1^2 eta2
      makes the integrand bounded.
    * "edge" (x2 = y2 = 0, x1 = y1 is the shared edge): split by which of x1,
      y1 is larger (xi is the larger one); in the half x1 >= y1 write
      x = xi (1, p), y = xi (1 - w, r) with r <= 1 - w, and split the prism
      (w, p, r) into {p >= w + r} (Jacobian xi^3 eta1^2 eta2) and
      {p <= w + r} (Jacobian xi^3 eta1^2); the other half is the mirror.
    * "vertex" (x = y = 0 is the shared vertex): split by which of x1, y1
      is larger; Jacobian xi^3 eta2.

    In every case the Jacobian vanishes to the order of the distance between
    the two points, which cancels the 1/|x - y| kernel.  Pinned by exact
    polynomial moments over K x K and by closed-form singular integrals."""
    xi, e1, e2, e3, ww = _grid4(n)
    regs = []
    if kind == "coincident":
        J = ww * xi ** 3 * e1 ** 2 * e2
        a = (xi, xi * (1 - e1 + e1 * e2))
        b = (xi * (1 - e1 * e2 * e3), xi * (1 - e1))
        c = (xi, xi * e1 * (1 - e2 + e2 * e3))
        d = (xi * (1 - e1 * e2), xi * e1 * (1 - e2))
        e = (xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3))
        f = (xi, xi * e1 * (1 - e2))
        regs = [(a, b, J), (b, a, J), (c, d, J), (d, c, J), (e, f, J), (f, e, J)]
    elif kind == "edge":
        JA = ww * xi ** 3 * e1 ** 2 * e2
        JB = ww * xi ** 3 * e1 ** 2
        ax = (xi, xi * e1)
        ay = (xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3))
        bx = (xi, xi * e1 * e3)
        by = (xi * (1 - e1 * e2), xi * e1 * (1 - e2))
        regs = [(ax, ay, JA), (bx, by, JB), (ay, ax, JA), (by, bx, JB)]
    elif kind == "vertex":
        J = ww * xi ** 3 * e2
        ax = (xi, xi * e1)
        ay = (xi * e2, xi * e2 * e3)
        regs = [(ax, ay, J), (ay, ax, J)]
    else:
        raise ValueError(kind)
    X = np.concatenate([np.stack(r[0], axis=1) for r in regs])
    Y = np.concatenate([np.stack(r[1], axis=1) for r in regs])
    W = np.concatenate([r[2] for r in regs])
    return X, Y, W
