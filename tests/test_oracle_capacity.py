"""Pins of the oracle's capacity, ZZ indicators and Doerfler marking against
the paper's printed values, the capacity proposition, monotonicity under
nested refinement, the sphere's exact capacity, brute force and closed forms."""

import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def cap_of(mesh):
    V = oracle.assemble(mesh.verts, mesh.tris)
    b = oracle.rhs(mesh.verts, mesh.tris)
    x = oracle.solve_direct(V, b)
    return oracle.capacity(x, b), V, b, x


def test_sphere_capacity_converges_from_below():
    # Cap(ball of radius r) = r; an inscribed polyhedron has smaller capacity
    # and the P0 Galerkin value is smaller still (capacity proposition).
    r = 1.37
    caps = [cap_of(synth.icosphere(k, r))[0] for k in (1, 2, 3)]
    assert all(c < r for c in caps)
    assert caps[0] < caps[1] < caps[2]
    gaps = [r - c for c in caps]
    ratio = gaps[1] / gaps[2]
    assert 2.5 < ratio < 6.0, ratio  # O(h^2) geometric + discretisation error
    assert gaps[2] / r < 1.5e-2


def test_capacity_scales_linearly():
    m = synth.icosphere(1)
    c1 = cap_of(m)[0]
    c2 = cap_of(m.scaled(2.5))[0]
    assert abs(c2 - 2.5 * c1) < 1e-13 * c2


def test_cube_capacity_below_literature_and_monotone():
    lit = GOLDEN["cube_capacity_literature"]["value"]
    lo = GOLDEN["cube_polya_bounds"]["lower"]
    caps = [cap_of(synth.cube(n))[0] for n in (2, 4, 8)]  # nested meshes
    assert caps[0] < caps[1] < caps[2] < lit
    assert caps[2] > lo
    # the gap shrinks like N^(-2/3) under uniform refinement (ratio ~ 4^(2/3))
    r = (lit - caps[1]) / (lit - caps[2])
    assert 1.8 < r < 3.2, r


def test_energy_identity_nested_meshes():
    # Pythagoras in the energy norm for nested P0 spaces:
    # 4 pi (Cap_{l+1} - Cap_l) = (x_f - P x_c)^T V_f (x_f - P x_c)
    m = synth.voxel_union(2, 0.4, 3)
    t0 = synth.init_reference_edges(m.verts, m.tris)
    v1, t1, _ = synth.refine_uniform(m.verts, t0, 1)
    rng = np.random.default_rng(2)
    v2, t2, parent = synth.refine_nvb(v1, t1, rng.choice(len(t1), len(t1) // 3, replace=False))
    cc, _, _, xc = cap_of(synth.Mesh(v1, t1))
    cf, Vf, _, xf = cap_of(synth.Mesh(v2, t2))
    e = xf - xc[parent]
    lhs = 4 * math.pi * (cf - cc)
    rhs = e @ Vf @ e
    assert lhs > 0
    assert abs(lhs - rhs) / rhs < 2e-2


def test_capacity_positive_and_rhs_is_area():
    m = synth.convex_hull(10, 2)
    c, V, b, x = cap_of(m)
    g = oracle.element_geometry(m.verts, m.tris)
    assert np.array_equal(b, g["area"])
    assert c > 0
    # 4 pi Cap = b^T V^{-1} b = x^T V x (Galerkin energy of the solution)
    assert abs(4 * math.pi * c - x @ V @ x) < 1e-12 * abs(x @ V @ x)


# ------------------------------------------------------------------ ZZ

def test_zz_zero_for_constant_density():
    m = synth.voxel_union(3, 0.4, 5)
    eta2 = oracle.zz_indicators(m.verts, m.tris, np.full(m.N, 3.7))
    assert np.all(np.abs(eta2) < 1e-25)


def _zz_bruteforce(verts, tris, sigma, h_mode="diam"):
    # incidence-matrix nodal averages + high-order quadrature of (sigma_T - I sigma)^2
    N, M = len(tris), len(verts)
    g = oracle.element_geometry(verts, tris)
    A = np.zeros((M, N))
    for e, t in enumerate(tris):
        A[t, e] = g["area"][e]
    nodal = (A @ sigma) / A.sum(axis=1)
    s, t, w = oracle.triangle_rule(8)
    lam = np.stack([1 - s - t, s, t], axis=1)
    out = np.empty(N)
    for e, tri in enumerate(tris):
        Is = lam @ nodal[tri]
        l2 = 2 * g["area"][e] * np.sum(w * (sigma[e] - Is) ** 2)
        h = g["diam"][e] if h_mode == "diam" else math.sqrt(g["area"][e])
        out[e] = h * l2
    return out


@pytest.mark.parametrize("h_mode", ["diam", "area"])
def test_zz_closed_form_vs_quadrature(h_mode):
    m = synth.convex_hull(14, 9)
    rng = np.random.default_rng(4)
    sigma = rng.uniform(0.5, 2.0, m.N)
    got = oracle.zz_indicators(m.verts, m.tris, sigma, h_mode)
    ref = _zz_bruteforce(m.verts, m.tris, sigma, h_mode)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15 * ref.max())


def test_zz_single_vertex_hand_value():
    # tetrahedron, sigma = 1 except element 0 = 2: every vertex average is
    # a hand-computable weighted mean
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    tris = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]])
    sigma = np.array([2.0, 1.0, 1.0, 1.0])
    g = oracle.element_geometry(verts, tris)
    a = g["area"]
    # vertex 3 is not in element 0: its average is 1, vertices 0, 1, 2 are
    nodal = np.array([(2 * a[0] + a[1] + a[2]) / (a[0] + a[1] + a[2]),
                      (2 * a[0] + a[1] + a[3]) / (a[0] + a[1] + a[3]),
                      (2 * a[0] + a[2] + a[3]) / (a[0] + a[2] + a[3]), 1.0])
    d = nodal[tris[1]] - 1.0
    expect1 = g["diam"][1] * a[1] / 12 * (d.sum() ** 2 + (d ** 2).sum())
    assert oracle.zz_indicators(verts, tris, sigma)[1] == pytest.approx(expect1, rel=1e-14)


# -------------------------------------------------------------- Doerfler

@pytest.mark.parametrize("seed", range(12))
def test_doerfler_minimal_cardinality(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 11))
    eta2 = rng.choice([0.5, 1.0, 2.0, 3.0], size=n) if seed % 3 == 0 else rng.uniform(0, 1, n)
    theta = float(rng.choice([0.25, 0.5, 0.7, 1.0]))
    got = oracle.doerfler(eta2, theta)
    total = eta2.sum()
    best = min(k for k in range(1, n + 1)
               if any(eta2[list(c)].sum() >= theta * total * (1 - 1e-15) for c in itertools.combinations(range(n), k)))
    assert len(got) == best
    assert eta2[got].sum() >= theta * total * (1 - 1e-15)


def test_doerfler_ties_lower_index():
    got = oracle.doerfler(np.array([1.0, 2.0, 2.0, 2.0, 1.0]), 0.5)
    assert got.tolist() == [1, 2]


# ------------------------------------------------------------ mesh check

def test_mesh_check_cases():
    m = synth.cube(2)
    assert oracle.mesh_check(m.verts, m.tris)[0]
    bad = m.tris.copy()
    bad[0, 0] = m.M
    assert not oracle.mesh_check(m.verts, bad)[0]
    v = m.verts.copy()
    v[3, 1] = np.nan
    assert not oracle.mesh_check(v, m.tris)[0]
    assert not oracle.mesh_check(m.verts, m.tris[:-1])[0]  # open surface


def test_cg_solve_matches_cholesky():
    """The oracle's CG solve (for matrices of more than 2^31 entries) reaches
    the Cholesky solution: capacities within 1e-14, the solution within
    1e-12 of its largest entry, and the reported bound on the capacity's
    error holds."""
    for m in (synth.cube(8), synth.voxel_union(3, 0.4, 21), synth.icosphere(3, 1.0)):
        V = oracle.assemble(m.verts, m.tris)
        b = oracle.rhs(m.verts, m.tris)
        x1 = oracle.solve_direct(V, b)
        x2, rr, its = oracle.solve_cg(V, b, rows=100)
        assert rr <= 1e-14 and its > 1
        c1, c2 = oracle.capacity(x1, b), oracle.capacity(x2, b)
        assert abs(c1 - c2) <= 1e-14 * c1
        assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x1))
        r = b - V @ x2
        assert abs(c1 - c2) / c1 <= 2 * np.linalg.norm(x2) * np.linalg.norm(r) / abs(b @ x2) + 1e-16
