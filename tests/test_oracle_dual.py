"""Pins of the dual-mesh oracle (oracle/dual.py) against facts fixed by the
geometry and the mathematics, not by re-evaluating its own formulas:

* the barycentric refinement splits every triangle into six of equal area
  |T|/6 (the medians cut a triangle into six triangles of equal area) and is
  a closed conforming surface; each son touches the vertex whose dual cell
  it belongs to;
* the dual cell of a vertex has the area of the hat function's integral,
  sum_{T ni z} |T|/3 (two independent computations), and the cells tile the
  surface;
* the mass matrix <phi_j, chi_i^dual> has row sums |T_i^dual| and column
  sums <phi_j, 1> (partition of unity, dual cells tile Gamma), is symmetric,
  and has the hand-derived entries 11|T|/54 (own vertex) and 7|T|/108
  (other vertex of the triangle) per triangle;
* surface curls are tangential, sum to zero over a triangle's three hat
  functions and equal (P_{a+1} - P_{a+2}) / (2|T|) (derived by hand from
  the gradient of a barycentric coordinate);
* the hypersingular matrix annihilates constants, is symmetric positive
  semi-definite, and on spheres <D z, z> converges to the exact value
  (2/3) ||z||^2 = 8 pi / 9 (z is a degree-1 spherical harmonic, for which
  the Laplace hypersingular operator on the unit sphere has eigenvalue
  l (l + 1) / (2 l + 1) = 2/3);
* the dual capacity of spheres increases towards r at the same rate as the
  primal one and the two agree to the discretisation error;
* the dual ZZ indicators vanish for constant solutions and match a
  brute-force quadrature of (Phi - I Phi)^2.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import dual

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def ico():
    out = {}
    for L in (1, 2):
        m = synth.icosphere(L, 1.0)
        Vb, P, bv, bt = dual.assemble_dual(m.verts, m.tris)
        out[L] = (m, Vb, P)
    return out


def test_barycentric_refinement():
    for m in (synth.cube(2), synth.icosphere(1, 0.7), synth.voxel_union(2, 0.4, 7)):
        bv, bt, parent, owner = dual.barycentric_mesh(m.verts, m.tris)
        assert bt.shape[0] == 6 * m.N
        ok, info = synth.mesh_topology_ok(bv, bt)
        assert ok and info["euler"] == 2
        a = oracle.element_geometry(m.verts, m.tris)["area"]
        ab = oracle.element_geometry(bv, bt)["area"]
        assert np.allclose(ab, np.repeat(a, 6) / 6.0, rtol=1e-13, atol=0)
        assert all(owner[k] in bt[k] for k in range(bt.shape[0]))
        assert all(owner[k] in m.tris[parent[k]] for k in range(bt.shape[0]))


def test_barycentric_generator_matches_oracle():
    """The GPU side takes the barycentric mesh from synth.barycentric
    (vectorised); the oracle builds it triangle by triangle from the
    definition.  Vertices, sons, parents and owners agree bitwise, and each
    son has its parent's orientation (the same normal direction)."""
    for m in (synth.cube12(), synth.fichera48(), synth.voxel_union(3, 0.4, 21), synth.convex_hull(17, 5)):
        bv, bt, parent, owner = dual.barycentric_mesh(m.verts, m.tris)
        sm, spar, sown = synth.barycentric(m.verts, m.tris)
        assert np.array_equal(bv, sm.verts) and np.array_equal(bt, sm.tris)
        assert np.array_equal(parent, spar) and np.array_equal(owner, sown)
        P = bv[bt]
        n_son = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        Q = np.asarray(m.verts)[np.asarray(m.tris)][parent]
        n_par = np.cross(Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0])
        assert np.all(np.einsum("ij,ij->i", n_son, n_par) > 0)


def test_dual_cells_tile_the_surface():
    m = synth.voxel_union(2, 0.4, 7)
    f = dual.dual_load(m.verts, m.tris)
    a = dual.hat_integrals(m.verts, m.tris)
    area = oracle.element_geometry(m.verts, m.tris)["area"]
    assert np.allclose(f, a, rtol=1e-13, atol=0)
    assert math.isclose(f.sum(), area.sum(), rel_tol=1e-13)


def test_mass_matrix():
    m = synth.cube(1)
    Mm = dual.dual_mass(m.verts, m.tris)
    f = dual.dual_load(m.verts, m.tris)
    a = dual.hat_integrals(m.verts, m.tris)
    assert np.allclose(Mm.sum(1), f, rtol=1e-13) and np.allclose(Mm.sum(0), a, rtol=1e-13)
    assert np.allclose(Mm, Mm.T, rtol=0, atol=1e-15)
    # hand-derived entries: per triangle 11|T|/54 on its vertices' diagonal,
    # 7|T|/108 between two of its vertices
    area = oracle.element_geometry(m.verts, m.tris)["area"]
    ref = np.zeros_like(Mm)
    for t, tri in enumerate(m.tris):
        for i in tri:
            for j in tri:
                ref[i, j] += area[t] * (11.0 / 54.0 if i == j else 7.0 / 108.0)
    assert np.allclose(Mm, ref, rtol=1e-13, atol=1e-16)


def test_surface_curls():
    m = synth.convex_hull(12, 3)
    C = dual.surface_curls(m.verts, m.tris)
    P = m.verts[m.tris]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    A2 = np.linalg.norm(n, axis=1)
    n /= A2[:, None]
    assert np.abs((C * n[:, None, :]).sum(-1)).max() < 1e-12 * np.abs(C).max()
    assert np.abs(C.sum(1)).max() < 1e-12 * np.abs(C).max()
    for a in range(3):
        ref = (P[:, (a + 1) % 3] - P[:, (a + 2) % 3]) / A2[:, None]
        assert np.allclose(C[:, a], ref, rtol=1e-12, atol=1e-12)


def test_hypersingular_matrix(ico):
    errs = []
    for L in (1, 2):
        m, Vb, P = ico[L]
        Q = dual.curl_matrices(m.verts, m.tris)
        D = dual.hypersingular(Vb, Q)
        assert np.abs(D.sum(1)).max() <= 1e-12 * np.abs(D).max()
        assert np.allclose(D, D.T, rtol=0, atol=1e-14 * np.abs(D).max())
        w = np.linalg.eigvalsh(D)
        assert w[0] > -1e-12 * w[-1] and w[1] > 0
        a = dual.hat_integrals(m.verts, m.tris)
        assert np.linalg.eigvalsh(D + np.outer(a, a))[0] > 0
        z = m.verts[:, 2]
        errs.append(abs(z @ D @ z - 8.0 * math.pi / 9.0))
    assert errs[1] < errs[0] / 3.0 and errs[1] < 0.1, errs


def test_dual_capacity_of_spheres(ico):
    caps, gaps = [], []
    for L in (1, 2):
        m, Vb, P = ico[L]
        f = dual.dual_load(m.verts, m.tris)
        x, Vd = dual.solve_dual(Vb, P, f)
        assert np.linalg.eigvalsh(Vd)[0] > 0
        cap = dual.capacity_dual(x, f)
        V = oracle.assemble(m.verts, m.tris)
        b = oracle.rhs(m.verts, m.tris)
        capp = oracle.capacity(oracle.solve_direct(V, b), b)
        caps.append(cap)
        gaps.append(abs(cap - capp))
    assert caps[0] < caps[1] < 1.0
    assert (1.0 - caps[1]) < (1.0 - caps[0]) / 3.0
    assert gaps[1] < gaps[0]


def test_zz_dual():
    m = synth.cube(1)
    assert np.abs(dual.zz_dual(m.verts, m.tris, np.full(m.verts.shape[0], 2.5))).max() < 1e-28
    rng = np.random.default_rng(0)
    x = rng.standard_normal(m.verts.shape[0])
    eta2 = dual.zz_dual(m.verts, m.tris, x)
    # brute force: midpoint sampling of (Phi - I Phi)^2 on a fine grid of each
    # barycentric son (where Phi is constant and the integrand smooth)
    geo = oracle.element_geometry(m.verts, m.tris)
    bv, bt, parent, owner = dual.barycentric_mesh(m.verts, m.tris)
    ab = oracle.element_geometry(bv, bt)["area"]
    ref = np.zeros(m.N)
    n = 48
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = ii + jj < n
    lower = np.stack([(ii[keep] + 1 / 3) / n, (jj[keep] + 1 / 3) / n], 1)
    keep2 = ii + jj < n - 1
    upper = np.stack([(ii[keep2] + 2 / 3) / n, (jj[keep2] + 2 / 3) / n], 1)
    uv = np.concatenate([lower, upper])  # n^2 cells of equal area
    for k in range(bt.shape[0]):
        t = parent[k]
        Q = bv[bt[k]]
        pts = Q[0] + uv[:, :1] * (Q[1] - Q[0]) + uv[:, 1:] * (Q[2] - Q[0])
        P = m.verts[m.tris[t]]
        e1, e2 = P[1] - P[0], P[2] - P[0]
        G = np.array([[e1 @ e1, e1 @ e2], [e2 @ e1, e2 @ e2]])
        d = pts - P[0]
        su = np.linalg.solve(G, np.stack([d @ e1, d @ e2]))
        lam = np.stack([1 - su[0] - su[1], su[0], su[1]], 1)
        g = x[owner[k]] - lam @ x[m.tris[t]]
        ref[t] += ab[k] * np.mean(g * g)
    ref *= geo["diam"]
    assert np.allclose(eta2, ref, rtol=1e-3), (eta2, ref)


def test_table1_first_step():
    """Section 3.1, Table 1, l = 0: the dual-mesh capacity and estimator of
    the 12-triangle unit cube.  The printed values depend on the face
    diagonals of T_0 (eight classes, capacities 0.64889 .. 0.64971 at the
    same quadrature); on the class built by synth.cube12 the converged
    capacity lies 2.3e-6 below the printed one (the paper's quadrature
    orders are not stated; our own order 4 -> 8 changes the value by 2e-5).
    eta^2 uses the mesh size |T|^(1/2) of the paper's implementation listing
    (Appendix B); with diam(T)^(1/2) it would be twice as large on this mesh,
    and on every other diagonal class it is off by more than a factor 2.
    (This row's error column, 1.114e-2, does not equal the literature value
    minus its capacity column, 1.1397e-2; later rows do.  The capacity column
    is the one pinned.)"""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    row = g["cube_table1"]["rows"][0]
    m = synth.cube12()
    assert m.N == row["N"]
    Vb, P, bv, bt = dual.assemble_dual(m.verts, m.tris, 8, 8)
    f = dual.dual_load(m.verts, m.tris)
    x, Vd = dual.solve_dual(Vb, P, f)
    cap = dual.capacity_dual(x, f)
    assert abs(cap - row["cap"]) < 1e-5, cap
    eta2 = dual.zz_dual(m.verts, m.tris, x, "area").sum()
    assert abs(eta2 / row["eta2"] - 1.0) < 2e-3, eta2


def test_table2_first_step():
    """Section 3.2, Table 2, l = 0: the dual-mesh capacity and estimator of
    the 48-triangle Fichera cube (synth.fichera48).  Converged quadrature
    (order 8) gives 1.2813949, 3.6e-6 below the printed 1.2813985240 (order
    4: 1.28141130, so the paper's unstated orders explain the gap), and
    eta^2 = 0.323868 with |T|^(1/2), inside the printed 3.239e-1's rounding
    interval."""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    row = g["fichera_table2"]["rows"][0]
    m = synth.fichera48()
    assert m.N == row["N"]
    Vb, P, bv, bt = dual.assemble_dual(m.verts, m.tris, 8, 8)
    f = dual.dual_load(m.verts, m.tris)
    x, Vd = dual.solve_dual(Vb, P, f)
    cap = dual.capacity_dual(x, f)
    assert abs(cap - row["cap"]) < 1e-5, cap
    eta2 = dual.zz_dual(m.verts, m.tris, x, "area").sum()
    assert abs(eta2 - row["eta2"]) <= 5e-5, eta2
