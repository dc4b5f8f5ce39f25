"""Pins of the oracle's Galerkin matrix: far-field multipole limit, exact
scaling, rigid-motion invariance, symmetry and definiteness, brute-force pair
classification and mesh independence of 1^T V 1."""

import math

import numpy as np
import pytest

import oracle
import synth

P = lambda *a: np.array(a, dtype=np.float64)  # noqa: E731


def test_far_pair_limit_slope_two():
    # V_ij -> |T_i||T_j| / (4 pi |c_i - c_j|); the centroid expansion has no
    # dipole term, so the relative deviation decays like (diam / dist)^2.
    T1 = [P(0, 0, 0), P(1, 0.1, 0), P(0.2, 0.9, 0.1)]
    T2 = [P(0, 0, 0), P(0.8, 0, 0.3), P(0.1, 0.7, 0.5)]
    dists = np.array([8.0, 16.0, 32.0, 64.0])
    dirn = np.array([0.3, -0.5, 0.81])
    dirn /= np.linalg.norm(dirn)
    devs = []
    for d in dists:
        verts = np.array(T1 + [p + d * dirn for p in T2])
        tris = np.array([[0, 1, 2], [3, 4, 5]])
        g = oracle.element_geometry(verts, tris)
        v = oracle.entry(verts, tris, 0, 1)
        mono = g["area"][0] * g["area"][1] / (4 * math.pi * np.linalg.norm(g["centroid"][0] - g["centroid"][1]))
        devs.append(abs(v - mono) / mono)
    slope = np.polyfit(np.log(dists), np.log(devs), 1)[0]
    assert -2.15 < slope < -1.85, slope


@pytest.fixture(scope="module")
def cube2():
    m = synth.cube(2)
    return m, oracle.assemble(m.verts, m.tris)


def test_exact_scaling(cube2):
    m, V = cube2
    for s in (0.5, 3.0):
        Vs = oracle.assemble(m.verts * s, m.tris)
        assert np.allclose(Vs, s ** 3 * V, rtol=1e-13, atol=0)


def test_rigid_motion_invariance(cube2):
    m, V = cube2
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    verts = m.verts @ Q.T + np.array([0.3, -1.2, 2.5])
    V2 = oracle.assemble(verts, m.tris)
    assert np.allclose(V2, V, rtol=1e-12, atol=0)


def test_symmetric_positive_definite(cube2):
    m, V = cube2
    assert np.array_equal(V, V.T)
    assert np.all(V > 0)
    assert np.linalg.eigvalsh(V).min() > 0
    oracle.solve_direct(V, oracle.rhs(m.verts, m.tris))  # Cholesky succeeds


def _brute_classes(tris):
    out = {}
    for i in range(len(tris)):
        for j in range(i, len(tris)):
            s = len(set(tris[i].tolist()) & set(tris[j].tolist()))
            if s:
                out[(i, j)] = {3: "coincident", 2: "edge", 1: "vertex"}[s]
    return out


@pytest.mark.parametrize("mesh", ["ico2", "voxel", "hull"])
def test_classification_brute_force(mesh):
    m = {"ico2": lambda: synth.icosphere(2), "voxel": lambda: synth.voxel_union(3, 0.4, 11),
         "hull": lambda: synth.convex_hull(15, 4)}[mesh]()
    got = {(i, j): k for (i, j, k, _, _) in oracle.classify_pairs(m.tris)}
    assert got == _brute_classes(m.tris)
    # canonical orders: shared vertices lead, in the documented order
    for (i, j, kind, Ti, Tj) in oracle.classify_pairs(m.tris):
        assert sorted(Ti) == sorted(m.tris[i].tolist()) and sorted(Tj) == sorted(m.tris[j].tolist())
        if kind == "edge":
            assert Ti[:2] == Tj[:2] and Ti[0] < Ti[1]
        if kind == "vertex":
            assert Ti[0] == Tj[0]
            k = m.tris[i].tolist().index(Ti[0])
            assert Ti == tuple(m.tris[i].tolist()[k:] + m.tris[i].tolist()[:k])


def test_icosphere_pair_counts():
    m = synth.icosphere(2)
    cl = oracle.classify_pairs(m.tris)
    N, M = m.N, m.M
    deg = np.bincount(m.tris.ravel(), minlength=M)
    E = 3 * N // 2
    n_vertex = int(sum(d * (d - 1) // 2 for d in deg)) - 2 * E  # pairs through a vertex, minus edge pairs twice
    kinds = [c[2] for c in cl]
    assert kinds.count("coincident") == N
    assert kinds.count("edge") == E
    assert kinds.count("vertex") == n_vertex - 0  # each edge pair appears in both its vertices' counts


def test_one_V_one_mesh_independent():
    # 1^T V 1 = (1/4pi) int int 1/|x-y| over the whole surface, for any
    # triangulation of the same surface (up to quadrature error)
    vals = []
    for n in (3, 6):
        m = synth.cube(n)
        V = oracle.assemble(m.verts, m.tris)
        vals.append(V.sum())
    assert abs(vals[0] - vals[1]) / vals[1] < 2e-4


def test_entry_matches_assemble(cube2):
    m, V = cube2
    rng = np.random.default_rng(3)
    for _ in range(12):
        i, j = rng.integers(0, m.N, size=2)
        assert oracle.entry(m.verts, m.tris, int(i), int(j)) == pytest.approx(V[i, j], rel=1e-14)
    rows = oracle.assemble_rows(m.verts, m.tris, [0, 7, 40])
    assert np.allclose(rows, V[[0, 7, 40]], rtol=1e-14, atol=0)


def test_assemble_parallel_equals_serial():
    m = synth.icosphere(1)
    a = oracle.assemble(m.verts, m.tris, workers=1)
    b = oracle.assemble(m.verts, m.tris, workers=3)
    assert np.array_equal(a, b)


def test_near_pairs_hand_built():
    """Two unit right triangles in the plane z = 0 and a third one far away:
    the first two share no vertex, their centroids are a known distance
    apart, and they are near exactly when that distance is below
    near_factor times the common diameter sqrt(2)."""
    for gap, factor, expect in ((0.5, 1.5, True), (0.5, 0.9, False), (3.0, 1.5, False), (0.6, 1.2, True),
                                (2.0, 1.2, False)):
        verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0],
                          [1 + gap, 0, 0], [2 + gap, 0, 0], [1 + gap, 1, 0],
                          [50, 0, 0], [51, 0, 0], [50, 1, 0]], dtype=np.float64)
        tris = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]])
        # both centroids at height 1/3; x = 1/3 and 1 + gap + 1/3
        dist = 1.0 + gap
        assert (dist < factor * math.sqrt(2.0)) == expect
        got = set(oracle.near_pairs(verts, tris, factor))
        assert got == ({(0, 1), (1, 0)} if expect else set())


def test_near_pairs_spatial_search():
    """The pair list against a k-d tree search (scipy), a different
    enumeration of the same definition, on meshes with graded elements."""
    from scipy.spatial import cKDTree

    for m in (synth.icosphere(2), synth.voxel_union(3, 0.4, 21)):
        v, t = m.verts, m.tris
        if m.name.startswith("voxel"):
            v, t, _ = synth.refine_nvb(v, synth.init_reference_edges(v, t), [0, 5, 9], "bisec3")
        g = oracle.element_geometry(v, t)
        c, d2 = g["centroid"], g["diam2"]
        tree = cKDTree(c)
        cand = tree.query_pairs(1.5 * np.sqrt(d2.max()) * (1 + 1e-9))
        shared = lambda i, j: bool(set(t[i].tolist()) & set(t[j].tolist()))  # noqa: E731
        ref = set()
        for i, j in cand:
            dd = c[i] - c[j]
            # on squares, as defined: lattice meshes have pairs exactly at the threshold
            if (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2] < 2.25 * max(d2[i], d2[j]) and not shared(i, j):
                ref |= {(i, j), (j, i)}
        assert set(oracle.near_pairs(v, t, 1.5)) == ref and len(ref) > 0


def test_near_pairs_definition():
    m = synth.icosphere(2)
    g = oracle.element_geometry(m.verts, m.tris)
    near = set(oracle.near_pairs(m.verts, m.tris, 1.5))
    touching = {(i, j) for (i, j, *_r) in oracle.classify_pairs(m.tris)}
    touching |= {(j, i) for (i, j) in touching}
    for i in range(0, m.N, 7):
        for j in range(m.N):
            d = np.linalg.norm(g["centroid"][i] - g["centroid"][j])
            inside = d < 1.5 * max(g["diam"][i], g["diam"][j])
            expect = inside and (i, j) not in touching and i != j
            assert ((i, j) in near) == expect


def test_per_pair_orders_select_by_class_and_shape():
    """Singular-rule orders chosen per touching pair (oracle.SSOrders): every
    entry of the matrix equals, bitwise, the entry of the uniform-order
    matrix whose order that pair calls for: 6 / 5 / 3 points for pairs that
    share 3 / 2 / 1 vertices, at least 8 where either element is thin
    (diam^2 > 12 |T|); regular entries do not depend on the orders.  Shared
    vertices and thinness are counted here directly from the triangles."""
    h = synth.convex_hull(14, 0, min_angle=0.0)  # facets down to a few degrees
    verts, tris, _ = synth.refine_uniform(h.verts, synth.init_reference_edges(h.verts, h.tris), 1)
    verts, tris = np.asarray(verts), np.asarray(tris)
    P = verts[tris]
    d2 = np.max(np.sum((P[:, [1, 2, 0]] - P) ** 2, axis=2), axis=1)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    thin = d2 > 12.0 * area
    assert thin.any() and (~thin).any()
    got = oracle.assemble(verts, tris, 4, oracle.SSOrders(6, 5, 3, sliver=8, sliver_ratio=12.0))
    uniform = {n: oracle.assemble(verts, tris, 4, n) for n in (3, 5, 6, 8)}
    N = len(tris)
    seen = set()
    for i in range(N):
        for j in range(N):
            shared = len(set(tris[i].tolist()) & set(tris[j].tolist()))
            if shared == 0:
                assert got[i, j] == uniform[3][i, j] == uniform[8][i, j]
                continue
            n = {3: 6, 2: 5, 1: 3}[shared]
            if thin[i] or thin[j]:
                n = max(n, 8)
            seen.add(n)
            assert got[i, j] == uniform[n][i, j], (i, j, shared, n)
    assert seen == {3, 5, 6, 8}
