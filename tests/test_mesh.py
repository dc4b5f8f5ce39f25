"""Seeded input generators and newest-vertex bisection."""

import numpy as np
import pytest

import synth


def test_cube_768_counts_and_topology():
    m = synth.cube(8)
    assert (m.N, m.M) == (768, 386)
    ok, info = synth.mesh_topology_ok(m.verts, m.tris)
    assert ok and info["euler"] == 2
    assert m.verts.min() == 0.0 and m.verts.max() == 1.0


@pytest.mark.parametrize("level,N,M", [(0, 20, 12), (2, 320, 162), (4, 5120, 2562)])
def test_icosphere_counts(level, N, M):
    r = 1.7
    m = synth.icosphere(level, r)
    assert (m.N, m.M) == (N, M)
    assert np.allclose(np.linalg.norm(m.verts, axis=1), r, rtol=1e-15)
    assert synth.mesh_topology_ok(m.verts, m.tris)[0]


@pytest.mark.parametrize("seed", [3, 4, 5, 17])
def test_voxel_union_manifold_and_seeded(seed):
    a = synth.voxel_union(4, 0.4, seed)
    b = synth.voxel_union(4, 0.4, seed)
    assert np.array_equal(a.verts, b.verts) and np.array_equal(a.tris, b.tris)
    assert a.meta["voxels"] >= 26
    ok, info = synth.mesh_topology_ok(a.verts, a.tris)
    assert ok
    assert info["euler"] % 2 == 0 and info["euler"] <= 2


def test_hull_and_box():
    h = synth.convex_hull(20, 1)
    ok, info = synth.mesh_topology_ok(h.verts, h.tris)
    assert ok and info["euler"] == 2
    b = synth.box(3.0, 7.5)
    assert b.N == 12 and synth.mesh_topology_ok(b.verts, b.tris)[0]
    assert np.allclose(b.verts.max(0), [1.0, 3.0, 7.5])


def _areas(v, t):
    P = v[t]
    return 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)


@pytest.mark.parametrize("mode", ["bisec3", "bisec1"])
def test_nvb_conforming_area_preserving(mode):
    m = synth.voxel_union(3, 0.4, 8)
    v, t = m.verts, synth.init_reference_edges(m.verts, m.tris)
    rng = np.random.default_rng(0)
    for _ in range(4):
        marked = rng.choice(len(t), max(1, len(t) // 8), replace=False)
        v2, t2, parent = synth.refine_nvb(v, t, marked, mode)
        ok, info = synth.mesh_topology_ok(v2, t2)
        assert ok, info
        a1, a2 = _areas(v, t), _areas(v2, t2)
        # sons tile their parent
        assert np.allclose(np.bincount(parent, weights=a2, minlength=len(t)), a1, rtol=1e-13)
        # marked elements are bisected
        counts = np.bincount(parent, minlength=len(t))
        assert np.all(counts[marked] >= (4 if mode == "bisec3" else 2))
        assert np.all(np.isin(counts, [1, 2, 3, 4]))
        v, t = v2, t2


def test_nvb_shape_regularity():
    # NVB generates finitely many similarity classes: min angle stays bounded
    m = synth.convex_hull(12, 3)
    v, t = m.verts, synth.init_reference_edges(m.verts, m.tris)

    def min_angle(v, t):
        P = v[t]
        out = []
        for k in range(3):
            a = P[:, (k + 1) % 3] - P[:, k]
            b = P[:, (k + 2) % 3] - P[:, k]
            c = np.einsum("ij,ij->i", a, b) / np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1)
            out.append(np.arccos(np.clip(c, -1, 1)))
        return np.min(out)

    a0 = min_angle(v, t)
    rng = np.random.default_rng(1)
    for _ in range(6):
        v, t, _ = synth.refine_nvb(v, t, rng.choice(len(t), len(t) // 4, replace=False))
    assert min_angle(v, t) >= a0 / 4 - 1e-12


def test_uniform_refinement_counts():
    m = synth.cube(2)
    v, t, parent = synth.refine_uniform(m.verts, synth.init_reference_edges(m.verts, m.tris), 2)
    assert len(t) == 16 * m.N
    assert synth.mesh_topology_ok(v, t)[0]


def test_refine_to_size_and_requests():
    reqs = synth.request_stream(6, seed=5, rate=10.0)
    assert all(reqs[k].arrival < reqs[k + 1].arrival for k in range(5))
    again = synth.request_stream(6, seed=5, rate=10.0)
    assert [(r.kind, r.n_target, r.seed) for r in reqs] == [(r.kind, r.n_target, r.seed) for r in again]
    # the requests do not depend on the arrival rate (a Poisson run serves the
    # same meshes as the saturated one)
    sat = synth.request_stream(6, seed=5)
    assert all(r.arrival == 0.0 for r in sat)
    assert [(r.kind, r.params, r.n_target, r.seed) for r in reqs] == [(r.kind, r.params, r.n_target, r.seed) for r in sat]
    small = [r for r in reqs if r.n_target < 4000][:2]
    for r in small:
        mesh = r.build_mesh()
        assert mesh.N >= r.n_target
        assert synth.mesh_topology_ok(mesh.verts, mesh.tris)[0]
