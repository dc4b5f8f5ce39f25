"""Adaptive loop (solve, ZZ, Doerfler, NVB) on the GPU against the oracle at
every step, on a small voxel union; capacities increase monotonically
(nested P0 spaces, Appendix A corollary)."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_adaptive_steps_match_oracle():
    from paper_1901_08393_amd.adaptive import adaptive_capacity

    m = synth.voxel_union(2, 0.4, 3)
    t0 = synth.init_reference_edges(m.verts, m.tris)
    v, t, _ = synth.refine_uniform(m.verts, t0, 1)
    steps = adaptive_capacity(v, t, steps=3, theta=0.5, precision="fp64", keep=True)
    caps = [s.cap for s in steps]
    assert all(caps[k] < caps[k + 1] for k in range(len(caps) - 1)), caps
    for s in steps:
        print(f"level {s.level} N={s.N} cap={s.cap:.12f} eta2={s.eta2:.3e} marked={s.n_marked}", flush=True)
        V = oracle.assemble(s.verts, s.tris)
        b = oracle.rhs(s.verts, s.tris)
        x = oracle.solve_direct(V, b)
        cap_ref = oracle.capacity(x, b)
        assert abs(s.cap - cap_ref) <= 1e-12 * cap_ref
        eta_ref = oracle.zz_indicators(s.verts, s.tris, x)
        assert np.allclose(s.eta2_elem, eta_ref, rtol=1e-9, atol=1e-12 * eta_ref.max())
        if s.n_marked:
            mk = oracle.doerfler(eta_ref, 0.5)
            from paper_1901_08393_amd.adaptive import doerfler

            assert np.array_equal(doerfler(s.eta2_elem, 0.5), mk)
    # the meshes really are nested refinements with growing N
    assert all(steps[k].N < steps[k + 1].N for k in range(len(steps) - 1))


def test_residual_driven_steps_match_oracle():
    """Appendix A's algorithm (weighted-residual indicators, Doerfler, NVB)
    on the GPU: capacities and mu^2 against the oracle at every step; the
    marked set has the oracle's minimal size and satisfies Doerfler for the
    oracle's indicators (equal indicators may be ordered differently)."""
    from paper_1901_08393_amd.adaptive import adaptive_capacity, doerfler
    from oracle import residual as R

    m = synth.voxel_union(2, 0.4, 3)
    t0 = synth.init_reference_edges(m.verts, m.tris)
    steps = adaptive_capacity(m.verts, t0, steps=3, theta=0.5, precision="fp64", keep=True, estimator="residual")
    caps = [s.cap for s in steps]
    assert all(caps[k] < caps[k + 1] for k in range(len(caps) - 1)), caps
    for s in steps:
        print(f"level {s.level} N={s.N} cap={s.cap:.12f} mu2={s.eta2:.3e} marked={s.n_marked}", flush=True)
        V = oracle.assemble(s.verts, s.tris)
        b = oracle.rhs(s.verts, s.tris)
        x = oracle.solve_direct(V, b)
        cap_ref = oracle.capacity(x, b)
        assert abs(s.cap - cap_ref) <= 1e-12 * cap_ref
        mu_ref, _ = R.residual_indicators(s.verts, s.tris, x)
        # the GPU solution (not the oracle's) went in: compare at the solver's accuracy
        assert np.allclose(s.eta2_elem, mu_ref, rtol=1e-6, atol=1e-9 * mu_ref.max())
        if s.n_marked:
            mk = oracle.doerfler(mu_ref, 0.5)
            got = doerfler(s.eta2_elem, 0.5)
            assert got.size == mk.size
            assert mu_ref[got].sum() >= 0.5 * mu_ref.sum() * (1 - 1e-9)
    assert all(steps[k].N < steps[k + 1].N for k in range(len(steps) - 1))
