"""GPU weighted-residual estimator (bc_residual_indicators, Appendix A,
eq. "residual:indicator") against the oracle (oracle/residual.py), on the
oracle's own solution so that only the estimator is compared.

Bars: the first moments m_k = <V Phi, lambda_k>_T within 1e-13 of the same
moments of |Phi| (FP64 rounding of sums over N columns of 256 point pairs);
mu(T) = 6 diam^(1/2) |sum_k m_k e_k| / |T|^(3/2) then differs by at most
6 diam^(1/2) (sum_k |dm_k| |e_k|) / |T|^(3/2), the moments' bound carried
through (the sum cancels the moments' common part, so a relative bound on
mu itself would not follow from the arithmetic)."""

import numpy as np
import pytest

import oracle
import synth
from oracle import residual as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MESHES = {
    "voxel": lambda: synth.voxel_union(3, 0.4, 21),   # N = 104, not a multiple of 64
    "hull": lambda: synth.convex_hull(17, 5),
    "cube4": lambda: synth.cube(4),
    "ico2": lambda: synth.icosphere(2, 0.8),
    "cube768": lambda: synth.cube(8),
}


def _check(m, prec, ss_order=4):
    from paper_1901_08393_amd import api

    V = oracle.assemble(m.verts, m.tris, 4, ss_order)
    b = oracle.rhs(m.verts, m.tris)
    x = oracle.solve_direct(V, b)
    mu2_ref, mom_ref = R.residual_indicators(m.verts, m.tris, x, 4, ss_order)
    mag = R.p1_moments(m.verts, m.tris, np.abs(x), 4, ss_order)
    p = api.CapacityProblem(m.verts, m.tris, prec, ss_order=ss_order)
    p.assemble()
    xd = torch.from_numpy(x).to("cuda")
    mu2, mom = p.residual(xd, moments=True)
    mu2, mom = mu2.cpu().numpy(), mom.cpu().numpy()
    dm = np.abs(mom - mom_ref)
    assert np.max(dm / mag) <= 1e-13, np.max(dm / mag)
    P = np.asarray(m.verts)[np.asarray(m.tris)]
    e = np.stack([P[:, 2] - P[:, 1], P[:, 0] - P[:, 2], P[:, 1] - P[:, 0]], axis=1)
    g = oracle.element_geometry(m.verts, m.tris)
    bound = 6 * np.sqrt(g["diam"]) * np.sum(1e-13 * mag * np.linalg.norm(e, axis=2), axis=1) / g["area"] ** 1.5
    dmu = np.abs(np.sqrt(mu2) - np.sqrt(mu2_ref))
    assert np.all(dmu <= bound + 1e-13 * np.sqrt(mu2_ref)), np.max(dmu / bound)
    print(f"  max moment err {np.max(dm / mag):.1e}, max mu err / bound {np.max(dmu / bound):.2f}, "
          f"sum mu2 {mu2.sum():.6e} (oracle {mu2_ref.sum():.6e})", flush=True)
    return mu2, mu2_ref


@pytest.mark.parametrize("name", list(MESHES))
def test_residual_matches_oracle(name):
    print(f"residual {name}", flush=True)
    _check(MESHES[name](), "fp64")


def test_residual_mixed_pattern_and_order8():
    """A mixed-precision pattern (near entries, which take the regular rule
    here) and order-8 singular rules."""
    print("residual voxel mixed pattern", flush=True)
    _check(MESHES["voxel"](), "mixed")
    print("residual hull order 8", flush=True)
    _check(MESHES["hull"](), "fp64", ss_order=8)


def test_residual_bitwise_reproducible():
    from paper_1901_08393_amd import api

    m = MESHES["ico2"]()
    p = api.CapacityProblem(m.verts, m.tris, "fp64")
    p.assemble()
    p.solve()
    a = p.residual().cpu().numpy()
    b = p.residual().cpu().numpy()
    assert np.array_equal(a, b)
