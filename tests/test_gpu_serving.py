"""Continuous-batching server: every result is bitwise the same alone and in
the mix (saturated and Poisson arrivals, memory budget small enough to force
queueing), and the FP64 form matches the CPU oracle."""

import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests(n=14, seed=11, rate=math.inf):
    reqs = synth.request_stream(n, seed=seed, rate=rate, n_min=200, n_max=2500)
    return reqs, [r.build_mesh() for r in reqs]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_serving_alone_equals_mix(precision):
    from paper_1901_08393_amd import api
    from paper_1901_08393_amd.serve import CapacityServer, summarize

    print(f"serving {precision}", flush=True)
    reqs, meshes = _requests(rate=400.0)
    # results alone
    alone = []
    for m in meshes:
        p = api.CapacityProblem(m.verts, m.tris, precision)
        p.assemble()
        r = p.solve()
        alone.append((r.cap, r.iters, p.sigma.cpu().numpy().copy()))
    srv = CapacityServer(precision, chunk_ms=0.05)
    # budget for about three of the largest requests at a time: forces queueing
    srv.budget = 3 * max(srv.footprint(m.N) for m in meshes)
    for realtime in (False, True):  # saturated (all at t = 0), then Poisson arrivals
        recs = srv.run(reqs, meshes, realtime=realtime)
        s = summarize(recs)
        print(s, flush=True)
        assert s["ok"] == len(reqs)
        assert max(r.chunks for r in recs) > 1  # systems were interleaved over several chunks
        for rec, (cap, iters, _sig) in zip(recs, alone):
            assert rec.cap == cap and rec.iters == iters, (rec, cap)
            assert rec.latency > 0


def test_serving_sigma_bitwise_and_oracle():
    from paper_1901_08393_amd import api
    from paper_1901_08393_amd.serve import CapacityServer

    reqs, meshes = _requests(n=6, seed=4)
    srv = CapacityServer("fp64", chunk_ms=0.05, keep_sigma=True)
    recs = srv.run(reqs, meshes, realtime=False)
    for rec, m in zip(recs, meshes):
        p = api.CapacityProblem(m.verts, m.tris, "fp64")
        p.assemble()
        r = p.solve()
        assert np.array_equal(rec.sigma, p.sigma.cpu().numpy())
        if m.N <= 1200:
            V = oracle.assemble(m.verts, m.tris)
            b = oracle.rhs(m.verts, m.tris)
            cap_ref = oracle.capacity(oracle.solve_direct(V, b), b)
            assert abs(rec.cap - cap_ref) <= 1e-12 * cap_ref
        assert r.cap == rec.cap


def test_serving_rejects_oversize():
    from paper_1901_08393_amd.serve import CapacityServer

    reqs, meshes = _requests(n=3, seed=9)
    srv = CapacityServer("mixed")
    srv.budget = min(srv.footprint(m.N) for m in meshes) - 1  # nothing fits
    recs = srv.run(reqs, meshes, realtime=False)
    assert all(r.status == -3 for r in recs)
