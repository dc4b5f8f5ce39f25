"""bc_solve_static (the solve whose workspace is a device array of
libbemcap_static.so, for callers that cannot allocate) against bc_solve,
through the C ABI: two calls in a row, the second on a smaller system, each bitwise equal
to bc_solve's result (same kernels, same fixed-order reductions), in both
precisions; and the size limit returns BC_ENOMEM."""

import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _run(L, _lib, api, p, static):
    o = api.default_solve_opts(p.precision, cap_rtol=1e-8 if p.precision == "mixed" else None)
    sigma = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    res = torch.zeros(C.sizeof(_lib.bc_result), dtype=torch.uint8, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if static:
        st = _lib.lib_static().bc_solve_static(_ptr(p.V), p.N, p.prec, _ptr(p.pattern), p.nnz, _ptr(p.area), _ptr(sigma), C.byref(o),
                               _ptr(res), stream)
    else:
        nb = L.bc_solve_workspace_bytes(p.N, p.prec)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        st = L.bc_solve(_ptr(p.V), p.N, p.prec, _ptr(p.pattern), p.nnz, _ptr(p.area), _ptr(sigma), C.byref(o),
                        _ptr(ws), nb, _ptr(res), stream)
    assert st == _lib.BC_OK
    torch.cuda.synchronize()
    return api.SolveResult.from_bytes(res.cpu().numpy().tobytes()), sigma.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_solve_equals_solve(prec):
    from paper_1901_08393_amd import _lib, api

    L = _lib.lib()
    meshes = [synth.icosphere(4, 0.9), synth.voxel_union(3, 0.4, 21)]  # N = 5120, then N = 104
    for m in meshes:
        print(f"static solve {prec} N={m.N}", flush=True)
        p = api.CapacityProblem(m.verts, m.tris, prec)
        p.assemble()
        r_ref, s_ref = _run(L, _lib, api, p, static=False)
        r_st, s_st = _run(L, _lib, api, p, static=True)
        assert r_ref.ok and r_st.ok
        assert r_st.cap == r_ref.cap and r_st.iters == r_ref.iters and r_st.outer == r_ref.outer
        assert np.array_equal(s_st, s_ref)


def test_static_solve_size_limit():
    from paper_1901_08393_amd import _lib, api

    S = _lib.lib_static()
    o = api.default_solve_opts("mixed")
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = S.bc_solve_static(_ptr(dummy), 40000, _lib.BC_MIXED, _ptr(dummy), 40000, _ptr(dummy), _ptr(dummy),
                           C.byref(o), _ptr(dummy), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.BC_ENOMEM
