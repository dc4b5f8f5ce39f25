"""The C-ABI library loads, exports every symbol include/bemcap.h declares,
and its host-only functions (sizes, status text, mesh validation, argument
checks) behave as documented.  No device work is launched here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1901_08393_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libbemcap.so not built (run __graft_entry__.build())")
    return _lib.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bemcap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_exported(L):
    from paper_1901_08393_amd import _lib

    names = declared_functions()
    assert len(names) >= 15
    S = _lib.lib_static()
    for n in names:
        assert hasattr(S if n in _lib.STATIC_SIGNATURES else L, n), n
    assert set(names) == set(_lib.SIGNATURES) | set(_lib.STATIC_SIGNATURES)
    # the main library does not carry the allocation-free entry point's array
    assert not hasattr(L, "bc_solve_static")


def test_version_and_status_strings(L):
    assert L.bc_version() >= 10000
    for s in (0, -1, -2, -3, -4, -5, -6, -7, 1):
        assert L.bc_status_string(s)
    assert L.bc_status_string(-99) == b"unknown status"


def test_sizes(L):
    assert L.bc_matrix_ld(1) == 64 and L.bc_matrix_ld(64) == 64 and L.bc_matrix_ld(65) == 128
    assert L.bc_matrix_bytes(768, 0) == 768 * 768 * 8
    assert L.bc_matrix_bytes(1000, 1) == 1000 * 1024 * 4
    assert L.bc_matrix_bytes(10, 7) == 0
    assert L.bc_mesh_workspace_bytes(1000) > 1000 * (16 + 32 + 8 + 4 * 16 * (8 + 8 + 4 + 4))
    assert L.bc_pattern_bytes(100, 1000, 1) > L.bc_pattern_bytes(100, 1000, 0)
    assert L.bc_solve_workspace_bytes(1000, 0) > L.bc_solve_workspace_bytes(1000, 1)
    assert L.bc_solve_workgroups(1) == 1 and L.bc_solve_workgroups(80) == 1 and L.bc_solve_workgroups(81) == 2
    assert L.bc_solve_workgroups(10 ** 6) == 256
    assert L.bc_batch_scratch_bytes(3) >= 3 * 96
    # products with several vectors: FP64 with 1 or 3, mixed with 1
    one, three = L.bc_matvec_workspace_bytes(5000, 0, 1), L.bc_matvec_workspace_bytes(5000, 0, 3)
    assert one > 0 and three > 2 * one
    assert L.bc_matvec_workspace_bytes(5000, 1, 1) > 0
    assert L.bc_matvec_workspace_bytes(5000, 0, 2) == 0 and L.bc_matvec_workspace_bytes(5000, 1, 3) == 0
    # FP32 matrix with FP64 vectors: 1 or 3
    assert L.bc_matvec_workspace_bytes(5000, 2, 1) > 0 and L.bc_matvec_workspace_bytes(5000, 2, 3) > 0


def _check(L, verts, tris):
    v = np.ascontiguousarray(verts, np.float64)
    t = np.ascontiguousarray(tris, np.int32)
    bad = C.c_int64(0)
    st = L.bc_mesh_check(v.ctypes.data_as(C.c_void_p), v.shape[0], t.ctypes.data_as(C.c_void_p), t.shape[0],
                         C.byref(bad))
    return st, bad.value


def test_mesh_check(L):
    import oracle

    for m in (synth.cube(3), synth.icosphere(2), synth.voxel_union(3, 0.4, 2), synth.convex_hull(11, 1)):
        assert _check(L, m.verts, m.tris) == (0, -1)
        assert oracle.mesh_check(m.verts, m.tris)[0]
    m = synth.cube(2)
    t = m.tris.copy()
    t[5, 2] = m.M + 3
    assert _check(L, m.verts, t) == (-2, 5)
    t = m.tris.copy()
    t[7, 1] = t[7, 0]
    assert _check(L, m.verts, t) == (-2, 7)
    v = m.verts.copy()
    v[4, 2] = np.inf
    assert _check(L, v, m.tris) == (-2, 4)
    assert _check(L, m.verts, m.tris[:-2])[0] == -2  # open
    v = np.concatenate([m.verts, m.verts[:1]])
    t = m.tris.copy()
    t[t == 0] = m.M  # duplicate vertex position, unwelded
    assert _check(L, v, t)[0] == -2
    flat = m.verts.copy()
    flat[:, 2] = 0.0  # every triangle on z=0 faces... zero-area ones appear
    assert _check(L, flat, m.tris)[0] == -2


def test_argument_errors_without_device(L):
    from paper_1901_08393_amd import _lib

    o = _lib.bc_assembly_opts(4, 4, 0, 0, 0.0)
    info = _lib.bc_pattern_info()
    null = C.c_void_p(0)
    assert L.bc_prepare(null, 8, null, 12, C.byref(o), null, 0, C.byref(info), null) == -1
    bad = _lib.bc_assembly_opts(9, 4, 0, 0, 0.0)
    assert L.bc_prepare(C.c_void_p(16), 8, C.c_void_p(16), 12, C.byref(bad), C.c_void_p(16), 1 << 30,
                        C.byref(info), null) == -1
    for bad in (_lib.bc_assembly_opts(4, 4, 0, 2, 0.0), _lib.bc_assembly_opts(4, 4, 1, 2, 1.5)):
        # the 7-point rule for distant blocks is an option (0 or 1)
        assert L.bc_prepare(C.c_void_p(16), 8, C.c_void_p(16), 12, C.byref(bad), C.c_void_p(16), 1 << 30,
                            C.byref(info), null) == -1
    # per-pair singular orders: orders within 0..8, a ratio with the sliver order, reserved 0
    for bad in (_lib.bc_assembly_opts(4, 4, 0, 0, 0.0, 9, 0, 0, 0, 0.0),
                _lib.bc_assembly_opts(4, 4, 0, 0, 0.0, 0, -1, 0, 0, 0.0),
                _lib.bc_assembly_opts(4, 4, 0, 0, 0.0, 0, 0, 8, 0, 0.0),
                _lib.bc_assembly_opts(4, 4, 0, 0, 0.0, 0, 0, 8, 0, float("nan")),
                _lib.bc_assembly_opts(4, 4, 0, 0, 0.0, 0, 0, 0, 1, 0.0)):
        assert L.bc_prepare(C.c_void_p(16), 8, C.c_void_p(16), 12, C.byref(bad), C.c_void_p(16), 1 << 30,
                            C.byref(info), null) == -1
    fp64_near = _lib.bc_assembly_opts(4, 4, 0, 0, 1.5)
    assert L.bc_prepare(C.c_void_p(16), 8, C.c_void_p(16), 12, C.byref(fp64_near), C.c_void_p(16), 1 << 30,
                        C.byref(info), null) == -1
    assert L.bc_prepare(C.c_void_p(16), 8, C.c_void_p(16), 12, C.byref(o), C.c_void_p(16), 10,
                        C.byref(info), null) == -3
    so = _lib.bc_solve_opts(1e-12, 1e-11, 0, 1, 1, 0)  # max_iter 0 invalid
    assert L.bc_solve(C.c_void_p(16), 12, 0, null, 0, C.c_void_p(16), C.c_void_p(16), C.byref(so), C.c_void_p(16),
                      1 << 30, C.c_void_p(16), null) == -1
    so = _lib.bc_solve_opts(1e-12, 1e-11, 10, 1, 1, 0)
    assert L.bc_solve(C.c_void_p(16), 12, 0, null, 0, C.c_void_p(16), C.c_void_p(16), C.byref(so), C.c_void_p(16),
                      100, C.c_void_p(16), null) == -3
    for cap_rtol in (-1e-8, 1.0, float("nan"), float("inf")):  # capacity tolerance outside [0, 1)
        so = _lib.bc_solve_opts(1e-12, 1e-11, 10, 1, 1, 0, cap_rtol)
        assert L.bc_solve(C.c_void_p(16), 12, 0, null, 0, C.c_void_p(16), C.c_void_p(16), C.byref(so),
                          C.c_void_p(16), 1 << 30, C.c_void_p(16), null) == -1
    for spin, res in ((-1, 0), (0, 1)):  # negative spin limit, reserved field set
        so = _lib.bc_solve_opts(1e-12, 1e-11, 10, 1, 1, 0, 0.0, spin, res)
        assert L.bc_solve(C.c_void_p(16), 12, 0, null, 0, C.c_void_p(16), C.c_void_p(16), C.byref(so),
                          C.c_void_p(16), 1 << 30, C.c_void_p(16), null) == -1
    assert L.bc_zz_indicators(null, 12, null, null, 12, null, 0, null, null) == -1
    assert L.bc_capacity(null, null, 5, null, null) == -1
    assert L.bc_matvec(C.c_void_p(16), 100, 0, 2, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 1 << 30,
                       null) == -1
    # dual solve options: negative lambda and unknown h_mode are argument errors
    res = _lib.bc_dual_result()
    v = C.c_void_p(16)
    for o in (_lib.bc_dual_opts(1e-10, -1.0, 10, 20, 30, 1), _lib.bc_dual_opts(1e-10, 1e-3, 10, 20, 30, 2),
              _lib.bc_dual_opts(1e-10, 0.0, 30, 20, 30, 1)):
        assert L.bc_dual_solve(v, 0, null, 0, v, 100, 60, v, v, v, v, 1 << 40, C.byref(o), v, C.byref(res),
                               null) == -1
    # mixed dual solve without its pattern; unknown precision
    o = _lib.bc_dual_opts(1e-10, 0.0, 10, 20, 30, 1)
    for prec, pat in ((1, null), (7, v)):
        assert L.bc_dual_solve(v, prec, pat, 10, v, 100, 60, v, v, v, v, 1 << 40, C.byref(o), v, C.byref(res),
                               null) == -1
    assert L.bc_matvec(C.c_void_p(16), 100, 0, 3, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 10, null) == -3
