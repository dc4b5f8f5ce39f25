"""Python front end of libbemcap.

PyTorch provides device memory and streams; every numerical step runs in the
library's HIP kernels.  One :class:`CapacityProblem` holds a mesh resident in
HBM together with its geometry tables, sparse pattern, dense matrix and
solver state:

    prob = CapacityProblem(verts, tris, precision="mixed")
    prob.assemble()
    res = prob.solve()          # res.cap = (1/4pi) sum sigma_i |T_i|
    eta2 = prob.zz(prob.sigma)  # ZZ-type indicators per element
"""

from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

PRECISION = {"fp64": _lib.BC_FP64, "mixed": _lib.BC_MIXED}


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclasses.dataclass
class SolveResult:
    cap: float
    rel_residual: float
    iters: int
    outer: int
    status: int
    precision: int
    cap_bound: float = 0.0  # ||sigma|| ||r|| / |b^T sigma|: first-order bound on Cap's relative algebraic error

    @property
    def ok(self) -> bool:
        return self.status == _lib.BC_OK

    @staticmethod
    def from_bytes(b: bytes) -> "SolveResult":
        r = _lib.bc_result.from_buffer_copy(b)
        return SolveResult(r.cap, r.rel_residual, r.iters, r.outer, r.status, r.precision, r.cap_bound)


def default_solve_opts(precision: str, **over) -> _lib.bc_solve_opts:
    if precision == "fp64":
        o = dict(rtol=1e-12, inner_rtol=1e-11, max_iter=20000, max_outer=40, jacobi=1, x0_given=0, cap_rtol=0.0)
    else:
        o = dict(rtol=1e-10, inner_rtol=1e-5, max_iter=20000, max_outer=60, jacobi=1, x0_given=0, cap_rtol=0.0)
    o.update({k: v for k, v in over.items() if v is not None})
    return _lib.bc_solve_opts(**o)


def mesh_check(verts: np.ndarray, tris: np.ndarray):
    """Host validation of a closed conforming triangulation.  Returns
    (status, bad_index)."""
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    bad = C.c_int64(-1)
    st = lib().bc_mesh_check(v.ctypes.data_as(C.c_void_p), v.shape[0], t.ctypes.data_as(C.c_void_p), t.shape[0],
                             C.byref(bad))
    return st, bad.value


class CapacityProblem:
    """A mesh on the GPU with everything the capacity computation needs."""

    def __init__(self, verts, tris, precision: str = "fp64", far_order: int = 4, ss_order: int = 4,
                 near_factor: Optional[float] = None, device: str = "cuda", validate: bool = True, stream=None,
                 far_low: Optional[bool] = None, ss_order_edge: int = 0, ss_order_vertex: int = 0,
                 ss_order_sliver: int = 0, sliver_ratio: float = 0.0):
        """ss_order: points per coordinate of the singular rules (coincident
        pairs, and every touching pair unless the next three say otherwise);
        ss_order_edge / ss_order_vertex: the orders of edge- and
        vertex-adjacent pairs (0: ss_order); ss_order_sliver with
        sliver_ratio: at least that order for touching pairs with an element
        whose diam^2 exceeds sliver_ratio |T| (0: off)."""
        if precision not in PRECISION:
            raise ValueError(f"precision must be one of {list(PRECISION)}")
        L = lib()
        verts = np.ascontiguousarray(verts, dtype=np.float64)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        if validate:
            st, bad = mesh_check(verts, tris)
            if st != _lib.BC_OK:
                raise _lib.BemcapError(f"bc_mesh_check (index {bad})", st)
        self.precision = precision
        self.prec = PRECISION[precision]
        self.N = int(tris.shape[0])
        self.M = int(verts.shape[0])
        self.ld = int(L.bc_matrix_ld(self.N))
        self.device = torch.device(device)
        if near_factor is None:
            near_factor = 1.5 if precision == "mixed" else 0.0
        if far_low is None:  # Radon's 7-point rule on distant blocks (8 diameters mixed, 32 FP64), 4 x 4 far rule
            far_low = far_order == 4
        self.opts = _lib.bc_assembly_opts(far_order, ss_order, self.prec, int(bool(far_low)), float(near_factor),
                                          int(ss_order_edge), int(ss_order_vertex), int(ss_order_sliver), 0,
                                          float(sliver_ratio))
        self.d_verts = torch.from_numpy(verts).to(self.device)
        self.d_tris = torch.from_numpy(tris).to(self.device)
        nb = L.bc_mesh_workspace_bytes(self.N)
        self.mesh_ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.pattern = None
        self.area = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self.prepare(stream)
        self.V: Optional[torch.Tensor] = None
        self.sigma = torch.zeros(self.N, dtype=torch.float64, device=self.device)
        self.solve_ws: Optional[torch.Tensor] = None
        self.result_buf = torch.zeros(C.sizeof(_lib.bc_result), dtype=torch.uint8, device=self.device)

    def prepare(self, stream=None):
        """Geometry tables and pair classification (bc_prepare; waits for
        the stream), then the element areas."""
        L = lib()
        info = _lib.bc_pattern_info()
        check("bc_prepare", L.bc_prepare(_ptr(self.d_verts), self.M, _ptr(self.d_tris), self.N, C.byref(self.opts),
                                         _ptr(self.mesh_ws), self.mesh_ws.numel(), C.byref(info), _stream(stream)))
        self.info = info
        self.nnz = int(info.nnz)
        self.pattern_bytes = L.bc_pattern_bytes(self.N, self.nnz, self.prec)
        if self.pattern is None or self.pattern.numel() < self.pattern_bytes:
            self.pattern = torch.empty(self.pattern_bytes, dtype=torch.uint8, device=self.device)
        check("bc_areas", L.bc_areas(_ptr(self.mesh_ws), self.N, _ptr(self.area), _stream(stream)))

    # ------------------------------------------------------------ assembly
    @property
    def matrix_dtype(self):
        return torch.float64 if self.precision == "fp64" else torch.float32

    def matrix_bytes(self) -> int:
        return int(lib().bc_matrix_bytes(self.N, self.prec))

    def allocate(self):
        """Device memory of the matrix and of the solver, allocated once;
        assemble() and solve() allocate whatever is missing themselves.
        Calling this first keeps allocation (which may release cached blocks
        and wait for the device) out of a timed assemble or solve."""
        if self.V is None:
            self.V = torch.empty((self.N, self.ld), dtype=self.matrix_dtype, device=self.device)
        self._ensure_solve_ws()

    def assemble(self, stream=None) -> torch.Tensor:
        if self.V is None:
            self.V = torch.empty((self.N, self.ld), dtype=self.matrix_dtype, device=self.device)
        L = lib()
        check("bc_assemble", L.bc_assemble(_ptr(self.d_verts), self.M, _ptr(self.d_tris), self.N, C.byref(self.opts),
                                           _ptr(self.mesh_ws), self.mesh_ws.numel(), _ptr(self.pattern),
                                           self.pattern_bytes, self.nnz, _ptr(self.V), _stream(stream)))
        return self.V

    def dense(self) -> torch.Tensor:
        """The N x N matrix (a view without the padding columns)."""
        return self.V[:, : self.N]

    def pattern_arrays(self):
        """(rowptr, col, row, kind, corr) views into the pattern buffer."""
        N, nnz = self.N, self.nnz

        def off(n):
            return (n + 255) // 256 * 256

        o_rowptr = 0
        o_col = off(4 * (N + 1))
        o_row = o_col + off(4 * nnz)
        o_kind = o_row + off(4 * nnz)
        o_corr = o_kind + off(4 * nnz)
        b = self.pattern
        rowptr = b[o_rowptr:o_rowptr + 4 * (N + 1)].view(torch.int32)
        col = b[o_col:o_col + 4 * nnz].view(torch.int32)
        row = b[o_row:o_row + 4 * nnz].view(torch.int32)
        kind = b[o_kind:o_kind + 4 * nnz].view(torch.int32)
        corr = b[o_corr:o_corr + 8 * nnz].view(torch.float64) if self.precision == "mixed" else None
        return rowptr, col, row, kind, corr

    # --------------------------------------------------------------- solve
    def _ensure_solve_ws(self):
        if self.solve_ws is None:
            nb = lib().bc_solve_workspace_bytes(self.N, self.prec)
            self.solve_ws = torch.empty(nb, dtype=torch.uint8, device=self.device)

    def solve(self, stream=None, x0: Optional[torch.Tensor] = None, sync: bool = True, **opts) -> Optional[SolveResult]:
        if self.V is None:
            raise RuntimeError("assemble() first")
        self._ensure_solve_ws()
        o = default_solve_opts(self.precision, **opts)
        if x0 is not None:
            self.sigma.copy_(x0)
            o.x0_given = 1
        L = lib()
        check("bc_solve", L.bc_solve(_ptr(self.V), self.N, self.prec, _ptr(self.pattern), self.nnz, _ptr(self.area),
                                     _ptr(self.sigma), C.byref(o), _ptr(self.solve_ws), self.solve_ws.numel(),
                                     _ptr(self.result_buf), _stream(stream)))
        if not sync:
            return None
        return self.result(stream)

    def result(self, stream=None) -> SolveResult:
        (stream or torch.cuda.current_stream()).synchronize()
        return SolveResult.from_bytes(self.result_buf.cpu().numpy().tobytes())

    def capacity_of(self, sigma: torch.Tensor, stream=None) -> float:
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        check("bc_capacity", lib().bc_capacity(_ptr(sigma), _ptr(self.area), self.N, _ptr(out), _stream(stream)))
        return float(out.item())

    # ------------------------------------------------------------------ ZZ
    def zz(self, sigma: Optional[torch.Tensor] = None, h_mode: int = 0, stream=None) -> torch.Tensor:
        sigma = self.sigma if sigma is None else sigma
        eta2 = torch.empty(self.N, dtype=torch.float64, device=self.device)
        check("bc_zz_indicators", lib().bc_zz_indicators(_ptr(self.d_tris), self.N, _ptr(self.mesh_ws),
                                                         _ptr(self.pattern), self.nnz, _ptr(sigma), h_mode,
                                                         _ptr(eta2), _stream(stream)))
        return eta2

    # ------------------------------------------------- residual estimator
    def residual(self, sigma: Optional[torch.Tensor] = None, moments: bool = False, stream=None):
        """Weighted-residual indicators mu(T)^2 (Appendix A, eq.
        "residual:indicator"; bc_residual_indicators) of the density sigma
        (default: the last solution), in FP64.  With moments=True also
        returns the first moments <V sigma, lambda_k>_T (N x 3)."""
        sigma = self.sigma if sigma is None else sigma
        L = lib()
        nb = L.bc_residual_workspace_bytes(self.N, self.nnz)
        ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        mu2 = torch.empty(self.N, dtype=torch.float64, device=self.device)
        mom = torch.empty((self.N, 3), dtype=torch.float64, device=self.device) if moments else None
        check("bc_residual_indicators", L.bc_residual_indicators(
            _ptr(self.d_verts), _ptr(self.d_tris), self.N, C.byref(self.opts), _ptr(self.mesh_ws),
            _ptr(self.pattern), self.nnz, _ptr(sigma), _ptr(mu2), _ptr(mom), _ptr(ws), nb, _stream(stream)))
        return (mu2, mom) if moments else mu2

    def release_matrix(self):
        self.V = None
        self.solve_ws = None


def matvec(problem: "CapacityProblem", x: torch.Tensor, stream=None) -> torch.Tensor:
    """y = V x with the problem's assembled matrix (bc_matvec): the symmetric
    product of the solver as a standalone call.  x has N entries, or shape
    (k, N) for k vectors that share one pass over V (k = 1 or 3 with FP64
    vectors).  x in the matrix precision, or FP64 with a mixed problem's
    FP32 matrix (FP64 sums; the sparse FP64 correction is not applied)."""
    L = lib()
    nr = 1 if x.dim() == 1 else int(x.shape[0])
    prec = problem.prec
    if problem.precision == "mixed" and x.dtype == torch.float64:
        prec = _lib.BC_F32_F64
    elif x.dtype != problem.matrix_dtype:
        raise ValueError("x: the matrix precision, or FP64 with a mixed problem")
    if x.shape[-1] != problem.N or not x.is_contiguous():
        raise ValueError("x: contiguous, N entries per vector")
    nb = L.bc_matvec_workspace_bytes(problem.N, prec, nr)
    if nb == 0:
        raise ValueError(f"bc_matvec: {nr} vectors not supported in this precision")
    ws = torch.empty(nb, dtype=torch.uint8, device=problem.device)
    y = torch.empty_like(x)
    check("bc_matvec", L.bc_matvec(_ptr(problem.V), problem.N, prec, nr, _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                   _stream(stream)))
    return y


@dataclasses.dataclass
class DualResult:
    cap: float
    rel_residual: float
    iters: int
    status: int
    energy_step: float = 0.0  # ||x_k - x_{k-1}||_V of the last step (inexact stop)
    eta: float = 0.0  # ZZ estimator of the returned iterate (inexact stop)
    stop: int = 0  # 1 residual, 2 inexact-solve criterion, 3 invariant subspace, 0 step limit

    @property
    def ok(self) -> bool:
        return self.status == _lib.BC_OK


class DualProblem:
    """The paper's dual-mesh Galerkin system (Algorithm 1, step (i)): V on
    the barycentric refinement (FP64, or FP32 with FP64 corrections of the
    touching and near entries for precision="mixed", assembled by the
    library like any mesh), the unknowns on the dual cells of the vertices,
    solved by GMRES with the hypersingular operator as preconditioner
    (Section 2.6); vectors and sums are FP64 in both precisions."""

    def __init__(self, verts, tris, far_order: int = 4, ss_order: int = 4, restart: int = 200, device: str = "cuda",
                 stream=None, precision: str = "fp64"):
        import synth

        L = lib()
        verts = np.ascontiguousarray(verts, dtype=np.float64)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        st, bad = mesh_check(verts, tris)
        if st != _lib.BC_OK:
            raise _lib.BemcapError(f"bc_mesh_check (index {bad})", st)
        self.N, self.M = int(tris.shape[0]), int(verts.shape[0])
        self.restart = int(restart)
        self.device = torch.device(device)
        bary, _, _ = synth.barycentric(verts, tris)
        # V_bary in FP64, or FP32 with the FP64 correction of touching and near entries
        self.precision = precision
        self.bary = CapacityProblem(bary.verts, bary.tris, precision, far_order, ss_order, device=device,
                                    validate=False, stream=stream)
        iptr, itri, icor = synth.vertex_incidence(tris, self.M)
        self.d_verts = torch.from_numpy(verts).to(self.device)
        self.d_tris = torch.from_numpy(tris).to(self.device)
        self.d_iptr = torch.from_numpy(iptr).to(self.device)
        self.d_itri = torch.from_numpy(itri).to(self.device)
        self.d_icor = torch.from_numpy(icor).to(self.device)
        nb = L.bc_dual_workspace_bytes(self.N, self.M, self.restart)
        if nb == 0:
            raise ValueError("mesh too large or too small for the dual system")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check("bc_dual_setup", L.bc_dual_setup(_ptr(self.d_verts), self.M, _ptr(self.d_tris), self.N,
                                               _ptr(self.d_iptr), _ptr(self.d_itri), _ptr(self.ws), self.ws.numel(),
                                               self.restart, _stream(stream)))
        self.x = torch.zeros(self.M, dtype=torch.float64, device=self.device)

    def allocate(self):
        """Device memory of V_bary, allocated once (assemble() allocates it
        itself when missing); keeps allocation out of a timed assembly."""
        b = self.bary
        if b.V is None:
            b.V = torch.empty((b.N, b.ld), dtype=b.matrix_dtype, device=b.device)

    def assemble(self, stream=None) -> torch.Tensor:
        """V_bary (6N x 6N, FP64)."""
        return self.bary.assemble(stream)

    def solve(self, rtol: float = 1e-12, max_iter: Optional[int] = None, jacobi_sweeps: int = 2,
              inexact_lambda: float = 0.0, h_mode: int = 1, stream=None) -> DualResult:
        """GMRES to the relative residual rtol; with inexact_lambda > 0 also
        stops once the energy norm of the last update is at most
        inexact_lambda times the ZZ estimator (mesh size h_mode) of the
        current iterate (Section 2.5, Remark (i))."""
        if self.bary.V is None:
            raise RuntimeError("assemble() first")
        o = _lib.bc_dual_opts(rtol, inexact_lambda, int(max_iter or self.restart), self.restart, jacobi_sweeps, h_mode)
        r = _lib.bc_dual_result()
        check("bc_dual_solve", lib().bc_dual_solve(_ptr(self.bary.V), self.bary.prec, _ptr(self.bary.pattern),
                                                   self.bary.nnz, _ptr(self.d_tris), self.N, self.M,
                                                   _ptr(self.d_iptr), _ptr(self.d_itri), _ptr(self.d_icor),
                                                   _ptr(self.ws), self.ws.numel(), C.byref(o), _ptr(self.x),
                                                   C.byref(r), _stream(stream)))
        return DualResult(r.cap, r.rel_residual, r.iters, r.status, r.energy_step, r.eta, r.stop)

    def zz(self, h_mode: int = 0, stream=None) -> torch.Tensor:
        eta2 = torch.empty(self.N, dtype=torch.float64, device=self.device)
        check("bc_dual_zz", lib().bc_dual_zz(_ptr(self.ws), self.ws.numel(), _ptr(self.d_tris), self.N, self.M,
                                             self.restart, _ptr(self.x), h_mode, _ptr(eta2), _stream(stream)))
        return eta2


def solve_batched(problems, precision: str, iter_budget: int = 0, start=None, budgets=None, stream=None,
                  **opts):
    """One persistent launch over several assembled problems (same precision).
    start[k] = 1 (re)initialises problem k, 0 resumes it; budgets[k] > 0
    bounds problem k's matrix products in this launch.  Asynchronous: read
    each problem's result with problem.result() after the stream syncs."""
    L = lib()
    n = len(problems)
    arr = (_lib.bc_system * n)()
    for k, p in enumerate(problems):
        p._ensure_solve_ws()
        arr[k] = _lib.bc_system(p.V.data_ptr(), p.pattern.data_ptr(), p.area.data_ptr(), p.sigma.data_ptr(),
                                p.solve_ws.data_ptr(), p.result_buf.data_ptr(), p.N, p.nnz, PRECISION[precision],
                                1 if start is None else int(start[k]), 0 if budgets is None else int(budgets[k]), 0)
    o = default_solve_opts(precision, **opts)
    nb = L.bc_batch_scratch_bytes(n)
    scratch = torch.empty(nb, dtype=torch.uint8, device=problems[0].device)
    check("bc_solve_batched", L.bc_solve_batched(n, arr, C.byref(o), iter_budget, _ptr(scratch), nb,
                                                 _stream(stream)))
    return scratch  # keep alive until the launch completes


def capacity(verts, tris, precision: str = "fp64", return_problem: bool = False, **kw):
    """Assemble, solve and return the capacity of one polyhedron."""
    solve_kw = {k: kw.pop(k) for k in list(kw) if k in ("rtol", "inner_rtol", "max_iter", "max_outer", "jacobi")}
    p = CapacityProblem(verts, tris, precision=precision, **kw)
    p.assemble()
    r = p.solve(**solve_kw)
    return (r, p) if return_problem else r
