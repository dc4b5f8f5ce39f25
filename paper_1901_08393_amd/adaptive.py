"""Adaptive loop solve -> estimate -> mark -> refine (Algorithm 1, steps
(i)-(iv)), on the primal P0 discretisation (adaptive_capacity) and on the
dual mesh as the algorithm states it (adaptive_dual).

(i)   solve: dense assembly and persistent Krylov solve on the GPU, warm
      started from the previous mesh's solution (the P0 spaces of NVB meshes
      are nested, so every son inherits its parent's value);
(ii)  estimate: ZZ-type indicators eta(T)^2 on the GPU (eq. "zz:T"), or
      on the primal path the weighted-residual indicators mu(T)^2 of
      Appendix A (eq. "residual:indicator"), which drive the standard
      adaptive algorithm stated there;
(iii) mark: Doerfler marking (eq. "doerfler") on the host;
(iv)  refine: newest-vertex bisection of the marked elements with closure.

By the corollary in Appendix A the discrete capacities of nested P0 spaces
increase monotonically; the loops report them per step.
"""

from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np
import torch

import synth

from .api import CapacityProblem


def doerfler(eta2: np.ndarray, theta: float) -> np.ndarray:
    """Smallest set M with theta * sum eta^2 <= sum_{M} eta^2, chosen greedily
    by decreasing eta^2 with ties to the lower index (eq. "doerfler" with
    C_mark = 1).  Returns sorted element indices."""
    eta2 = np.asarray(eta2, dtype=np.float64)
    if eta2.size == 0:
        return np.zeros(0, dtype=np.int64)
    order = np.lexsort((np.arange(eta2.size), -eta2))
    total = math.fsum(eta2.tolist())  # exactly rounded total
    cum = np.cumsum(eta2[order])  # sequential, in marking order
    k = int(np.searchsorted(cum, theta * total, side="left")) + 1
    return np.sort(order[: min(k, eta2.size)])


@dataclasses.dataclass
class Step:
    level: int
    N: int
    cap: float
    eta2: float
    iters: int
    outer: int
    n_marked: int
    t_assemble_ms: float
    t_solve_ms: float
    t_zz_ms: float
    t_refine_ms: float
    verts: Optional[np.ndarray] = None
    tris: Optional[np.ndarray] = None
    sigma: Optional[np.ndarray] = None
    eta2_elem: Optional[np.ndarray] = None
    marked: Optional[np.ndarray] = None


def adaptive_capacity(verts, tris, steps: int = 5, theta: float = 0.5, precision: str = "fp64",
                      h_mode: int = 0, warm_start: bool = True, keep: bool = False, refine: str = "bisec1",
                      max_elements: Optional[int] = None, far_order: int = 4, ss_order: int = 4,
                      estimator: str = "zz", ss_order_edge: int = 0, ss_order_vertex: int = 0,
                      **solve_opts) -> List[Step]:
    """Run `steps` refinements (steps + 1 solves), or stop before the first
    mesh with more than `max_elements` triangles.  `tris` must be in NVB form
    (reference edge first); use synth.init_reference_edges on a new mesh.
    refine "bisec1" bisects every marked element once and closes the mesh
    (the coarsest conforming refinement of step (iv)); "bisec3" splits
    marked elements into four.  estimator "zz" marks by the ZZ-type
    indicators (h_mode as in bc_zz_indicators); "residual" by the
    weighted-residual indicators mu(T)^2 (Appendix A's algorithm; always
    with diam(T)), reported in the eta2 fields.  ss_order_edge /
    ss_order_vertex: singular-rule orders of edge- and vertex-adjacent pairs
    (0: ss_order)."""
    if estimator not in ("zz", "residual"):
        raise ValueError("estimator: 'zz' or 'residual'")
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int32)
    x0 = None
    out: List[Step] = []
    for level in range(steps + 1):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        prob = CapacityProblem(verts, tris, precision, far_order, ss_order, ss_order_edge=ss_order_edge,
                               ss_order_vertex=ss_order_vertex)
        prob.allocate()  # allocation (tens of GB at large N) is not assembly time
        ev[0].record()
        prob.assemble()
        ev[1].record()
        res = prob.solve(x0=x0 if warm_start else None, sync=False, **solve_opts)
        ev[2].record()
        eta2_d = prob.zz(h_mode=h_mode) if estimator == "zz" else prob.residual()
        ev[3].record()
        res = prob.result()
        if not res.ok:
            raise RuntimeError(f"solve failed at level {level}: {res}")
        eta2 = eta2_d.cpu().numpy()
        sigma = prob.sigma.cpu().numpy()
        t0 = time.perf_counter()
        last = level == steps
        marked = np.zeros(0, dtype=np.int64) if last else doerfler(eta2, theta)
        step = Step(level, int(tris.shape[0]), res.cap, float(eta2.sum()), res.iters, res.outer, int(marked.size),
                    ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]), 0.0)
        if keep:
            step.verts, step.tris, step.sigma, step.eta2_elem, step.marked = verts, tris, sigma, eta2, marked
        device = prob.device
        del prob, eta2_d
        if not last:
            nv, nt, parent = synth.refine_nvb(verts, tris, marked, refine)
            if max_elements is not None and nt.shape[0] > max_elements:
                last = True
            else:
                verts, tris = nv, nt
                x0 = torch.from_numpy(sigma[parent]).to(device)
        step.t_refine_ms = (time.perf_counter() - t0) * 1e3
        out.append(step)
        if last:
            break
    return out


def adaptive_dual(verts, tris, steps: int = 5, theta: float = 0.5, h_mode: int = 1, rtol: float = 1e-10,
                  max_elements: Optional[int] = None, keep: bool = False, far_order: int = 4, ss_order: int = 4,
                  jacobi_sweeps: int = 2, restart: int = 200, refine: str = "bisec1",
                  inexact_lambda: float = 0.0, precision: str = "fp64") -> List[Step]:
    """Algorithm 1 as stated: (i) the Galerkin solution on the dual mesh,
    computed from V on the barycentric refinement by GMRES with the
    hypersingular operator as preconditioner (Section 2.6); (ii) the ZZ
    indicators of the dual solution (eq. "zz:T"); (iii) Doerfler marking;
    (iv) NVB.  h_mode 1 weights the indicators with |T|^(1/2), as the
    implementation in Appendix B does (0: diam(T)^(1/2), as eq. "zz:T" is
    written).  Stops after `steps` refinements, or before the first mesh
    with more than `max_elements` triangles.  `iters` of each step is the
    number of GMRES steps; the dual unknowns are not carried over between
    meshes (each solve starts from zero).  refine as in adaptive_capacity.
    inexact_lambda > 0 couples the solver to the estimator (Section 2.5,
    Remark (i)): GMRES also stops once the energy norm of its last update is
    at most inexact_lambda times the estimator of the current iterate.
    precision "mixed" stores V_bary in FP32 with FP64 corrections of the
    touching and near entries (half the memory, about twice as fast)."""
    from .api import DualProblem

    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int32)
    out: List[Step] = []
    for level in range(steps + 1):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        prob = DualProblem(verts, tris, far_order=far_order, ss_order=ss_order, restart=restart, precision=precision)
        prob.allocate()  # allocation is not assembly time
        ev[0].record()
        prob.assemble()
        ev[1].record()
        res = prob.solve(rtol=rtol, jacobi_sweeps=jacobi_sweeps, inexact_lambda=inexact_lambda, h_mode=h_mode)
        ev[2].record()
        eta2_d = prob.zz(h_mode=h_mode)
        ev[3].record()
        if not res.ok:
            raise RuntimeError(f"dual solve failed at level {level}: {res}")
        eta2 = eta2_d.cpu().numpy()
        t0 = time.perf_counter()
        last = level == steps
        marked = np.zeros(0, dtype=np.int64)
        if not last:
            marked = doerfler(eta2, theta)
        step = Step(level, int(tris.shape[0]), res.cap, float(eta2.sum()), res.iters, 0, int(marked.size),
                    ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]), 0.0)
        if keep:
            step.verts, step.tris, step.eta2_elem, step.marked = verts, tris, eta2, marked
            step.sigma = prob.x.cpu().numpy()
        del prob
        if not last:
            nv, nt, _ = synth.refine_nvb(verts, tris, marked, refine)
            if max_elements is not None and nt.shape[0] > max_elements:
                last = True
            else:
                verts, tris = nv, nt
        step.t_refine_ms = (time.perf_counter() - t0) * 1e3
        out.append(step)
        if last:
            break
    return out
