"""Capacity-solve server with continuous batching.

Requests (a polyhedron already meshed on the host) arrive over time.  The
server keeps every admitted mesh, its dense matrix and its Krylov state
resident in HBM and works on many of them at once:

* admission: FIFO, while the sum of the admitted requests' footprints
  (N x ld matrix plus geometry, pattern and solver workspaces) stays within
  the memory budget (free HBM, at most 288 GB); a request that can never fit
  is rejected;
* assembly: geometry, classification and the dense matrix of each admitted
  request are built on an assembly stream, overlapping the solves;
* solving: assembled systems join the next cooperative solver launch on the
  solve stream.  A launch ("chunk") packs systems up to the number of
  co-resident workgroups; each system gets a bound on its matrix products
  sized so that a chunk streams about `chunk_ms` of HBM traffic.  Between
  chunks finished systems retire (their memory is released and their Cap is
  reported), unfinished ones resume bitwise where they stopped, and newly
  assembled ones start.  A system's arithmetic depends only on its own N, so
  every result is the same alone and in the mix.

Latency of a request = from its arrival (mesh already built) to its Cap
being available on the host.
"""

from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import List, Optional

import torch

from . import _lib
from .api import CapacityProblem, solve_batched
from ._lib import lib


@dataclasses.dataclass
class Record:
    rid: int
    N: int
    kind: str = ""
    arrival: float = 0.0
    admitted: float = math.nan
    assembled: float = math.nan
    started: float = math.nan
    done: float = math.nan
    cap: float = math.nan
    iters: int = 0
    outer: int = 0
    status: int = _lib.BC_RUNNING
    rel_residual: float = math.nan
    chunks: int = 0
    sigma: Optional[object] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Live:
    __slots__ = ("rec", "prob", "event", "foot", "started", "G")

    def __init__(self, rec, prob, event, foot, G):
        self.rec, self.prob, self.event, self.foot, self.G = rec, prob, event, foot, G
        self.started = False


class CapacityServer:
    def __init__(self, precision: str = "mixed", budget_bytes: Optional[float] = None, chunk_ms: float = 2.0,
                 stream_gbs: float = 5000.0, device: str = "cuda", solve_opts: Optional[dict] = None,
                 keep_sigma: bool = False):
        self.precision = precision
        self.prec = 0 if precision == "fp64" else 1
        self.device = torch.device(device)
        free, _total = torch.cuda.mem_get_info(self.device)
        cap = 288e9
        self.budget = float(min(budget_bytes if budget_bytes is not None else 0.9 * free, cap))
        self.capacity_wg = int(lib().bc_solve_capacity(self.prec))
        if self.capacity_wg <= 0:
            raise RuntimeError("bc_solve_capacity: no co-resident solver workgroups")
        self.chunk_ms = chunk_ms
        self.stream_gbs = stream_gbs
        self.asm_stream = torch.cuda.Stream(self.device)
        self.solve_stream = torch.cuda.Stream(self.device)
        self.solve_opts = solve_opts or {}
        self.keep_sigma = keep_sigma

    # ------------------------------------------------------------- sizes
    def footprint(self, N: int) -> int:
        L = lib()
        return int(L.bc_matrix_bytes(N, self.prec) + L.bc_mesh_workspace_bytes(N)
                   + L.bc_solve_workspace_bytes(N, self.prec) + 2048 * N)

    def product_budget(self, N: int) -> int:
        elem = 8 if self.prec == 0 else 4
        per = elem * N * lib().bc_matrix_ld(N)
        return max(2, int(self.chunk_ms * 1e-3 * self.stream_gbs * 1e9 / per))

    # --------------------------------------------------------------- run
    def run(self, requests, meshes, realtime: bool = True) -> List[Record]:
        """Serve `requests` (objects with rid, arrival, kind) whose meshes
        are meshes[k] (objects with verts, tris).  realtime=False treats
        every request as arrived at t = 0."""
        L = lib()
        order = sorted(range(len(requests)), key=lambda k: (requests[k].arrival if realtime else 0.0, k))
        recs = [Record(requests[k].rid, int(meshes[k].tris.shape[0]), requests[k].kind,
                       requests[k].arrival if realtime else 0.0) for k in range(len(requests))]
        waiting = collections.deque()
        assembling: List[_Live] = []
        ready: List[_Live] = []  # assembled or running, in service order
        inflight = None
        used = 0
        nxt = 0
        n_done = 0
        t0 = time.perf_counter()
        while n_done < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(order) and recs[order[nxt]].arrival <= now:
                waiting.append(order[nxt])
                nxt += 1
            progressed = False
            # admission (one per pass keeps the loop responsive)
            if waiting:
                k = waiting[0]
                foot = self.footprint(recs[k].N)
                G = int(L.bc_solve_workgroups(recs[k].N))
                if foot > self.budget or G > self.capacity_wg:
                    waiting.popleft()
                    recs[k].status = _lib.BC_ENOMEM
                    recs[k].done = time.perf_counter() - t0
                    n_done += 1
                    progressed = True
                elif used + foot <= self.budget:
                    waiting.popleft()
                    used += foot
                    recs[k].admitted = time.perf_counter() - t0
                    with torch.cuda.stream(self.asm_stream):
                        prob = CapacityProblem(meshes[k].verts, meshes[k].tris, self.precision,
                                               device=str(self.device), stream=self.asm_stream)
                        prob.assemble(stream=self.asm_stream)
                        prob._ensure_solve_ws()
                        ev = torch.cuda.Event()
                        ev.record(self.asm_stream)
                    assembling.append(_Live(recs[k], prob, ev, foot, G))
                    progressed = True
            # assembly completion
            still = []
            for lv in assembling:
                if lv.event.query():
                    lv.rec.assembled = time.perf_counter() - t0
                    for tns in (lv.prob.V, lv.prob.pattern, lv.prob.area, lv.prob.sigma, lv.prob.solve_ws,
                                lv.prob.result_buf):
                        tns.record_stream(self.solve_stream)
                    ready.append(lv)
                    progressed = True
                else:
                    still.append(lv)
            assembling = still
            # retire a finished chunk
            if inflight is not None and inflight[1].query():
                batch, _ev, _keep = inflight
                with torch.cuda.stream(self.solve_stream):
                    res = torch.stack([lv.prob.result_buf for lv in batch]).cpu().numpy()
                tnow = time.perf_counter() - t0
                for lv, row in zip(batch, res):
                    r = _lib.bc_result.from_buffer_copy(row.tobytes())
                    lv.rec.chunks += 1
                    if r.status != _lib.BC_RUNNING:
                        lv.rec.done = tnow
                        lv.rec.cap, lv.rec.iters, lv.rec.outer = r.cap, r.iters, r.outer
                        lv.rec.status, lv.rec.rel_residual = r.status, r.rel_residual
                        if self.keep_sigma:
                            with torch.cuda.stream(self.solve_stream):
                                lv.rec.sigma = lv.prob.sigma.cpu().numpy().copy()
                        ready.remove(lv)
                        used -= lv.foot
                        n_done += 1
                    else:
                        # served systems go to the back of the queue
                        ready.remove(lv)
                        ready.append(lv)
                inflight = None
                progressed = True
            # launch the next chunk
            if inflight is None and ready:
                batch, wg = [], 0
                for lv in ready:
                    if wg + lv.G <= self.capacity_wg:
                        batch.append(lv)
                        wg += lv.G
                start = [0 if lv.started else 1 for lv in batch]
                budgets = [self.product_budget(lv.rec.N) for lv in batch]
                tnow = time.perf_counter() - t0
                for lv in batch:
                    if not lv.started:
                        lv.started = True
                        lv.rec.started = tnow
                with torch.cuda.stream(self.solve_stream):
                    keep = solve_batched([lv.prob for lv in batch], self.precision, start=start, budgets=budgets,
                                         stream=self.solve_stream, **self.solve_opts)
                    ev = torch.cuda.Event()
                    ev.record(self.solve_stream)
                inflight = (batch, ev, keep)
                progressed = True
            if not progressed:
                if nxt < len(order) and not waiting and not assembling and not ready and inflight is None:
                    wait = recs[order[nxt]].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                else:
                    time.sleep(5e-5)
        torch.cuda.synchronize(self.device)
        return recs


def summarize(recs: List[Record]) -> dict:
    import numpy as np

    ok = [r for r in recs if r.status == _lib.BC_OK]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done for r in recs) - min(r.arrival for r in recs)
    return {
        "requests": len(recs),
        "ok": len(ok),
        "rejected": sum(1 for r in recs if r.status == _lib.BC_ENOMEM),
        "failed": sum(1 for r in recs if r.status not in (_lib.BC_OK, _lib.BC_ENOMEM)),
        "solves_per_s": len(ok) / span if span > 0 else float("nan"),
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else float("nan"),
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else float("nan"),
        "makespan_s": span,
        "mean_iters": float(np.mean([r.iters for r in ok])) if ok else float("nan"),
    }
