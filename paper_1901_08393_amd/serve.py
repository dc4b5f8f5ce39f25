"""Capacity-solve server with continuous batching.

Requests (a polyhedron already meshed on the host) arrive over time.  The
server keeps every admitted mesh, its dense matrix and its Krylov state
resident in HBM and works on many of them at once:

* admission: FIFO, while the sum of the admitted requests' footprints
  (N x ld matrix plus geometry, pattern and solver workspaces) stays within
  the memory budget (free HBM, at most 288 GB); a request that can never fit
  is rejected.  Several requests are admitted per loop pass (up to
  `admit_ms` of host time);
* set-up and assembly: geometry and classification (bc_prepare, which waits
  for its own stream) on a set-up stream, then the dense matrix on an
  assembly stream, overlapping the solves;
* solving: assembled systems join the next cooperative solver launch on the
  solve stream.  A launch ("chunk") packs systems up to the number of
  co-resident workgroups, in the order of the scheduling policy (round
  robin by default, or the least remaining work first); each system gets a bound on its matrix
  products sized so that a chunk streams about `chunk_ms` of HBM traffic.
  Two chunks are kept in flight, so that the GPU does not wait for the host
  between them.  As chunks complete, finished systems retire (their memory
  is released and their Cap is reported), unfinished ones resume bitwise
  where they stopped, and newly assembled ones start.  A system's arithmetic
  depends only on its own N, so every result is the same alone and in the
  mix.

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
    __slots__ = ("rec", "prob", "event", "foot", "started", "G", "finished", "products")

    def __init__(self, rec, prob, event, foot, G):
        self.rec, self.prob, self.event, self.foot, self.G = rec, prob, event, foot, G
        self.started = False
        self.finished = False
        self.products = 0  # matrix products granted so far (budgets of launched chunks)


class CapacityServer:
    """policy: order in which ready systems are packed into a chunk.
    "rr" serves them round robin (a system that took part in a chunk goes to
    the back); "srpt" takes the least remaining work first, estimated as
    N ld (expected products - products granted so far).  pipeline: chunks
    kept in flight on the solve stream (2: the next chunk is queued while
    the current one runs, so the host's retire-and-launch turnaround does not
    leave the GPU idle; a system that finished in the running chunk is a
    no-op in the queued one).  admit_ms: host time one loop pass may spend
    admitting requests (each admission runs bc_prepare, which waits for its
    own stream)."""

    def __init__(self, precision: str = "mixed", budget_bytes: Optional[float] = None, chunk_ms: float = 2.0,
                 stream_gbs: float = 5000.0, device: str = "cuda", solve_opts: Optional[dict] = None,
                 keep_sigma: bool = False, policy: str = "rr", pipeline: int = 2, admit_ms: float = 1.0,
                 expected_products: int = 60):
        if policy not in ("rr", "srpt"):
            raise ValueError("policy: 'rr' or 'srpt'")
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
        self.prep_stream = torch.cuda.Stream(self.device)
        self.asm_stream = torch.cuda.Stream(self.device)
        self.solve_stream = torch.cuda.Stream(self.device)
        self.solve_opts = solve_opts or {}
        self.keep_sigma = keep_sigma
        self.policy = policy
        self.pipeline = max(1, int(pipeline))
        self.admit_ms = admit_ms
        self.expected_products = expected_products
        # pinned host slots for the results of the chunks in flight (one
        # system per workgroup at most)
        rs = ctypes_sizeof_result()
        self._pinned = [torch.empty((self.capacity_wg, rs), dtype=torch.uint8, pin_memory=True)
                        for _ in range(self.pipeline)]

    # ------------------------------------------------------------- sizes
    def footprint(self, N: int) -> int:
        L = lib()
        return int(L.bc_matrix_bytes(N, self.prec) + L.bc_mesh_workspace_bytes(N)
                   + L.bc_solve_workspace_bytes(N, self.prec) + 2048 * N)

    def product_budget(self, N: int) -> int:
        elem = 8 if self.prec == 0 else 4
        per = elem * N * lib().bc_matrix_ld(N)
        return max(2, int(self.chunk_ms * 1e-3 * self.stream_gbs * 1e9 / per))

    def _remaining(self, lv: "_Live") -> float:
        return float(lv.rec.N) * float(lv.rec.N) * max(1, self.expected_products - lv.products)

    def _admit(self, rec: "Record", mesh, foot: int, G: int, t0: float) -> "_Live":
        rec.admitted = time.perf_counter() - t0
        # bc_prepare waits for its stream: its own stream, so that it does not
        # wait for queued assemblies; the assembly follows on the assembly
        # stream (prepare has completed when the constructor returns)
        with torch.cuda.stream(self.prep_stream):
            prob = CapacityProblem(mesh.verts, mesh.tris, self.precision, device=str(self.device),
                                   stream=self.prep_stream)
        for tns in (prob.d_verts, prob.d_tris, prob.mesh_ws, prob.pattern, prob.area, prob.sigma, prob.result_buf):
            tns.record_stream(self.asm_stream)
        with torch.cuda.stream(self.asm_stream):
            prob.assemble(stream=self.asm_stream)
            prob._ensure_solve_ws()
            ev = torch.cuda.Event()
            ev.record(self.asm_stream)
        return _Live(rec, prob, ev, foot, G)

    # --------------------------------------------------------------- run
    def run(self, requests, meshes, realtime: bool = True) -> List[Record]:
        """Serve `requests` (objects with rid, arrival, kind) whose meshes
        are meshes[k] (objects with verts, tris).  realtime=False treats
        every request as arrived at t = 0."""
        L = lib()
        rsize = ctypes_sizeof_result()
        order = sorted(range(len(requests)), key=lambda k: (requests[k].arrival if realtime else 0.0, k))
        recs = [Record(requests[k].rid, int(meshes[k].tris.shape[0]), requests[k].kind,
                       requests[k].arrival if realtime else 0.0) for k in range(len(requests))]
        waiting = collections.deque()
        assembling: List[_Live] = []
        ready: List[_Live] = []  # assembled or running, in service order
        inflight = collections.deque()  # (batch, event, scratch, slot)
        slot_free = list(range(self.pipeline))
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
            # admission: FIFO, as long as memory allows and this pass's time lasts
            ta = time.perf_counter()
            while waiting and (time.perf_counter() - ta) * 1e3 < self.admit_ms:
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
                    assembling.append(self._admit(recs[k], meshes[k], foot, G, t0))
                    progressed = True
                else:
                    break
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
            # retire finished chunks, oldest first
            while inflight and inflight[0][1].query():
                batch, _ev, _keep, slot = inflight.popleft()
                res = self._pinned[slot][: len(batch)].numpy()
                tnow = time.perf_counter() - t0
                for lv, row in zip(batch, res):
                    if lv.finished:
                        continue  # finished in an earlier chunk (a no-op in this one)
                    r = _lib.bc_result.from_buffer_copy(row.tobytes())
                    lv.rec.chunks += 1
                    if r.status != _lib.BC_RUNNING:
                        lv.finished = True
                        lv.rec.done = tnow
                        lv.rec.cap, lv.rec.iters, lv.rec.outer = r.cap, r.iters, r.outer
                        lv.rec.status, lv.rec.rel_residual = r.status, r.rel_residual
                        if self.keep_sigma:
                            with torch.cuda.stream(self.solve_stream):
                                lv.rec.sigma = lv.prob.sigma.cpu().numpy().copy()
                        ready.remove(lv)
                        used -= lv.foot
                        n_done += 1
                slot_free.append(slot)
                progressed = True
            # launch chunks until `pipeline` are in flight
            while len(inflight) < self.pipeline and ready and slot_free:
                cand = ready if self.policy == "rr" else sorted(ready, key=self._remaining)
                batch, wg = [], 0
                for lv in cand:
                    if wg + lv.G <= self.capacity_wg:
                        batch.append(lv)
                        wg += lv.G
                start = [0 if lv.started else 1 for lv in batch]
                budgets = [self.product_budget(lv.rec.N) for lv in batch]
                tnow = time.perf_counter() - t0
                for lv, bdg in zip(batch, budgets):
                    lv.products += bdg
                    if not lv.started:
                        lv.started = True
                        lv.rec.started = tnow
                slot = slot_free.pop()
                with torch.cuda.stream(self.solve_stream):
                    keep = solve_batched([lv.prob for lv in batch], self.precision, start=start, budgets=budgets,
                                         stream=self.solve_stream, **self.solve_opts)
                    host = self._pinned[slot]
                    for q, lv in enumerate(batch):
                        host[q].copy_(lv.prob.result_buf, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(self.solve_stream)
                inflight.append((batch, ev, keep, slot))
                progressed = True
                if self.policy == "rr":
                    for lv in batch:  # the queued chunk's systems yield to the others for the next one
                        ready.remove(lv)
                        ready.append(lv)
            if not progressed:
                if nxt < len(order) and not waiting and not assembling and not ready and not inflight:
                    wait = recs[order[nxt]].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                else:
                    time.sleep(5e-5)
        torch.cuda.synchronize(self.device)
        assert rsize == self._pinned[0].shape[1]
        return recs


def ctypes_sizeof_result() -> int:
    import ctypes

    return ctypes.sizeof(_lib.bc_result)


def summarize(recs: List[Record]) -> dict:
    """Rate, latency percentiles, and the latency split into queueing
    (arrival to admission), set-up and assembly (admission to assembled),
    waiting for the first chunk and solving (first chunk to Cap on the
    host), each as p50 / p99 over the requests; and the latency p99 of the
    smallest and the largest half of the requests by N."""
    import numpy as np

    ok = [r for r in recs if r.status == _lib.BC_OK]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done for r in recs) - min(r.arrival for r in recs)

    def pp(x):
        x = np.asarray(x) * 1e3
        return {"p50": round(float(np.percentile(x, 50)), 3), "p99": round(float(np.percentile(x, 99)), 3)} \
            if len(x) else {}

    out = {
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
    if ok:
        out["breakdown_ms"] = {
            "queue": pp([r.admitted - r.arrival for r in ok]),
            "setup_assembly": pp([r.assembled - r.admitted for r in ok]),
            "wait_first_chunk": pp([r.started - r.assembled for r in ok]),
            "solve": pp([r.done - r.started for r in ok]),
        }
        Ns = np.array([r.N for r in ok])
        med = np.median(Ns)
        small = lat[Ns <= med]
        large = lat[Ns > med]
        out["p99_ms_by_size"] = {"N<=median": float(np.percentile(small, 99)) if len(small) else None,
                                 "N>median": float(np.percentile(large, 99)) if len(large) else None,
                                 "median_N": float(med)}
    return out
