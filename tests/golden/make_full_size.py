"""Writes tests/golden/full_size.json: FP64 oracle results of the full-size
workloads, for the GPU tests that check the benchmark configurations.

Calls only ``oracle`` (the CPU FP64 reference) and ``synth`` (the seeded mesh
generators); nothing here touches the GPU library.  Run on the CPU:

    python tests/golden/make_full_size.py [--only sphere_L5|voxel_60k]

Workloads (each recorded with a SHA-256 of its mesh arrays, so that a test
can tell whether ``synth`` still builds the same mesh):

* ``sphere_L5``: the sphere of radius r ~ U[0.5, 2] (numpy default_rng(2)) as
  a level-5 icosphere, N = 20480 (the headline workload);
* ``sphere_L4``: the same sphere as a level-4 icosphere, N = 5120 (the
  configuration's smaller mesh);
* ``voxel_60k``: the voxel union of 26 unit voxels in a 4^3 lattice
  (seed 4), NVB-refined uniformly and then by bisection of the largest
  elements until N >= 60000 (``synth.refine_to_size``), N = 60000.
* ``serve_voxel``, ``serve_hull``, ``serve_box``: the largest request of each
  kind in the serving stream (``synth.request_stream(512, seed=5)``: requests
  2, 151 and 307, N = 29900, 29442 and 29800 or near), at the top of the
  serving workload's size range.
* ``dual_cube``: Algorithm 1's dual system (Section 2.6) on the 12-triangle
  cube of Table 1 refined uniformly four times (N = 3072, N_bary = 18432):
  the dual capacity, the dual solution at 64 seeded vertices and the ZZ
  indicators (|T|^(1/2)) at 64 seeded elements and in total.
* ``adaptive_voxel``: configuration 3 run by the oracle (five steps of
  solve, ZZ, Doerfler with theta = 1/2 and NVB from about 2.5k to about 28k
  triangles): per step the mesh's hash, Cap, the sum of eta^2 and the number
  of marked elements.

For each: the capacity of the FP64 Galerkin solution (eq. "cap:ell"; 4 x 4
regular rule, order-4 singular rules; dense Cholesky, or for more than 2^31
matrix entries Jacobi-preconditioned CG to a relative residual of 1e-14 with
the resulting bound on the capacity's error recorded), the sum of all
entries 1^T V 1, and the row sums (V 1)_i at 64 seeded rows.  The voxel case
holds a 28.8 GB matrix and takes about an hour on 8 cores.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")


def mesh_sha(verts, tris) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(verts, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(tris, dtype=np.int32).tobytes())
    return h.hexdigest()[:16]


def sphere_L5():
    r = float(np.random.default_rng(2).uniform(0.5, 2.0))
    m = synth.icosphere(5, r)
    return m.verts, m.tris, {"recipe": "icosphere(5, r), r = default_rng(2).uniform(0.5, 2)", "r": r}


def sphere_L4():
    r = float(np.random.default_rng(2).uniform(0.5, 2.0))
    m = synth.icosphere(4, r)
    return m.verts, m.tris, {"recipe": "icosphere(4, r), r = default_rng(2).uniform(0.5, 2)", "r": r}


def voxel_60k():
    m = synth.voxel_union(4, 0.4, 4)
    t0 = synth.init_reference_edges(m.verts, m.tris)
    v, t = synth.refine_to_size(m.verts, t0, 60000)
    return v, t, {"recipe": "refine_to_size(voxel_union(4, 0.4, 4) with longest-edge references, 60000)",
                  "voxels": int(m.meta["voxels"])}


def _serving_request(rid: int):
    reqs = {q.rid: q for q in synth.request_stream(512, seed=5)}
    r = reqs[rid]
    m = r.build_mesh()
    return m.verts, m.tris, {"recipe": f"synth.request_stream(512, seed=5), request {rid}: {r.kind} {r.params}",
                             "kind": r.kind}


def serve_voxel():
    return _serving_request(2)


def serve_hull():
    return _serving_request(151)


def serve_box():
    return _serving_request(307)


WORKLOADS = {"sphere_L4": sphere_L4, "sphere_L5": sphere_L5, "voxel_60k": voxel_60k, "serve_voxel": serve_voxel, "serve_hull": serve_hull,
             "serve_box": serve_box}


def dual_cube():
    m = synth.cube12()
    v, t, _ = synth.refine_uniform(m.verts, m.tris, 4)
    return v, t, {"recipe": "refine_uniform(cube12, 4): the 12-triangle cube of Table 1 refined uniformly four times"}


DUAL_WORKLOADS = {"dual_cube": dual_cube}


def adaptive_voxel_start():
    """Configuration 3's start: the voxel union of 26 unit voxels (4^3
    lattice, seed 3), uniformly refined to about 2.5k triangles."""
    m = synth.voxel_union(4, 0.4, 3)
    v, t = m.verts, synth.init_reference_edges(m.verts, m.tris)
    while len(t) * 4 <= 2600:
        v, t, _ = synth.refine_uniform(v, t, 1)
    return v, t


def run_adaptive(name: str) -> dict:
    """Configuration 3 run by the oracle: five steps of the FP64 Galerkin
    solution, ZZ indicators (eq. "zz:T", diameter weights), Doerfler marking
    (theta = 1/2) and NVB with the marked elements split into four, then the
    last mesh's solution; per step the mesh's hash, Cap, the sum of eta^2 and
    the number of marked elements."""
    v, t = adaptive_voxel_start()
    steps = []
    t_all = time.perf_counter()
    for level in range(6):
        V = oracle.assemble(v, t, 4, 4)
        b = oracle.rhs(v, t)
        x = oracle.solve_direct(V, b, overwrite=True)
        del V
        cap = oracle.capacity(x, b)
        eta2 = oracle.zz_indicators(v, t, x, "diam")
        rec = {"level": level, "N": int(len(t)), "mesh_sha": mesh_sha(v, t), "cap": cap,
               "eta2_sum": math.fsum(eta2.tolist())}
        if level < 5:
            mk = oracle.doerfler(eta2, 0.5)
            rec["marked"] = int(len(mk))
            v, t, _ = synth.refine_nvb(v, t, mk, "bisec3")
        steps.append(rec)
        print(f"{name} level {level}: N={rec['N']} cap={cap!r} marked={rec.get('marked')}", flush=True)
    return {"recipe": "voxel_union(4, 0.4, 3), uniform NVB to ~2.5k, then 5 x (solve, ZZ diam, Doerfler 1/2, "
                      "NVB bisec3)", "steps": steps, "far_order": 4, "ss_order": 4,
            "oracle_seconds": round(time.perf_counter() - t_all, 1), "cores": os.cpu_count()}


ADAPTIVE_WORKLOADS = {"adaptive_voxel": run_adaptive}


def run_dual(name: str) -> dict:
    """Algorithm 1's dual system on the barycentric refinement (Section 2.6):
    V_bary assembled densely, the dual matrix P^T V_bary P solved by Cholesky,
    the capacity and the ZZ indicators of the dual solution."""
    verts, tris, meta = DUAL_WORKLOADS[name]()
    N = len(tris)
    t0 = time.perf_counter()
    Vb, P, bv, bt = oracle.dual.assemble_dual(verts, tris)
    t_asm = time.perf_counter() - t0
    f = oracle.dual.dual_load(verts, tris)
    t0 = time.perf_counter()
    x, _ = oracle.dual.solve_dual(Vb, P, f)
    t_solve = time.perf_counter() - t0
    del Vb
    cap = oracle.dual.capacity_dual(x, f)
    eta2 = oracle.dual.zz_dual(verts, tris, x, "area")
    M = np.asarray(verts).shape[0]
    vrows = np.sort(np.random.default_rng(7).choice(M, size=64, replace=False))
    erows = np.sort(np.random.default_rng(8).choice(N, size=64, replace=False))
    print(f"{name}: N={N} N_bary={len(bt)} cap={cap!r} assemble {t_asm:.0f} s solve {t_solve:.0f} s", flush=True)
    return dict(meta, N=N, N_bary=len(bt), M=int(M), mesh_sha=mesh_sha(verts, tris), far_order=4, ss_order=4,
                cap=cap, x_rows=vrows.tolist(), x=[float(x[i]) for i in vrows.tolist()],
                eta2_rows=erows.tolist(), eta2=[float(eta2[i]) for i in erows.tolist()],
                eta2_sum=math.fsum(eta2.tolist()), solver="cholesky",
                oracle_seconds={"assemble": round(t_asm, 1), "solve": round(t_solve, 1)}, cores=os.cpu_count())


def run(name: str) -> dict:
    verts, tris, meta = WORKLOADS[name]()
    N = len(tris)
    t0 = time.perf_counter()
    V = oracle.assemble(verts, tris, 4, 4)
    t_asm = time.perf_counter() - t0
    rows = np.sort(np.random.default_rng(7).choice(N, size=64, replace=False))
    rowsum = [math.fsum(V[i].tolist()) for i in rows.tolist()]
    total = float(np.sum(V))  # pairwise summation
    b = oracle.rhs(verts, tris)
    t0 = time.perf_counter()
    solver = {}
    if N * N < 2 ** 31:
        x = oracle.solve_direct(V, b, overwrite=True)
        solver = {"solver": "cholesky"}
    else:
        # more than 2^31 entries: beyond the dense LAPACK factorisation's
        # 32-bit indexing here (it reports a spurious non-positive minor)
        x, rr, its = oracle.solve_cg(V, b, rtol=1e-14)
        r = b - np.concatenate([V[r0:r0 + 4096] @ x for r0 in range(0, N, 4096)])
        solver = {"solver": "cg", "cg_iterations": its, "rel_residual": rr,
                  "cap_error_bound": float(np.linalg.norm(x) * np.linalg.norm(r) / abs(b @ x))}
    t_solve = time.perf_counter() - t0
    del V
    cap = oracle.capacity(x, b)
    print(f"{name}: N={N} cap={cap!r} assemble {t_asm:.0f} s solve {t_solve:.0f} s {solver}", flush=True)
    return dict(meta, N=N, mesh_sha=mesh_sha(verts, tris), far_order=4, ss_order=4, cap=cap, one_V_one=total,
                rows=rows.tolist(), rowsum=rowsum, x_rows=[float(x[i]) for i in rows.tolist()],
                oracle_seconds={"assemble": round(t_asm, 1), "solve": round(t_solve, 1)}, cores=os.cpu_count(),
                **solver)


def main():
    ap = argparse.ArgumentParser()
    names = sorted(WORKLOADS) + sorted(DUAL_WORKLOADS) + sorted(ADAPTIVE_WORKLOADS)
    ap.add_argument("--only", choices=names, default=None)
    a = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in ([a.only] if a.only else names):
        if name in ADAPTIVE_WORKLOADS:
            data[name] = ADAPTIVE_WORKLOADS[name](name)
        else:
            data[name] = run_dual(name) if name in DUAL_WORKLOADS else run(name)
        data["_about"] = ("FP64 oracle results (tests/golden/make_full_size.py; oracle/ and synth/ only): "
                          "Cap, 1^T V 1 and sampled row sums of V")
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
