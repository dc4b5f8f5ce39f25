"""Seeded request streams for the capacity-solve server.

A request is one polyhedron meshed to a target size.  Shapes are drawn
uniformly from three families: voxel unions on a k^3 lattice (k in 2..5) at
40% occupancy, convex hulls of 8..20 uniform points in [-1, 1]^3, and boxes
with sides (1, a, b), a and b uniform in [1, 8].  Target sizes are
log-uniform in [n_min, n_max]; meshing is uniform newest-vertex bisection
followed by bisection of the largest elements until N >= target.  Arrival
times are a Poisson process (exponential inter-arrival times) of a given
rate; rate = inf puts every request at t = 0.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from .meshes import Mesh, box, convex_hull, voxel_union
from .nvb import init_reference_edges, refine_to_size


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after stream start
    kind: str
    params: dict
    n_target: int
    seed: int

    def build_mesh(self) -> Mesh:
        if self.kind == "voxel":
            base = voxel_union(self.params["L"], 0.4, self.seed)
        elif self.kind == "hull":
            base = convex_hull(self.params["npts"], self.seed)
        elif self.kind == "box":
            base = box(self.params["a"], self.params["b"])
        else:
            raise ValueError(self.kind)
        t0 = init_reference_edges(base.verts, base.tris)
        v, t = refine_to_size(base.verts, t0, self.n_target)
        return Mesh(v, t, f"req{self.rid}_{self.kind}", dict(base.meta, n_target=self.n_target))


def request_stream(n: int = 512, seed: int = 5, rate: float = math.inf,
                   n_min: int = 500, n_max: int = 30000):
    rng = np.random.default_rng(seed)
    # arrival times from a generator of their own, so that the requests
    # themselves (kind, parameters, size, mesh seed) do not depend on the rate
    arrivals = np.random.default_rng([seed, 1])
    out = []
    t = 0.0
    for rid in range(n):
        kind = ("voxel", "hull", "box")[int(rng.integers(0, 3))]
        if kind == "voxel":
            params = {"L": int(rng.integers(2, 6))}
        elif kind == "hull":
            params = {"npts": int(rng.integers(8, 21))}
        else:
            params = {"a": float(rng.uniform(1, 8)), "b": float(rng.uniform(1, 8))}
        n_target = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        sub_seed = int(rng.integers(0, 2 ** 31 - 1))
        if math.isfinite(rate):
            t += float(arrivals.exponential(1.0 / rate))
        out.append(Request(rid, t if math.isfinite(rate) else 0.0, kind, params, n_target, sub_seed))
    return out
