"""Build libbemcap.so, and libbemcap_static.so beside it, for gfx950 with
hipcc (in-tree, no JIT cache).

libbemcap_static.so holds only bc_solve_static and the device array that is
its workspace; it links against libbemcap.so.  Keeping the array out of the
main library means that a process holds its 96 MiB per GPU only when it
loads the companion library, i.e. when it uses the allocation-free entry
point.

    python -m paper_1901_08393_amd.build [--jobs N]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbemcap.so")
LIB_STATIC = os.path.join(HERE, "libbemcap_static.so")
SOURCES = ["abi.hip", "geometry.hip", "assemble.hip", "solve.hip", "zz.hip", "dual.hip", "residual.hip"]
SOURCES_STATIC = ["solve_static.hip"]
ARCH = os.environ.get("BEMCAP_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _link(objs, out: str, extra=()) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *extra, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of {os.path.basename(out)} failed:\n{r.stderr}")
    os.replace(tmp, out)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + SOURCES_STATIC
    jobs = jobs or min(len(srcs), os.cpu_count() or 1, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    _link([objs[s] for s in SOURCES], LIB)
    # the companion library finds libbemcap.so next to itself
    _link([objs[s] for s in SOURCES_STATIC], LIB_STATIC, ["-L" + HERE, "-l:libbemcap.so", "-Wl,-rpath,$ORIGIN"])
    if verbose:
        print(f"built {LIB} and {LIB_STATIC}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
