"""Builds libbg.so for gfx950 in-tree: one object per multiplicity (kernels fully unrolled
per n) plus the C-ABI layer, compiled in parallel with hipcc, then linked shared.

Usage: python -m paper_1002_3446_amd.build [--jobs J]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay disabled (only scalar FP32 VALU forms are emitted)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the recursion is unrolled completely per multiplicity so currents stay in registers
    "-mllvm", "-pragma-unroll-threshold=100000000",
]


def _compile(src: str, obj: str, defines: list[str]) -> str:
    cmd = [HIPCC, *FLAGS, *defines, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {obj}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


KINDS = (0, 1, 2)  # 0 generate, 1 amp2, 2 gradient
GRAD_MAX_N = 10    # the fully unrolled adjoint of n = 11, 12 would need 4-8x the register file


def units_for(ns, precs=(32, 64), kinds=KINDS):
    units = [(os.path.join(CSRC, "bg_capi.hip"), os.path.join(OUT_DIR, "bg_capi.o"), [], 0),
             (os.path.join(CSRC, "bg_finalize.hip"), os.path.join(OUT_DIR, "bg_finalize.o"), [], 0)]
    # the persistent multi-class kernel holds every multiplicity: start it first
    units.append((os.path.join(CSRC, "bg_multi.hip"), os.path.join(OUT_DIR, "bg_multi_p32.o"), [], 1000))
    for n in ns:
        for p in precs:
            for k in kinds:
                if k == 2 and n > GRAD_MAX_N:
                    continue
                obj = os.path.join(OUT_DIR, f"bg_n{n:02d}_p{p}_k{k}.o")
                units.append((os.path.join(CSRC, "bg_inst.hip"), obj,
                              [f"-DBG_N={n}", f"-DBG_PREC={p}", f"-DBG_KIND={k}"], n * (2 if p == 64 else 1)))
    # the largest multiplicities take longest to compile: start them first
    units.sort(key=lambda u: -u[3])
    return units


def _deps_mtime(src: str) -> float:
    """Newest modification time of a unit's inputs: its own source, every header in csrc/
    and include/bg.h (other .hip files are not inputs)."""
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    hdrs.append(os.path.join(PKG, "..", "include", "bg.h"))
    return max(os.path.getmtime(f) for f in hdrs + [src])


def build(jobs: int | None = None, verbose: bool = True, ns=range(4, 13), incremental: bool = False) -> str:
    """Compiles every unit for the multiplicities ns and links libbg.so.  incremental=True
    keeps objects newer than their unit's inputs (developer convenience; the default
    rebuilds all)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    units = units_for(list(ns))
    if incremental:
        done = [u for u in units if os.path.exists(u[1]) and os.path.getmtime(u[1]) > _deps_mtime(u[0])]
        units_todo = [u for u in units if u not in done]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(lambda u: _compile(u[0], u[1], u[2]), units_todo))
        objs = [u[1] for u in units]
        return _link(objs, verbose)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u[0], u[1], u[2]), units))
    return _link(objs, verbose)


def _link(objs, verbose) -> str:
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--ns", type=str, default="4,5,6,7,8,9,10,11,12",
                    help="comma-separated multiplicities to build (others report BG_ENOTSUP)")
    ap.add_argument("--incremental", action="store_true", help="reuse objects newer than their unit's inputs")
    a = ap.parse_args()
    build(a.jobs, ns=[int(x) for x in a.ns.split(",")], incremental=a.incremental)
