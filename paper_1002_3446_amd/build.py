"""Builds libbg.so for gfx950 in-tree: one object per kernel (kind, multiplicity, precision,
lane form; kernels fully unrolled per n), the persistent multi-class kernel, and the C-ABI
layer, compiled in parallel with hipcc, then linked shared.  The C-ABI layer embeds a hash
of the sources (source_hash), which the binding checks before it uses the library.

Usage: python -m paper_1002_3446_amd.build [--jobs J]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
HEADER = os.path.join(PKG, "..", "include", "bg.h")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay disabled (only scalar FP32 VALU forms are emitted)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # LLVM's CodeGenPrepare pass is quadratic on the recursion's straight-line code (half the
    # compile time of a unit) and changes nothing in its machine code: skipped
    "-mllvm", "-disable-cgp",
]


def source_hash() -> str:
    """sha256 (first 16 hex digits) over the kernel sources in csrc/ (sorted by name), the
    C header and this file (the compiler flags of every unit): the identity a built library
    carries and the binding checks."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(CSRC, f), "rb").read())
    h.update(open(HEADER, "rb").read())
    h.update(open(os.path.abspath(__file__), "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, obj: str, defines: list[str]) -> tuple[str, float]:
    cmd = [HIPCC, *FLAGS, *defines, "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {obj}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, time.time() - t0


KINDS = (0, 1, 2)  # 0 generate, 1 amp2, 2 gradient


def has_one_lane(n: int, p: int) -> bool:
    return n <= 9 if p == 32 else n <= 6


def has_lane_pairs(n: int, p: int) -> bool:
    return n >= 9 if p == 32 else n >= 6


def has_lane_quads(n: int, p: int) -> bool:
    return p == 64 and n >= 10


def has_real_pol(n: int, p: int) -> bool:
    return n <= 12 if p == 32 else n <= 8


def has_wtensor(n: int, p: int) -> bool:
    return (n == 8 or n >= 10) if p == 32 else n in (6, 10)


def unit_flags(n: int, p: int, k: int, f: int) -> list[str]:
    """Extra compiler flags of one kernel unit.  The generation and bg_amp2 units of FP32 n = 8
    (one lane) and of FP64 n >= 8 (two or four lanes) are built without LLVM's pre-RA machine
    scheduler: there the recursion fills the register file at one wave per SIMD, and the
    scheduler's reordering for latency raises register pressure, which costs more (scratch
    spill, AGPR copies) than the latency it hides.  Measured on generation, alternating runs
    on one GPU: FP32 n = 8 6.69 -> 6.53-6.61 ms per 2^24 events; FP64 n = 8 11.1 -> 11.0 ms per
    2^24, n = 9 5.23 -> 5.01, n = 10 unchanged, n = 11 12.99 -> 12.71, n = 12 20.57 -> 18.45 ms
    per 2^22 (scratch 400 -> 248 B per lane).  FP32 n = 12 lost 0.8% without it and keeps it."""
    if k < 2 and ((p == 32 and f == 1 and n == 8) or (p == 64 and f in (2, 5) and n >= 8)):
        return ["-mllvm", "-enable-misched=0"]
    return []


def units_for(ns, precs=(32, 64), kinds=KINDS):
    """(source, object, defines, expected cost) of every unit; the costliest start first."""
    units = [(os.path.join(CSRC, "bg_capi.hip"), os.path.join(OUT_DIR, "bg_capi.o"),
              [f'-DBG_SOURCE_HASH="{source_hash()}"'], 0),
             (os.path.join(CSRC, "bg_finalize.hip"), os.path.join(OUT_DIR, "bg_finalize.o"), [], 0),
             (os.path.join(CSRC, "bg_hist.hip"), os.path.join(OUT_DIR, "bg_hist.o"), [], 0),
             (os.path.join(CSRC, "bg_probe.hip"), os.path.join(OUT_DIR, "bg_probe.o"), [], 0)]
    if set(range(4, 13)) <= set(ns) and 32 in precs:
        units.append((os.path.join(CSRC, "bg_multi.hip"), os.path.join(OUT_DIR, "bg_multi_p32.o"), [], 1000))
    for n in ns:
        for p in precs:
            for k in kinds:
                if k == 2:
                    forms = (1,)
                else:
                    forms = tuple(f for f, ok in ((1, has_one_lane(n, p)), (2, has_lane_pairs(n, p)),
                                                  (3, k == 0 and has_real_pol(n, p)),
                                                  (4, has_wtensor(n, p)),
                                                  (5, k < 2 and has_lane_quads(n, p))) if ok)
                for f in forms:
                    obj = os.path.join(OUT_DIR, f"bg_n{n:02d}_p{p}_k{k}_f{f}.o")
                    cost = n ** 3 * (2 if p == 64 else 1) * (4 if k == 2 else 1)
                    units.append((os.path.join(CSRC, "bg_inst.hip"), obj,
                                  [f"-DBG_N={n}", f"-DBG_PREC={p}", f"-DBG_KIND={k}", f"-DBG_FORM={f}"]
                                  + unit_flags(n, p, k, f), cost))
    units.sort(key=lambda u: -u[3])
    return units


def build(jobs: int | None = None, verbose: bool = True, ns=range(4, 13)) -> str:
    """Compiles every unit for the multiplicities ns and links libbg.so (always a full build)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    units = units_for(list(ns))
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        done = list(ex.map(lambda u: _compile(u[0], u[1], u[2]), units))
    if verbose:
        slow = sorted(done, key=lambda d: -d[1])[:3]
        print(f"compiled {len(done)} units in {time.time() - t0:.0f} s (slowest: "
              + ", ".join(f"{os.path.basename(o)} {t:.0f} s" for o, t in slow) + ")", file=sys.stderr)
    return _link([d[0] for d in done], verbose)


def _link(objs, verbose) -> str:
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} (sources {source_hash()})", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--ns", type=str, default="4,5,6,7,8,9,10,11,12",
                    help="comma-separated multiplicities to build (others report BG_ENOTSUP)")
    a = ap.parse_args()
    build(a.jobs, ns=[int(x) for x in a.ns.split(",")])
