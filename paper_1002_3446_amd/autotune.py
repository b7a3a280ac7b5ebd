"""Launch-shape autotuner for libbg (needs a GPU).

For every multiplicity n and recursion precision it times single-class bg_generate with
64, 128 and 256 threads per workgroup and, where the library holds both, one or two lanes
per event, and keeps the fastest; then, on the FP32 mixed workload
(n = 4..12 with 2^(26-n) events each, one persistent launch), it tunes each class's tile
length (events per lane per tile) by coordinate search, and finally records which of the
three strategies for several classes (one after another, one persistent launch, classes on
concurrent streams) is fastest for that workload.  The result is written to
autotune.json next to this file, which the binding applies on import.

Usage: python -m paper_1002_3446_amd.autotune [--prec 32|64|both] [--out PATH] [--scale S]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import torch

from . import bg

NS = list(range(4, 13))


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def mixed_workload(prec, scale=0):
    cfgs = [bg.config(n, prec=prec, seed=0xB6000003 + n) for n in NS]
    counts = [1 << (26 - n - scale) for n in NS]
    return cfgs, counts


def lane_forms(n, prec):
    """Lanes-per-event forms the library holds for (n, prec)."""
    grouped = (prec == 32 and n >= 9) or (prec == 64 and n >= 6)
    one = (prec == 32 and n <= 9) or (prec == 64 and n <= 6)
    return ((1,) if one else ()) + ((2,) if grouped else ()) + ((4,) if prec == 64 and n >= 10 else ())


def wtensor_forms(n, prec):
    """Multiplicities whose W-tensor form the library holds."""
    return (prec == 32 and n in (8, 10, 11, 12)) or (prec == 64 and n in (6, 10))


def tune_single(prec=32, scale=0, log=print):
    """Workgroup size, lanes per event and recursion form of every single-class kernel."""
    shapes = {}
    for n in NS:
        N = 1 << max(20 - scale, 26 - n - scale)
        cfg = bg.config(n, prec=prec, seed=0xB6000003 + n)
        out = bg.generate(cfg, N, outputs=("weight", "acc"))
        cands = [(lanes, 0, block) for lanes in lane_forms(n, prec) for block in (64, 128, 256)]
        if wtensor_forms(n, prec):
            cands.append((0, 1, 64))   # W-tensor: fixed 64-lane workgroups, lanes unused
        best = None
        for lanes, form, block in cands:
            bg.set_form(n, prec, form)
            if lanes:
                bg.set_lanes(n, prec, lanes)
            bg.set_launch(n, prec, block, bg.get_launch(n, prec)[1] or 1)
            t = _time(lambda: bg.generate(cfg, N, outputs=("weight", "acc"), out_tensors=[out]))
            log(f"n={n} prec={prec} form={form} lanes={lanes} block={block}: {t:.3f} ms for {N} events")
            if best is None or t < best[0]:
                best = (t, block, lanes, form)
        shapes[n] = [best[1], bg.get_launch(n, prec)[1], best[2], best[3]]
        bg.set_launch(n, prec, shapes[n][0], shapes[n][1])
        if shapes[n][2]:
            bg.set_lanes(n, prec, shapes[n][2])
        bg.set_form(n, prec, shapes[n][3])
    return shapes


def tune(prec=32, scale=0, log=print):
    shapes = tune_single(prec, scale, log)
    if prec != 32:   # the persistent multi-class kernel is FP32 only
        return [dict(n=n, prec=prec, block=b, tile_iters=i, lanes=l, form=f) for n, (b, i, l, f) in shapes.items()], None
    cfgs, counts = mixed_workload(prec, scale)
    outs = bg.generate(cfgs, counts, outputs=("weight", "acc"))
    run = lambda: bg.generate(cfgs, counts, outputs=("weight", "acc"), out_tensors=outs)
    base = _time(run)
    log(f"mixed launch, default tiles: {base:.3f} ms")
    for n in NS:
        best = (base, shapes[n][1])
        for it in (1, 2, 4, 8, 16):
            bg.set_launch(n, prec, shapes[n][0], it)
            t = _time(run)
            if t < best[0] * 0.995:
                best = (t, it)
        shapes[n][1] = best[1]
        bg.set_launch(n, prec, shapes[n][0], best[1])
        base = best[0]
        log(f"n={n}: tile_iters={best[1]} -> mixed {base:.3f} ms")
    modes = {"persistent": base}
    for name, m in (("sequential", bg.MIXED_SEQUENTIAL), ("concurrent", bg.MIXED_CONCURRENT)):
        bg.set_mixed_launch(m)
        modes[name] = _time(run)
    bg.set_mixed_launch(bg.MIXED_PERSISTENT)
    log("mixed workload: " + ", ".join(f"{k} {v:.3f} ms" for k, v in modes.items()))
    return [dict(n=n, prec=prec, block=b, tile_iters=i, lanes=l, form=f) for n, (b, i, l, f) in shapes.items()], modes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--prec", default="both", choices=("32", "64", "both"))
    ap.add_argument("--scale", type=int, default=0, help="shrink every workload by 2^scale")
    ap.add_argument("--out", default=bg.TUNING_PATH)
    a = ap.parse_args()
    precs = (32, 64) if a.prec == "both" else (int(a.prec),)
    t0 = time.time()
    for prec in precs:
        for n in NS:
            bg.set_launch(n, prec, 0, 0)   # start from the built-in defaults
            bg.set_lanes(n, prec, 0)
            bg.set_form(n, prec, 0)
    bg.set_mixed_launch(bg.MIXED_PERSISTENT)
    doc = json.load(open(a.out)) if os.path.exists(a.out) else {}
    shapes = [e for e in doc.get("shapes", []) if e["prec"] not in precs]
    for prec in precs:
        sh, modes = tune(prec, a.scale)
        shapes += sh
        if modes is not None:
            ids = {"sequential": bg.MIXED_SEQUENTIAL, "persistent": bg.MIXED_PERSISTENT,
                   "concurrent": bg.MIXED_CONCURRENT}
            best = min(modes, key=modes.get)
            doc.update({"mixed_ms": modes, "mixed_mode": ids[best], "mixed_mode_name": best})
    doc.update({"device": torch.cuda.get_device_name(0), "tuned_in_s": time.time() - t0, "shapes": shapes})
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc))


if __name__ == "__main__":
    main()
