#!/usr/bin/env python3
"""Benchmark of the event-generation path on one MI355X.

One step = one bg_generate call over 2^24 gg -> 6g events (n = 8 external gluons):
Philox draws, x1/x2 from f(x) = x^-1.3 (1-x)^5, RAMBO at sqrt(S) = 14 TeV, the boost, jet
cuts (pT > 20 GeV, |eta| < 2.5, dR > 0.4) and observables, helicity sources, the
Berends-Giele recursion in FP32 (kinematics, K^2 and weights in FP64), |A|^2, weights and
the compensated weight sums.  Inputs are generated on the device from the seed; nothing
is copied from the host inside the timed region.

Prints one JSON line (see the keys below).  Extra keys report the FP64 run of the same
workload, the FP32 / FP64 runs of gg -> 10g (n = 12, 2^22 events), the FP32-versus-FP64
relative error on identical events, and the forward+adjoint rate when available.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12   # MI355X vector FP32 (counts packed FP32; this build emits scalar FP32 only)
PEAK_FP32_SCALAR = 78.6e12  # the same without packed FP32: 256 CUs x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_FP64 = 78.6e12    # MI355X vector FP64
PAPER_N8_EVENTS_PER_S = 1.0 / 3.546e-7   # Table 1 of the paper, NVIDIA Tesla, FP32 (context only)


def comb(n, k):
    return math.comb(n, k)


def flops_plain(n: int) -> int:
    """Per-event flops of the recursion in the printed form (3- and 4-gluon brackets summed
    term by term, complex helicity currents): 146 C(n,3) + 188 C(n,4) + 20 (L(L-1)/2 - 1) + 40 n + 30."""
    L = n - 1
    return 146 * comb(n, 3) + 188 * comb(n, 4) + 20 * (L * (L - 1) // 2 - 1) + 40 * n + 30


def flops_executed(n: int) -> int:
    """Per-event floating-point operations of the recursion and closure as the kernel
    executes them (fma = 2; span momenta and propagators come precomputed): per split of a
    span, complex dot 30, two complex-real dots 28, two complex axpys 64, K_A - K_B 4 and
    its axpy 16, the span scalar 2 (144); per pair of splits, dot 30 + axpy 32; 2(l-2)
    span-scalar axpys of 32; V = 2X + Y 16; then the propagator 8, or the closure dot 30."""
    L = n - 1
    tot = 0
    for length in range(2, L + 1):
        spans = L - length + 1
        per = 144 * (length - 1) + 62 * comb(length - 1, 2) + 64 * (length - 2) + 16
        per += 8 if length < L else 30
        tot += spans * per
    return tot


def flops_real(n: int) -> int:
    """Per-event flops of the recursion with real currents (random real polarisations) in the
    printed form: about 51 per three-gluon and 46 per four-gluon bracket term (real dots of
    7, axpys of 8), 5 per propagator, 20 n for the sources and the closure."""
    L = n - 1
    return 51 * comb(n, 3) + 46 * comb(n, 4) + 5 * (L * (L - 1) // 2 - 1) + 20 * n


def kernel_hash() -> str:
    """Hash of the kernel sources (the one the loaded library embeds, bg_source_hash)."""
    from paper_1002_3446_amd.build import source_hash
    return source_hash()


def traffic_from_profile(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they were taken
    on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def run_steps(bg, torch, cfg, N, steps, warmup, outputs):
    """Returns (wall seconds over the timed steps, list of per-launch device ms, outputs)."""
    first = cfg.first_event
    out = bg.generate(cfg, N, outputs=outputs)          # first call allocates the outputs
    torch.cuda.synchronize()
    for s in range(warmup):
        cfg.first_event = first + (s + 1) * N
        out["acc"].zero_()
        bg.generate(cfg, N, outputs=outputs, out_tensors=[out])
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for s in range(steps):
        cfg.first_event = first + (warmup + 1 + s) * N
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        bg.generate(cfg, N, outputs=outputs, out_tensors=[out])
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cfg.first_event = first
    return wall, [a.elapsed_time(b) for a, b in evs], out


def scaling_measure(t_n: float, t_prev: float, n: int, m: int) -> float:
    """Polynomial scaling measure of Table 1 (Sec. 4): P_n(m) = ((n-1)/n) (T_n / T_(n-1))^(1/m)
    for per-event times T; it approaches 1 when T grows like n^m."""
    return (n - 1) / n * (t_n / t_prev) ** (1.0 / m)


def mixed_rate(bg, torch):
    """n = 4..12 with 2^(26-n) events each (8,372,224 events), FP32: one persistent launch,
    one class after another, and classes on concurrent streams; the rate is the fastest."""
    ns = list(range(4, 13))
    cfgs = [bg.config(n, prec=32, seed=0xB6000003 + n) for n in ns]
    counts = [1 << (26 - n) for n in ns]
    outputs = ("weight", "amp2", "obs", "pass", "acc")
    outs = bg.generate(cfgs, counts, outputs=outputs)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    mode = bg.get_mixed_launch()
    ms_modes = {}
    for name, m in (("persistent", bg.MIXED_PERSISTENT), ("sequential", bg.MIXED_SEQUENTIAL),
                    ("concurrent", bg.MIXED_CONCURRENT)):
        bg.set_mixed_launch(m)
        ms_modes[name] = timed(lambda: bg.generate(cfgs, counts, outputs=outputs, out_tensors=outs))
    bg.set_mixed_launch(mode)
    per_n = {}
    for c, N, o in zip(cfgs, counts, outs):
        per_n[c.n] = timed(lambda: bg.generate(c, N, outputs=outputs, out_tensors=[o]))
    total = sum(counts)
    return {"mixed_n4_12_fp32_events_per_s": total / (min(ms_modes.values()) * 1e-3),
            "mixed_n4_12_ms_by_mode": ms_modes, "mixed_n4_12_tuned_mode": mode,
            "mixed_n4_12_sum_of_single_ms": sum(per_n.values()),
            "single_class_fp32_events_per_s": {str(n): counts[i] / (per_n[n] * 1e-3) for i, n in enumerate(ns)},
            # the paper's GPU scaling measure P_n(3) (Table 1) for these per-event times
            "single_class_fp32_scaling_P3": {str(n): scaling_measure(per_n[n] / counts[i], per_n[n - 1] / counts[i - 1], n, 3)
                                             for i, n in enumerate(ns) if i > 0}}


def adjoint_rate(bg, torch, N=1 << 20, steps=5, n=8, prec=32):
    """Forward + backward of log w_int through the torch Function (gg -> 6g, FP32, unless
    n and prec say otherwise), on phase-space points the GPU draws first (untimed)."""
    from paper_1002_3446_amd.autograd import log_weight
    cfg = bg.config(n, prec=prec, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000004)
    d = bg.generate(cfg, N, outputs=("uniforms", "x12", "hel", "order"))
    u = d["uniforms"].requires_grad_(True)
    x = d["x12"].requires_grad_(True)
    evs = []
    for s in range(steps + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        u.grad = None
        x.grad = None
        a.record()
        lw = log_weight(u, x, cfg, d["hel"], d["order"])
        lw.sum().backward()
        b.record()
        if s > 0:
            evs.append((a, b))
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in evs) / len(evs)
    tag = f"n{n}_fwd_adjoint_fp{prec}"
    return {f"{tag}_events_per_s": N / (ms * 1e-3), f"{tag}_ms_per_2^{N.bit_length() - 1}": ms}


def recursion_rate(bg, torch, n=8, N=1 << 22, reps=5):
    """bg_amp2 alone (helicity sources, recursion, closure; FP32) on phase-space points the
    generator draws first (untimed): the recursion kernel's own FLOP rate."""
    cfg = bg.config(n, prec=32, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000005)
    d = bg.generate(cfg, N, outputs=("momenta", "hel", "order"))
    out = bg.amp2(n, 32, d["momenta"], d["hel"], d["order"])
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        bg.amp2(n, 32, d["momenta"], d["hel"], d["order"], out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    fp, fe = flops_plain(n), flops_executed(n)
    return {"kernel": f"k_amp2<{n},float>", "events": N, "launch_ms": ms, "events_per_s": N / (ms * 1e-3),
            "achieved_plain_tflops": fp * N / (ms * 1e-3) / 1e12, "frac_plain": fp * N / (ms * 1e-3) / PEAK_FP32,
            "achieved_executed_tflops": fe * N / (ms * 1e-3) / 1e12,
            "frac_executed": fe * N / (ms * 1e-3) / PEAK_FP32,
            "frac_executed_of_scalar_fp32": fe * N / (ms * 1e-3) / PEAK_FP32_SCALAR,
            "hbm_bytes_per_event": 8 * 4 * n + 4 + n + 8}


def hist_rate(bg, torch, out, N, reps=5):
    """Exact histograms of H_T (40 bins) and R_min (36 bins) over one step's events (weights
    and observables already in device memory): one bg_hist_accumulate call; algorithmic
    bytes 24 per event (weight + two observables read)."""
    axes = [(bg.OBS_HT, 40, 0.0, 2000.0), (bg.OBS_RMIN, 36, 0.4, 4.0)]
    limbs = bg.hist_limbs(axes)
    bg.hist_accumulate(out["weight"], out["obs"], axes, limbs)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        bg.hist_accumulate(out["weight"], out["obs"], axes, limbs)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"hist_2axes_ms_per_step": ms, "hist_2axes_GBps": 24 * N / (ms * 1e-3) / 1e9}


def live_helicities(hel, n, torch):
    """Mask of helicity words with at least two of each helicity (non-vanishing amplitudes)."""
    bits = (hel.unsqueeze(1) >> torch.arange(n, device=hel.device, dtype=hel.dtype)) & 1
    plus = bits.sum(1)
    return (plus >= 2) & (plus <= n - 2)


def host_cores() -> int:
    """Host threads the CPU legs use: all the host's cores, at most the 16 a one-GPU share
    of the machine provides."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


BENCH_SEED = {8: 0xB6000001, 12: 0xB6000002}
BENCH_SEED.update({n: 0xB6000003 + n for n in (4, 5, 6, 7, 9, 10, 11)})  # the mixed workload's
CHUNK = 4096


def _oracle_cfg(n):
    from oracle import event
    return event.config(n=n, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=BENCH_SEED[n])


def _oracle_timed(args):
    """Worker: oracle event generation over chunks w, w + W, ... of the n = 8 workload for
    about `seconds`; returns (events, seconds)."""
    import numpy as np

    from oracle import event
    w, W, seconds = args
    oc = _oracle_cfg(8)
    done, k = 0, w
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        event.generate(oc, np.arange(k * CHUNK, (k + 1) * CHUNK))
        done += CHUNK
        k += W
    return done, time.perf_counter() - t0


def _oracle_amp2(args):
    """Worker: the oracle's |A|^2 and helicity words of events lo..hi-1 of a workload."""
    import numpy as np

    from oracle import event
    from oracle.recursion import mdot
    n, lo, hi = args
    o = event.generate(_oracle_cfg(n), np.arange(lo, hi))
    # the event's size for FP32 tails: the Parke-Taylor |A|^2 of its colour ordering with
    # legs 0 and 1 of opposite helicity
    k = o["mom_cm"] * np.array([-1.0, -1.0] + [1.0] * (n - 2))[None, :, None]
    ko = np.take_along_axis(k, o["order"].astype(np.int64)[:, :, None], axis=1)
    den = np.ones(len(k))
    for t in range(n):
        den = den * np.abs(2 * mdot(ko[:, t], ko[:, (t + 1) % n]))
    size = np.maximum(o["amp2"], (2 * mdot(k[:, 0], k[:, 1])) ** 4 / den)
    return o["amp2"], o["hel"], size


def cpu_legs(seconds: float = 10.0, accuracy_events: int = 1 << 16):
    """Runs before the GPU is touched (the worker processes are forked).  Returns the CPU
    baseline (the oracle on all host cores and on one, a bounded sample of the n = 8
    workload) and the oracle's |A|^2 of the first accuracy_events events of the n = 8 and
    n = 12 workloads and of 2^13 events of every other n = 4..11 (the reference of the
    accuracy block)."""
    import multiprocessing as mp

    import numpy as np

    cores = host_cores()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        single = _oracle_timed((0, 1, seconds / 4))
        res = pool.map(_oracle_timed, [(w, cores, seconds) for w in range(cores)])
        ref = {}
        for n in range(4, 13):
            ne = accuracy_events if n in (8, 12) else accuracy_events // 8
            parts = pool.map(_oracle_amp2, [(n, lo, lo + CHUNK) for lo in range(0, ne, CHUNK)])
            ref[n] = tuple(np.concatenate([p[i] for p in parts]) for i in range(3))
    events = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    base = dict(value=events / wall, unit="events/s", cores=cores, kind="oracle",
                sample=f"{events} events of the n=8 workload (seed 0xB6000001, chunks of {CHUNK} events "
                       f"interleaved over {cores} processes, numpy float64, {wall:.1f} s)",
                single_core_events_per_s=single[0] / single[1], host_nproc=os.cpu_count(), host_cpu=cpu_model())
    return base, ref


def accuracy_block(bg, torch, ref):
    """Per-event relative error of |A|^2 against the oracle (float64) on the first events of
    the workloads (2^16 at n = 8 and 12, 2^13 at the other n), FP32 and FP64 recursion, over the helicity
    configurations whose amplitude does not vanish identically; the maximum also relative
    to the event's size max(|A|^2, Parke-Taylor |A|^2 of its ordering), which bounds the
    FP32 tail of events near a zero of the amplitude."""
    import numpy as np
    out = {}
    for n, (oa, oh, size) in ref.items():
        N = len(oa)
        bits = (oh.astype(np.int64)[:, None] >> np.arange(n)) & 1
        live = (bits.sum(1) >= 2) & (bits.sum(1) <= n - 2) & (oa > 0)
        for prec in (32, 64):
            c = bg.config(n, prec=prec, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=BENCH_SEED[n])
            r = bg.generate(c, N, outputs=("amp2", "hel"))
            g = r["amp2"].cpu().numpy()
            gh = r["hel"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(gh, oh.astype(np.int64)), "helicity draws differ from the oracle's"
            rel = np.abs(g[live] - oa[live]) / oa[live]
            sc = np.abs(g[live] - oa[live]) / size[live]
            q = np.quantile(rel, [0.5, 0.9, 0.99])
            out[f"n{n}_fp{prec}"] = dict(p50=float(q[0]), p90=float(q[1]), p99=float(q[2]), max=float(rel.max()),
                                         max_rel_to_event_size=float(sc.max()),
                                         frac_within_1e12=float(np.mean(rel <= 1e-12)), events=int(live.sum()))
    return out


def sigma_block(bg, torch, N):
    """sigma = sum w / N from one untimed call of the benchmark workload (events 0..N-1),
    checked against the exact sum of that call's weights; the same events with FP64
    recursion; their difference in units of the statistical error delta sigma."""
    out = {}
    for prec in (32, 64):
        c = bg.config(8, prec=prec, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=BENCH_SEED[8])
        r = bg.generate(c, N, outputs=("weight", "acc"))
        acc = r["acc"].cpu().numpy()
        exact = math.fsum(r["weight"].cpu().numpy().tolist())
        s, s2 = acc[0] + acc[1], acc[2] + acc[3]
        sig = s / N
        out[prec] = dict(sigma_pb=sig, delta_sigma_pb=math.sqrt(max(s2 / N - sig * sig, 0.0) / (N - 1)),
                         exact_sum_rel_diff=abs(s - exact) / abs(exact))
    d = out[32]["sigma_pb"] - out[64]["sigma_pb"]
    return {"events": N, "sigma_pb_fp32": out[32]["sigma_pb"], "delta_sigma_pb": out[64]["delta_sigma_pb"],
            "sigma_pb_fp64": out[64]["sigma_pb"], "fp32_minus_fp64_over_delta_sigma": d / out[64]["delta_sigma_pb"],
            "fp32_minus_fp64_rel": d / out[64]["sigma_pb"],
            "compensated_vs_exact_sum_rel": max(out[32]["exact_sum_rel_diff"], out[64]["exact_sum_rel_diff"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=1 << 24)
    ap.add_argument("--n", type=int, default=8,
                    help="multiplicity of the main line (8, the benchmark workload; others for profiling)")
    ap.add_argument("--prec", type=int, default=32, choices=(32, 64),
                    help="recursion precision of the main line (32, the benchmark workload; 64 for profiling)")
    ap.add_argument("--mixed-only", type=int, default=-1, metavar="MODE",
                    help="only run the mixed n = 4..12 workload three times in one mixed-launch mode (profiling)")
    ap.add_argument("--no-extras", action="store_true", help="main line only (used under profilers)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--recursion", action="store_true",
                    help="with --no-extras: still time the recursion kernel (bg_amp2) alone")
    ap.add_argument("--adjoint", action="store_true",
                    help="with --no-extras: still time the forward + adjoint through the torch Function")
    ap.add_argument("--adjoint-n", type=int, default=8, help="multiplicity of the --adjoint timing")
    ap.add_argument("--adjoint-prec", type=int, default=32, choices=(32, 64), help="precision of the --adjoint timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scales HBM counters)")
    a = ap.parse_args()
    if a.copy_calibration:
        import torch
        src = torch.ones(a.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4}), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); events are independent, "
              "so N GPUs would run disjoint Philox event ranges and add their compensated sums.", file=sys.stderr)
        sys.exit(2)

    # CPU legs first: their worker processes are forked before anything touches the GPU
    cpu, ref = (None, None) if a.no_cpu else cpu_legs()

    import torch

    from paper_1002_3446_amd import bg

    torch.cuda.set_device(0)
    outputs = ("weight", "amp2", "obs", "pass", "acc")
    n, N = a.n, a.events
    if a.mixed_only >= 0:
        bg.set_mixed_launch(a.mixed_only)
        ns = list(range(4, 13))
        cfgs = [bg.config(m, prec=32, seed=0xB6000003 + m) for m in ns]
        counts = [1 << (26 - m) for m in ns]
        outs = bg.generate(cfgs, counts, outputs=outputs)
        for _ in range(3):
            bg.generate(cfgs, counts, outputs=outputs, out_tensors=outs)
        torch.cuda.synchronize()
        print(json.dumps({"mixed_mode": a.mixed_only, "events": sum(counts)}), flush=True)
        return
    cfg = bg.config(n, prec=a.prec, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=BENCH_SEED.get(n, 0xB6000001))
    wall, ms, out = run_steps(bg, torch, cfg, N, a.steps, a.warmup, outputs)
    ms_step = 1e3 * wall / a.steps
    value = N * a.steps / wall
    launch_ms = sum(ms) / len(ms)
    fp = flops_plain(n)
    fe = flops_executed(n)
    # FP32 n <= 8 runs as a kinematics and a recursion kernel per chunk of 2^22 events: the
    # timed unit is then the whole bg_generate call (both kernels, every chunk)
    real_t = "float" if a.prec == 32 else "double"
    peak = PEAK_FP32 if a.prec == 32 else PEAK_FP64
    lanes = bg.get_lanes(n, a.prec)
    if n <= 8 and a.prec == 32:
        kname = f"k_kin<{n}>+k_rec<{n}>"
    elif lanes == 1:
        kname = f"k_generate<{n},{real_t}>"
    else:
        kname = f"k_kin<{n}>+k_rec_g<{n},{real_t},{lanes}>"
    achieved = fp * N / (launch_ms * 1e-3)
    line = {
        "metric": f"events/s at gg->{n - 2}g (n={n}) FP{a.prec} recursion (FP64 kinematics and weights), full generation path",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f{a.prec} recursion + f64 kinematics/weights",
        "data": "synthetic: Philox-seeded RAMBO events generated on the device",
        "config": {"workload": f"gg->{n - 2}g ({n} external gluons), {N} events per step, sqrt(S)=14 TeV, "
                               f"x ~ x^-1.3 (1-x)^5 on [{((n - 2) * 20.0 / 14000.0) ** 2:.3g},1), alpha_s=0.118, random helicity and "
                               "colour ordering per event, cuts pT>20 GeV |eta|<2.5 dR>0.4",
                   "n": n, "events_per_step": N, "prec": a.prec, "parallelism": "one event per lane, 1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic_from_profile(kname),
                     "kernel": kname, "launch_ms": launch_ms,
                     "flops_per_event_plain": fp, "flops_per_event_executed": fe,
                     "executed_tflops": fe * N / (launch_ms * 1e-3) / 1e12,
                     "executed_frac": fe * N / (launch_ms * 1e-3) / peak},
        "paper_context": {"tesla_fp32_n8_events_per_s": PAPER_N8_EVENTS_PER_S,
                          "note": "paper Table 1, NVIDIA Tesla, real polarisations, LHAPDF; not the same workload"},
    }
    # the ceilings as this GPU sustains them: plain multiply-add chains (scalar FP32, FP64)
    fma32, fma64 = bg.fma_rate(32), bg.fma_rate(64)
    exe = fe * N / (launch_ms * 1e-3) / 1e12
    line["calibration"] = {"fma_fp32_tflops": fma32, "fma_fp64_tflops": fma64,
                           "executed_frac_of_measured_fma": exe / (fma32 if a.prec == 32 else fma64),
                           "note": "bg_fma_rate: chains of independent FMAs, all CUs, 8 waves/SIMD; scalar FP32"}
    if n == 8:
        line["sigma"] = sigma_block(bg, torch, N)
    if ref is not None:
        line["accuracy_vs_oracle"] = accuracy_block(bg, torch, ref)

    if a.recursion and a.no_extras:
        line["recursion_kernel"] = recursion_rate(bg, torch)
    if a.adjoint and a.no_extras:
        line["adjoint"] = adjoint_rate(bg, torch, N=1 << (20 if a.adjoint_n <= 8 else 18), steps=2,
                                       n=a.adjoint_n, prec=a.adjoint_prec)
    if not a.no_extras:
        extras = {}
        cfg64 = bg.config(n, prec=64, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000001)
        w64, ms64, out64 = run_steps(bg, torch, cfg64, N, max(2, a.steps // 3), 1, outputs)
        extras["n8_fp64_events_per_s"] = N * max(2, a.steps // 3) / w64
        extras["n8_fp64_launch_ms"] = sum(ms64) / len(ms64)
        # FP32 versus FP64 on identical events (kinematics are FP64 in both), over helicity
        # configurations whose amplitude does not vanish identically
        r32 = bg.generate(cfg, 1 << 20, outputs=("amp2", "hel"))
        a32, hel = r32["amp2"], r32["hel"]
        a64 = bg.generate(cfg64, 1 << 20, outputs=("amp2",))["amp2"]
        rel = ((a32 - a64).abs() / a64.abs())[live_helicities(hel, n, torch)]
        q = torch.quantile(rel.float(), torch.tensor([0.5, 0.9, 0.99], device=rel.device))
        extras["n8_fp32_vs_fp64_rel_err_p50_p90_p99"] = [float(x) for x in q]
        n12, N12 = 12, 1 << 22
        for prec in (32, 64):
            c12 = bg.config(n12, prec=prec, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000002)
            st = 3 if prec == 32 else 2
            w12, ms12, _ = run_steps(bg, torch, c12, N12, st, 1, outputs)
            extras[f"n12_fp{prec}_events_per_s"] = N12 * st / w12
            extras[f"n12_fp{prec}_launch_ms"] = sum(ms12) / len(ms12)
            extras[f"n12_fp{prec}_frac_plain"] = flops_plain(12) * N12 / (sum(ms12) / len(ms12) * 1e-3) / (PEAK_FP32 if prec == 32 else PEAK_FP64)
        # the W-tensor form of the recursion (Eqs. 3.3-3.4, 16 lanes per event)
        for nw, pw in ((12, 32), (10, 32), (10, 64)):
            cw = bg.config(nw, prec=pw, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000002)
            old = bg.get_form(nw, pw)
            bg.set_form(nw, pw, bg.FORM_WTENSOR)
            try:
                ww, msw, _ = run_steps(bg, torch, cw, 1 << 22, 2, 1, outputs)
            finally:
                bg.set_form(nw, pw, old)
            extras[f"n{nw}_fp{pw}_wtensor_events_per_s"] = (1 << 22) * 2 / ww
            extras[f"n{nw}_fp{pw}_wtensor_launch_ms"] = sum(msw) / len(msw)
        c12a = bg.config(12, prec=32, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000002)
        c12b = bg.config(12, prec=64, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=0xB6000002)
        r32 = bg.generate(c12a, 1 << 18, outputs=("amp2", "hel"))
        b64 = bg.generate(c12b, 1 << 18, outputs=("amp2",))["amp2"]
        rel = ((r32["amp2"] - b64).abs() / b64.abs())[live_helicities(r32["hel"], 12, torch)]
        q = torch.quantile(rel.float(), torch.tensor([0.5, 0.9, 0.99], device=rel.device))
        extras["n12_fp32_vs_fp64_rel_err_p50_p90_p99"] = [float(x) for x in q]
        # the paper's own sources: random real polarisation vectors (real currents)
        for nr, Nr in ((8, N), (12, 1 << 22)):
            cr = bg.config(nr, prec=32, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=BENCH_SEED[nr], polarisation=1)
            wr, msr, _ = run_steps(bg, torch, cr, Nr, 3, 1, outputs)
            lm = sum(msr) / len(msr)
            extras[f"n{nr}_realpol_fp32_events_per_s"] = Nr * 3 / wr
            extras[f"n{nr}_realpol_fp32_launch_ms"] = lm
            extras[f"n{nr}_realpol_fp32_frac_plain"] = flops_real(nr) * Nr / (lm * 1e-3) / PEAK_FP32
        # the dynamic scale mu = H_T (alpha_s and the density from grids)
        cd = bg.config(n, prec=32, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=BENCH_SEED[8], dynamic_scale=1)
        wd, msd, _ = run_steps(bg, torch, cd, N, 3, 1, outputs)
        extras["n8_dynamic_scale_fp32_events_per_s"] = N * 3 / wd
        line["recursion_kernel"] = recursion_rate(bg, torch)
        extras.update(hist_rate(bg, torch, out, N))
        extras.update(adjoint_rate(bg, torch))
        extras.update(adjoint_rate(bg, torch, N=1 << 18, steps=2, n=12, prec=32))
        extras.update(adjoint_rate(bg, torch, N=1 << 18, steps=2, n=12, prec=64))
        extras.update(mixed_rate(bg, torch))
        line["extras"] = extras

    if cpu is not None:
        line["cpu_baseline"] = cpu
    line["source_hash"] = bg.source_hash()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
