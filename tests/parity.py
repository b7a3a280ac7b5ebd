"""Shared comparison rules for GPU-versus-oracle parity tests.

FP64 |A|^2 (the 1e-12 bar, read against the conditioning of each event):
  1. at least 96% of the non-vanishing events lie within 1e-12 relative of the float64
     oracle (measured: 97-100% for n = 4..12; uncut RAMBO points include soft and collinear
     ones where no two float64 evaluations in different operation orders agree that
     closely: the float64 oracle itself misses 1e-12 against its long-double value for
     1-2% of the events);
  2. measured against the oracle's long-double evaluation (64-bit mantissa), the GPU's
     relative-error quantiles (50, 90, 99%) are at most 4x those of the float64 oracle
     (+1e-16), and the 99.9% quantile at most 20x: the GPU is as accurate as a plain
     float64 evaluation (single extreme events differ by ~10x between any two
     equivalent operation orders, so the far tail gets the wider factor);
  3. no event is off by more than max(1e-9, 1e4 x the oracle's own error).
Helicity configurations whose amplitude vanishes identically (fewer than two minority
helicities) must come out below 1e-12 of the MHV size at the same point.
FP32 |A|^2: relative error against the long-double value, median <= 1e-4.
"""
from __future__ import annotations

import numpy as np

from oracle import event, recursion
from oracle.ops import NPLD

EPS = 2.0**-52


def lane_forms(n, prec):
    """Lanes-per-event forms the library holds for (n, prec): one lane for FP32 n <= 9 and
    FP64 n <= 6, two lanes for FP32 n >= 9 and FP64 n >= 6, four for FP64 n >= 10."""
    return [l for l, ok in ((1, n <= (9 if prec == 32 else 6)), (2, n >= (9 if prec == 32 else 6)),
                            (4, prec == 64 and n >= 10)) if ok]


def popcount(words, n):
    w = np.asarray(words, dtype=np.uint64)
    return np.array([bin(int(x) & ((1 << n) - 1)).count("1") for x in w])


def mhv_scale(mom):
    n = mom.shape[1]
    k = mom * np.array([-1.0, -1.0] + [1.0] * (n - 2))[None, :, None]
    return recursion.parke_taylor(k, 0, 1)


def oracle_amp2(mom, hel, order):
    """(float64 oracle, long-double oracle) |A|^2."""
    a64 = event.amp2(mom, hel, order)
    ald = event.amp2(np.asarray(mom, dtype=np.longdouble), hel, order, NPLD)
    return a64, ald


def check_amp2_fp64(gpu, mom, hel, order, extra_rel=None):
    """Asserts FP64 parity (rules 1-3 above); extra_rel [B] widens every bound by a known
    input difference (the inverse-CDF conditioning of x1, x2).  Returns statistics."""
    n = mom.shape[1]
    a64, ald = oracle_amp2(mom, hel, order)
    pc = popcount(hel, n)
    live = (pc >= 2) & (pc <= n - 2)
    scale = mhv_scale(mom)
    extra = np.zeros(len(gpu)) if extra_rel is None else np.asarray(extra_rel, dtype=np.float64)
    own = (np.abs(a64 - ald) / np.abs(ald)).astype(np.float64)
    err = np.maximum((np.abs(gpu - ald) / np.abs(ald)).astype(np.float64) - extra, 0.0)
    rel = np.abs(gpu - a64) / np.abs(a64)
    L = live
    frac = float(np.mean(rel[L] <= 1e-12 + extra[L]))
    assert frac >= 0.96, f"only {frac:.4f} of events within 1e-12 of the oracle"
    for q, fac in ((0.5, 4), (0.9, 4), (0.99, 4), (0.999, 20)):
        gq, oq = np.quantile(err[L], q), np.quantile(own[L], q)
        assert gq <= fac * oq + 1e-16, f"GPU error quantile {q}: {gq:.3e} vs float64 oracle {oq:.3e}"
    gross = L & (rel > np.maximum(1e-9, 1e4 * own) + extra)
    assert not gross.any(), f"{gross.sum()} events grossly off: worst {rel[gross].max():.3e}"
    dead = ~live
    if dead.any():
        assert np.all(np.abs(gpu[dead]) <= 1e-12 * scale[dead]), "vanishing helicities not ~0"
    ratio = err[L] / np.maximum(own[L], 1e-17)
    return dict(frac_within_1e12=frac, median=float(np.median(rel[L])), max=float(rel[L].max()),
                gpu_err_p99=float(np.quantile(err[L], 0.99)), oracle_err_p99=float(np.quantile(own[L], 0.99)),
                worst_ratio_to_oracle_err=float(ratio.max()))


def oracle_amp2_real(mom, psi, order):
    """(float64 oracle, long-double oracle) |A|^2 with real polarisations at angles psi."""
    a64 = event.amp2_real(mom, psi, order)
    u = np.asarray(psi, dtype=np.float64) / (2 * np.pi)          # the drawn uniforms
    psi_ld = 2 * NPLD.pi * np.asarray(u, dtype=np.longdouble)
    ald = event.amp2_real(np.asarray(mom, dtype=np.longdouble), psi_ld, order, NPLD)
    return a64, ald


def check_amp2_fp64_real(gpu, mom, psi, order, extra_rel=None):
    """FP64 parity (rules 1-3 above) for real polarisations, where no amplitude vanishes
    identically; returns statistics."""
    a64, ald = oracle_amp2_real(mom, psi, order)
    extra = np.zeros(len(gpu)) if extra_rel is None else np.asarray(extra_rel, dtype=np.float64)
    L = np.asarray(ald > 0)
    own = (np.abs(a64 - ald) / np.abs(ald)).astype(np.float64)
    err = np.maximum((np.abs(gpu - ald) / np.abs(ald)).astype(np.float64) - extra, 0.0)
    rel = np.abs(gpu - a64) / np.abs(a64)
    frac = float(np.mean(rel[L] <= 1e-12 + extra[L]))
    assert frac >= 0.96, f"only {frac:.4f} of events within 1e-12 of the oracle"
    for q, fac in ((0.5, 4), (0.9, 4), (0.99, 4), (0.999, 20)):
        gq, oq = np.quantile(err[L], q), np.quantile(own[L], q)
        assert gq <= fac * oq + 1e-16, f"GPU error quantile {q}: {gq:.3e} vs float64 oracle {oq:.3e}"
    gross = L & (rel > np.maximum(1e-9, 1e4 * own) + extra)
    assert not gross.any(), f"{gross.sum()} events grossly off: worst {rel[gross].max():.3e}"
    return dict(frac_within_1e12=frac, median=float(np.median(rel[L])), max=float(rel[L].max()))


def fp32_errors_real(gpu, mom, psi, order):
    _, ald = oracle_amp2_real(mom, psi, order)
    return (np.abs(gpu - ald) / np.abs(ald)).astype(np.float64)


def fp32_errors(gpu, mom, hel, order, scaled=False):
    """Relative FP32 error against the long-double value on the non-vanishing helicities;
    with scaled, also the error relative to max(|A|^2, the Parke-Taylor size of the event's
    own colour ordering with legs 0, 1 of opposite helicity), which stays bounded where
    |A|^2 sits near a zero of the amplitude and its relative error does not."""
    n = mom.shape[1]
    _, ald = oracle_amp2(mom, hel, order)
    live = (popcount(hel, n) >= 2) & (popcount(hel, n) <= n - 2)
    rel = (np.abs(gpu - ald) / np.abs(ald)).astype(np.float64)[live]
    if not scaled:
        return rel
    k = np.asarray(mom, dtype=np.float64) * np.array([-1.0, -1.0] + [1.0] * (n - 2))[None, :, None]
    ko = np.take_along_axis(k, np.asarray(order, dtype=np.int64)[:, :, None], axis=1)
    den = np.ones(len(k))
    for t in range(n):
        den = den * np.abs(2 * recursion.mdot(ko[:, t], ko[:, (t + 1) % n]))
    pt = (2 * recursion.mdot(k[:, 0], k[:, 1])) ** 4 / den
    ref = np.maximum(np.abs(ald).astype(np.float64), pt)
    return rel, (np.abs(gpu - ald).astype(np.float64) / ref)[live]
