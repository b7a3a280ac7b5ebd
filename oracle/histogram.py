"""Weighted histograms of an observable (TEST INFRASTRUCTURE ONLY, like all of oracle/).

The paper fills its distributions (Sec. 4, Fig. 3: H_T and R_min) on the CPU with
compensated sums.  The plain definition: bin b of an axis (lo, hi, nbins) collects the
events with lo + (b-1) (hi-lo)/nbins <= x < lo + b (hi-lo)/nbins, b = 1..nbins, with an
underflow bin 0 (x < lo) and an overflow bin nbins+1 (x >= hi, or x not a number); its
contents are sum w and sum w^2 over those events, here the exact sums rounded once
(math.fsum).  The bin of x is floor((x - lo) / (hi - lo) * nbins) + 1, evaluated in
float64 as written (so that an event exactly at an edge has one well-defined bin).
"""
from __future__ import annotations

import math

import numpy as np


def bin_index(x, lo: float, hi: float, nbins: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        t = (x - lo) / (hi - lo) * float(nbins)
        b = np.where(np.isfinite(t), np.floor(t), 0.0).astype(np.int64)
        b = np.minimum(b, nbins - 1) + 1
        b = np.where(x < lo, 0, b)
        b = np.where(~(x < hi), nbins + 1, b)
    return b


def histogram(weight, x, lo: float, hi: float, nbins: int) -> np.ndarray:
    """[nbins + 2, 2]: (sum w, sum w^2) per bin over the events with w != 0."""
    w = np.asarray(weight, dtype=np.float64)
    keep = w != 0.0
    b = bin_index(np.asarray(x)[keep], lo, hi, nbins)
    w = w[keep]
    out = np.zeros((nbins + 2, 2))
    order = np.argsort(b, kind="stable")
    b, w = b[order], w[order]
    edges = np.searchsorted(b, np.arange(nbins + 3))
    for k in range(nbins + 2):
        seg = w[edges[k]:edges[k + 1]]
        out[k, 0] = math.fsum(seg.tolist())
        out[k, 1] = math.fsum((seg * seg).tolist())
    return out
