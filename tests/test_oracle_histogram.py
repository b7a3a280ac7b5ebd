"""Pins for the oracle's histogram (oracle/histogram.py): bins against a brute-force
assignment with exact rational edges away from the edges themselves, totals against the
sum over all events, and exact sums against rational arithmetic."""
from fractions import Fraction

import numpy as np

from oracle import histogram


def test_bins_match_exact_edges():
    rng = np.random.default_rng(1)
    lo, hi, nb = 0.4, 4.0, 36
    x = np.concatenate([rng.uniform(-1, 6, 5000), [np.nan, np.inf, -np.inf, lo, hi]])
    b = histogram.bin_index(x, lo, hi, nb)
    w = (Fraction(hi) - Fraction(lo)) / nb
    for xi, bi in zip(x, b):
        if xi < lo:                      # -inf included
            assert bi == 0
            continue
        if not np.isfinite(xi) or xi >= hi:
            assert bi == nb + 1
            continue
        t = (Fraction(xi) - Fraction(lo)) / w
        if abs(t - round(t)) < Fraction(1, 10**9):
            continue                     # within rounding of an edge: either neighbour
        assert bi == int(t) + 1


def test_totals_and_exact_sums():
    rng = np.random.default_rng(2)
    w = rng.lognormal(0, 5, 3000) * (rng.random(3000) < 0.7)
    x = rng.uniform(0, 2000, 3000)
    h = histogram.histogram(w, x, 0.0, 1500.0, 30)
    exact_all = sum(Fraction(v) for v in w)
    assert abs(Fraction(float(h[:, 0].sum())) - exact_all) <= exact_all * Fraction(2 ** -50)
    b = histogram.bin_index(x, 0.0, 1500.0, 30)
    for k in (0, 1, 15, 31):
        ex = sum(Fraction(v) for v, bi in zip(w, b) if bi == k and v != 0)
        ex2 = sum(Fraction(v * v) for v, bi in zip(w, b) if bi == k and v != 0)
        assert h[k, 0] == float(ex) and h[k, 1] == float(ex2)
