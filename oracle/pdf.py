"""Synthetic gluon density and its inverse-CDF sampler.

The paper folds the gluon densities F_g(x1) F_g(x2) into the hadronic integrand
(Sec. 3, Eq. 3.8) and reads them from LHAPDF grids (Sec. 3).  Here the density is
the synthetic f(x) = x^a (1-x)^b (a = -1.3, b = 5), truncated to [tau_min, 1) with
tau_min = (n_f * pT_min)^2 / S: below it no event can pass the jet cuts, because
the sum of the final-state transverse momenta never exceeds sqrt(s_hat).

For integer b >= 0 the primitive is the finite sum
   F(x) = sum_{k=0}^{b} C(b,k) (-1)^k x^(a+k+1) / (a+k+1).
Sampling solves F(x) - F(tau) = u * Z with Z = F(1) - F(tau) by Newton steps kept
inside a shrinking bisection bracket.
"""
from __future__ import annotations

from math import comb

import numpy as np


def density(x, a: float, b: int):
    return x ** a * (1.0 - x) ** b


def primitive(x, a: float, b: int):
    out = 0.0
    for k in range(b + 1):
        e = a + k + 1.0
        out = out + comb(b, k) * (-1.0) ** k * x ** e / e
    return out


def norm(tau: float, a: float, b: int) -> float:
    return float(primitive(1.0, a, b) - primitive(tau, a, b))


def sample(u: np.ndarray, tau: float, a: float, b: int, iters: int = 80) -> np.ndarray:
    """Inverse CDF of f on [tau, 1) at uniforms u (float64 arrays)."""
    u = np.asarray(u, dtype=np.float64)
    Ftau = primitive(tau, a, b)
    T = u * (primitive(1.0, a, b) - Ftau)
    lo = np.full_like(u, tau)
    hi = np.ones_like(u)
    # start from the leading power only: x^(a+1)/(a+1) - tau^(a+1)/(a+1) = T
    base = tau ** (a + 1.0) + (a + 1.0) * T
    with np.errstate(invalid="ignore", divide="ignore"):
        x = np.where(base > 0, np.abs(base) ** (1.0 / (a + 1.0)), 0.5 * (lo + hi))
    x = np.where((x > lo) & (x < hi), x, 0.5 * (lo + hi))
    for _ in range(iters):
        g = primitive(x, a, b) - Ftau - T
        hi = np.where(g > 0, x, hi)
        lo = np.where(g > 0, lo, x)
        xn = x - g / density(x, a, b)
        xn = np.where((xn > lo) & (xn < hi), xn, 0.5 * (lo + hi))
        x = xn
    return x


def tau_min(n: int, pt_min: float, sqrt_s: float) -> float:
    return ((n - 2) * pt_min / sqrt_s) ** 2
