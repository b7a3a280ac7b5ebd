"""Pins for the oracle's event weight and compensated sum (Eqs. 3.7, 3.8; Sec. 4):
the n = 4 cross section with cuts from Monte Carlo over the oracle's own weights
against a one-dimensional quadrature of the textbook gg -> gg |M|^2; the hadronic
version against a three-dimensional quadrature with the synthetic density; and
Neumaier summation against exact rational sums."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

from oracle import event, pdf, weight
from oracle.weight import HBARC2_PB


def textbook_me(s, t, u, alpha_s):
    g2 = 4 * math.pi * alpha_s
    return g2 * g2 * 4.5 * (3 - t * u / s**2 - s * u / t**2 - s * t / u**2)


def sigma_hat_quad(rs, alpha_s, pt_min, eta_max):
    """(1/2s) (1/2!) int dPhi_2 |M|^2 with the cuts; dPhi_2 = dcos dphi / (32 pi^2)."""
    s = rs * rs
    cmax = min(math.tanh(eta_max), math.sqrt(max(0.0, 1 - (2 * pt_min / rs) ** 2)))
    f = lambda c: textbook_me(s, -s * (1 - c) / 2, -s * (1 + c) / 2, alpha_s)
    val, _ = integrate.quad(f, -cmax, cmax, limit=200)
    return HBARC2_PB / (2 * s) * 0.5 * (2 * math.pi) / (32 * math.pi**2) * val


def test_fixed_energy_cross_section_n4():
    cfg = event.config(n=4, use_pdf=0, sqrt_s=1000.0, seed=2024)
    N = 800000
    w = np.concatenate([event.generate(cfg, np.arange(i, i + 50000))["weight"] for i in range(0, N, 50000)])
    mc, err = w.mean(), w.std() / math.sqrt(N)
    ref = sigma_hat_quad(1000.0, 0.118, 20.0, 2.5)
    assert abs(mc - ref) < 4 * err, (mc, ref, err)
    assert err / ref < 0.02


@pytest.mark.slow
def test_hadronic_cross_section_n4():
    """With x1, x2 from the synthetic density, sigma = int dx1 dx2 f f sigma_hat(x1 x2 S)
    with the cuts applied in the lab frame (boost along z by y = ln(x1/x2)/2)."""
    S = 14000.0
    cfg = event.config(n=4, use_pdf=1, sqrt_s=S, seed=77)
    N = 150000
    w = np.concatenate([event.generate(cfg, np.arange(i, i + 50000))["weight"] for i in range(0, N, 50000)])
    mc, err = w.mean(), w.std() / math.sqrt(N)
    tau = cfg["tau_min"]
    a, b = cfg["pdf_a"], int(cfg["pdf_b"])
    f = lambda x: pdf.density(x, a, b)

    lt = math.log(tau)

    def over_c(y1, y2):
        # the cuts bound |cos theta*| by the pT and |eta| conditions (eta1,2 = y +- atanh c)
        x1, x2 = math.exp(y1), math.exp(y2)
        s = x1 * x2 * S * S
        y = 0.5 * (y1 - y2)
        if s <= (2 * 20.0) ** 2 or abs(y) >= 2.5:
            return 0.0
        cmax = min(math.sqrt(1 - (2 * 20.0) ** 2 / s), math.tanh(2.5 - abs(y)))
        me = lambda c: textbook_me(s, -s * (1 - c) / 2, -s * (1 + c) / 2, 0.118)
        v, _ = integrate.quad(me, -cmax, cmax, epsrel=1e-7)
        return x1 * x2 * f(x1) * f(x2) * HBARC2_PB / (2 * s) * 0.5 / (16 * math.pi) * v

    val, _ = integrate.dblquad(over_c, lt, 0.0, lambda y1: lt, lambda y1: 0.0, epsrel=1e-5)
    assert abs(mc - val) < 4 * err, (mc, val, err)


def test_neumaier_exact_on_adversarial():
    cases = [[1e16, 1.0, -1e16], [1.0, 1e100, 1.0, -1e100], [0.1] * 10 + [1e20, -1e20]]
    for xs in cases:
        s, c = weight.neumaier(xs)
        exact = float(sum(Fraction(x) for x in xs))
        assert s + c == exact


def test_neumaier_bound_and_fp32_failure():
    rng = np.random.default_rng(1)
    xs = rng.lognormal(0, 3, 200000)
    s, c = weight.neumaier(xs)
    exact = float(sum(Fraction(float(x)) for x in xs))
    assert abs((s + c) - exact) <= 2 * 2.0**-53 * np.abs(xs).sum()
    naive32 = np.float32(0)
    for x in xs.astype(np.float32):
        naive32 = np.float32(naive32 + x)
    assert abs(float(naive32) / exact - 1) > 1e-4   # a single-precision running sum drifts


def test_weight_zero_when_cut():
    a2 = np.array([1.0, 2.0])
    w = weight.weight(a2, np.array([1e6, 1e6]), 5, 0.118, 1.0, np.array([True, False]))
    assert w[1] == 0.0 and w[0] > 0
