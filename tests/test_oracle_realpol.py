"""Pins for the oracle's random real polarisations (the paper's choice of sources, Sec. 3):
the transverse basis, the relation to the helicity vectors, gauge invariance of the real
amplitude, and -- the point of the estimator -- that 2^n |A(eps_psi)|^2 averaged over the
angles equals the helicity sum: |A|^2 is a trigonometric polynomial of degree two in each
angle, so the average over three equally spaced angles per leg is exact (3^n evaluations),
compared with the sum over all 2^n helicities, and at n = 4 with the textbook gg -> gg
|M|^2; plus the cross section of a Monte Carlo run against the helicity mode's."""
from itertools import permutations, product
from math import pi, sqrt

import numpy as np
import pytest
from scipy import stats

from oracle import draws, event, recursion
from oracle.helicity import linear_polarisation, polarisation, transverse_basis
from oracle.recursion import mdot
from paper_1002_3446_amd import inputs


def points(n, B, seed, rs=1000.0):
    u = inputs.rambo_uniforms(seed, B, n).reshape(B, n - 2, 4)
    mom, _ = event.kinematics(event.config(n=n, use_pdf=0, sqrt_s=rs), u, None)
    return mom


def test_transverse_basis():
    mom = points(6, 50, 3)
    e1, e2 = transverse_basis(mom)
    for a, b, v in ((e1, e1, -1.0), (e2, e2, -1.0), (e1, e2, 0.0)):
        assert np.allclose(mdot(a, b), v, atol=1e-14)
    assert np.allclose(mdot(e1, mom) / mom[..., 0], 0, atol=1e-14)
    assert np.allclose(mdot(e2, mom) / mom[..., 0], 0, atol=1e-14)
    for h in (1.0, -1.0):
        eh = polarisation(mom, np.full(mom.shape[:2], h))
        assert np.allclose(eh, (-h * e1 - 1j * e2) / sqrt(2), atol=1e-15)
    psi = np.random.default_rng(1).uniform(0, 2 * pi, mom.shape[:2])
    ep = linear_polarisation(mom, psi)
    assert np.allclose(mdot(ep, ep), -1.0, atol=1e-14) and np.isrealobj(ep)


def _amp2_real(mom, psi, order):
    return event.amp2_real(mom, psi, order)


@pytest.mark.parametrize("n", [4, 5, 6])
def test_angle_average_equals_helicity_sum(n):
    mom = points(n, B=3, seed=20 + n)
    B = mom.shape[0]
    order = inputs.orderings(20 + n, B, n)
    hsum = sum(event.amp2(mom, np.full(B, w, dtype=np.uint32), order) for w in range(1 << n))
    off = np.random.default_rng(n).uniform(0, 2 * pi, n)
    avg = np.zeros(B)
    for ks in product(range(3), repeat=n):
        psi = np.tile(off + 2 * pi * np.array(ks) / 3.0, (B, 1))
        avg += _amp2_real(mom, psi, order)
    avg /= 3 ** n
    assert np.allclose(2 ** n * avg, hsum, rtol=1e-11), np.abs(2 ** n * avg / hsum - 1).max()


def test_textbook_gg_to_gg_with_real_polarisations():
    """n = 4: (1/256) g^4 N^2 (N^2-1) 2^4 sum_sigma <|A(1,sigma;eps_psi)|^2>_psi equals the
    textbook averaged |M|^2 = g^4 (9/2)(3 - tu/s^2 - su/t^2 - st/u^2)."""
    n = 4
    mom = points(n, B=8, seed=11)
    B = mom.shape[0]
    tot = np.zeros(B)
    for p in permutations([1, 2, 3]):
        order = np.tile(np.array((0,) + p), (B, 1))
        for ks in product(range(3), repeat=n):
            tot += _amp2_real(mom, np.tile(2 * pi * np.array(ks) / 3.0 + 0.3, (B, 1)), order) / 3 ** n
    N = 3.0
    lhs = N ** 2 * (N ** 2 - 1) * 2 ** n * tot / 256.0
    k = mom * np.array([-1.0, -1.0, 1.0, 1.0])[None, :, None]
    s = 2 * mdot(k[:, 0], k[:, 1])
    t = 2 * mdot(k[:, 0], k[:, 2])
    u = 2 * mdot(k[:, 0], k[:, 3])
    rhs = 4.5 * (3 - t * u / s**2 - s * u / t**2 - s * t / u**2)
    assert np.allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("n", [5, 8])
def test_real_amplitude_gauge_invariance(n):
    mom = points(n, B=20, seed=5 + n)
    B = mom.shape[0]
    rng = np.random.default_rng(n)
    psi = rng.uniform(0, 2 * pi, (B, n))
    eps = linear_polarisation(mom, psi)
    k = mom * np.array([-1.0, -1.0] + [1.0] * (n - 2))[None, :, None]
    m0 = recursion.ordered_amplitude(k, eps)
    for leg in (0, 1, n - 1):
        e2 = eps.copy()
        e2[:, leg] = e2[:, leg] + rng.normal(size=(B, 1)) * k[:, leg] / k[:, leg, :1]
        m1 = recursion.ordered_amplitude(k, e2)
        assert np.median(np.abs(m1 - m0) / np.abs(m0)) < 1e-12
    assert np.isrealobj(m0)


def test_angle_draws_uniform():
    n = 7
    w = draws.event_words(5, np.arange(20000), n, real_pol=True)
    psi = draws.polarisation_angles(w, n)
    assert psi.shape == (20000, n) and np.all((psi > 0) & (psi < 2 * pi))
    for k in range(n):
        assert stats.kstest(psi[:, k] / (2 * pi), "uniform").pvalue > 1e-4
    # the helicity, x and RAMBO words are those of the helicity mode
    w0 = draws.event_words(5, np.arange(20000), n)
    assert np.array_equal(w[:, :w0.shape[1]], w0)


def test_cross_section_same_as_helicity_mode():
    """A Monte Carlo cross section (n = 5, fixed energy) with real polarisations agrees with
    the helicity-mode estimate within their combined error."""
    res = {}
    for pol in (0, 1):
        cfg = event.config(n=5, use_pdf=0, sqrt_s=1000.0, seed=77, polarisation=pol)
        w = np.concatenate([event.generate(cfg, np.arange(i, i + 50000))["weight"] for i in range(0, 300000, 50000)])
        res[pol] = (w.mean(), w.std() / sqrt(len(w)))
    d = abs(res[0][0] - res[1][0])
    assert d < 4 * sqrt(res[0][1] ** 2 + res[1][1] ** 2), res
