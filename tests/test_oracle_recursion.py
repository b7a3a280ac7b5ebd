"""Pins for the oracle's Berends-Giele recursion and closure (Eqs. 3.1, 3.2, 3.6):
Parke-Taylor closed form, vanishing helicity amplitudes, gauge invariance, the
paper's Ward diagnostic, cyclic / reflection / U(1)-decoupling identities, the
W-tensor form (Eqs. 3.3, 3.4), scaling and Lorentz invariance, and the textbook
n = 4 colour- and spin-summed |M|^2 (the absolute normalisation)."""
from itertools import permutations
from math import pi

import numpy as np
import pytest

from oracle import event, recursion
from oracle.helicity import polarisation
from oracle.ops import NPLD
from oracle.recursion import mdot
from paper_1002_3446_amd import inputs


def points(n, B=64, seed=1, rs=1000.0):
    u = inputs.rambo_uniforms(seed, B, n).reshape(B, n - 2, 4)
    cfg = event.config(n=n, use_pdf=0, sqrt_s=rs)
    mom, _ = event.kinematics(cfg, u, None)
    return mom


def outgoing(mom):
    n = mom.shape[1]
    return mom * np.array([-1.0, -1.0] + [1.0] * (n - 2))[None, :, None]


def hel_word(n, minus):
    return (1 << n) - 1 - sum(1 << i for i in minus)


def ident(B, n):
    return np.tile(np.arange(n), (B, 1))


def eps_of(mom, hel):
    return polarisation(mom, event.helicity_signs(hel, mom.shape[1]))


def live_mask(m, k, rel=1e-8):
    """events whose |m| is well above rounding noise, judged against the MHV size."""
    n = k.shape[1]
    scale = np.sqrt(recursion.parke_taylor(k, 0, 1) * 2.0 ** (n - 2))
    return np.abs(m) > rel * scale


def m_of(k, eps, order):
    """complex amplitude m for legs in the given colour order (position 0 closes)."""
    return recursion.ordered_amplitude(k[:, order], eps[:, order])


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 9, 10, 11, 12])
def test_parke_taylor(n):
    mom = points(n)
    B = mom.shape[0]
    k = outgoing(mom)
    rng = np.random.default_rng(n)
    for trial in range(4):
        i, j = sorted(rng.choice(n, 2, replace=False))
        for anti in (False, True):
            word = hel_word(n, [i, j]) if not anti else (1 << i) | (1 << j)
            a2 = event.amp2(mom, np.full(B, word, dtype=np.uint32), ident(B, n))
            rel = np.abs(a2 / recursion.parke_taylor(k, i, j) - 1)
            assert np.median(rel) < 1e-12 and np.quantile(rel, 0.9) < 1e-10, (n, i, j, rel.max())


@pytest.mark.parametrize("n", [4, 5, 6, 8, 12])
def test_vanishing_amplitudes(n):
    mom = points(n, seed=2)
    B = mom.shape[0]
    k = outgoing(mom)
    scale = recursion.parke_taylor(k, 0, 1)
    full = (1 << n) - 1
    for word in [full, 0, full - 1, full - (1 << (n - 1)), 1, 1 << 2]:
        a2 = event.amp2(mom, np.full(B, word, dtype=np.uint32), ident(B, n))
        assert np.median(a2 / scale) < 1e-22 and np.max(a2 / scale) < 1e-14


def test_n5_all_helicities_are_mhv_or_zero():
    n = 5
    mom = points(n, B=32, seed=4)
    B = mom.shape[0]
    k = outgoing(mom)
    for word in range(1 << n):
        minus = [i for i in range(n) if not (word >> i) & 1]
        plus = [i for i in range(n) if (word >> i) & 1]
        a2 = event.amp2(mom, np.full(B, word, dtype=np.uint32), ident(B, n))
        if len(minus) == 2 or len(plus) == 2:
            odd = minus if len(minus) == 2 else plus
            ref = recursion.parke_taylor(k, *odd)
            assert np.median(np.abs(a2 / ref - 1)) < 1e-12
        else:
            assert np.max(a2 / recursion.parke_taylor(k, 0, 1)) < 1e-14


@pytest.mark.parametrize("n", [5, 7, 10])
def test_gauge_invariance_shift(n):
    """eps_i -> eps_i + c k_i (a change of reference vector) leaves m unchanged."""
    mom = points(n, seed=5)
    B = mom.shape[0]
    hel = inputs.helicity_words(5, B, n)
    k = outgoing(mom)
    eps = eps_of(mom, hel)
    order = np.arange(n)
    m0 = m_of(k, eps, order)
    rng = np.random.default_rng(0)
    for leg in (0, 1, n - 1):
        c = (rng.normal(size=B) + 1j * rng.normal(size=B)) / mom[:, leg, 0]
        e2 = eps.copy()
        e2[:, leg] = e2[:, leg] + c[:, None] * k[:, leg]
        m1 = m_of(k, e2, order)
        rel = np.abs(m1 - m0) / np.abs(m0)
        ok = live_mask(m0, k)
        assert np.median(rel[ok]) < 1e-12


@pytest.mark.parametrize("n", [5, 8, 11])
def test_ward_diagnostic(n):
    """Replacing the closing polarisation by k_1 / E_1 gives zero (Sec. 4 diagnostic)."""
    mom = points(n, seed=6)
    B = mom.shape[0]
    hel = inputs.helicity_words(6, B, n)
    k = outgoing(mom)
    eps = eps_of(mom, hel)
    V, _, _ = recursion.currents(k[:, 1:], eps[:, 1:])
    m = mdot(eps[:, 0], V)
    w = mdot(k[:, 0] / mom[:, 0, 0:1], V)
    ratio = np.abs(w) ** 2 / np.abs(m) ** 2
    live = live_mask(m, k, 1e-3)
    assert np.median(ratio[live]) < 1e-24


@pytest.mark.parametrize("n", [4, 6, 9])
def test_cyclic_and_reflection(n):
    mom = points(n, seed=7)
    B = mom.shape[0]
    hel = inputs.helicity_words(7, B, n)
    k = outgoing(mom)
    eps = eps_of(mom, hel)
    base = np.arange(n)
    m0 = m_of(k, eps, base)
    scale = np.abs(m0) + 1e-300
    live = live_mask(m0, k)
    for shift in (1, 2, n - 1):
        m1 = m_of(k, eps, np.roll(base, -shift))
        assert np.median((np.abs(m1 - m0) / scale)[live]) < 1e-12
    refl = np.concatenate([[0], base[:0:-1]])
    m2 = m_of(k, eps, refl)
    assert np.median((np.abs(m2 - (-1) ** n * m0) / scale)[live]) < 1e-12


@pytest.mark.parametrize("n", [5, 6, 8])
def test_u1_decoupling(n):
    """sum of the orderings that insert leg 1 at every place among 2..n vanishes."""
    mom = points(n, seed=8)
    B = mom.shape[0]
    hel = inputs.helicity_words(8, B, n)
    k = outgoing(mom)
    eps = eps_of(mom, hel)
    rest = list(range(1, n))
    tot = 0
    mag = 0
    for pos in range(n - 1):
        order = np.array(rest[:pos] + [0] + rest[pos:])
        m = m_of(k, eps, order)
        tot = tot + m
        mag = mag + np.abs(m)
    live = live_mask(mag, k)
    assert np.median((np.abs(tot) / mag)[live]) < 1e-12


@pytest.mark.parametrize("n", [4, 6, 9])
def test_wtensor_form_matches(n):
    mom = points(n, seed=9)
    B = mom.shape[0]
    hel = inputs.helicity_words(9, B, n)
    k = outgoing(mom)
    eps = eps_of(mom, hel)
    V1, _, _ = recursion.currents(k[:, 1:], eps[:, 1:])
    V2 = recursion.currents_wtensor(k[:, 1:], eps[:, 1:])
    m1, m2 = mdot(eps[:, 0], V1), mdot(eps[:, 0], V2)
    live = live_mask(m1, k)
    assert np.median((np.abs(m1 - m2) / np.abs(m1))[live]) < 1e-12


@pytest.mark.parametrize("n", [5, 8])
def test_scaling_and_lorentz_invariance(n):
    mom = points(n, seed=10)
    B = mom.shape[0]
    hel = inputs.helicity_words(10, B, n)
    order = inputs.orderings(10, B, n)
    a0 = event.amp2(mom, hel, order)
    lam = 3.7
    a1 = event.amp2(lam * mom, hel, order)
    live = a0 > 1e-16 * recursion.parke_taylor(outgoing(mom), 0, 1)
    assert np.median(np.abs(a1 / (a0 * lam ** (2 * (4 - n))) - 1)[live]) < 1e-12
    # a general boost along x then a rotation about y
    b = 0.6
    g = 1 / np.sqrt(1 - b * b)
    Lx = np.array([[g, g * b, 0, 0], [g * b, g, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]])
    th = 0.7
    Ry = np.array([[1, 0, 0, 0], [0, np.cos(th), 0, np.sin(th)], [0, 0, 1, 0], [0, -np.sin(th), 0, np.cos(th)]])
    mom2 = mom @ (Ry @ Lx).T
    a2 = event.amp2(mom2, hel, order)
    assert np.median(np.abs(a2 / a0 - 1)[live]) < 1e-11


def test_textbook_gg_to_gg_absolute():
    """n = 4: (1/256) g^4 N^2 (N^2-1) sum_h sum_sigma |A(1,sigma;h)|^2 equals the
    textbook averaged |M|^2 = g^4 (9/2)(3 - tu/s^2 - su/t^2 - st/u^2)."""
    n = 4
    mom = points(n, B=16, seed=11)
    B = mom.shape[0]
    tot = np.zeros(B)
    for word in range(16):
        for p in permutations([1, 2, 3]):
            order = np.tile(np.array((0,) + p), (B, 1))
            tot += event.amp2(mom, np.full(B, word, dtype=np.uint32), order)
    g4 = 1.0
    N = 3.0
    lhs = g4 * N**2 * (N**2 - 1) * tot / 256.0
    k = outgoing(mom)
    s = 2 * mdot(k[:, 0], k[:, 1])
    t = 2 * mdot(k[:, 0], k[:, 2])
    u = 2 * mdot(k[:, 0], k[:, 3])
    rhs = g4 * 4.5 * (3 - t * u / s**2 - s * u / t**2 - s * t / u**2)
    assert np.allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("n", [6, 10])
def test_long_double_ground_truth(n):
    """The float64 oracle agrees with its own long-double evaluation (64-bit mantissa)
    on non-vanishing helicities for nearly all events."""
    mom = points(n, B=400, seed=12)
    B = mom.shape[0]
    hel = inputs.helicity_words(12, B, n)
    order = inputs.orderings(12, B, n)
    pc = np.array([bin(int(h)).count("1") for h in hel])
    nz = (pc >= 2) & (pc <= n - 2)
    a64 = event.amp2(mom, hel, order)
    ald = event.amp2(mom.astype(np.longdouble), hel, order, NPLD)
    rel = (np.abs(a64 - ald) / np.abs(ald)).astype(np.float64)[nz]
    assert np.median(rel) < 1e-13 and np.mean(rel < 1e-12) > 0.95
