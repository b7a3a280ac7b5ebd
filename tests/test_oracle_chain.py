"""Pins for the n-dependence of the oracle's weight chain (Eqs. 3.7, 3.8), each against
something other than the oracle's own formulas:

* the full-colour squared amplitude, summed by brute force over every colour assignment
  with explicit SU(3) generators (T^a = lambda^a / sqrt 2, Tr(T^a T^b) = delta^ab) and
  the colour-ordered amplitudes of the recursion, equals the leading-colour form
  N^(n-2) (N^2-1) sum |A|^2 at n = 4 and n = 5 (Sec. 4: leading colour is exact there),
  and the spin- and colour-averaged result equals the mean of the oracle's per-event
  estimator over all helicities and orderings -- which pins 2^n, (n-1)!, g^(2(n-2)) and
  N^(n-2) at n = 5 as well as n = 4;
* the random-ordering identity behind the factor (n-1) of Eq. 3.8: the mean of
  (n-1) |A(1, sigma)|^2 over the generator's random orderings equals the sum over all
  orderings divided by (n-2)!, and that sum equals the sum over orderings closing on the
  last leg (the paper's form of the permutation sum);
* the massless k-body phase-space volume V_k of RAMBO's weight, k = 2..10, against the
  textbook recursive factorisation dPhi_k = dPhi_2 x dM^2 / (2 pi) x dPhi_(k-1),
  integrated numerically;
* the log integrand weight of the gradient path against the event weight itself.
"""
from itertools import permutations
from math import factorial, pi, sqrt

import numpy as np
import pytest
from scipy import integrate

from oracle import draws, event, pdf, recursion, weight
from oracle.rambo import volume
from paper_1002_3446_amd import inputs


def gell_mann():
    """The eight Gell-Mann matrices lambda^a (Tr(lambda^a lambda^b) = 2 delta^ab)."""
    l = np.zeros((8, 3, 3), dtype=complex)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / sqrt(3)
    l[7][2, 2] = -2 / sqrt(3)
    return l


def test_gell_mann_normalisation():
    T = gell_mann() / sqrt(2)
    tr = np.einsum("aij,bji->ab", T, T)
    assert np.allclose(tr, np.eye(8), atol=1e-15)
    # Casimir: sum_a T^a T^a = C_F 1 with C_F = (N^2 - 1)/(2N) * 2 = 8/3 in this normalisation
    assert np.allclose(np.einsum("aij,ajk->ik", T, T), (8.0 / 3.0) * np.eye(3), atol=1e-14)


def trace_tensor(n):
    """Tr(T^{a_1} ... T^{a_n}) for every colour assignment: complex [8]*n."""
    T = gell_mann() / sqrt(2)
    letters = "abcdefg"[:n]
    idx = "ijklmnop"
    terms = [letters[p] + idx[p] + idx[(p + 1) % n] for p in range(n)]
    return np.einsum(",".join(terms) + "->" + letters, *([T] * n))


def colour_matrix(n, orders):
    """C[s, t] = sum over colours of conj(Tr_s) Tr_t for the given orderings of legs 0..n-1."""
    base = trace_tensor(n)
    letters = "abcdefg"[:n]
    cols = []
    for o in orders:
        sub = "".join(letters[l] for l in o)
        cols.append(np.einsum(sub + "->" + letters, base).reshape(-1))
    C = np.array(cols)
    return C.conj() @ C.T


def points(n, B, seed, rs=1000.0):
    u = inputs.rambo_uniforms(seed, B, n).reshape(B, n - 2, 4)
    mom, _ = event.kinematics(event.config(n=n, use_pdf=0, sqrt_s=rs), u, None)
    return mom


def ordered_amplitudes(mom, word, orders):
    """Colour-ordered amplitudes A(sigma) (|A|^2 in the Parke-Taylor normalisation) for
    every ordering, sharing one set of polarisation vectors: [B, len(orders)] complex."""
    B, n = mom.shape[:2]
    k, eps = event.ordered_legs(mom, np.full(B, word, dtype=np.uint32), np.tile(np.arange(n), (B, 1)))
    out = []
    for o in orders:
        o = list(o)
        m = recursion.ordered_amplitude(k[:, o], eps[:, o])
        out.append(m * 2.0 ** (-(n - 2) / 2))
    return np.stack(out, axis=1)


@pytest.mark.parametrize("n", [4, 5])
def test_full_colour_brute_force(n):
    N, alpha_s = 3.0, 0.118
    g2 = 4 * pi * alpha_s
    orders = [(0,) + p for p in permutations(range(1, n))]
    CM = colour_matrix(n, orders)
    mom = points(n, B=6, seed=31 + n)
    B = mom.shape[0]
    full = np.zeros(B)
    lead = np.zeros(B)
    est = np.zeros(B)
    for word in range(1 << n):
        A = ordered_amplitudes(mom, word, orders)
        full += np.real(np.einsum("bs,st,bt->b", A.conj(), CM, A))
        a2 = np.abs(A) ** 2
        lead += N ** (n - 2) * (N * N - 1) * a2.sum(1)
        est += weight.me_estimate(a2, n, alpha_s).sum(1)
    # leading colour is exact for four and five gluons
    assert np.allclose(full, lead, rtol=1e-11), np.max(np.abs(full / lead - 1))
    # spin (1/4) and colour (1/(N^2-1)^2) averaged |M|^2 = mean of the per-event estimator
    averaged = g2 ** (n - 2) * full / (4 * (N * N - 1) ** 2)
    mean_est = est / ((1 << n) * factorial(n - 1))
    assert np.allclose(mean_est, averaged, rtol=1e-11), np.max(np.abs(mean_est / averaged - 1))


@pytest.mark.parametrize("n", [5, 6])
def test_random_ordering_identity(n):
    mom = points(n, B=4, seed=41 + n)
    B = mom.shape[0]
    word = 0b10110 if n == 5 else 0b101100
    orders = [(0,) + p for p in permutations(range(1, n))]
    a2 = np.abs(ordered_amplitudes(mom, word, orders)) ** 2        # [B, (n-1)!]
    exact = a2.sum(1) / factorial(n - 2)
    # the same permutation sum with the last leg closing (the paper's form, Eq. 3.6)
    last = [tuple(p) + (n - 1,) for p in permutations(range(n - 1))]
    rot = [o[-1:] + o[:-1] for o in last]                           # cyclic: closing leg first
    a2_last = np.abs(ordered_amplitudes(mom, word, rot)) ** 2
    assert np.allclose(a2_last.sum(1), a2.sum(1), rtol=1e-12)
    # the generator's Fisher-Yates orderings (Philox draws), many per point
    M = 40000
    w = draws.event_words(97, np.arange(M), n)
    _, _, _, ords = draws.split_draws(w, n, True)
    index = {o: i for i, o in enumerate(orders)}
    pick = np.array([index[tuple(int(v) for v in o)] for o in ords])
    counts = np.bincount(pick, minlength=len(orders))
    for b in range(B):
        x = (n - 1) * a2[b, pick]
        mc, err = x.mean(), x.std() / sqrt(M)
        assert abs(mc - exact[b]) < 4.5 * err, (b, mc, exact[b], err)
    # every ordering is reached, with multinomial spread
    exp_c = M / len(orders)
    assert counts.min() > 0 and np.all(np.abs(counts - exp_c) < 6 * sqrt(exp_c))


def _volume_step(k, s):
    """int_0^s dM^2/(2 pi) dPhi_2(s; M^2, 0) V_(k-1)(M^2): one step of the factorisation, with
    the two-body volume of one massive and one massless particle, (1 - M^2/s) / (8 pi)."""
    f = lambda m2: (1.0 - m2 / s) / (8 * pi) * volume(k - 1, m2) / (2 * pi)
    v, _ = integrate.quad(f, 0.0, s, epsabs=0.0, epsrel=1e-12, limit=200)
    return v


@pytest.mark.parametrize("k", [3, 4, 5, 6, 8, 10])
def test_phase_space_volume_recursion(k):
    """Induction on k from V_2 = 1/(8 pi): each V_k is the factorisation integral of V_(k-1)."""
    for s in (7.3e5, 2.0e8):
        assert abs(_volume_step(k, s) / volume(k, s) - 1) < 1e-10


def test_phase_space_volume_two_body_closed_forms():
    # k = 2: int d^3p1 d^3p2 / ((2pi)^6 4 E1 E2) (2pi)^4 delta^4 = 1/(8 pi), independent of s
    assert abs(volume(2, 3.0) * 8 * pi - 1) < 1e-15
    assert abs(volume(2, 1e6) * 8 * pi - 1) < 1e-15


@pytest.mark.parametrize("n", [5, 8])
def test_log_weight_int_matches_weight(n):
    cfg = event.config(n=n, seed=0xB6000001 + n)
    o = event.generate(cfg, np.arange(30000))
    sel = o["pass_"] & (o["amp2"] > 0)
    assert sel.sum() > 20
    u = o["rho"].reshape(len(o["rho"]), -1)
    lw = event.log_weight_int(cfg, u[sel], o["x12"][sel], o["hel"][sel], o["order"][sel])
    a, b, tau = cfg["pdf_a"], int(cfg["pdf_b"]), cfg["tau_min"]
    x1, x2 = o["x12"][sel, 0], o["x12"][sel, 1]
    Z = pdf.norm(tau, a, b)
    w = np.exp(lw) * Z * Z / (pdf.density(x1, a, b) * pdf.density(x2, a, b))
    assert np.allclose(w, o["weight"][sel], rtol=1e-12)
