"""Berends-Giele recursion for colour-ordered gluon currents, as printed in Sec. 3.

Eq. 3.1 (with the shorthand of Eq. 3.2):
  J[m..n] = 1/K[m..n]^2 * ( sum_{i=m}^{n-1} [ J[m..i], J[i+1..n] ]
                          + sum_{i=m}^{n-2} sum_{j=i+1}^{n-1} { J[m..i], J[i+1..j], J[j+1..n] } )
  K[m..n] = sum_{i=m}^{n} k_i
  [Ja, Jb] = 2 (Ja.Kb) Jb - 2 (Ka.Jb) Ja + (Ja.Jb)(Ka - Kb)
  {Ja, Jb, Jc} = 2 (Ja.Jc) Jb - (Ja.Jb) Jc - (Jc.Jb) Ja
Sources J[i] are the polarisation vectors and k_i the all-outgoing momenta
(sum of all n momenta = 0).

Closure (Eq. 3.6): the amputated current of the n-1 recursion legs is contracted with
the closing leg's polarisation, m = J[closing] . V, where V is the bracket sum of the
last level, never divided by its propagator (its K^2 vanishes by momentum
conservation).

Normalisation: the printed brackets carry coefficient 1 where the usual
colour-ordered Feynman rules (Tr(T^a T^b) = delta^ab) carry 1/sqrt(2) (three-gluon)
and 1/2 (four-gluon); so a current of k legs is (sqrt 2)^(k-1) times the usual one and
|m|^2 = 2^(n-2) |A|^2.  The squared partial amplitude reported is |A|^2 = 2^-(n-2) |m|^2,
the normalisation in which the MHV amplitude obeys the Parke-Taylor formula (pinned
by tests/test_oracle_recursion.py).
"""
from __future__ import annotations

import numpy as np

from .ops import NP64


def mdot(a, b):
    """Minkowski product over the last axis, metric (+,-,-,-), no conjugation."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def bracket3(Ja, Ka, Jb, Kb):
    """[Ja, Jb] of Eq. 3.2."""
    return (2.0 * mdot(Ja, Kb)[..., None] * Jb
            - 2.0 * mdot(Ka, Jb)[..., None] * Ja
            + mdot(Ja, Jb)[..., None] * (Ka - Kb))


def bracket4(Ja, Jb, Jc):
    """{Ja, Jb, Jc} of Eq. 3.2."""
    return (2.0 * mdot(Ja, Jc)[..., None] * Jb
            - mdot(Ja, Jb)[..., None] * Jc
            - mdot(Jc, Jb)[..., None] * Ja)


def currents(k, eps):
    """k [B, L, 4] real momenta and eps [B, L, 4] complex sources of the ordered
    recursion legs.  Returns (V, J, K): V the undivided bracket sum of the full span
    [0..L-1], and dicts of all currents J[(a, b)] and span momenta K[(a, b)]."""
    L = k.shape[1]
    J = {(i, i): eps[:, i] for i in range(L)}
    K = {(i, i): k[:, i] for i in range(L)}
    V = None
    for length in range(2, L + 1):
        for a in range(0, L - length + 1):
            b = a + length - 1
            K[(a, b)] = K[(a, b - 1)] + k[:, b]
            acc = 0.0
            for i in range(a, b):
                acc = acc + bracket3(J[(a, i)], K[(a, i)], J[(i + 1, b)], K[(i + 1, b)])
            for i in range(a, b - 1):
                for j in range(i + 1, b):
                    acc = acc + bracket4(J[(a, i)], J[(i + 1, j)], J[(j + 1, b)])
            if length < L:
                J[(a, b)] = acc / mdot(K[(a, b)], K[(a, b)])[..., None]
            else:
                V = acc
    return V, J, K


def ordered_amplitude(k_ord, eps_ord):
    """m of Eq. 3.6 for legs already in colour order; position 0 closes.
    k_ord [B, n, 4] all-outgoing momenta, eps_ord [B, n, 4] polarisations."""
    V, _, _ = currents(k_ord[:, 1:], eps_ord[:, 1:])
    return mdot(eps_ord[:, 0], V)


def amp2_from_m(m, n: int, ops=NP64):
    return (ops.real(m) ** 2 + ops.imag(m) ** 2) * ops.const(2.0 ** -(n - 2))


def ordered_amp2(k_ord, eps_ord, ops=NP64):
    n = k_ord.shape[1]
    return amp2_from_m(ordered_amplitude(k_ord, eps_ord), n, ops)


# ----------------------------------------------------------------------------
# Checks that are independent formulations, used only by the oracle's own tests.
# ----------------------------------------------------------------------------

def parke_taylor(k_ord, i: int, j: int):
    """|A|^2 of an MHV (or anti-MHV) configuration whose two odd-helicity legs sit at
    colour positions i, j:  s_ij^4 / prod_t |s_{t,t+1}| (cyclic), s_ab = 2 k_a.k_b."""
    n = k_ord.shape[1]
    s = lambda a, b: 2.0 * mdot(k_ord[:, a], k_ord[:, b])
    den = 1.0
    for t in range(n):
        den = den * np.abs(s(t, (t + 1) % n))
    return s(i, j) ** 4 / den


def _outer(a, b):
    return a[..., :, None] * b[..., None, :]


def _wdot(W, J):
    """(W . J)^mu = sum_nu W^{mu nu} g_{nu nu} J^nu."""
    g = np.array([1.0, -1.0, -1.0, -1.0])
    return (W * (g * J)[..., None, :]).sum(-1)


def currents_wtensor(k, eps):
    """The same V via the W-tensor form of Eqs. 3.3-3.4, with the propagator 1/K^2
    that the printed Eq. 3.3 leaves implicit:
      J[m..n] = 1/K^2 sum_i [ W[i+1..n].J[m..i] - W[m..i].J[i+1..n] ],
      W[m..n] = 2 J K - K J + sum_i ( J[m..i] J[i+1..n] - J[i+1..n] J[m..i] )."""
    L = k.shape[1]
    J = {(i, i): eps[:, i] for i in range(L)}
    K = {(i, i): k[:, i] for i in range(L)}
    W = {(i, i): 2.0 * _outer(J[(i, i)], K[(i, i)]) - _outer(K[(i, i)], J[(i, i)]) for i in range(L)}
    V = None
    for length in range(2, L + 1):
        for a in range(0, L - length + 1):
            b = a + length - 1
            K[(a, b)] = K[(a, b - 1)] + k[:, b]
            acc = 0.0
            for i in range(a, b):
                acc = acc + _wdot(W[(i + 1, b)], J[(a, i)]) - _wdot(W[(a, i)], J[(i + 1, b)])
            if length < L:
                J[(a, b)] = acc / mdot(K[(a, b)], K[(a, b)])[..., None]
                Wab = 2.0 * _outer(J[(a, b)], K[(a, b)]) - _outer(K[(a, b)], J[(a, b)])
                for i in range(a, b):
                    Wab = Wab + _outer(J[(a, i)], J[(i + 1, b)]) - _outer(J[(i + 1, b)], J[(a, i)])
                W[(a, b)] = Wab
            else:
                V = acc
    return V
