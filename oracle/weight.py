"""Event weight and compensated summation.

Leading colour (Eq. 3.7): sum over colours of |amplitude|^2 = g^(2(n-2)) N^(n-2) (N^2-1)
sum over the (n-1)! orderings with leg 1 fixed of |A|^2, up to O(1/N^2).
Averaging over 4 initial helicity states and (N^2-1)^2 initial colours, and drawing
the helicities uniformly from 2^n states and the ordering uniformly from (n-1)!,
the per-event estimate of the averaged |M|^2 is
   2^n (n-1)! |A(1, sigma; h)|^2 g^(2(n-2)) N^(n-2) (N^2-1) / (4 (N^2-1)^2).
Hadronic cross section (Eq. 3.8): flux 1/(4 p1.p2) = 1/(2 s_hat), the identical-gluon
factor 1/(n-2)! (which with (n-1)! gives the paper's factor n-1), the RAMBO weight
V_{n-2}(s_hat), the density ratio f(x1) f(x2) / (p(x1) p(x2)) = Z^2 for x ~ p = f/Z,
and (hbar c)^2 = 0.3893793721e9 pb GeV^2.  Failing events get exactly 0.

Summation (Sec. 4): the paper uses Kahan's compensated sum; this is the
Neumaier (Kahan-Babuska) variant, in event order.
"""
from __future__ import annotations

from math import factorial, pi

import numpy as np

from .rambo import volume

NC = 3.0
HBARC2_PB = 0.3893793721e9


def me_estimate(amp2, n: int, alpha_s: float):
    """Spin- and colour-averaged leading-colour |M|^2 estimate from one |A(1,sigma;h)|^2."""
    g2 = 4.0 * pi * alpha_s
    col = g2 ** (n - 2) * NC ** (n - 2) * (NC * NC - 1.0) / (4.0 * (NC * NC - 1.0) ** 2)
    return 2.0 ** n * factorial(n - 1) * amp2 * col


def weight(amp2, s_hat, n: int, alpha_s: float, pdf_ratio, passed):
    """Event weight in pb."""
    w = pdf_ratio / (2.0 * s_hat) * volume(n - 2, s_hat) / factorial(n - 2) \
        * me_estimate(amp2, n, alpha_s) * HBARC2_PB
    return np.where(passed, w, 0.0)


def neumaier(xs):
    """Compensated sum of a 1-d float64 sequence, in order: returns (sum, compensation)."""
    s = 0.0
    c = 0.0
    for x in np.asarray(xs, dtype=np.float64).tolist():
        t = s + x
        if abs(s) >= abs(x):
            c += (s - t) + x
        else:
            c += (x - t) + s
        s = t
    return s, c
