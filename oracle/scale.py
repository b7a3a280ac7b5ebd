"""Running coupling and scale-dependent density for a dynamic scale (TEST INFRASTRUCTURE).

The paper reads alpha_s from a 1-D grid in the renormalisation scale and the gluon density
from a 2-D grid in (factorisation scale, x), interpolating linearly between nodes (Sec. 3),
and sets the scale of each event to H_T for its distributions (Sec. 4).  With the synthetic
density the grids are filled from closed forms:
  alpha_s(mu) = alpha_s(mu0) / (1 + alpha_s(mu0) b0 ln(mu^2/mu0^2)),  b0 = (33 - 2 n_f)/(12 pi),
                n_f = 5  (one-loop running, textbook)
  ln f(x, mu) = (a + da L) ln x + (b + db L) ln(1 - x),  L = ln(mu/mu0)
Nodes: alpha_s at 512 points uniform in ln mu over [5, 20000] GeV; ln f at 64 x 1024 points
uniform in ln mu (same range) and in y = ln(x/(1-x)) over x in [1e-6, 1 - 1e-9].  A point
between nodes takes the linear (alpha_s) or bilinear (ln f) interpolation of the node values;
points outside take the edge values.  The event weight then carries
  (alpha_s(mu)/alpha_s(mu0))^(n-2) f(x1, mu) f(x2, mu) / (f(x1, mu0) f(x2, mu0)),
the ratio to the fixed-scale factors, with mu = H_T.
"""
from __future__ import annotations

import math

import numpy as np

MU_LO, MU_HI = 5.0, 20000.0
X_LO, X_HI = 1e-6, 1.0 - 1e-9
N_ALPHA, N_MU, N_Y = 512, 64, 1024
NF = 5


def alpha_exact(mu, alpha0: float, mu0: float):
    b0 = (33.0 - 2.0 * NF) / (12.0 * math.pi)
    return alpha0 / (1.0 + alpha0 * b0 * np.log(np.asarray(mu, dtype=np.float64) ** 2 / mu0 ** 2))


def lnf_exact(x, mu, a: float, b: int, da: float, db: float, mu0: float):
    L = np.log(np.asarray(mu, dtype=np.float64) / mu0)
    x = np.asarray(x, dtype=np.float64)
    return (a + da * L) * np.log(x) + (b + db * L) * np.log1p(-x)


class Grids:
    """The node values of one configuration and their interpolation."""

    def __init__(self, alpha0, mu0, a=0.0, b=0, da=0.0, db=0.0, use_pdf=True):
        if not use_pdf:
            a, b, da, db = 0.0, 0, 0.0, 0.0
        self.lmu = np.linspace(math.log(MU_LO), math.log(MU_HI), N_ALPHA)
        self.lmu_pdf = np.linspace(math.log(MU_LO), math.log(MU_HI), N_MU)
        ylo = math.log(X_LO) - math.log1p(-X_LO)
        yhi = math.log(X_HI) - math.log1p(-X_HI)
        self.y = np.linspace(ylo, yhi, N_Y)
        self.alpha = alpha_exact(np.exp(self.lmu), alpha0, mu0)
        x = 1.0 / (1.0 + np.exp(-self.y))
        lx, l1x = -np.log1p(np.exp(-self.y)), -np.log1p(np.exp(self.y))
        L = self.lmu_pdf - math.log(mu0)
        self.lnf = (a + da * L)[:, None] * lx[None, :] + (b + db * L)[:, None] * l1x[None, :]
        self.x_nodes = x

    @staticmethod
    def _cell(v, nodes):
        lo, h = nodes[0], (nodes[-1] - nodes[0]) / (len(nodes) - 1)
        s = np.clip((np.asarray(v, dtype=np.float64) - lo) / h, 0.0, len(nodes) - 1.0)
        i = np.minimum(np.floor(s).astype(np.int64), len(nodes) - 2)
        return i, s - i

    def alpha_at(self, mu):
        i, t = self._cell(np.log(mu), self.lmu)
        return (1.0 - t) * self.alpha[i] + t * self.alpha[i + 1]

    def lnf_at(self, x, mu):
        x = np.asarray(x, dtype=np.float64)
        im, tm = self._cell(np.log(mu), self.lmu_pdf)
        iy, ty = self._cell(np.log(x) - np.log1p(-x), self.y)
        f0 = (1.0 - ty) * self.lnf[im, iy] + ty * self.lnf[im, iy + 1]
        f1 = (1.0 - ty) * self.lnf[im + 1, iy] + ty * self.lnf[im + 1, iy + 1]
        return (1.0 - tm) * f0 + tm * f1


def weight_ratio(grids: Grids, n: int, mu, x1, x2, alpha0: float, a: float, b: int, use_pdf: bool):
    """alpha_s(mu)^(n-2) f(x1, mu) f(x2, mu) over the same at mu0 (the sampled density)."""
    r = (n - 2) * (np.log(grids.alpha_at(mu)) - math.log(alpha0))
    if use_pdf:
        for x in (x1, x2):
            r = r + grids.lnf_at(x, mu) - (a * np.log(x) + b * np.log1p(-x))
    return np.exp(r)
