"""Pins for the oracle's dynamic scale (oracle/scale.py): the one-loop coupling against its
renormalisation-group equation and its value at mu0; the grid interpolation against the
closed forms within the bound linear interpolation allows; and the event weight with
mu = H_T against the fixed-scale weight times the closed-form ratio."""
import math

import numpy as np
import pytest

from oracle import event, scale

A0, MU0 = 0.118, 91.188


def test_alpha_rge_and_reference_value():
    assert scale.alpha_exact(MU0, A0, MU0) == A0
    b0 = 23.0 / (12.0 * math.pi)
    for mu in (10.0, 91.188, 500.0, 5000.0):
        h = 1e-5
        d = (scale.alpha_exact(mu * math.exp(h), A0, MU0) - scale.alpha_exact(mu * math.exp(-h), A0, MU0)) / (2 * h)
        a = scale.alpha_exact(mu, A0, MU0)
        assert abs(d / (-2.0 * b0 * a * a) - 1) < 1e-8   # d alpha / d ln mu = -2 b0 alpha^2


def test_alpha_grid_within_interpolation_bound():
    g = scale.Grids(A0, MU0)
    mu = np.exp(np.random.default_rng(1).uniform(math.log(5.0), math.log(20000.0), 20000))
    ex = scale.alpha_exact(mu, A0, MU0)
    err = np.abs(g.alpha_at(mu) - ex)
    # |alpha''| in ln mu is 8 b0^2 alpha^3; linear interpolation errs by at most h^2/8 of it
    b0 = 23.0 / (12.0 * math.pi)
    h = (math.log(20000.0) - math.log(5.0)) / (scale.N_ALPHA - 1)
    bound = h * h / 8 * 8 * b0 * b0 * scale.alpha_exact(5.0, A0, MU0) ** 3
    assert err.max() <= bound and err.max() > 0


@pytest.mark.parametrize("da,db", [(-0.05, 0.4), (0.0, 0.0)])
def test_density_grid_within_interpolation_bound(da, db):
    a, b = -1.3, 5
    g = scale.Grids(A0, MU0, a, b, da, db)
    rng = np.random.default_rng(2)
    x = np.exp(rng.uniform(math.log(1e-6), 0.0, 20000))
    x = x[x < 1 - 1e-6]
    mu = np.exp(rng.uniform(math.log(5.0), math.log(20000.0), len(x)))
    ex = scale.lnf_exact(x, mu, a, b, da, db, MU0)
    err = np.abs(g.lnf_at(x, mu) - ex)
    # ln f is linear in ln mu (exact between mu nodes) and has |d^2/dy^2| = |A + B| x (1 - x)
    # <= |A + B| / 4 in y; the bilinear interpolation errs by at most h_y^2/8 of that
    L = np.log(mu / MU0)
    hy = (g.y[-1] - g.y[0]) / (scale.N_Y - 1)
    bound = hy * hy / 8 * np.abs((a + da * L) + (b + db * L)) / 4 * (1 + 1e-9) + 1e-12
    assert np.all(err <= bound), (err / bound).max()


def test_dynamic_weight_is_fixed_weight_times_ratio():
    base = dict(n=6, seed=9)
    fixed = event.generate(event.config(**base), np.arange(12000))
    dyn = event.generate(event.config(dynamic_scale=1, **base), np.arange(12000))
    sel = fixed["pass_"]
    assert sel.sum() > 50 and np.array_equal(sel, dyn["pass_"])
    mu = fixed["ht"][sel]
    x1, x2 = fixed["x12"][sel, 0], fixed["x12"][sel, 1]
    ratio = (scale.alpha_exact(mu, A0, MU0) / A0) ** 4 * np.exp(
        scale.lnf_exact(x1, mu, -1.3, 5, -0.05, 0.4, MU0) + scale.lnf_exact(x2, mu, -1.3, 5, -0.05, 0.4, MU0)
        - (-1.3 * np.log(x1 * x2) + 5 * np.log((1 - x1) * (1 - x2))))
    got = dyn["weight"][sel] / fixed["weight"][sel]
    assert np.allclose(got, ratio, rtol=2e-3)           # the grids' interpolation error
    assert np.all(dyn["weight"][~sel] == 0.0)
