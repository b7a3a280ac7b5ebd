"""Pins for the oracle's log-weight gradient: torch autograd of the plain code against
central finite differences (h = 1e-6), the closed form in x1, x2 (|A|^2 is boost
invariant and scales as s_hat^(4-n), so d log w / dx = (a-1)/x - b/(1-x)), and the sum
rules from azimuthal symmetry and RAMBO's scale invariance."""
import numpy as np
import pytest

from oracle import event
from paper_1002_3446_amd import inputs


def setup(n, B, seed):
    cfg = event.config(n=n, use_pdf=1)
    u = inputs.rambo_uniforms(seed, B, n)
    x = inputs.x_fractions(seed, B, 0.003)
    hel = inputs.helicity_words(seed, B, n)
    # keep non-vanishing helicity configurations (log of a zero is not differentiable)
    pc = np.array([bin(int(h)).count("1") for h in hel])
    hel = np.where((pc >= 2) & (pc <= n - 2), hel, np.uint32(0b11))
    order = inputs.orderings(seed, B, n)
    return cfg, u, x, hel, order


@pytest.mark.parametrize("n", [5, 8])
def test_grad_vs_central_differences(n):
    cfg, u, x, hel, order = setup(n, 16, 3)
    lw, gu, gx = event.log_weight_grad(cfg, u, x, hel, order)
    h = 1e-6
    fd_u = np.zeros_like(u)
    for j in range(u.shape[1]):
        up, um = u.copy(), u.copy()
        up[:, j] += h
        um[:, j] -= h
        fd_u[:, j] = (event.log_weight_int(cfg, up, x, hel, order) - event.log_weight_int(cfg, um, x, hel, order)) / (2 * h)
    fd_x = np.zeros_like(x)
    for j in range(2):
        xp, xm = x.copy(), x.copy()
        hx = h * x[:, j]
        xp[:, j] += hx
        xm[:, j] -= hx
        fd_x[:, j] = (event.log_weight_int(cfg, u, xp, hel, order) - event.log_weight_int(cfg, u, xm, hel, order)) / (2 * hx)
    scale = np.abs(gu).max(1, keepdims=True)
    assert np.median(np.abs(gu - fd_u) / scale) < 1e-6
    assert np.max(np.abs(gx - fd_x) / np.abs(gx)) < 1e-5


@pytest.mark.parametrize("n", [5, 8])
def test_grad_x_closed_form(n):
    cfg, u, x, hel, order = setup(n, 32, 4)
    _, _, gx = event.log_weight_grad(cfg, u, x, hel, order)
    a, b = cfg["pdf_a"], cfg["pdf_b"]
    ref = (a - 1) / x - b / (1 - x)
    assert np.max(np.abs(gx - ref) / np.abs(ref)) < 1e-8


@pytest.mark.parametrize("n", [5, 8])
def test_grad_sum_rules(n):
    cfg, u, x, hel, order = setup(n, 32, 5)
    _, gu, _ = event.log_weight_grad(cfg, u, x, hel, order)
    B = u.shape[0]
    rho = u.reshape(B, n - 2, 4)
    g = gu.reshape(B, n - 2, 4)
    scale = np.abs(gu).max(1)
    # a common azimuthal rotation of all final-state momenta leaves w unchanged
    assert np.median(np.abs(g[:, :, 1].sum(1)) / scale) < 1e-9
    # only the product rho3*rho4 enters each particle
    assert np.median(np.abs(rho[:, :, 2] * g[:, :, 2] - rho[:, :, 3] * g[:, :, 3]).max(1) / scale) < 1e-9
    # a common rescaling of RAMBO's q0 leaves the conformally mapped momenta unchanged
    q0 = -np.log(rho[:, :, 2] * rho[:, :, 3])
    assert np.median(np.abs((q0 * rho[:, :, 2] * g[:, :, 2]).sum(1)) / scale) < 1e-9
