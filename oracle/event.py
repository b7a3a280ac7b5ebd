"""Whole-event pipelines of the oracle.

generate():  draws (Philox) -> parton fractions -> RAMBO -> boost -> cuts and observables
             -> helicity vectors -> recursion -> |A|^2 -> weight   (Secs. 3 and 4)
             |A|^2 is a Lorentz scalar; it is evaluated on the partonic centre-of-mass
             momenta that RAMBO produces (before the boost), where no precision is lost
             to large rapidities.  Cuts and observables use the lab momenta.
amp2():      |A|^2 from given momenta, helicity word and colour ordering
log_weight_int() / log_weight_grad():
             log of the integrand weight without the cut step function and without the
             sampling density, as a function of the RAMBO uniforms and x1, x2; its
             gradient comes from torch autograd over the same plain code.

Configuration dictionaries use the keys of the C-ABI's bg_config:
  n, prec (ignored: the oracle is always double), sqrt_s, use_pdf, pdf_a, pdf_b,
  tau_min, alpha_s, pt_min, eta_max, dr_min, random_order, seed, first_event,
  polarisation (0: helicity states, 1: random real unit vectors, Sec. 3),
  dynamic_scale (1: alpha_s and the density at mu = H_T from grids), mu0, pdf_da, pdf_db.
"""
from __future__ import annotations

from math import factorial, lgamma, log, pi

import numpy as np

from . import cuts as _cuts
from . import draws, pdf, scale
from .helicity import linear_polarisation, polarisation
from .ops import NP64, TorchOps
from .rambo import beams, boost_z, rambo
from .recursion import amp2_from_m, mdot, ordered_amplitude
from .weight import HBARC2_PB, NC, weight

DEFAULTS = dict(prec=64, sqrt_s=14000.0, use_pdf=1, pdf_a=-1.3, pdf_b=5, tau_min=0.0,
                alpha_s=0.118, pt_min=20.0, eta_max=2.5, dr_min=0.4, random_order=1,
                seed=0, first_event=0, polarisation=0, dynamic_scale=0, mu0=91.188, pdf_da=-0.05,
                pdf_db=0.4)


def config(**kw) -> dict:
    c = dict(DEFAULTS)
    c.update(kw)
    if c["use_pdf"] and c["tau_min"] <= 0:
        c["tau_min"] = pdf.tau_min(c["n"], c["pt_min"], c["sqrt_s"])
    return c


def helicity_signs(hel, n: int):
    """uint32 word -> [B, n] of +1/-1 (bit i set: leg i has helicity +)."""
    bits = (np.asarray(hel, dtype=np.uint64)[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)
    return np.where(bits == 1, 1.0, -1.0)


def ordered_legs(mom, hel, order, ops=NP64):
    """Physical momenta [B, n, 4] -> (k_ord, eps_ord) in colour order; k all-outgoing."""
    n = mom.shape[1]
    h = ops.asarray(helicity_signs(hel, n))
    eps = polarisation(mom, h, ops)
    sign = ops.asarray(np.array([-1.0, -1.0] + [1.0] * (n - 2)))
    k = mom * sign[None, :, None]
    return ops.gather_legs(k, order), ops.gather_legs(eps, order)


def amp2(mom, hel, order, ops=NP64):
    """|A(sigma; h)|^2 (Parke-Taylor normalisation) from physical momenta [B, n, 4]."""
    mom = ops.asarray(mom)
    k, e = ordered_legs(mom, hel, order, ops)
    return amp2_from_m(ordered_amplitude(k, e), mom.shape[1], ops)


def amp2_real(mom, psi, order, ops=NP64):
    """|A(sigma; eps_psi)|^2 with real polarisation vectors at angles psi [B, n]."""
    mom = ops.asarray(mom)
    n = mom.shape[1]
    eps = linear_polarisation(mom, ops.asarray(psi), ops)
    sign = ops.asarray(np.array([-1.0, -1.0] + [1.0] * (n - 2)))
    k = mom * sign[None, :, None]
    m = ordered_amplitude(ops.gather_legs(k, order), ops.gather_legs(eps, order))
    return m * m * ops.const(2.0 ** -(n - 2))


def _cat(b, p):
    return np.concatenate([b, p], axis=1) if isinstance(p, np.ndarray) else __import__("torch").cat([b, p], dim=1)


def kinematics(cfg: dict, rho, x12, ops=NP64, cm=False):
    """RAMBO uniforms [B, n-2, 4] and x12 [B, 2] -> (lab momenta [B, n, 4], s_hat [B]);
    with cm=True also the partonic centre-of-mass momenta [B, n, 4]."""
    if cfg["use_pdf"]:
        x1, x2 = x12[:, 0], x12[:, 1]
        s_hat = x1 * x2 * cfg["sqrt_s"] ** 2
        pc = rambo(rho, ops.sqrt(s_hat), ops)
        p = boost_z(pc, x1, x2, ops)
        b = beams(x1, x2, cfg["sqrt_s"], ops)
        one = 1.0 + 0.0 * x1
        bc = beams(one, one, ops.sqrt(s_hat), ops)
    else:
        one = 1.0 + 0.0 * rho[:, 0, 0]
        s_hat = one * cfg["sqrt_s"] ** 2
        pc = p = rambo(rho, ops.sqrt(s_hat), ops)
        bc = b = beams(one, one, cfg["sqrt_s"], ops)
    if cm:
        return _cat(b, p), s_hat, _cat(bc, pc)
    return _cat(b, p), s_hat


def generate(cfg: dict, events) -> dict:
    """Full event generation for the given absolute event indices (float64)."""
    n = cfg["n"]
    real = bool(cfg.get("polarisation", 0))
    events = np.asarray(events, dtype=np.uint64)
    words = draws.event_words(cfg["seed"], events, n, real_pol=real)
    ux, rho, hel, order = draws.split_draws(words, n, bool(cfg["random_order"]))
    if cfg["use_pdf"]:
        a, b, tau = cfg["pdf_a"], int(cfg["pdf_b"]), cfg["tau_min"]
        x12 = np.stack([pdf.sample(ux[:, 0], tau, a, b), pdf.sample(ux[:, 1], tau, a, b)], axis=1)
        ratio = pdf.norm(tau, a, b) ** 2
    else:
        x12 = np.ones((len(events), 2))
        ratio = 1.0
    mom, s_hat, mom_cm = kinematics(cfg, rho, x12, cm=True)
    cut = _cuts.cuts(mom[:, 2:], cfg["pt_min"], cfg["eta_max"], cfg["dr_min"])
    psi = draws.polarisation_angles(words, n) if real else None
    a2 = amp2_real(mom_cm, psi, order) if real else amp2(mom_cm, hel, order)
    w = weight(a2, s_hat, n, cfg["alpha_s"], ratio, cut["pass_"])
    if cfg.get("dynamic_scale", 0):
        g = scale.Grids(cfg["alpha_s"], cfg["mu0"], cfg["pdf_a"], int(cfg["pdf_b"]), cfg["pdf_da"], cfg["pdf_db"],
                        bool(cfg["use_pdf"]))
        w = w * np.where(cut["pass_"], scale.weight_ratio(g, n, cut["ht"], x12[:, 0], x12[:, 1], cfg["alpha_s"],
                                                          cfg["pdf_a"], int(cfg["pdf_b"]), bool(cfg["use_pdf"])), 0.0)
    return dict(x12=x12, rho=rho, hel=hel, order=order, mom=mom, mom_cm=mom_cm, s_hat=s_hat, amp2=a2,
                weight=w, pass_=cut["pass_"], ht=cut["ht"], rmin=cut["rmin"],
                margin=cut["margin"], words=words, psi=psi)


def log_const(n: int, alpha_s: float) -> float:
    """log of the event-independent factors of the integrand weight."""
    g2 = 4.0 * pi * alpha_s
    nf = n - 2
    lv = (4 - 3 * nf) * log(2 * pi) + (nf - 1) * log(pi / 2) - lgamma(nf) - lgamma(nf - 1)
    lme = n * log(2.0) + lgamma(n) + (n - 2) * log(g2) + (n - 2) * log(NC) - log(4.0 * (NC * NC - 1.0))
    return lv - lgamma(n - 1) + lme + log(HBARC2_PB) - log(2.0)


def log_weight_int(cfg: dict, u, x12, hel, order, ops=NP64):
    """log w_int: log f(x1) + log f(x2) - log s_hat + log(s_hat^(n-4)) + log |A|^2 + const
    (the (2 pi, pi/2, factorial) parts of V_{n-2}, the flux 1/2 and the colour and
    helicity factors sit in log_const).  u [B, 4(n-2)], x12 [B, 2]."""
    n = cfg["n"]
    B = u.shape[0]
    rho = u.reshape(B, n - 2, 4)
    _, s_hat, mom_cm = kinematics(cfg, rho, x12, ops, cm=True)
    k, e = ordered_legs(mom_cm, hel, order, ops)
    m = ordered_amplitude(k, e)
    la2 = ops.log(amp2_from_m(m, n, ops))
    out = la2 + (n - 5) * ops.log(s_hat) + log_const(n, cfg["alpha_s"])
    if cfg["use_pdf"]:
        a, b = cfg["pdf_a"], int(cfg["pdf_b"])
        for i in range(2):
            x = x12[:, i]
            out = out + a * ops.log(x) + b * ops.log(1.0 - x)
    return out


def log_weight_grad(cfg: dict, u, x12, hel, order):
    """(log w_int [B], d/du [B, 4(n-2)], d/dx12 [B, 2]) via torch float64 autograd."""
    import torch
    ops = TorchOps()
    ut = torch.tensor(np.asarray(u, dtype=np.float64), requires_grad=True)
    xt = torch.tensor(np.asarray(x12, dtype=np.float64), requires_grad=True)
    lw = log_weight_int(cfg, ut, xt, hel, order, ops)
    lw.sum().backward()
    gx = xt.grad.numpy() if cfg["use_pdf"] else np.zeros_like(np.asarray(x12))
    return lw.detach().numpy(), ut.grad.numpy(), gx
