"""Jet cuts and observables (Sec. 4: pT > 20 GeV, |eta| < 2.5, Delta R > 0.4; H_T and
R_min = min Delta R_ij).  Failing events are flagged only; their matrix element is
still evaluated (Sec. 3).

On lab momenta of the final-state gluons:
  pT = sqrt(px^2 + py^2),  eta = asinh(pz / pT),  phi = atan2(py, px),
  Delta R_ij = sqrt(Delta eta^2 + Delta phi^2), Delta phi folded into [0, pi];
  pass = all(pT > pt_min) and all(|eta| < eta_max) and all(Delta R > dr_min), strict.
"""
from __future__ import annotations

import numpy as np


def cuts(p, pt_min, eta_max, dr_min):
    """p [B, k, 4] float64 final-state lab momenta -> dict(pass_, ht, rmin, pt, eta, phi, margin)."""
    px, py, pz = p[..., 1], p[..., 2], p[..., 3]
    pt = np.sqrt(px * px + py * py)
    with np.errstate(divide="ignore", invalid="ignore"):
        eta = np.arcsinh(pz / pt)
    phi = np.arctan2(py, px)
    k = p.shape[-2]
    drs = []
    for i in range(k):
        for j in range(i + 1, k):
            dphi = np.abs(phi[..., i] - phi[..., j])
            dphi = np.where(dphi > np.pi, 2 * np.pi - dphi, dphi)
            deta = eta[..., i] - eta[..., j]
            drs.append(np.sqrt(deta * deta + dphi * dphi))
    dr = np.stack(drs, axis=-1)
    ok = (pt > pt_min).all(-1) & (np.abs(eta) < eta_max).all(-1) & (dr > dr_min).all(-1)
    # distance of the decision from its nearest threshold, relative (for parity checks)
    with np.errstate(invalid="ignore"):
        margin = np.minimum(np.minimum(np.abs(pt - pt_min).min(-1) / pt_min,
                                       np.abs(np.abs(eta) - eta_max).min(-1) / eta_max),
                            np.abs(dr - dr_min).min(-1) / dr_min)
    return dict(pass_=ok, ht=pt.sum(-1), rmin=dr.min(-1), pt=pt, eta=eta, phi=phi, margin=margin)
