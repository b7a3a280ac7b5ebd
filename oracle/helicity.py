"""Polarisation vectors of the external gluons.

The paper's sources J[i] are polarisation vectors orthogonal to k_i (Sec. 3).  Two
choices are implemented, both from the transverse basis of a physical momentum p with
direction (sin t cos f, sin t sin f, cos t):
   e1(p) = (0, cos t cos f, cos t sin f, -sin t),   e2(p) = (0, -sin f, cos f, 0),
with (cos f, sin f) = (1, 0) when pT = 0; e1.p = e2.p = 0, e1.e1 = e2.e2 = -1, e1.e2 = 0.

Helicity states (the default):
   eps_h(p) = (-h e1 - i e2) / sqrt(2)
            = (0, -h cos t cos f + i sin f, -h cos t sin f - i cos f, h sin t) / sqrt(2).
Properties: eps.p = 0, eps_h.eps_h = 0, eps_h.conj(eps_h) = -1.  The label h is the
all-outgoing helicity: the vector is built from the physical momentum p of every leg,
incoming legs included.

Random real unit vectors (the paper's own choice, which makes every current real):
   eps_psi(p) = cos(psi) e1 + sin(psi) e2,   psi uniform in [0, 2 pi).
Averaged over psi, eps^mu eps^nu = (e1 e1 + e2 e2) / 2 = (1/2) sum_h eps_h^mu conj(eps_h)^nu,
so for n legs 2^n |A(eps_psi)|^2 averages to the helicity sum, the same factor 2^n as for
a uniformly drawn helicity.
"""
from __future__ import annotations

from .ops import NP64


def transverse_basis(p, ops=NP64):
    """(e1, e2) of physical momenta p [..., 4]: real [..., 4] each."""
    px, py, pz = p[..., 1], p[..., 2], p[..., 3]
    pt2 = px * px + py * py
    safe = pt2 > 0
    one = 1.0 + 0.0 * pt2
    ptd = ops.sqrt(ops.where(safe, pt2, one))
    pt = ops.where(safe, ptd, 0.0 * pt2)
    pa = ops.sqrt(pt2 + pz * pz)
    ct = pz / pa
    st = pt / pa
    cf = ops.where(safe, px / ptd, one)
    sf = ops.where(safe, py / ptd, 0.0 * pt)
    zero = 0.0 * pt
    return ops.stack([zero, ct * cf, ct * sf, -st], axis=-1), ops.stack([zero, -sf, cf, zero], axis=-1)


def linear_polarisation(p, psi, ops=NP64):
    """p [..., 4] physical momenta, psi [...] angles -> real [..., 4] unit vectors."""
    e1, e2 = transverse_basis(p, ops)
    return ops.cos(psi)[..., None] * e1 + ops.sin(psi)[..., None] * e2


def polarisation(p, h, ops=NP64):
    """p [..., 4] physical momenta, h [...] in {+1, -1} -> complex [..., 4]."""
    px, py, pz = p[..., 1], p[..., 2], p[..., 3]
    pt2 = px * px + py * py
    safe = pt2 > 0
    one = 1.0 + 0.0 * pt2
    # sqrt of a guarded argument keeps autograd finite on the beam axis (pT = 0)
    ptd = ops.sqrt(ops.where(safe, pt2, one))
    pt = ops.where(safe, ptd, 0.0 * pt2)
    pa = ops.sqrt(pt2 + pz * pz)
    ct = pz / pa
    st = pt / pa
    cf = ops.where(safe, px / ptd, one)
    sf = ops.where(safe, py / ptd, 0.0 * pt)
    r = 1.0 / ops.sqrt(ops.const(2.0))
    zero = 0.0 * pt
    e0 = ops.cplx(zero, zero)
    e1 = ops.cplx(-h * ct * cf * r, sf * r)
    e2 = ops.cplx(-h * ct * sf * r, -cf * r)
    e3 = ops.cplx(h * st * r, zero)
    return ops.stack([e0, e1, e2, e3], axis=-1)
