"""Helicity polarisation vectors of the external gluons.

The paper's sources J[i] are polarisation vectors orthogonal to k_i (Sec. 3); it
uses random real unit vectors, whereas this path uses helicity states.  For a
physical momentum p with direction (sin t cos f, sin t sin f, cos t):
   eps_h(p) = (0, -h cos t cos f + i sin f, -h cos t sin f - i cos f, h sin t) / sqrt(2)
with (cos f, sin f) = (1, 0) when pT = 0.  Properties: eps.p = 0, eps_h.eps_h = 0,
eps_h.conj(eps_h) = -1.  The label h is the all-outgoing helicity: the vector is
built from the physical momentum p of every leg, incoming legs included.
"""
from __future__ import annotations

from .ops import NP64


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
