"""RAMBO flat massless phase space and the longitudinal boost to the lab frame.

The paper generates its final-state momenta with RAMBO (Sec. 1 and Sec. 3; Kleiss,
Stirling, Ellis 1986).  For k massless particles with total momentum (sqrt_s, 0):
  per particle, from (rho1, rho2, rho3, rho4):
     c = 2 rho1 - 1,  phi = 2 pi rho2,  q0 = -ln(rho3 rho4),
     q = q0 (sqrt(1-c^2) cos phi, sqrt(1-c^2) sin phi, c)
  Q = sum q,  M = sqrt(Q^2),  b = -Q_vec / M,  gamma = Q0 / M,  a = 1/(1+gamma),
  X = sqrt_s / M,
  p0 = X (gamma q0 + b.q),   p_vec = X (q_vec + b q0 + a (b.q) b).
Every point carries the same weight, the volume of massless k-body phase space
  V_k(s) = (2 pi)^(4-3k) (pi/2)^(k-1) s^(k-2) / ((k-1)! (k-2)!)
for the measure prod d^3p / ((2 pi)^3 2E) (2 pi)^4 delta^4.
Momenta are (E, px, py, pz) in GeV, metric (+,-,-,-).
"""
from __future__ import annotations

from math import factorial, pi

from .ops import NP64


def rambo(rho, sqrt_s, ops=NP64):
    """rho [B, k, 4] uniforms, sqrt_s [B] or scalar -> momenta [B, k, 4] in the CM frame."""
    r1, r2, r3, r4 = rho[..., 0], rho[..., 1], rho[..., 2], rho[..., 3]
    c = 2.0 * r1 - 1.0
    phi = 2.0 * ops.pi * r2
    q0 = -ops.log(r3 * r4)
    st = ops.sqrt(1.0 - c * c)
    qx = q0 * st * ops.cos(phi)
    qy = q0 * st * ops.sin(phi)
    qz = q0 * c
    Q0, Qx, Qy, Qz = q0.sum(-1), qx.sum(-1), qy.sum(-1), qz.sum(-1)
    M = ops.sqrt(Q0 * Q0 - Qx * Qx - Qy * Qy - Qz * Qz)
    bx, by, bz = -Qx / M, -Qy / M, -Qz / M
    gamma = Q0 / M
    a = 1.0 / (1.0 + gamma)
    X = sqrt_s / M
    bq = bx[..., None] * qx + by[..., None] * qy + bz[..., None] * qz
    E = X[..., None] * (gamma[..., None] * q0 + bq)
    px = X[..., None] * (qx + bx[..., None] * q0 + a[..., None] * bq * bx[..., None])
    py = X[..., None] * (qy + by[..., None] * q0 + a[..., None] * bq * by[..., None])
    pz = X[..., None] * (qz + bz[..., None] * q0 + a[..., None] * bq * bz[..., None])
    return ops.stack([E, px, py, pz], axis=-1)


def volume(k: int, s):
    """Massless k-body phase-space volume V_k(s)."""
    return (2 * pi) ** (4 - 3 * k) * (pi / 2) ** (k - 1) * s ** (k - 2) / (factorial(k - 1) * factorial(k - 2))


def boost_z(p, x1, x2, ops=NP64):
    """Boost CM momenta p [B, k, 4] to the lab, rapidity y = ln(x1/x2)/2:
    E' = E cosh y + pz sinh y,  pz' = pz cosh y + E sinh y, with
    cosh y = (x1+x2)/(2 sqrt(x1 x2)),  sinh y = (x1-x2)/(2 sqrt(x1 x2))."""
    r = 2.0 * ops.sqrt(x1 * x2)
    ch = ((x1 + x2) / r)[..., None]
    sh = ((x1 - x2) / r)[..., None]
    E, px, py, pz = p[..., 0], p[..., 1], p[..., 2], p[..., 3]
    return ops.stack([E * ch + pz * sh, px, py, pz * ch + E * sh], axis=-1)


def beams(x1, x2, sqrt_S, ops=NP64):
    """Incoming parton momenta p_i = x_i P_i with P_1,2 = (sqrt_S/2)(1, 0, 0, +-1): [B, 2, 4]."""
    e1 = 0.5 * sqrt_S * x1
    e2 = 0.5 * sqrt_S * x2
    z = 0.0 * e1
    p1 = ops.stack([e1, z, z, e1], axis=-1)
    p2 = ops.stack([e2, z, z, -e2], axis=-1)
    return ops.stack([p1, p2], axis=-2)
