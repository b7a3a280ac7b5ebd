"""Which Philox words feed which random choice of one event.

The paper draws, per event, the RAMBO momenta (Sec. 3), the parton fractions
(Sec. 3, Eq. 3.8), the external polarisation states and a random colour ordering
{sigma_2..sigma_n} of {2..n} (Sec. 3, below Eq. 3.8).  This module fixes a layout
for those draws so that every event is a pure function of (seed, event index, n):

  key     = (seed mod 2**32, seed div 2**32)
  counter = (block, event mod 2**32, event div 2**32, n)
  block 0             : word 0 -> x1 uniform, word 1 -> x2 uniform,
                        word 2 -> helicity bits (bit i = 1: leg i has helicity +),
                        word 3 unused
  block 1 .. n-2      : the four RAMBO uniforms (rho1..rho4) of final gluon 3 .. n
  block n-1 ...       : shuffle words r_t, consumed for t = n-2, n-3, ..., 1
  block n_blocks(n)+k/4, word k%4 (real polarisations only): the angle of leg k,
                        psi_k = 2 pi u_k, k = 0 .. n-1

Colour ordering (Fisher-Yates on the 0-based legs 1..n-1, leg 0 always closes):
  a = [1, 2, ..., n-1];  for t = n-2 down to 1:  j = (r_t * (t+1)) >> 32; swap a[t], a[j]
  order = [0] + a.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32, uniform01


def n_blocks(n: int) -> int:
    nf = n - 2
    return 1 + nf + (n - 2 + 3) // 4


def angle_blocks(n: int) -> int:
    return (n + 3) // 4


def event_words(seed: int, events: np.ndarray, n: int, real_pol: bool = False) -> np.ndarray:
    """[B, 4*blocks] uint32 words of the given event indices (blocks = n_blocks, plus the
    angle blocks with real polarisations)."""
    events = np.asarray(events, dtype=np.uint64)
    B = events.shape[0]
    nb = n_blocks(n) + (angle_blocks(n) if real_pol else 0)
    ctr = np.zeros((B, nb, 4), dtype=np.uint64)
    ctr[:, :, 0] = np.arange(nb, dtype=np.uint64)[None, :]
    ctr[:, :, 1] = (events & np.uint64(0xFFFFFFFF))[:, None]
    ctr[:, :, 2] = (events >> np.uint64(32))[:, None]
    ctr[:, :, 3] = np.uint64(n)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    out = philox4x32(ctr.reshape(-1, 4), key)
    return out.reshape(B, nb * 4)


def polarisation_angles(words: np.ndarray, n: int) -> np.ndarray:
    """Words of event_words(..., real_pol=True) -> [B, n] angles psi_k = 2 pi u_k."""
    a = 4 * n_blocks(n)
    return 2.0 * np.pi * uniform01(words[:, a:a + n])


def split_draws(words: np.ndarray, n: int, random_order: bool = True):
    """Words -> (x uniforms [B,2], rho [B, n-2, 4], helicity word [B], order [B, n])."""
    B = words.shape[0]
    nf = n - 2
    ux = uniform01(words[:, 0:2])
    hel = (words[:, 2].astype(np.uint64) & np.uint64((1 << n) - 1)).astype(np.uint32)
    rho = uniform01(words[:, 4:4 + 4 * nf]).reshape(B, nf, 4)
    order = np.tile(np.arange(n, dtype=np.int64), (B, 1))
    if random_order:
        sw = words[:, 4 * (1 + nf):4 * (1 + nf) + (n - 2)].astype(np.uint64)
        a = order[:, 1:].copy()
        rows = np.arange(B)
        for k, t in enumerate(range(n - 2, 0, -1)):
            j = ((sw[:, k] * np.uint64(t + 1)) >> np.uint64(32)).astype(np.int64)
            at = a[:, t].copy()
            a[:, t] = a[rows, j]
            a[rows, j] = at
        order[:, 1:] = a
    return ux, rho, hel, order.astype(np.uint8)
