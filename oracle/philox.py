"""Philox-4x32-10 counter-based generator, restated from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).

The paper does not name its generator; it only requires that the number of draws
stay far below the generator's period (Sec. 4).  Philox is counter based, so any
event's draws can be recomputed from (seed, event index) alone.

One round maps a 128-bit counter (c0, c1, c2, c3) under a 64-bit key (k0, k1) to
  (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
and the key is advanced by the Weyl constants (W0, W1) between rounds.

Pinned word for word against the independent implementation in ROCm's rocRAND
headers (tests/test_oracle_philox.py, 2^14 counter/key pairs), plus structural and
statistical checks.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF
ROUNDS = 10


def philox4x32(ctr: np.ndarray, key: np.ndarray, rounds: int = ROUNDS) -> np.ndarray:
    """ctr [B, 4] and key [B, 2] (or [2]) of 32-bit words -> [B, 4] uint32."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.broadcast_to(np.asarray(key, dtype=np.uint64), ctr.shape[:-1] + (2,))
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = key[..., 0].copy(), key[..., 1].copy()
    m = np.uint64(MASK)
    for r in range(rounds):
        p0 = np.uint64(M0) * c0          # < 2**64: exact 32x32 -> 64 product
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & m
        k1 = (k1 + np.uint64(W1)) & m
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def uniform01(r: np.ndarray) -> np.ndarray:
    """32-bit word -> double (r + 1/2) / 2**32, exact and strictly inside (0, 1)."""
    return (np.asarray(r, dtype=np.float64) + 0.5) * 2.0**-32
