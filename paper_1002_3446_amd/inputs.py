"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle's checks.

This module holds random-number plumbing only: uniforms in (0,1), parton momentum
fractions drawn log-uniformly, helicity bit words and colour orderings.  None of the
method's arithmetic lives here (no phase space, no recursion, no weights), so both the
HIP path and the oracle can be fed from it without sharing any of the method's code.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, int(seed) >> 32, stream]))


def open_uniforms(seed: int, shape) -> np.ndarray:
    """float64 uniforms strictly inside (0,1): (r + 0.5) * 2**-32 for a 32-bit integer r."""
    r = _rng(seed, 1).integers(0, 2**32, size=shape, dtype=np.uint64)
    return (r.astype(np.float64) + 0.5) * 2.0**-32


def rambo_uniforms(seed: int, N: int, n: int) -> np.ndarray:
    """[N, 4*(n-2)] uniforms, four per final-state gluon."""
    return open_uniforms(seed, (N, 4 * (n - 2)))


def x_fractions(seed: int, N: int, tau_min: float) -> np.ndarray:
    """[N, 2] momentum fractions, log-uniform on [tau_min, 1)."""
    u = open_uniforms(seed + 7919, (N, 2))
    return np.exp(np.log(tau_min) * (1.0 - u))


def helicity_words(seed: int, N: int, n: int) -> np.ndarray:
    """[N] uint32 whose low n bits are uniform helicity bits."""
    r = _rng(seed, 2).integers(0, 2**n, size=N, dtype=np.uint64)
    return r.astype(np.uint32)


def orderings(seed: int, N: int, n: int, shuffle: bool = True) -> np.ndarray:
    """[N, n] uint8 colour orderings: column 0 is leg 0, the rest a permutation of 1..n-1."""
    base = np.tile(np.arange(n, dtype=np.uint8), (N, 1))
    if not shuffle:
        return base
    keys = _rng(seed, 3).random((N, n - 1))
    perm = np.argsort(keys, axis=1).astype(np.uint8) + 1
    base[:, 1:] = perm
    return base
