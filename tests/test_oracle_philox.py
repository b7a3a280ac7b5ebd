"""Pins for the oracle's generator and draw layout.

Philox's bit pattern is parity unpinned against published known-answer vectors (none
are available here); these checks pin what a plausible slip would break: every
counter word and key word must be mixed in (no collisions, full avalanche), the
output must be uniform, and the draw layout must give uniform permutations and
helicity bits.
"""
import itertools
from math import factorial

import numpy as np
from scipy import stats

from oracle import draws, philox


def test_uniform01_open_interval():
    r = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint32)
    u = philox.uniform01(r)
    assert u[0] == 0.5 * 2.0**-32 and u[-1] == 1.0 - 0.5 * 2.0**-32
    assert np.all((u > 0) & (u < 1))


def _ctrs(N):
    c = np.zeros((N, 4), dtype=np.uint64)
    c[:, 0] = np.arange(N)
    return c


def test_no_collisions_any_counter_word():
    # counters that differ in only one word must give different outputs, for each word
    key = np.array([123, 456], dtype=np.uint64)
    for w in range(4):
        c = np.zeros((4096, 4), dtype=np.uint64)
        c[:, w] = np.arange(4096)
        out = philox.philox4x32(c, key)
        assert len({tuple(r) for r in out.tolist()}) == 4096, f"counter word {w} not mixed"


def test_key_words_mixed():
    c = _ctrs(64)
    base = philox.philox4x32(c, np.array([1, 2], dtype=np.uint64))
    for k in ([2, 2], [1, 3]):
        other = philox.philox4x32(c, np.array(k, dtype=np.uint64))
        assert np.all(np.any(base != other, axis=1))


def test_avalanche():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64)
    key = np.array([0xDEADBEEF, 0x12345678], dtype=np.uint64)
    a = philox.philox4x32(c, key)
    for w in range(4):
        for bit in (0, 13, 31):
            c2 = c.copy()
            c2[:, w] ^= np.uint64(1 << bit)
            b = philox.philox4x32(c2, key)
            flips = np.unpackbits((a ^ b).view(np.uint8), axis=1).sum(1)
            assert abs(flips.mean() - 64) < 1.5, (w, bit, flips.mean())


def test_uniformity_chi2():
    out = philox.philox4x32(_ctrs(1 << 15), np.array([7, 9], dtype=np.uint64))
    bytes_ = out.view(np.uint8).ravel()
    counts = np.bincount(bytes_, minlength=256)
    p = stats.chisquare(counts).pvalue
    assert 1e-4 < p
    u = philox.uniform01(out.ravel())
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_rounds_matter():
    c = _ctrs(16)
    key = np.array([1, 1], dtype=np.uint64)
    assert not np.array_equal(philox.philox4x32(c, key, rounds=9), philox.philox4x32(c, key, rounds=10))


def test_block_count():
    assert [draws.n_blocks(n) for n in (4, 5, 8, 12)] == [1 + 2 + 1, 1 + 3 + 1, 1 + 6 + 2, 1 + 10 + 3]


def test_orderings_are_uniform_permutations():
    n = 5
    w = draws.event_words(99, np.arange(24000), n)
    _, rho, hel, order = draws.split_draws(w, n, True)
    assert np.all(order[:, 0] == 0)
    assert np.all(np.sort(order[:, 1:], axis=1) == np.arange(1, n))
    perms = {p: i for i, p in enumerate(itertools.permutations(range(1, n)))}
    idx = np.array([perms[tuple(r)] for r in order[:, 1:].tolist()])
    counts = np.bincount(idx, minlength=factorial(n - 1))
    assert stats.chisquare(counts).pvalue > 1e-4
    bits = (hel[:, None] >> np.arange(n)) & 1
    assert np.all(hel < (1 << n))
    assert np.all(np.abs(bits.mean(0) - 0.5) < 0.02)
    assert np.all((rho > 0) & (rho < 1))


def test_fixed_order_identity():
    w = draws.event_words(1, np.arange(10), 6)
    _, _, _, order = draws.split_draws(w, 6, False)
    assert np.all(order == np.arange(6))


def test_event_counter_high_word():
    # events beyond 2**32 must use the counter's third word
    a = draws.event_words(3, np.array([5], dtype=np.uint64), 5)
    b = draws.event_words(3, np.array([5 + (1 << 32)], dtype=np.uint64), 5)
    assert not np.array_equal(a, b)
