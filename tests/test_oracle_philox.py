"""Pins for the oracle's generator and draw layout.

Philox's bit pattern is pinned word for word against an independent implementation of
the published generator, the one in ROCm's rocRAND headers (compiled for the host from
tests/native/philox_ref.hip), on 2^14 random (counter, key) pairs, counters with high
words set and the all-zero / all-one inputs.  The structural checks pin what a plausible
slip would break independently of any reference: every counter word and key word must be
mixed in (no collisions, full avalanche), the output must be uniform, and the draw layout
must give uniform permutations and helicity bits.
"""
import itertools
import os
import shutil
import subprocess
from math import factorial

import numpy as np
import pytest
from scipy import stats

from oracle import draws, philox


def test_uniform01_open_interval():
    r = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint32)
    u = philox.uniform01(r)
    assert u[0] == 0.5 * 2.0**-32 and u[-1] == 1.0 - 0.5 * 2.0**-32
    assert np.all((u > 0) & (u < 1))


HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCRAND_PHILOX = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    """Runs rocRAND's Philox-4x32-10 (host build) on rows of (counter, key) words."""
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)) or not os.path.exists(ROCRAND_PHILOX):
        pytest.skip("hipcc or the rocRAND headers are not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([HIPCC, "-O2", "--offload-arch=gfx950", "-std=c++17", os.path.join(HERE, "native", "philox_ref.hip"),
                    "-o", exe], check=True, capture_output=True)

    def run(ctr, key):
        rows = np.concatenate([ctr, key], axis=1).astype(np.uint64)
        inp = "\n".join(" ".join(f"{int(v):x}" for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, check=True, capture_output=True, text=True).stdout.split()
        return np.array([int(v, 16) for v in out], dtype=np.uint64).reshape(-1, 4).astype(np.uint32)
    return run


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(20240611)
    N = 1 << 14
    ctr = rng.integers(0, 2**32, size=(N, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(N, 2), dtype=np.uint64)
    # the event layout: small block index, event words, multiplicity tag
    ctr[:1024, 0] = rng.integers(0, 16, 1024)
    ctr[:1024, 3] = rng.integers(4, 13, 1024)
    ctr[1024:1100, 1:3] = 0xFFFFFFFF                  # high counter words set
    ctr[-2] = 0
    key[-2] = 0
    ctr[-1] = 0xFFFFFFFF
    key[-1] = 0xFFFFFFFF
    ref = rocrand_philox(ctr, key)
    ours = np.concatenate([philox.philox4x32(ctr[i:i + 1], key[i]) for i in range(0, 64)] +
                          [philox.philox4x32(ctr[64:], key[64:])])
    assert ours.shape == ref.shape
    bad = np.nonzero(np.any(ours != ref, axis=1))[0]
    assert bad.size == 0, f"{bad.size} of {N} outputs differ, first at row {bad[:4]}"


def test_event_words_match_rocrand(rocrand_philox):
    # the per-event draw layout through the reference generator: counter (block, event lo,
    # event hi, n), key (seed lo, seed hi)
    seed, n = 0xB6000001 + (7 << 40), 8
    ev = np.array([0, 1, 77, (1 << 32) + 5, (1 << 40) + 3], dtype=np.uint64)
    w = draws.event_words(seed, ev, n)
    nb = draws.n_blocks(n)
    ctr = np.array([[b, int(e) & 0xFFFFFFFF, int(e) >> 32, n] for e in ev for b in range(nb)], dtype=np.uint64)
    key = np.tile(np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64), (len(ctr), 1))
    assert np.array_equal(w.reshape(-1, 4), rocrand_philox(ctr, key))


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
