"""Exactness of the library's fixed-point histogram sums (bg_hist.hpp), checked on the CPU:
the header compiled for the host adds groups of doubles into limbs and rounds the total
once; every total must equal math.fsum of the same values (the correctly rounded exact
sum), including groups over 400 binades, halfway cases and values below the grid."""
import math
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def hist_sum(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("histcheck") / "hist_check")
    subprocess.run([HIPCC, "-O2", "--offload-arch=gfx950", "-std=c++17", os.path.join(HERE, "native", "hist_check.hip"),
                    "-o", exe], check=True, capture_output=True)

    def run(groups):
        inp = "\n".join(f"{len(g)} " + " ".join(float(x).hex() for x in g) for g in groups) + "\n"
        out = subprocess.run([exe], input=inp, check=True, capture_output=True, text=True).stdout.split("\n")
        res = []
        for line in out[:len(groups)]:
            tag, v = line.split()
            res.append((tag, float.fromhex(v)))
        return res
    return run


def test_random_groups_equal_fsum(hist_sum):
    rng = np.random.default_rng(3)
    groups = []
    for _ in range(300):
        k = int(rng.integers(1, 400))
        e = rng.uniform(-120, 100, k)
        groups.append((rng.uniform(0.5, 1.0, k) * 2.0 ** np.floor(e)).tolist())
    for _ in range(100):   # realistic weights: lognormal over many decades
        groups.append(rng.lognormal(0, 6, int(rng.integers(1, 2000))).tolist())
    res = hist_sum(groups)
    for g, (tag, v) in zip(groups, res):
        assert tag == "ok" and v == math.fsum(g), (v, math.fsum(g))


def test_halfway_cases_round_to_even(hist_sum):
    ulp = 2.0 ** -52
    groups = [[1.0, ulp / 2], [1.0 + ulp, ulp / 2], [1.0, ulp / 2, 2.0 ** -200], [1.0, ulp / 2, 2.0 ** -150],
              [2.0 ** 60, 2.0 ** 7], [2.0 ** 60, 2.0 ** 7, 2.0 ** -100], [3.0 * 2.0 ** 100, 1.0]]
    res = hist_sum(groups)
    for g, (tag, v) in zip(groups, res):
        exact_tail = [x for x in g if x >= 2.0 ** -160]   # bits below 2^-160 are not kept
        assert tag == "ok" and v == math.fsum(exact_tail), (g, v)


def test_rejects_negative_and_huge(hist_sum):
    res = hist_sum([[1.0, -1.0], [2.0 ** 224], [float("inf")], [float("nan")], [2.0 ** 223]])
    assert [t for t, _ in res] == ["rejected", "rejected", "rejected", "rejected", "ok"]
    assert res[0][1] == 1.0 and res[4][1] == 2.0 ** 223
