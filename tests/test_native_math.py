"""Accuracy of the library's own FP64 logarithm (used for RAMBO energies, pseudorapidities
and the parton sampler) and of its sin(pi t), cos(pi t) (RAMBO's azimuth), checked on the
CPU: the same header compiled for the host, against the exact value from 40-digit decimal
arithmetic.  The device build performs the identical
IEEE operations (frexp, correctly rounded division, fused multiply-adds)."""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def math_lines(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("mathcheck") / "math_check")
    subprocess.run([HIPCC, "-O2", "--offload-arch=gfx950", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", os.path.join(HERE, "native", "math_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    return [l.split() for l in subprocess.run([exe], check=True, capture_output=True, text=True).stdout.splitlines()]


@pytest.fixture(scope="module")
def log_samples(math_lines):
    return [(float.fromhex(a), float.fromhex(b)) for tag, a, b in (l for l in math_lines if l[0] == "L")]


@pytest.fixture(scope="module")
def sincos_samples(math_lines):
    return [tuple(float.fromhex(v) for v in l[1:]) for l in math_lines if l[0] == "S"]


PI40 = Decimal("3.141592653589793238462643383279502884197169399375")


def _sin_cos_pi(t):
    """sin(pi t), cos(pi t) from their Taylor series in 40-digit decimal arithmetic."""
    x = PI40 * Decimal(t)
    x2 = x * x
    s, c, ts, tc = Decimal(0), Decimal(0), x, Decimal(1)
    for k in range(1, 60):
        s += ts
        c += tc
        ts = -ts * x2 / ((2 * k) * (2 * k + 1))
        tc = -tc * x2 / ((2 * k - 1) * (2 * k))
    return s, c


def test_log_within_one_ulp(log_samples):
    getcontext().prec = 40
    worst = 0.0
    for x, y in log_samples[::13] + log_samples[-8:]:
        t = Decimal(x).ln()
        ulp = math.ulp(float(t)) if t != 0 else 2.0**-1074
        worst = max(worst, float(abs(Decimal(y) - t) / Decimal(ulp)))
    assert worst < 1.0, worst


def test_log_special_values(log_samples):
    vals = dict(log_samples[-8:])
    assert vals[1.0] == 0.0
    assert vals[2.0] == np.log(2.0) and vals[0.5] == -np.log(2.0)
    assert abs(vals[2.0**-1074] - (-1074 * math.log(2.0))) <= 2 * math.ulp(744.0)


def test_sincospi_accuracy(sincos_samples):
    """Absolute error within 2^-52 (what RAMBO's directions need), relative error within two
    ulp wherever the value is at least 1/16 in size, and the exact values at the multiples
    of 1/4 where they are representable."""
    getcontext().prec = 40
    worst_abs = worst_ulp = 0.0
    for t, s, c in sincos_samples:
        es, ec = _sin_cos_pi(t)
        for y, e in ((s, es), (c, ec)):
            err = abs(Decimal(y) - e)
            worst_abs = max(worst_abs, float(err))
            if abs(e) >= Decimal(1) / 16:
                worst_ulp = max(worst_ulp, float(err / Decimal(math.ulp(float(e)))))
    assert worst_abs <= 2.0**-52, worst_abs
    assert worst_ulp <= 2.0, worst_ulp
    exact = {0.0: (0.0, 1.0), 0.5: (1.0, 0.0), 1.0: (0.0, -1.0), 1.5: (-1.0, 0.0), 2.0: (0.0, 1.0)}
    got = {t: (s, c) for t, s, c in sincos_samples[-9:]}
    for t, (es, ec) in exact.items():
        assert got[t][0] == es and got[t][1] == ec, (t, got[t])
    half = math.sqrt(0.5)
    for t in (0.25, 0.75, 1.25, 1.75):
        assert abs(abs(got[t][0]) - half) <= 2 * math.ulp(half) and abs(abs(got[t][1]) - half) <= 2 * math.ulp(half)
