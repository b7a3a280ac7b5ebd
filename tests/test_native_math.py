"""Accuracy of the library's own FP64 logarithm (used for RAMBO energies, pseudorapidities
and the parton sampler), checked on the CPU: the same header compiled for the host, against
the exact value from 40-digit decimal arithmetic.  The device build performs the identical
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
def log_samples(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("mathcheck") / "math_check")
    subprocess.run([HIPCC, "-O2", "--offload-arch=gfx950", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", os.path.join(HERE, "native", "math_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [(float.fromhex(a), float.fromhex(b)) for a, b in zip(out[0::2], out[1::2])]


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
