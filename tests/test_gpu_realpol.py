"""GPU parity of bg_generate with random real polarisations (the paper's sources, Sec. 3:
real currents) against the oracle, event by event: draws bit-exact, kinematics and cuts
as in the helicity mode, |A|^2 and weights to the FP64 rules or the FP32 bound; the FP32
and FP64 runs on identical events; the cross section against the helicity mode's."""
import math

import numpy as np
import pytest
import torch

from oracle import event, pdf
from tests.test_gpu_generate import ALL, EPS, cfg_c0, cfg_c1, compare_events, oracle_cfg, to_np

pytestmark = pytest.mark.gpu


def test_c0_real_fp64(gpu_lib):
    """n = 5 at fixed energy, identity ordering, FP64 real currents: 16384 events."""
    c = cfg_c0(gpu_lib, polarisation=1)
    N = 16384
    print("generate real-pol c0 n=5 fp64", flush=True)
    g = to_np(gpu_lib.generate(c, N, outputs=ALL))
    oc = oracle_cfg(c)
    o = event.generate(oc, np.arange(N))
    print(compare_events(g, o, oc, 64))
    exact = math.fsum(g["weight"].tolist())
    assert abs(g["acc"][0] + g["acc"][1] - exact) <= 2 * EPS * np.abs(g["weight"]).sum()


@pytest.mark.parametrize("n,prec", [(8, 64), (8, 32), (4, 32), (6, 64), (9, 32), (12, 32)])
def test_real_pdf_events(gpu_lib, n, prec):
    c = cfg_c1(gpu_lib, n=n, prec=prec, first_event=777, polarisation=1)
    N = 4 * 256 + 77
    print(f"generate real-pol n={n} prec={prec} N={N}", flush=True)
    g = to_np(gpu_lib.generate(c, N, outputs=ALL))
    oc = oracle_cfg(c)
    oc["tau_min"] = pdf.tau_min(n, 20.0, 14000.0)
    o = event.generate(oc, 777 + np.arange(N))
    print(compare_events(g, o, oc, prec))


def test_real_fp32_vs_fp64_same_events(gpu_lib):
    n, N = 8, 1 << 18
    r = {}
    for prec in (32, 64):
        print(f"generate real-pol n=8 prec={prec} N=2^18", flush=True)
        r[prec] = to_np(gpu_lib.generate(cfg_c1(gpu_lib, n=n, prec=prec, seed=91, polarisation=1), N,
                                         outputs=("amp2", "pass", "x12", "obs", "hel", "order")))
    for k in ("pass", "x12", "obs", "hel", "order"):
        assert np.array_equal(r[32][k], r[64][k]), k
    a32, a64 = r[32]["amp2"], r[64]["amp2"]
    live = a64 > 0
    q = np.quantile(np.abs(a32[live] - a64[live]) / a64[live], [0.5, 0.9, 0.99])
    print("real-pol n=8 fp32 vs fp64 rel err p50/p90/p99", q)
    assert q[0] <= 1e-4 and q[2] <= 1e-2


def test_real_cross_section_matches_helicity_mode(gpu_lib):
    """n = 5 at 1 TeV, 2^22 events each: sigma with real polarisations equals sigma with
    uniformly drawn helicities within four combined standard errors."""
    N = 1 << 22
    res = {}
    for pol in (0, 1):
        c = gpu_lib.config(5, prec=32, sqrt_s=1000.0, use_pdf=0, random_order=1, seed=4711, polarisation=pol)
        print(f"generate n=5 polarisation={pol} N=2^22", flush=True)
        acc = gpu_lib.generate(c, N, outputs=("acc",))["acc"].cpu().numpy()
        s, s2 = acc[0] + acc[1], acc[2] + acc[3]
        res[pol] = (s / N, math.sqrt((s2 / N - (s / N) ** 2) / (N - 1)))
    print("sigma (pb) helicity / real:", res)
    d = abs(res[0][0] - res[1][0])
    assert d < 4 * math.sqrt(res[0][1] ** 2 + res[1][1] ** 2), res


def test_real_unsupported(gpu_lib):
    c = cfg_c1(gpu_lib, n=10, prec=64, polarisation=1)
    with pytest.raises(gpu_lib.BgError) as e:
        gpu_lib.generate(c, 16, outputs=("weight",))
    assert e.value.status == gpu_lib.BG_ENOTSUP
