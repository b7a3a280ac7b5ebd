"""GPU parity of the W-tensor form of the recursion (Eqs. 3.3-3.4, 16 lanes per event,
bg_set_form) against the oracle: bg_amp2 on given momenta to the FP64 rules (n = 6, 10)
and the FP32 bound (n = 8, 10, 11, 12); bg_generate with the form against the oracle event
by event; the same events as the direct form (draws, kinematics, cuts identical)."""
import contextlib

import numpy as np
import pytest

from oracle import event, pdf
from tests.parity import check_amp2_fp64, fp32_errors
from tests.test_gpu_amp2 import make_points, run_gpu
from tests.test_gpu_generate import ALL, cfg_c1, compare_events, oracle_cfg, same_events, to_np

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def form_set(bg, n, prec, form):
    old = bg.get_form(n, prec)
    bg.set_form(n, prec, form)
    try:
        yield
    finally:
        bg.set_form(n, prec, old)


@pytest.mark.parametrize("n", [6, 10])
def test_wtensor_amp2_fp64(gpu_lib, n):
    N = 4 * 256 + 13
    mom, hel, order = make_points(n, N, 300 + n)
    print(f"amp2 W-tensor fp64 n={n}", flush=True)
    with form_set(gpu_lib, n, 64, 1):
        got = run_gpu(gpu_lib, n, 64, mom, hel, order)
    print(check_amp2_fp64(got, mom, hel, order))


@pytest.mark.parametrize("n", [8, 10, 11, 12])
def test_wtensor_amp2_fp32(gpu_lib, n):
    N = 2 * 256 + 5
    mom, hel, order = make_points(n, N, 400 + n)
    print(f"amp2 W-tensor fp32 n={n}", flush=True)
    with form_set(gpu_lib, n, 32, 1):
        got = run_gpu(gpu_lib, n, 32, mom, hel, order)
    rel, sc = fp32_errors(got, mom, hel, order, scaled=True)
    print(f"n={n} rel err median {np.median(rel):.2e} p99 {np.quantile(rel, 0.99):.2e}, scaled max {sc.max():.2e}")
    assert np.median(rel) <= 1e-4 and sc.max() <= 1e-4


@pytest.mark.parametrize("n,prec", [(12, 32), (10, 64), (8, 32)])
def test_wtensor_generate_vs_oracle_and_direct(gpu_lib, n, prec):
    c = cfg_c1(gpu_lib, n=n, prec=prec, first_event=99)
    N = 3 * 256 + 41
    print(f"generate W-tensor n={n} prec={prec}", flush=True)
    with form_set(gpu_lib, n, prec, 1):
        w = to_np(gpu_lib.generate(c, N, outputs=ALL))
    oc = oracle_cfg(c)
    oc["tau_min"] = pdf.tau_min(n, 20.0, 14000.0)
    print(compare_events(w, event.generate(oc, 99 + np.arange(N)), oc, prec))
    d = to_np(gpu_lib.generate(c, N, outputs=ALL))
    if prec == 32:
        same_events(w, d, n, exact=False)
    else:
        for k in ("hel", "order", "pass", "momenta", "obs", "x12", "uniforms"):
            assert np.array_equal(w[k], d[k]), k


def test_wtensor_unsupported(gpu_lib):
    with pytest.raises(gpu_lib.BgError) as e:
        gpu_lib.set_form(9, 32, 1)
    assert e.value.status == gpu_lib.BG_ENOTSUP
    with pytest.raises(gpu_lib.BgError):
        gpu_lib.set_form(10, 32, 2)
    assert gpu_lib.get_form(10, 32) == 0
