"""GPU parity of bg_amp2 (recursion + closure on given momenta) against the oracle, for
the one-lane and (where built) the two-lane form of the recursion."""
import contextlib

import numpy as np
import pytest
import torch

from oracle import event
from paper_1002_3446_amd import inputs
from tests.parity import check_amp2_fp64, fp32_errors, lane_forms

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def lanes_set(bg, n, prec, lanes):
    old = bg.get_lanes(n, prec)
    bg.set_lanes(n, prec, lanes)
    try:
        yield
    finally:
        bg.set_lanes(n, prec, old)


def make_points(n, N, seed, rs=1000.0):
    u = inputs.rambo_uniforms(seed, N, n).reshape(N, n - 2, 4)
    cfg = event.config(n=n, use_pdf=0, sqrt_s=rs)
    mom, _ = event.kinematics(cfg, u, None)
    return mom, inputs.helicity_words(seed, N, n), inputs.orderings(seed, N, n)


def run_gpu(bg, n, prec, mom, hel, order):
    m = torch.tensor(mom, device="cuda")
    h = torch.tensor(hel.astype(np.int64), device="cuda").to(torch.int32)
    o = torch.tensor(order, device="cuda")
    out = bg.amp2(n, prec, m, h, o)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,lanes", [(n, l) for n in range(4, 13) for l in lane_forms(n, 64)])
def test_amp2_fp64_parity(gpu_lib, n, lanes):
    N = 8 * 256 + 37            # several workgroups and a ragged tail
    mom, hel, order = make_points(n, N, 100 + n)
    print(f"amp2 fp64 n={n} lanes={lanes} N={N}", flush=True)
    with lanes_set(gpu_lib, n, 64, lanes):
        got = run_gpu(gpu_lib, n, 64, mom, hel, order)
    stats = check_amp2_fp64(got, mom, hel, order)
    print(stats)


@pytest.mark.parametrize("n,lanes", [(n, l) for n in range(4, 13) for l in lane_forms(n, 32)])
def test_amp2_fp32_error(gpu_lib, n, lanes):
    N = 2 * 256 + 11
    mom, hel, order = make_points(n, N, 200 + n)
    print(f"amp2 fp32 n={n} lanes={lanes} N={N}", flush=True)
    with lanes_set(gpu_lib, n, 32, lanes):
        got = run_gpu(gpu_lib, n, 32, mom, hel, order)
    rel, sc = fp32_errors(got, mom, hel, order, scaled=True)
    q = np.quantile(rel, [0.5, 0.9, 0.99])
    print(f"n={n} fp32 rel err median {q[0]:.2e} p90 {q[1]:.2e} p99 {q[2]:.2e} max {rel.max():.2e}; "
          f"relative to the event's size: max {sc.max():.2e}")
    # the stated FP32 bound (median), and the tail in units of max(|A|^2, Parke-Taylor size):
    # events nearest a zero of the amplitude lose the most relative digits, not absolute ones
    assert q[0] <= 1e-4 and sc.max() <= 1e-4


def test_amp2_empty_and_single(gpu_lib):
    n = 6
    mom, _, order = make_points(n, 1, 7)
    hel = np.array([0b100101], dtype=np.uint32)   # three minus, three plus: non-vanishing
    out = run_gpu(gpu_lib, n, 64, mom, hel, order)
    ref = event.amp2(mom, hel, order)
    assert abs(out[0] / ref[0] - 1) < 1e-12
    z = torch.empty((0, n, 4), dtype=torch.float64, device="cuda")
    r = gpu_lib.amp2(n, 64, z, torch.empty(0, dtype=torch.int32, device="cuda"),
                     torch.empty((0, n), dtype=torch.uint8, device="cuda"))
    assert r.numel() == 0


def test_amp2_unsupported(gpu_lib):
    n = 3
    z = torch.zeros((4, n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.BgError) as e:
        gpu_lib.amp2(n, 64, z, torch.zeros(4, dtype=torch.int32, device="cuda"),
                     torch.zeros((4, n), dtype=torch.uint8, device="cuda"))
    assert e.value.status == gpu_lib.BG_ENOTSUP


def test_check_events(gpu_lib):
    """bg_check_events: well-formed inputs give -1; planted malformed rows (a repeated leg, a
    leg index n, a helicity bit n) give the smallest planted index; the binding's debug mode
    rejects a malformed call before any amplitude is computed."""
    n, N = 8, 5000 + 13
    hel = inputs.helicity_words(3, N, n)
    order = inputs.orderings(3, N, n)
    dev = lambda h, o: (torch.tensor(h.astype(np.int64), device="cuda").to(torch.int32), torch.tensor(o, device="cuda"))
    assert gpu_lib.check_events(n, *dev(hel, order)) == -1
    o2, h2 = order.copy(), hel.copy()
    o2[4000, 3] = o2[4000, 5]        # a repeated leg
    o2[4500, 7] = n                  # a leg index out of range
    h2[4200] |= np.uint32(1 << n)    # a helicity bit beyond the last leg
    assert gpu_lib.check_events(n, *dev(h2, o2)) == 4000
    h3 = hel.copy()
    h3[N - 1] |= np.uint32(1 << 31)
    assert gpu_lib.check_events(n, *dev(h3, order)) == N - 1
    o4 = order.copy()
    o4[17, 0] = 3                    # leg 3 twice, leg 0 missing
    assert gpu_lib.check_events(n, *dev(hel, o4)) == 17
    assert gpu_lib.check_events(n, torch.empty(0, dtype=torch.int32, device="cuda"),
                                torch.empty((0, n), dtype=torch.uint8, device="cuda")) == -1
    mom, _, _ = make_points(n, N, 3)
    old = gpu_lib.DEBUG_CHECKS
    gpu_lib.DEBUG_CHECKS = True
    try:
        with pytest.raises(ValueError, match="event 4000"):
            gpu_lib.amp2(n, 32, torch.tensor(mom, device="cuda"), *dev(h2, o2))
        good = gpu_lib.amp2(n, 32, torch.tensor(mom, device="cuda"), *dev(hel, order))
        assert good.numel() == N
    finally:
        gpu_lib.DEBUG_CHECKS = old
