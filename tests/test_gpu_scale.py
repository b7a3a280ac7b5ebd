"""GPU parity of bg_generate with the dynamic scale mu = H_T (alpha_s and the density read
from grids with linear interpolation, Secs. 3 and 4) against the oracle, event by event:
weights, |A|^2, cuts and draws as compare_events checks them, with the weight carrying
alpha_s(mu)^(n-2) f(x1, mu) f(x2, mu)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import event, pdf
from tests.test_gpu_generate import ALL, cfg_c0, cfg_c1, compare_events, oracle_cfg, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,prec,pol", [(8, 64, 0), (8, 32, 0), (12, 32, 0), (6, 64, 0), (8, 32, 1), (10, 32, 0)])
def test_dynamic_scale_pdf_events(gpu_lib, n, prec, pol):
    c = cfg_c1(gpu_lib, n=n, prec=prec, first_event=4321, dynamic_scale=1, polarisation=pol)
    N = 4 * 256 + 77
    print(f"generate dynamic scale n={n} prec={prec} pol={pol}", flush=True)
    g = to_np(gpu_lib.generate(c, N, outputs=ALL))
    oc = oracle_cfg(c)
    oc["tau_min"] = pdf.tau_min(n, 20.0, 14000.0)
    o = event.generate(oc, 4321 + np.arange(N))
    print(compare_events(g, o, oc, prec))
    # the scale changes the weights: most passing events differ from the fixed-scale weight
    fixed = to_np(gpu_lib.generate(cfg_c1(gpu_lib, n=n, prec=prec, first_event=4321, polarisation=pol), N,
                                   outputs=("weight", "pass")))
    ps = g["pass"].astype(bool)
    assert np.array_equal(ps, fixed["pass"].astype(bool))
    if ps.sum():
        assert np.mean(g["weight"][ps] != fixed["weight"][ps]) > 0.9


def test_dynamic_scale_fixed_energy_fp64(gpu_lib):
    c = cfg_c0(gpu_lib, dynamic_scale=1)
    N = 8192
    g = to_np(gpu_lib.generate(c, N, outputs=ALL))
    oc = oracle_cfg(c)
    print(compare_events(g, event.generate(oc, np.arange(N)), oc, 64))


def test_dynamic_scale_unsupported_paths(gpu_lib):
    c = cfg_c1(gpu_lib, n=6, prec=64, dynamic_scale=1)
    outs = gpu_lib.BgOutputs()
    assert gpu_lib.raw().bg_generate_noalloc(ctypes.byref(c), 16, None, ctypes.byref(outs), None) == gpu_lib.BG_ENOTSUP
    u = torch.full((4, 16), 0.5, dtype=torch.float64, device="cuda")
    x = torch.full((4, 2), 0.1, dtype=torch.float64, device="cuda")
    h = torch.full((4,), 0b110011, dtype=torch.int32, device="cuda")
    o = torch.tensor([list(range(6))] * 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu_lib.BgError) as e:
        gpu_lib.amp2_grad(c, u, x, h, o)
    assert e.value.status == gpu_lib.BG_ENOTSUP
