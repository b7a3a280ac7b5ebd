"""The allocation-free entry point bg_generate_noalloc, called through the C ABI, against
bg_generate on the same classes: every per-event output and the compensated totals equal
bitwise (same kernels, same partial layout), on calls in a row that shrink, over the split
form (staged in chunks of 2^16 events), the two-lane form, FP64 and real polarisations."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ALL = ("weight", "amp2", "obs", "pass", "momenta", "hel", "order", "x12", "uniforms", "acc", "logw")


def cfg(bg, n, prec, seed, **kw):
    return bg.config(n, prec=prec, sqrt_s=14000.0, use_pdf=1, random_order=1, seed=seed, **kw)


def noalloc(bg, c, N):
    """Output tensors allocated here, then one raw C-ABI call that fills them."""
    outs = bg.BgOutputs()
    keep = {}
    for name in ALL:
        dt, sh = bg._OUT_SPEC[name]
        t = torch.zeros(sh(N, c.n), dtype=dt, device="cuda")
        keep[name] = t
        setattr(outs, name, t.data_ptr())
    torch.cuda.synchronize()
    st = bg.raw().bg_generate_noalloc(ctypes.byref(c), N, None, ctypes.byref(outs),
                                      torch.cuda.current_stream().cuda_stream)
    assert st == bg.BG_OK, bg.strerror(st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in keep.items()}


@pytest.mark.parametrize("n,prec,N,pol", [(8, 32, (1 << 20) + 37, 0), (6, 32, 5000, 0), (10, 32, 3001, 0),
                                          (5, 64, 2000, 0), (7, 32, 70001, 1), (6, 32, 999, 0)])
def test_noalloc_matches_generate(gpu_lib, n, prec, N, pol):
    c = cfg(gpu_lib, n, prec, 0xA110C + n, first_event=17, polarisation=pol)
    print(f"noalloc n={n} prec={prec} N={N} pol={pol}", flush=True)
    a = noalloc(gpu_lib, c, N)
    ref = {k: v.cpu().numpy() for k, v in gpu_lib.generate(c, N, outputs=ALL).items()}
    for k in ALL:
        assert np.array_equal(a[k], ref[k], equal_nan=True), k


def test_noalloc_rejects_oversize(gpu_lib):
    c = cfg(gpu_lib, 8, 32, 1)
    outs = gpu_lib.BgOutputs()
    st = gpu_lib.raw().bg_generate_noalloc(ctypes.byref(c), (1 << 24) + 1, None, ctypes.byref(outs), None)
    assert st == gpu_lib.BG_EINVAL
