"""Host-side checks of the C-ABI that need no GPU: every function declared in
include/bg.h is exported by libbg.so, and argument errors are reported before any
device work is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1002_3446_amd", "libbg.so")
HDR = os.path.join(ROOT, "include", "bg.h")

need_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libbg.so not built")


def declared():
    text = open(HDR).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(bg_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    assert {"bg_generate", "bg_amp2", "bg_amp2_grad", "bg_strerror", "bg_version",
            "bg_set_launch", "bg_get_launch"} <= set(declared())


@need_lib
def test_all_declared_symbols_exported():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@need_lib
def test_host_error_paths():
    from paper_1002_3446_amd import bg
    lib = bg.raw()
    assert bg.version() >= 10000
    assert bg.strerror(bg.BG_ENOTSUP).startswith("unsupported")
    c = bg.config(3)
    counts = (ctypes.c_int64 * 1)(10)
    outs = (bg.BgOutputs * 1)()
    assert lib.bg_generate(ctypes.byref(c), 1, counts, None, outs, None) == bg.BG_ENOTSUP
    c = bg.config(8, prec=16)
    assert lib.bg_generate(ctypes.byref(c), 1, counts, None, outs, None) == bg.BG_ENOTSUP
    c = bg.config(8)
    c.polarisation = 2
    assert lib.bg_generate(ctypes.byref(c), 1, counts, None, outs, None) == bg.BG_EINVAL
    c = bg.config(8, pt_min=0.0)            # tau_min would be 0: the density is not integrable
    assert lib.bg_generate(ctypes.byref(c), 1, counts, None, outs, None) == bg.BG_EINVAL
    c = bg.config(8, pdf_a=-2.0, pdf_b=5)   # a + k + 1 = 0 at k = 1
    assert lib.bg_generate(ctypes.byref(c), 1, counts, None, outs, None) == bg.BG_EINVAL
    neg = (ctypes.c_int64 * 1)(-1)
    assert lib.bg_generate(ctypes.byref(bg.config(8)), 1, neg, None, outs, None) == bg.BG_EINVAL
    assert lib.bg_generate(None, 1, counts, None, outs, None) == bg.BG_EINVAL
    assert lib.bg_generate(ctypes.byref(bg.config(8)), 0, counts, None, outs, None) == bg.BG_EINVAL
    assert lib.bg_amp2(13, 64, 5, None, None, None, None, None) == bg.BG_ENOTSUP
    assert lib.bg_amp2(8, 64, -1, None, None, None, None, None) == bg.BG_EINVAL
    assert lib.bg_amp2(8, 64, 0, None, None, None, None, None) == bg.BG_OK
    assert lib.bg_amp2(8, 64, 4, None, None, None, None, None) == bg.BG_EINVAL
    assert lib.bg_check_events(3, 5, None, None, None, None) == bg.BG_ENOTSUP
    assert lib.bg_check_events(8, -1, None, None, None, None) == bg.BG_EINVAL
    assert lib.bg_check_events(8, 5, None, None, None, None) == bg.BG_EINVAL
    assert lib.bg_check_events(8, 1 << 40, 16, 16, 16, None) == bg.BG_EINVAL
    assert lib.bg_amp2_grad(None, 4, *([None] * 9)) == bg.BG_EINVAL
    assert lib.bg_set_launch(8, 32, 96, 1) == bg.BG_EINVAL
    assert lib.bg_set_launch(8, 32, 128, 0) == bg.BG_EINVAL
    assert lib.bg_set_launch(2, 32, 128, 1) == bg.BG_ENOTSUP
    assert lib.bg_set_mixed_launch(3) == bg.BG_EINVAL and lib.bg_set_mixed_launch(-1) == bg.BG_EINVAL
    assert lib.bg_set_mixed_launch(2) == bg.BG_OK and lib.bg_get_mixed_launch() == 2
    assert lib.bg_set_mixed_launch(0) == bg.BG_OK and lib.bg_get_mixed_launch() == 0
    assert lib.bg_set_mixed_launch(1) == bg.BG_OK and lib.bg_get_mixed_launch() == 1
    v = ctypes.c_int()
    assert lib.bg_set_lanes(8, 32, 3) == bg.BG_EINVAL
    assert lib.bg_set_lanes(3, 32, 1) == bg.BG_ENOTSUP
    assert lib.bg_get_lanes(8, 32, None) == bg.BG_EINVAL
    keep = {n: bg.get_lanes(n, 32) for n in (8, 12)}
    assert lib.bg_set_lanes(8, 32, 0) == bg.BG_OK and lib.bg_set_lanes(12, 32, 0) == bg.BG_OK
    assert lib.bg_get_lanes(8, 32, ctypes.byref(v)) == bg.BG_OK and v.value == 1    # defaults
    assert lib.bg_get_lanes(12, 32, ctypes.byref(v)) == bg.BG_OK and v.value == 2
    assert lib.bg_set_lanes(8, 32, 2) == bg.BG_ENOTSUP   # no grouped form at n = 8 FP32
    assert lib.bg_set_lanes(8, 32, 4) == bg.BG_ENOTSUP
    assert lib.bg_set_lanes(12, 32, 4) == bg.BG_ENOTSUP  # four lanes: FP64 n >= 10 only
    assert lib.bg_set_lanes(9, 64, 4) == bg.BG_ENOTSUP
    assert lib.bg_set_lanes(12, 64, 1) == bg.BG_ENOTSUP  # no one-lane form at n = 12 FP64
    assert lib.bg_set_lanes(12, 32, 8) == bg.BG_EINVAL
    keep64 = bg.get_lanes(12, 64)
    assert lib.bg_set_lanes(12, 64, 0) == bg.BG_OK
    assert lib.bg_get_lanes(12, 64, ctypes.byref(v)) == bg.BG_OK and v.value == 4   # default
    for l in (2, 4):
        assert lib.bg_set_lanes(12, 64, l) == bg.BG_OK
        assert lib.bg_get_lanes(12, 64, ctypes.byref(v)) == bg.BG_OK and v.value == l
    bg.set_lanes(12, 64, keep64)
    for n, l in keep.items():
        bg.set_lanes(n, 32, l)
    b, k = ctypes.c_int(), ctypes.c_int()
    assert lib.bg_get_launch(8, 32, ctypes.byref(b), ctypes.byref(k)) == bg.BG_OK and b.value in (64, 128, 192, 256)


@need_lib
def test_hip_error_path_without_device():
    """Without a GPU the first HIP call of a valid request fails: the entry points return
    BG_EHIP (nothing is enqueued, no pointer is dereferenced on the host)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    from paper_1002_3446_amd import bg
    lib = bg.raw()
    c = bg.config(8, prec=32)
    counts = (ctypes.c_int64 * 1)(1000)
    outs = bg.BgOutputs()
    outs.weight = ctypes.c_void_p(0x10000)
    assert lib.bg_generate(ctypes.byref(c), 1, counts, None, ctypes.byref(outs), None) == bg.BG_EHIP
    p = ctypes.c_void_p(0x10000)
    assert lib.bg_amp2(8, 32, 4, p, p, p, p, None) == bg.BG_EHIP
    assert lib.bg_generate_noalloc(ctypes.byref(c), 10, None, ctypes.byref(outs), None) == bg.BG_EHIP
