"""bg_fma_rate, the calibration of the roofline denominators: plain multiply-add chains reach
a stated fraction of the scalar ceiling 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz =
78.6 TFLOP/s (FP32 without packing, and FP64), and never exceed it by more than clock
tolerance."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [32, 64])
def test_fma_rate_within_ceiling(gpu_lib, prec):
    r = gpu_lib.fma_rate(prec)
    print(f"FP{prec} multiply-add chains: {r:.1f} TFLOP/s")
    assert 0.5 * 78.6 < r < 1.05 * 78.6


def test_fma_rate_rejects_bad_precision(gpu_lib):
    import ctypes
    v = ctypes.c_double()
    assert gpu_lib.raw().bg_fma_rate(16, ctypes.byref(v), None) == gpu_lib.BG_EINVAL
    assert gpu_lib.raw().bg_fma_rate(32, None, None) == gpu_lib.BG_EINVAL
