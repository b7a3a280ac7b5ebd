"""The host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: the
ABI layer's sources (bg_capi.hip, bg_finalize.hip, bg_hist.hip, bg_probe.hip, no kernel units, so every
recursion launcher is absent) are built with -fsanitize=address,undefined on the host code
and driven by tests/native/abi_check.cpp on a machine without a GPU.  Every argument check,
table lookup and, for valid arguments, the first HIP call (which fails without a device:
BG_EHIP) runs under the sanitizers; any report aborts the run.  Skipped where a GPU is
visible (the valid calls pass host buffers)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1002_3446_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

OK, EINVAL, ENOTSUP, EHIP = 0, -1, -2, -3

# status of each call in a library without kernel units
EXPECTED = {
    "generate_null_cfgs": EINVAL, "generate_ncfg0": EINVAL, "generate_ncfg17": EINVAL,
    "generate_negative_count": EINVAL, "generate_n3": ENOTSUP, "generate_n13": ENOTSUP,
    "generate_prec16": ENOTSUP, "generate_polarisation2": EINVAL, "generate_reserved": EINVAL,
    "generate_sqrt_s": EINVAL, "generate_empty": ENOTSUP, "generate_valid": ENOTSUP,
    "generate_two_valid": ENOTSUP, "noalloc_null": EINVAL, "noalloc_oversize": EINVAL,
    "noalloc_dynamic": ENOTSUP, "noalloc_valid": ENOTSUP, "amp2_n13": ENOTSUP, "amp2_negative": EINVAL,
    "amp2_empty": ENOTSUP, "amp2_null": ENOTSUP, "amp2_valid": ENOTSUP, "grad_null_cfg": EINVAL,
    "grad_empty": ENOTSUP, "grad_polarisation": ENOTSUP, "grad_valid": ENOTSUP,
    "hist_null_axes": EINVAL, "hist_bad_column": EINVAL, "hist_too_many_bins": EINVAL,
    "hist_lo_ge_hi": EINVAL, "hist_valid": EHIP, "hist_read_null": EINVAL,
    "set_launch_bad_block": EINVAL, "set_launch_n2": ENOTSUP, "set_launch_ok": OK, "get_launch": OK,
    "set_launch_default": OK, "set_lanes_3": EINVAL, "set_lanes_n8_2": ENOTSUP, "get_lanes": OK,
    "set_form_bad": EINVAL, "set_form_n9": ENOTSUP, "get_form": OK, "set_mixed_bad": EINVAL,
    "set_mixed_ok": OK, "check_n3": ENOTSUP, "check_null": EINVAL, "fma_prec16": EINVAL, "fma_null": EINVAL,
    "fma_valid": EHIP,
}


def gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_abi_host_code_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    if gpu_visible():
        pytest.skip("runs without a GPU only (valid calls pass host buffers)")
    exe = str(tmp_path / "abi_check")
    cmd = [HIPCC, "-O1", "-g", "--offload-arch=gfx950", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-mllvm", "-disable-cgp",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           '-DBG_SOURCE_HASH="sanitized"', os.path.join(CSRC, "bg_capi.hip"), os.path.join(CSRC, "bg_finalize.hip"),
           os.path.join(CSRC, "bg_hist.hip"), os.path.join(CSRC, "bg_probe.hip"),
           os.path.join(HERE, "native", "abi_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    got = {}
    for line in r.stdout.splitlines():
        parts = line.split()
        if len(parts) == 2 and parts[0] in EXPECTED:
            got[parts[0]] = int(parts[1])
    assert got == EXPECTED
    lines = r.stdout.splitlines()
    assert "launch 128 4" in lines and "lanes 4" in lines and "form 0" in lines and "mixed 0" in lines
    assert all(l.endswith("text") for l in lines if l.startswith("strerror"))
