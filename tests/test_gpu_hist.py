"""GPU exact histograms (bg_hist_accumulate / bg_hist_read) of H_T and R_min: bitwise equal
to the oracle's histogram (exact per-bin sums, rounded once) of the same weights and
observables, independent of how the events are split over calls; and the generator's
distributions against the oracle's own events."""
import math

import numpy as np
import pytest
import torch

from oracle import event, histogram, pdf

pytestmark = pytest.mark.gpu

AXES = [(0, 40, 0.0, 2000.0), (1, 36, 0.4, 4.0)]   # H_T in GeV, R_min


def oracle_hist(w, obs, axes=AXES):
    return np.concatenate([histogram.histogram(w, obs[:, c], lo, hi, nb) for c, nb, lo, hi in axes])


def test_hist_matches_oracle_bitwise_and_splits(gpu_lib):
    n, N = 8, (1 << 20) + 333
    c = gpu_lib.config(n, prec=32, seed=0xB6000001)
    print("generate n=8 fp32 for histograms", flush=True)
    r = gpu_lib.generate(c, N, outputs=("weight", "obs"))
    limbs = gpu_lib.hist_limbs(AXES)
    gpu_lib.hist_accumulate(r["weight"], r["obs"], AXES, limbs)
    h = gpu_lib.hist_read(AXES, limbs).cpu().numpy()
    w, obs = r["weight"].cpu().numpy(), r["obs"].cpu().numpy()
    ref = oracle_hist(w, obs)
    assert np.array_equal(h, ref), np.nonzero(h != ref)
    # the same events in three calls, accumulated: bitwise the same
    l2 = gpu_lib.hist_limbs(AXES)
    for a, b in ((0, 1000), (1000, N // 2), (N // 2, N)):
        gpu_lib.hist_accumulate(r["weight"][a:b].contiguous(), r["obs"][a:b].contiguous(), AXES, l2)
    assert torch.equal(limbs, l2)
    # totals: the bins of one axis hold every non-zero weight
    tot = math.fsum(w.tolist())
    assert abs(h[:42, 0].sum() - tot) <= 1e-12 * tot


def test_hist_generator_vs_oracle_events(gpu_lib):
    """n = 5, 2^16 events at 1 TeV, FP64: the GPU's histograms against the oracle's from its
    own events; bins agree to the per-event weight agreement except where an event's H_T
    or R_min straddles a bin edge between the two evaluations."""
    N = 1 << 16
    c = gpu_lib.config(5, prec=64, sqrt_s=1000.0, use_pdf=0, random_order=1, seed=33)
    r = gpu_lib.generate(c, N, outputs=("weight", "obs"))
    limbs = gpu_lib.hist_accumulate(r["weight"], r["obs"], AXES, gpu_lib.hist_limbs(AXES))
    h = gpu_lib.hist_read(AXES, limbs).cpu().numpy()
    o = event.generate(event.config(n=5, use_pdf=0, sqrt_s=1000.0, random_order=1, seed=33), np.arange(N))
    oobs = np.stack([o["ht"], o["rmin"]], 1)
    ref = oracle_hist(o["weight"], oobs)
    gobs = r["obs"].cpu().numpy()
    moved = np.zeros(len(ref), dtype=bool)
    base = 0
    for col, nb, lo, hi in AXES:
        bg_ = histogram.bin_index(gobs[:, col], lo, hi, nb)
        bo = histogram.bin_index(oobs[:, col], lo, hi, nb)
        for k in np.unique(np.concatenate([bg_[bg_ != bo], bo[bg_ != bo]])):
            moved[base + k] = True
        base += nb + 2
    ok = ~moved & (ref[:, 0] > 0)
    rel = np.abs(h[ok, 0] - ref[ok, 0]) / ref[ok, 0]
    print(f"bins compared {ok.sum()}, moved {moved.sum()}, max rel {rel.max():.2e}")
    assert ok.sum() > 40 and rel.max() < 1e-10


def test_hist_argument_errors(gpu_lib):
    w = torch.zeros(4, dtype=torch.float64, device="cuda")
    obs = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    limbs = gpu_lib.hist_limbs(AXES)
    for bad in ([(2, 10, 0.0, 1.0)], [(0, 0, 0.0, 1.0)], [(0, 10, 1.0, 1.0)], [(0, 399, 0.0, 1.0)]):
        with pytest.raises(gpu_lib.BgError) as e:
            gpu_lib.hist_accumulate(w, obs, bad, gpu_lib.hist_limbs(bad))
        assert e.value.status == gpu_lib.BG_EINVAL
