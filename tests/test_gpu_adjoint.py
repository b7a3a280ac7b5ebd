"""GPU parity of the hand-written adjoint (bg_amp2_grad; FP32 n = 6..8 run the two-lane
reverse sweep, the others one lane per event) and of the torch Function:
against the oracle's float64 autograd gradient, against central finite differences of
the GPU's own FP64 forward (h = 1e-6), the closed form in x1, x2, and the sum rules of
azimuthal symmetry and RAMBO's scale invariance."""
import numpy as np
import pytest
import torch

from oracle import event, pdf
from paper_1002_3446_amd import inputs

pytestmark = pytest.mark.gpu


def setup(n, N, seed):
    tau = pdf.tau_min(n, 20.0, 14000.0)
    u = inputs.rambo_uniforms(seed, N, n)
    x = inputs.x_fractions(seed, N, tau)
    hel = inputs.helicity_words(seed, N, n)
    pc = np.array([bin(int(h)).count("1") for h in hel])
    hel = np.where((pc >= 2) & (pc <= n - 2), hel, np.uint32(0b11)).astype(np.uint32)
    order = inputs.orderings(seed, N, n)
    return u, x, hel, order


def dev(u, x, hel, order):
    return (torch.tensor(u, device="cuda"), torch.tensor(x, device="cuda"),
            torch.tensor(hel.astype(np.int64), device="cuda").to(torch.int32), torch.tensor(order, device="cuda"))


@pytest.mark.parametrize("n,prec", [(5, 64), (8, 64), (8, 32), (6, 32), (7, 32), (4, 64), (4, 32), (6, 64),
                                    (5, 32), (9, 32), (10, 32), (11, 32), (12, 32), (9, 64), (10, 64), (12, 64)])
def test_grad_vs_oracle(gpu_lib, n, prec):
    N = 1024 + 17
    u, x, hel, order = setup(n, N, 40 + n)
    c = gpu_lib.config(n, prec=prec)
    print(f"grad n={n} prec={prec} N={N}", flush=True)
    gu, gx, lw = gpu_lib.amp2_grad(c, *dev(u, x, hel, order))
    torch.cuda.synchronize()
    oc = event.config(n=n, use_pdf=1)
    olw, ogu, ogx = event.log_weight_grad(oc, u, x, hel, order)
    gu, gx, lw = gu.cpu().numpy(), gx.cpu().numpy(), lw.cpu().numpy()
    scale = np.abs(ogu).max(1)
    err = np.abs(gu - ogu).max(1) / scale
    xerr = np.abs(gx - ogx) / np.abs(ogx)
    lerr = np.abs(lw - olw)
    q = np.quantile(err, [0.5, 0.9, 0.99])
    print(f"n={n} prec={prec} grad_u rel err p50/p90/p99 {q}, grad_x max {xerr.max():.2e}, logw max {lerr.max():.2e}")
    if prec == 64:
        # ill-conditioned events (soft/collinear) carry the same ~1e-10 tails as |A|^2 itself
        assert q[0] < 1e-12 and q[2] < 1e-8
        assert np.median(xerr) < 1e-12 and np.quantile(xerr, 0.99) < 1e-8 and xerr.max() < 1e-6
        assert np.median(lerr) < 1e-12 and np.quantile(lerr, 0.99) < 1e-9 and lerr.max() < 1e-6
    else:
        # FP32: the stated median bound; the 1% tail holds events near a zero of the
        # amplitude, where FP32 loses most digits (measured p99 3.6e-4 .. 2.5e-3 for n = 5..12)
        assert q[0] < 1e-4 and q[1] < 1e-3 and q[2] < 1e-2
        assert np.median(xerr) < 1e-5 and np.quantile(xerr, 0.99) < 1e-2
        assert np.median(lerr) < 1e-5 and np.quantile(lerr, 0.99) < 1e-2


def test_grad_full_size_sampled(gpu_lib):
    """The adjoint workload as timed (n = 8, FP32, 2^20 events, plus a ragged tail of 37):
    the oracle's gradient on sampled events, including the first and last."""
    n, N = 8, (1 << 20) + 37
    u, x, hel, order = setup(n, N, 23)
    print(f"grad full size n={n} N={N}", flush=True)
    gu, gx, lw = gpu_lib.amp2_grad(gpu_lib.config(n, prec=32), *dev(u, x, hel, order))
    torch.cuda.synchronize()
    gu, gx, lw = gu.cpu().numpy(), gx.cpu().numpy(), lw.cpu().numpy()
    assert np.all(np.isfinite(gu)) and np.all(np.isfinite(gx))
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, 1, N - 2, N - 1], rng.integers(0, N, 300)]))
    olw, ogu, ogx = event.log_weight_grad(event.config(n=n, use_pdf=1), u[idx], x[idx], hel[idx], order[idx])
    err = np.abs(gu[idx] - ogu).max(1) / np.abs(ogu).max(1)
    q = np.quantile(err, [0.5, 0.9])
    print(f"sampled grad_u rel err p50/p90 {q}")
    assert q[0] < 1e-4 and q[1] < 1e-2
    assert np.median(np.abs(gx[idx] - ogx) / np.abs(ogx)) < 1e-5
    assert np.median(np.abs(lw[idx] - olw)) < 1e-5


def test_grad_closed_form_and_sum_rules(gpu_lib):
    n, N = 8, 2048
    u, x, hel, order = setup(n, N, 7)
    gu, gx, _ = gpu_lib.amp2_grad(gpu_lib.config(n, prec=64), *dev(u, x, hel, order))
    gu, gx = gu.cpu().numpy(), gx.cpu().numpy()
    a, b = -1.3, 5.0
    ref = (a - 1) / x - b / (1 - x)
    # the -1/x of the s_hat dependence arrives through the momentum adjoint of |A|^2, so an
    # ill-conditioned event (soft or collinear gluons) carries its |A|^2 rounding tail here
    xr = np.abs(gx / ref - 1)
    assert np.median(xr) < 1e-13 and np.quantile(xr, 0.99) < 1e-10 and xr.max() < 1e-8, xr.max()
    rho = u.reshape(N, n - 2, 4)
    g = gu.reshape(N, n - 2, 4)
    scale = np.abs(gu).max(1)
    assert np.median(np.abs(g[:, :, 1].sum(1)) / scale) < 1e-10
    assert np.median(np.abs(rho[:, :, 2] * g[:, :, 2] - rho[:, :, 3] * g[:, :, 3]).max(1) / scale) < 1e-10
    q0 = -np.log(rho[:, :, 2] * rho[:, :, 3])
    assert np.median(np.abs((q0 * rho[:, :, 2] * g[:, :, 2]).sum(1)) / scale) < 1e-10


@pytest.mark.parametrize("n,prec,N", [(6, 64, 256), (8, 32, 1024), (12, 64, 128), (12, 32, 256)])
def test_grad_vs_finite_differences_of_gpu_forward(gpu_lib, n, prec, N):
    """Central differences (h = 1e-6) of log w from bg_generate's FP64 forward, against the
    FP64 adjoint (n = 6, 12), the FP32 adjoint of the timed workload (n = 8, 1024 events)
    and the FP32 adjoint at n = 12."""
    u, x, hel, order = setup(n, N, 9)
    c = gpu_lib.config(n, prec=64)
    U, X, H, O = dev(u, x, hel, order)
    print(f"finite differences n={n} adjoint prec={prec} N={N}", flush=True)
    gu, gx, _ = gpu_lib.amp2_grad(gpu_lib.config(n, prec=prec), U, X, H, O)

    def lw(Uv, Xv):
        return gpu_lib.generate(c, N, inputs=dict(uniforms=Uv, x12=Xv, hel=H, order=O), outputs=("logw",))["logw"]

    h = 1e-6
    fd = torch.zeros_like(gu)
    for j in range(u.shape[1]):
        up, um = U.clone(), U.clone()
        up[:, j] += h
        um[:, j] -= h
        fd[:, j] = (lw(up, X) - lw(um, X)) / (2 * h)
    fdx = torch.zeros_like(gx)
    for j in range(2):
        xp, xm = X.clone(), X.clone()
        hx = h * X[:, j]
        xp[:, j] += hx
        xm[:, j] -= hx
        fdx[:, j] = (lw(U, xp) - lw(U, xm)) / (2 * hx)
    scale = gu.abs().amax(1)
    err = ((gu - fd).abs().amax(1) / scale).cpu().numpy()
    xerr = ((gx - fdx).abs() / gx.abs()).cpu().numpy()
    print(f"n={n} prec={prec}: grad_u vs FD p50/p90/p99 {np.quantile(err, [0.5, 0.9, 0.99])}, grad_x max {xerr.max():.2e}")
    if prec == 64:
        assert np.median(err) < 1e-6, np.quantile(err, [0.5, 0.9])
        assert float(xerr.max()) < 1e-5
    else:
        assert np.median(err) < 1e-4 and np.quantile(err, 0.9) < 1e-2
        assert np.median(xerr) < 1e-5


@pytest.mark.parametrize("n,prec", [(3, 32), (13, 64)])
def test_grad_unsupported_multiplicity(gpu_lib, n, prec):
    N = 4
    U = torch.zeros((N, 4 * max(n - 2, 1)), dtype=torch.float64, device="cuda")
    X = torch.full((N, 2), 0.5, dtype=torch.float64, device="cuda")
    H = torch.zeros(N, dtype=torch.int32, device="cuda")
    O = torch.zeros((N, n), dtype=torch.uint8, device="cuda")
    c = gpu_lib.config(8, prec=prec)
    c.n = n
    with pytest.raises(gpu_lib.BgError) as e:
        gpu_lib.amp2_grad(c, U, X, H, O)
    assert e.value.status == gpu_lib.BG_ENOTSUP


def test_autograd_function(gpu_lib):
    from paper_1002_3446_amd.autograd import log_weight
    n, N = 8, 512
    u, x, hel, order = setup(n, N, 11)
    U, X, H, O = dev(u, x, hel, order)
    U.requires_grad_(True)
    X.requires_grad_(True)
    c = gpu_lib.config(n, prec=32)
    lw = log_weight(U, X, c, H, O)
    w = torch.linspace(0.5, 1.5, N, device="cuda", dtype=torch.float64)
    (lw * w).sum().backward()
    gu, gx, lw2 = gpu_lib.amp2_grad(c, U.detach(), X.detach(), H, O, gout=w)
    assert torch.equal(U.grad, gu) and torch.equal(X.grad, gx)
    # two FP32 evaluations of the same recursion (the generator's one-lane kernel and the
    # adjoint's two-lane forward): equal to FP32 rounding, which ill-conditioned events
    # (near a zero of the amplitude) amplify
    d = (lw - lw2).abs().detach()
    assert float(d.median()) < 1e-5 and float(torch.quantile(d, 0.95)) < 1e-3
    assert float((d > 1e-2).double().mean()) <= 0.02
