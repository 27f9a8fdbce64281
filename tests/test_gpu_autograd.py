"""Differentiable FFT: FFTFunction forward = eq. 1 on the GPU, backward = the
adjoint F^H (inverse direction, scale 1) on the GPU, checked against the FP64
oracle's analytic gradient and FP64 central finite differences."""
import math

import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import api, capi, workloads
from gpu_helpers import rel_l2_rows, require_gpu, to_gpu_c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def row_loss_fp64(x_row, w_row):
    """Sum over one signal of |W * F x|^2 in FP64 with the oracle."""
    X = oracle.fft(x_row)
    return float(np.sum((w_row * np.abs(X)) ** 2))


def test_autograd_64x65536_weighted_power_loss(dev):
    B, N = 64, 1 << 16
    x, w, coords = workloads.autograd_case(B, N, seed=4, probes=32)
    xc = x.astype(np.complex64)
    wf = w.astype(np.float32)
    xt = to_gpu_c64(xc, dev).requires_grad_(True)
    wt = torch.from_numpy(wf).to(dev)
    y = api.FFTFunction.apply(xt)
    loss = ((wt * y.abs()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = xt.grad.cpu().numpy().astype(np.complex128)

    # analytic gradient in torch's convention: 2 F^H (W^2 * F x)
    x64 = xc.astype(np.complex128)
    w64 = wf.astype(np.float64)
    ga = 2.0 * oracle.adjoint(w64 ** 2 * oracle.fft(x64))
    err = np.linalg.norm(g - ga) / np.linalg.norm(ga)
    print(f"64 x 2^16 analytic gradient rel-L2 {err:.3e}")
    assert err <= 5e-5, err

    # FP64 central differences of the affected row's loss, h = 1e-6
    h = 1e-6
    rms = float(np.sqrt(np.mean(np.abs(ga) ** 2)))
    worst = 0.0
    for c in coords:
        b, j = divmod(int(c), N)
        xr = x64[b].copy()
        for part, unit in (("re", 1.0), ("im", 1j)):
            xp = xr.copy()
            xm = xr.copy()
            xp[j] += h * unit
            xm[j] -= h * unit
            d = (row_loss_fp64(xp, w64[b]) - row_loss_fp64(xm, w64[b])) / (2 * h)
            gj = g[b, j].real if part == "re" else g[b, j].imag
            bound = 1e-4 * max(abs(gj), rms)
            worst = max(worst, abs(d - gj) / bound)
            assert abs(d - gj) <= bound, (b, j, part, d, gj)
    print(f"64 x 2^16 finite differences: worst |fd - g| / bound = {worst:.3f}")


def test_adjoint_dot_product(dev):
    n = 1 << 16
    x = workloads.normal_batch(n, 4, seed=51).astype(np.complex64)
    y = workloads.normal_batch(n, 4, seed=52).astype(np.complex64)
    xt, yt = to_gpu_c64(x, dev), to_gpu_c64(y, dev)
    fx = api.fft(xt).cpu().numpy().astype(np.complex128)
    fhy = api.fft(yt, inverse=True, scale=1.0).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y.astype(np.complex128), fx)
    rhs = np.vdot(fhy, x.astype(np.complex128))
    bound = 1e-6 * math.log2(n) * np.linalg.norm(fx) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= bound


def test_backward_matches_oracle_adjoint_small(dev):
    for n in (8, 1024, 1 << 15):
        x = workloads.normal_batch(n, 3, seed=n).astype(np.complex64)
        g = workloads.normal_batch(n, 3, seed=n + 1).astype(np.complex64)
        xt = to_gpu_c64(x, dev).requires_grad_(True)
        y = api.fft_autograd(xt)
        y.backward(to_gpu_c64(g, dev))
        torch.cuda.synchronize()
        ref = oracle.adjoint(g)
        assert rel_l2_rows(xt.grad.cpu().numpy(), ref, n).max() <= 1e-6 * max(1, math.log2(n))
