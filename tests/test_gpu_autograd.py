"""Differentiation through the forward SHT: the autograd function's backward
runs the library's adjoint kernels (transposed phi DFT, transposed ALT).

Pins: the loss L = sum_{l,j} w_l |f(theta_l, phi_j)|^2 equals M ||beta||^2
exactly (discrete orthonormality of the order functions under Gauss-Legendre
quadrature and of e^{i m phi_j} over the M equispaced phi), so PyTorch's
gradient is exactly 2 M beta; central differences of this quadratic in FP64;
and the oracle's transposed dense gradient 2 S^H W S beta."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _loss(f, w):
    return (w.view(1, -1, 1) * (f.real ** 2 + f.imag ** 2)).sum()


def test_gradcheck_small_f64():
    from paper_2004_11346_amd.autograd import sht_forward
    from paper_2004_11346_amd.sht import Plan
    print("autograd gradcheck N=3", flush=True)
    for method in ("dense", "idbf"):
        p = Plan(3, 1, dtype=torch.complex128, method=method)
        beta = torch.from_numpy(inputs.make_beta(3, 1, 5)).cuda().requires_grad_(True)
        assert torch.autograd.gradcheck(lambda b: sht_forward(b, p), (beta,), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_n512_batch8_f32():
    """N = 512, 8 fields, FP32 fast path (grid 1024 x 2047)."""
    from paper_2004_11346_amd.autograd import sht_forward
    from paper_2004_11346_amd.sht import Plan
    N, batch = 512, 8
    M = 4 * N - 1
    print("autograd N=512 batch 8 f32", flush=True)
    beta64 = inputs.make_beta(N, batch, 5).astype(np.complex64).astype(np.complex128)
    p32 = Plan(N, batch, dtype=torch.complex64, method="idbf")
    x, w = p32.nodes()
    wt32 = torch.from_numpy(w).float().cuda()
    beta = torch.from_numpy(beta64).to(torch.complex64).cuda().requires_grad_(True)
    f = sht_forward(beta, p32)
    loss = _loss(f, wt32)
    loss.backward()
    grad = beta.grad.detach().cpu().numpy().astype(np.complex128)

    # exact value of the gradient
    e_exact = rel_l2(grad, 2 * M * beta64)
    print("rel l2 vs 2 M beta:", e_exact, flush=True)
    assert e_exact <= 2e-6

    # FP64 central differences on 64 seeded coefficients, real and imaginary
    # directions.  |f+|^2 - |f-|^2 = Re(conj(f+ + f-) (f+ - f-)) avoids the
    # cancellation of two large losses.
    rng = np.random.default_rng(5064)
    picks = [(int(rng.integers(batch)), int(rng.integers(4 * N * N))) for _ in range(64)]
    dirs = [(b, i, d) for (b, i) in picks for d in (1.0, 1j)]
    chunk = 8
    p64 = Plan(N, 2 * chunk, dtype=torch.complex128, method="dense")
    wt64 = torch.from_numpy(w).cuda()
    h = 64.0  # any step is exact for a quadratic; a large one keeps f+ - f- well above rounding
    fd = np.empty(len(dirs), complex)
    for c0 in range(0, len(dirs), chunk):
        part = dirs[c0:c0 + chunk]
        bb = np.zeros((2 * chunk, 4 * N * N), complex)
        for j, (b, i, d) in enumerate(part):
            bb[2 * j] = beta64[b]
            bb[2 * j + 1] = beta64[b]
            bb[2 * j, i] += h * d
            bb[2 * j + 1, i] -= h * d
        for j in range(len(part), chunk):
            bb[2 * j] = bb[2 * j + 1] = beta64[0]
        ff = p64.forward(torch.from_numpy(bb).cuda())
        fp, fm = ff[0::2], ff[1::2]
        dl = (wt64.view(1, -1, 1) * (torch.conj(fp + fm) * (fp - fm)).real).sum(dim=(1, 2)) / (2 * h)
        fd[c0:c0 + len(part)] = dl.cpu().numpy()[:len(part)]
    got = np.array([grad[b, i].real if d == 1.0 else grad[b, i].imag for (b, i, d) in dirs])
    e_fd = rel_l2(got, fd.real)
    print("rel l2 vs FP64 central differences:", e_fd, flush=True)
    assert e_fd <= 2e-6
    # the differences themselves reproduce 2 M beta (a check of the FD harness)
    exact = np.array([(2 * M * beta64[b, i]).real if d == 1.0 else (2 * M * beta64[b, i]).imag
                      for (b, i, d) in dirs])
    assert rel_l2(fd.real, exact) <= 1e-10

    # the oracle's transposed dense gradient for field 0: 2 S^H W S beta
    f0 = oracle.sht_forward(N, beta64[0])
    g0 = 2 * oracle.sht_adjoint(N, w[:, None] * f0)
    e_or = rel_l2(grad[0], g0)
    print("rel l2 vs oracle adjoint gradient:", e_or, flush=True)
    assert e_or <= 2e-6
