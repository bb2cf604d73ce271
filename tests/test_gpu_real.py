"""Real fields (sht_forward_real / sht_inverse_real: coefficients of orders
m >= 0 only, real grids, two real fields per complex transform) against the
oracle's real-field transforms, through the C ABI: plain and fast form, FP64
and FP32, an odd number of real fields (the last pair half empty), and the
N = 1024 workload shape at sampled rows and orders."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-12, torch.complex64: 2e-6}


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _half(N, nreal, seed, dtype):
    h = inputs.make_beta(N, nreal, seed)[:, : N * (2 * N + 1)].copy()
    return h if dtype == torch.complex128 else h.astype(np.complex64).astype(np.complex128)


def _real_grid(N, nreal, seed, dtype):
    g = inputs.make_grid(N, nreal, seed).real.copy()
    return g if dtype == torch.complex128 else g.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("method,kw", [("dense", {}), ("idbf", {}), ("idbf", dict(n0=32, leaf=8))])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("N,batch,nreal", [(1, 1, 1), (2, 1, 2), (5, 2, 3), (16, 2, 4), (33, 1, 2), (64, 2, 3)])
def test_real_fields_vs_oracle(N, batch, nreal, method, kw, dtype):
    from paper_2004_11346_amd.sht import Plan
    if kw and N < 64:
        pytest.skip("small partition options need N >= 64")
    print(f"real fields N={N} batch={batch} nreal={nreal} {method} {kw} {dtype}", flush=True)
    p = Plan(N, batch, dtype=dtype, method=method, **kw)
    half = _half(N, nreal, 70, dtype)
    f = p.forward_real(torch.from_numpy(half).to(dtype).cuda())
    grid = _real_grid(N, nreal, 71, dtype)
    bh = p.inverse_real(torch.from_numpy(grid).to(p.real_dtype).cuda())
    back = p.inverse_real(f)
    torch.cuda.synchronize()
    fh, bhh, backh = f.cpu().numpy(), bh.cpu().numpy(), back.cpu().numpy()
    for b in range(nreal):
        assert rel_l2(fh[b], oracle.sht_forward_real(N, half[b])) <= TOL[dtype], ("forward", b)
        assert rel_l2(bhh[b], oracle.sht_inverse_real(N, grid[b])) <= TOL[dtype], ("inverse", b)
        ref = half[b].copy()
        ref[: 2 * N] = ref[: 2 * N].real
        assert rel_l2(backh[b], ref) <= TOL[dtype], ("round trip", b)
    p.close()


def test_real_fields_agree_with_complex_transform():
    """The real transform of fields (f1, f2) equals the complex transform of
    the extended coefficients, field by field (same kernels, same plan)."""
    from paper_2004_11346_amd.sht import Plan
    N, batch = 48, 2
    p = Plan(N, batch, method="idbf")
    half = _half(N, 4, 72, torch.complex128)
    full = np.stack([oracle.real_to_full(N, h) for h in half])
    fr = p.forward_real(torch.from_numpy(half).cuda()).cpu().numpy()
    for b0 in (0, 2):
        fc = p.forward(torch.from_numpy(full[b0:b0 + 2]).cuda()).cpu().numpy()
        for j in range(2):
            assert rel_l2(fr[b0 + j], fc[j].real) <= 1e-13
            assert np.abs(fc[j].imag).max() <= 1e-12 * np.abs(fc[j].real).max()
    p.close()


def test_real_fields_n1024_sampled():
    """N = 1024, 8 real fields on a plan of 4 complex fields (fast form):
    forward at sampled rows against the oracle's full ALT at those rows and its
    direct phi sums; inverse by round trip."""
    from paper_2004_11346_amd.sht import Plan
    N, batch, nreal = 1024, 4, 8
    print("real fields N=1024", flush=True)
    p = Plan(N, batch, method="idbf")
    half = inputs.make_beta(N, nreal, 73, dist="decay")[:, : N * (2 * N + 1)].copy()
    ft = p.forward_real(torch.from_numpy(half).cuda())
    rows = [0, 777, 2 * N - 1]
    worst = 0.0
    for b in (0, nreal - 1):
        full = oracle.real_to_full(N, half[b])
        g = oracle.alt_forward_rows(N, full, rows)
        gg = np.zeros((2 * N, 4 * N - 1), complex)
        gg[rows] = g
        ref = oracle.dft_synthesis(N, gg, rows=rows).real
        worst = max(worst, rel_l2(ft[b, rows].cpu().numpy(), ref))
    print(f"forward rel l2 at sampled rows: {worst:.3e}", flush=True)
    assert worst <= 1e-11
    back = p.inverse_real(ft).cpu().numpy()
    ref = half.copy()
    ref[:, : 2 * N] = ref[:, : 2 * N].real
    rt = rel_l2(back, ref)
    print(f"round trip: {rt:.3e}", flush=True)
    assert rt <= 1e-11
    p.close()
