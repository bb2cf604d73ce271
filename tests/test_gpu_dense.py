"""GPU parity of the plain (dense) ALT path and the phi DFT against the CPU
oracle, through the C-ABI.  Tolerances: FP64 relative l2 <= 1e-12 and relative
max <= 1e-11 (the dense path has no approximation, only rounding of a length-2N
recurrence and sum); FP32 storage (FP64 recurrence, FP32 DFT) <= 2e-6.
"""
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


def rel_max(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _plan(N, batch, dtype=torch.complex128, method="dense", **kw):
    from paper_2004_11346_amd.sht import Plan
    return Plan(N, batch, dtype=dtype, method=method, **kw)


def _to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


@pytest.mark.parametrize("N,batch", [(64, 1), (1, 1), (2, 2), (3, 1), (5, 3), (33, 5), (100, 2)])
def test_dense_forward_inverse_vs_oracle(N, batch):
    print(f"dense fwd/inv N={N} batch={batch}", flush=True)
    beta = inputs.make_beta(N, batch, 1)
    p = _plan(N, batch)
    f = p.forward(_to_dev(beta, torch.complex128)).cpu().numpy()
    for b in range(batch):
        ref = oracle.sht_forward(N, beta[b])
        assert rel_l2(f[b], ref) <= 1e-12, (b, rel_l2(f[b], ref))
        assert rel_max(f[b], ref) <= 1e-11
    # inverse of a generic (not band-limited) grid: same linear map as the oracle
    grid = inputs.make_grid(N, batch, 1)
    bi = p.inverse(_to_dev(grid, torch.complex128)).cpu().numpy()
    for b in range(batch):
        ref = oracle.sht_inverse(N, grid[b])
        assert rel_l2(bi[b], ref) <= 1e-12, (b, rel_l2(bi[b], ref))
    # round trip
    back = p.inverse(_to_dev(f, torch.complex128)).cpu().numpy()
    assert rel_l2(back, beta) <= 1e-12


@pytest.mark.parametrize("N,batch", [(16, 1), (70, 2)])
def test_dense_backward_is_adjoint(N, batch):
    print(f"dense adjoint N={N} batch={batch}", flush=True)
    p = _plan(N, batch)
    y = inputs.make_grid(N, batch, 7)
    gb = p.backward(_to_dev(y, torch.complex128)).cpu().numpy()
    for b in range(batch):
        ref = oracle.sht_adjoint(N, y[b])
        assert rel_l2(gb[b], ref) <= 1e-12


def test_dense_alt_apply_order_range():
    N, batch = 40, 2
    print("dense alt_apply range", flush=True)
    p = _plan(N, batch)
    beta = inputs.make_beta(N, batch, 3)
    M = 4 * N - 1
    g = torch.full((batch, 2 * N, M), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    lo, hi = 11, 29
    p.alt(lo, hi, "fwd", _to_dev(beta, torch.complex128), g)
    g = g.cpu().numpy()
    cols = set()
    for a in range(lo, hi + 1):
        cols.add(a % M)
        cols.add((-a) % M)
    for b in range(batch):
        ref = oracle.alt_forward(N, beta[b])
        for c in range(M):
            if c in cols:
                assert rel_l2(g[b][:, c], ref[:, c]) <= 1e-12
            else:
                assert np.all(g[b][:, c] == 7.0)
    # transposed with weights over the same range
    gin = inputs.make_grid(N, batch, 4)
    bo = torch.zeros((batch, 4 * N * N), dtype=torch.complex128, device="cuda")
    p.alt(lo, hi, "inv", _to_dev(gin, torch.complex128), bo)
    bo = bo.cpu().numpy()
    k_of, m_of = inputs.layout(N)
    sel = (np.abs(m_of) >= lo) & (np.abs(m_of) <= hi)
    for b in range(batch):
        ref = oracle.alt_transpose(N, gin[b], weights=True)
        assert rel_l2(bo[b][sel], ref[sel]) <= 1e-12
        assert np.all(bo[b][~sel] == 0)


@pytest.mark.parametrize("N,batch", [(64, 1), (48, 3)])
def test_dense_f32(N, batch):
    print(f"dense f32 N={N}", flush=True)
    beta = inputs.make_beta(N, batch, 1).astype(np.complex64)
    p = _plan(N, batch, dtype=torch.complex64)
    f = p.forward(_to_dev(beta, torch.complex64)).cpu().numpy()
    for b in range(batch):
        ref = oracle.sht_forward(N, beta[b].astype(np.complex128))
        assert rel_l2(f[b], ref) <= 2e-6
    back = p.inverse(_to_dev(f, torch.complex64)).cpu().numpy()
    assert rel_l2(back, beta) <= 4e-6


def test_dense_n1024_sampled():
    """Full-size plain path at N = 1024 (grid 2048 x 4095): the ALT at sampled
    orders and the full SHT at sampled latitude rows, against the oracle."""
    N = 1024
    print("dense N=1024 sampled", flush=True)
    beta = inputs.make_beta(N, 1, 2, dist="decay")
    p = _plan(N, 1)
    bd = _to_dev(beta, torch.complex128)
    M = 4 * N - 1
    g = torch.zeros((1, 2 * N, M), dtype=torch.complex128, device="cuda")
    p.alt(0, 2 * N - 1, "fwd", bd, g)
    g = g.cpu().numpy()[0]
    absm = [0, 1, N // 2, N, 3 * N // 2, 2 * N - 1] + list(inputs.sample_indices(2 * N, 6, 11))
    ref = oracle.alt_forward_orders(N, beta[0], absm)
    for i, a in enumerate(absm):
        got = np.stack([g[:, a % M], g[:, (-a) % M]])
        assert rel_l2(got, ref[i]) <= 1e-12, (a, rel_l2(got, ref[i]))
    f = p.forward(bd).cpu().numpy()[0]
    rows = inputs.sample_indices(2 * N, 8, 12)
    fr = oracle.dft_synthesis(N, g, rows=rows)  # DFT of the GPU's own (checked) g
    assert rel_l2(f[rows], fr) <= 1e-12


@pytest.mark.parametrize("N,batch", [(70, 8), (33, 33), (130, 4)])
def test_dense_matrix_core_paths(N, batch):
    """Many right-hand sides: pack -> MFMA forward -> combine and fold -> MFMA
    transpose -> scatter, including a partial last column pass."""
    print(f"dense mfma N={N} batch={batch}", flush=True)
    p = _plan(N, batch)
    beta = inputs.make_beta(N, batch, 8)
    f = p.forward(_to_dev(beta, torch.complex128)).cpu().numpy()
    grid = inputs.make_grid(N, batch, 8)
    bi = p.inverse(_to_dev(grid, torch.complex128)).cpu().numpy()
    ba = p.backward(_to_dev(grid, torch.complex128)).cpu().numpy()
    for b in sorted({0, batch // 2, batch - 1}):
        assert rel_l2(f[b], oracle.sht_forward(N, beta[b])) <= 1e-12
        assert rel_l2(bi[b], oracle.sht_inverse(N, grid[b])) <= 1e-12
        assert rel_l2(ba[b], oracle.sht_adjoint(N, grid[b])) <= 1e-12


def test_dense_n1024_four_fields_sampled():
    N, batch = 1024, 4
    print("dense N=1024 batch 4 sampled", flush=True)
    beta = inputs.make_beta(N, batch, 2, dist="decay")
    p = _plan(N, batch)
    M = 4 * N - 1
    g = torch.zeros((batch, 2 * N, M), dtype=torch.complex128, device="cuda")
    p.alt(0, 2 * N - 1, "fwd", _to_dev(beta, torch.complex128), g)
    g = g.cpu().numpy()
    absm = [0, 3, N - 1, 2 * N - 2]
    for b in (0, 3):
        ref = oracle.alt_forward_orders(N, beta[b], absm)
        got = np.stack([np.stack([g[b][:, a % M], g[b][:, (-a) % M]]) for a in absm])
        assert rel_l2(got, ref) <= 1e-12
    # transposed with weights at the same orders (inputs: the oracle's g)
    gin = np.zeros((batch, 2 * N, M), complex)
    refs = {}
    for b in (0, 3):
        refs[b] = oracle.alt_forward_orders(N, beta[b], absm)
        for i, a in enumerate(absm):
            gin[b][:, a % M] = refs[b][i, 0]
            gin[b][:, (-a) % M] = refs[b][i, 1]
    bo = torch.zeros((batch, 4 * N * N), dtype=torch.complex128, device="cuda")
    p.alt(0, 2 * N - 1, "inv", _to_dev(gin, torch.complex128), bo)
    bo = bo.cpu().numpy()
    k_of, m_of = inputs.layout(N)
    for b in (0, 3):
        bref = oracle.alt_transpose_orders(N, refs[b], absm, weights=True)
        for i, a in enumerate(absm):
            for sgn, m in enumerate((a, -a) if a else (0,)):
                assert rel_l2(bo[b][m_of == m], bref[i, sgn, : 2 * N - a]) <= 1e-12


@pytest.mark.parametrize("N,batch", [(70, 4), (130, 3)])
def test_dense_transpose_in_state_chunks(N, batch, monkeypatch):
    """The transposed product records its recurrence states a chunk of tasks
    at a time; a tiny state buffer forces one or two tasks per chunk."""
    monkeypatch.setenv("SHT_DENSE_CKPT_STATES", "1")
    print(f"dense transpose chunks N={N} batch={batch}", flush=True)
    p = _plan(N, batch)
    grid = inputs.make_grid(N, batch, 3)
    bi = p.inverse(_to_dev(grid, torch.complex128)).cpu().numpy()
    ba = p.backward(_to_dev(grid, torch.complex128)).cpu().numpy()
    for b in sorted({0, batch - 1}):
        assert rel_l2(bi[b], oracle.sht_inverse(N, grid[b])) <= 1e-12
        assert rel_l2(ba[b], oracle.sht_adjoint(N, grid[b])) <= 1e-12
