"""The three phi DFT schedules (Section 1, eq. `sht_fft`: rows in LDS, Rader's
convolution for prime M = 4N - 1, four-step through a grid-sized buffer)
against the oracle, through the C ABI.

* Every schedule is forced at small N, where the oracle computes the whole
  transform: forward SHT, adjoint and round trip, FP64 and FP32 (plain ALT,
  so only the DFT schedule changes).
* A prime factor R of a four-step length (R >= 41) or of a row (R >= 80)
  whose R - 1 splits into radices up to 13 runs as the last pass by Rader's
  convolution (four-step 73 x 7 for M = 511, 43 x 41 for 1763 = 41 43, and
  129 x 127 at N = 4096; rows of 267 = 3 89 and 2047 = 23 89); the plan stats
  name it.
* The persistent row kernel over more rows than its workgroups (N = 16,
  33 fields: a partial last round), both ALT forms, every field.
* At N = 1500 the forced four-step runs with partial chunks in both kernels.
* At N = 2048 (M = 8191 prime: Rader) and N = 4096 (M = 16383 = 3 43 127:
  four-step), where the full oracle transform takes too
  long, the forward SHT of coefficients that are non-zero at a few orders only
  is compared at sampled rows with the oracle's ALT of those orders followed by
  its direct phi sums; the inverse is checked by round trip and the adjoint by
  the dot-product identity <S b, y> = <b, S^H y>.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs
from paper_2004_11346_amd import lib as L

pytestmark = pytest.mark.gpu

SCHED = {"rows": L.SHT_DFT_ROWS, "rader": L.SHT_DFT_RADER, "four_step": L.SHT_DFT_FOUR_STEP}
TOL = {torch.complex128: 1e-12, torch.complex64: 2e-6}
# large N: the FP64 bar of the whole path (the plain ALT's recurrence over
# thousands of degrees dominates the error there)
TOL_LARGE = {torch.complex128: 1e-11, torch.complex64: 2e-6}


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _cast(a, dtype):
    return a if dtype == torch.complex128 else a.astype(np.complex64).astype(np.complex128)


# (N, schedule): M = 19 (prime), 63 = 3^2 7, 131 (prime), 255 = 3 5 17
# (17 as a generic pass; four-step 17 x 15), 519 = 3 173 (172 = 4 43: a
# generic pass / four-step 173 x 3), 511 = 7 73 (73 generic in the rows, by
# Rader's convolution in the four-step 73 x 7), 267 = 3 89 (89 by Rader's
# convolution in the rows)
CASES = [(5, "rows"), (5, "rader"), (16, "rows"), (16, "four_step"), (33, "rader"), (33, "rows"),
         (64, "rows"), (64, "four_step"), (130, "rows"), (130, "four_step"), (128, "rows"), (128, "four_step"),
         (67, "rows")]


@pytest.mark.parametrize("N,sched,dtype,kind,expect", [
    (64, "rows", torch.complex128, "rows", [0, 0]),         # 17: the direct sums are as fast
    (67, "rows", torch.complex128, "rows", [89, 0]),
    (128, "rows", torch.complex128, "rows", [0, 0]),        # 73 in rows: the direct sums are faster
    (128, "four_step", torch.complex128, "four_step", [73, 0]),  # M1 = 73, M2 = 7
    (130, "rows", torch.complex128, "rows", [0, 0]),        # 173 - 1 = 4 43: no register radices
    (441, None, torch.complex128, "rows", [0, 0]),          # 1763 = 41 43: rows with direct sums
    (441, "four_step", torch.complex128, "four_step", [43, 41]),
    (512, None, torch.complex128, "rows", [89, 0]),         # 2047 = 23 89: 23 stays a generic pass
    (4096, None, torch.complex128, "four_step", [43, 127]),  # 129 x 127
    (4096, None, torch.complex64, "four_step", [43, 127]),   # FP32 rows would keep 43 and 127 generic
    (1024, None, torch.complex128, "rows", [0, 0]),         # 4095: register radices only
])
def test_rader_last_pass_schedule(N, sched, dtype, kind, expect):
    """Which prime factor of M runs as a last pass by Rader's convolution, per
    pass list (rows or the first four-step kernel, then the second), and the
    schedule chosen by length."""
    from paper_2004_11346_amd.sht import Plan
    kw = {} if sched is None else {"dft_schedule": SCHED[sched]}
    p = Plan(N, 1, dtype=dtype, method="dense", **kw)
    st = p.stats()
    assert st["dft"] == kind
    assert st["dft_rader_last"] == expect


def test_rader_last_pass_in_both_four_step_kernels():
    """M = 1763 = 41 43: four-step 43 x 41 with a Rader last pass in each
    kernel; the whole FP64 transform against the oracle."""
    from paper_2004_11346_amd.sht import Plan
    N = 441
    print(f"dft four-step with two Rader last passes N={N}", flush=True)
    p = Plan(N, 1, dtype=torch.complex128, method="dense", dft_schedule=SCHED["four_step"])
    assert p.stats()["dft_rader_last"] == [43, 41]
    beta = inputs.make_beta(N, 1, 21)
    f = p.forward(torch.from_numpy(beta).cuda()).cpu().numpy()
    assert rel_l2(f[0], oracle.sht_forward(N, beta[0])) <= TOL[torch.complex128]
    grid = inputs.make_grid(N, 1, 22)
    adj = p.backward(torch.from_numpy(grid).cuda()).cpu().numpy()
    assert rel_l2(adj[0], oracle.sht_adjoint(N, grid[0])) <= TOL[torch.complex128]
    p.close()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("N,sched", CASES)
def test_forced_schedule_vs_oracle(N, sched, dtype):
    from paper_2004_11346_amd.sht import Plan
    print(f"dft schedule {sched} N={N} {dtype}", flush=True)
    batch = 2
    p = Plan(N, batch, dtype=dtype, method="dense", dft_schedule=SCHED[sched])
    beta = _cast(inputs.make_beta(N, batch, 1), dtype)
    bd = torch.from_numpy(beta).to(dtype).cuda()
    f = p.forward(bd)
    back = p.inverse(f)
    grid = _cast(inputs.make_grid(N, batch, 5), dtype)
    adj = p.backward(torch.from_numpy(grid).to(dtype).cuda())
    torch.cuda.synchronize()
    fh, bh, ah = f.cpu().numpy(), back.cpu().numpy(), adj.cpu().numpy()
    for b in range(batch):
        assert rel_l2(fh[b], oracle.sht_forward(N, beta[b])) <= TOL[dtype], b
        assert rel_l2(ah[b], oracle.sht_adjoint(N, grid[b])) <= TOL[dtype], b
    assert rel_l2(bh, beta) <= TOL[dtype]
    p.close()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("method", ["dense", "idbf"])
def test_persistent_rows_partial_last_round(dtype, method):
    """The persistent row kernel (rows of at most 4096 points with register
    radices, two workgroups per CU taking rows in turn, the next row loaded
    during the current one's passes) over 33 fields of N = 16 (M = 63 = 9 7):
    1056 rows, so the last round of the workgroups is partial; forward,
    inverse and adjoint against the oracle for every field."""
    from paper_2004_11346_amd.sht import Plan
    N, batch = 16, 33
    print(f"dft persistent rows N={N} batch={batch} {method} {dtype}", flush=True)
    kw = {"n0": 8, "leaf": 8} if method == "idbf" else {}
    p = Plan(N, batch, dtype=dtype, method=method, **kw)
    assert p.stats()["dft"] == "rows"
    beta = _cast(inputs.make_beta(N, batch, 41), dtype)
    grid = _cast(inputs.make_grid(N, batch, 42), dtype)
    f = p.forward(torch.from_numpy(beta).to(dtype).cuda()).cpu().numpy()
    bi = p.inverse(torch.from_numpy(grid).to(dtype).cuda()).cpu().numpy()
    ba = p.backward(torch.from_numpy(grid).to(dtype).cuda()).cpu().numpy()
    # the fast form's FP64 factors carry the 1e-12 ID tolerance
    tol = 1e-11 if (method == "idbf" and dtype == torch.complex128) else TOL[dtype]
    for b in range(batch):
        assert rel_l2(f[b], oracle.sht_forward(N, beta[b])) <= tol, b
        assert rel_l2(bi[b], oracle.sht_inverse(N, grid[b])) <= tol, b
        assert rel_l2(ba[b], oracle.sht_adjoint(N, grid[b])) <= tol, b
    p.close()


def test_schedule_that_does_not_apply_is_refused():
    from paper_2004_11346_amd.sht import Plan
    from paper_2004_11346_amd.lib import ShtError
    with pytest.raises(ShtError):
        Plan(16, 1, method="dense", dft_schedule=L.SHT_DFT_RADER)  # M = 63 is not prime
    with pytest.raises(ShtError):
        Plan(5, 1, method="dense", dft_schedule=L.SHT_DFT_FOUR_STEP)  # M = 19 has no split


def _sparse_beta(N, orders, seed):
    """Coefficients that are non-zero only at the listed signed orders, with the
    workloads' variance (k + 1)^-2."""
    k_of, m_of = inputs.layout(N)
    beta = inputs.make_beta(N, 1, seed, dist="decay")[0]
    keep = np.isin(m_of, orders)
    beta[~keep] = 0
    return beta


def _expected_rows(N, beta, orders, rows):
    """The oracle's f at the listed rows for coefficients supported on `orders`."""
    M = 4 * N - 1
    absm = sorted({abs(m) for m in orders})
    ga = oracle.alt_forward_orders(N, beta, absm)
    g = np.zeros((2 * N, M), dtype=np.complex128)
    for i, a in enumerate(absm):
        g[:, a % M] = ga[i, 0]
        if a:
            g[:, (-a) % M] = ga[i, 1]
    return oracle.dft_synthesis(N, g, rows=rows)


@pytest.mark.parametrize("N,dtype,sched", [(512, torch.complex128, None), (1500, torch.complex128, "four_step"),
                                           (2048, torch.complex128, None),
                                           (4096, torch.complex128, None), (4096, torch.complex64, None),
                                           (2048, torch.complex64, None)])
def test_large_rows_vs_oracle(N, dtype, sched):
    from paper_2004_11346_amd.sht import Plan
    kw = {} if sched is None else {"dft_schedule": SCHED[sched]}
    print(f"dft large N={N} {dtype} {sched or 'auto'}", flush=True)
    p = Plan(N, 1, dtype=dtype, method="dense", **kw)
    orders = [0, 1, -1, 7, -300, N, -(N + 1), 2 * N - 1, -(2 * N - 1)]
    beta = _cast(_sparse_beta(N, orders, 11), dtype)
    f = p.forward(torch.from_numpy(beta[None]).to(dtype).cuda())
    rows = [0, 1, N - 1, N, 2 * N - 3]
    got = f[0, rows].cpu().numpy()
    err = rel_l2(got, _expected_rows(N, beta, orders, rows))
    # the ALT alone at the same orders and rows, to separate the DFT's share
    M = 4 * N - 1
    g = torch.zeros((1, 2 * N, M), dtype=dtype, device="cuda")
    p.alt(0, 2 * N - 1, "fwd", torch.from_numpy(beta[None]).to(dtype).cuda(), g)
    absm = sorted({abs(m) for m in orders})
    ga = oracle.alt_forward_orders(N, beta, absm)
    cols = [c for a in absm for c in ((a % M, (-a) % M) if a else (0,))]
    ref_g = np.stack([ga[i, s][rows] for i, a in enumerate(absm) for s in ((0, 1) if a else (0,))])
    err_alt = rel_l2(g[0][rows][:, cols].cpu().numpy().T, ref_g)
    print(f"forward at sampled rows: {err:.3e} (ALT alone at those rows and orders: {err_alt:.3e})", flush=True)
    assert err <= TOL_LARGE[dtype]
    # round trip on generic coefficients
    bfull = _cast(inputs.make_beta(N, 1, 12, dist="decay"), dtype)
    bt = torch.from_numpy(bfull).to(dtype).cuda()
    back = p.inverse(p.forward(bt))
    rt = rel_l2(back.cpu().numpy(), bfull)
    print(f"round trip: {rt:.3e}", flush=True)
    assert rt <= TOL_LARGE[dtype]
    # adjoint: <S b, y> = <b, S^H y>
    y = torch.from_numpy(_cast(inputs.make_grid(N, 1, 13), dtype)).to(dtype).cuda()
    sb = p.forward(bt)
    shy = p.backward(y)
    lhs = torch.vdot(y.reshape(-1).to(torch.complex128), sb.reshape(-1).to(torch.complex128)).item()
    rhs = torch.vdot(shy.reshape(-1).to(torch.complex128), bt.reshape(-1).to(torch.complex128)).item()
    rel = abs(lhs - rhs) / abs(lhs)
    print(f"adjoint identity: {rel:.3e}", flush=True)
    assert rel <= TOL_LARGE[dtype]
    p.close()
