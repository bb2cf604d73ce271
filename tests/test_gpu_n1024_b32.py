"""N = 1024 with 32 fields (grid 2048 x 4095, R = 128 right-hand sides per
task): the configuration the benchmark times, in its launch configuration,
through the C ABI.  The forward ALT of seeded coefficients and the weighted
transposed ALT of a seeded grid that is nonzero at the sampled orders only are
compared with the oracle at those orders, for three fields, in both forms.
Bars: 1e-12 (plain form, rounding only) and 1e-11 (fast form)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


@pytest.mark.parametrize("method,tol,kw", [("dense", 1e-12, {}), ("idbf", 1e-11, {}), ("idbf", 1e-11, {"leaf": 32})])
def test_n1024_32_fields_sampled_orders(method, tol, kw):
    from paper_2004_11346_amd.sht import Plan
    N, batch = 1024, 32
    M = 4 * N - 1
    print(f"{method} {kw} N=1024 batch 32 sampled (plan build)", flush=True)
    p = Plan(N, batch, dtype=torch.complex128, method=method, **kw)
    beta = inputs.make_beta(N, batch, 2, dist="decay")
    absm = sorted({0, 1, N // 2, N, 3 * N // 2, 2 * N - 1} | {int(a) for a in inputs.sample_indices(2 * N, 6, 21)})
    fields = (0, 17, 31)
    g = torch.zeros((batch, 2 * N, M), dtype=torch.complex128, device="cuda")
    p.alt(0, 2 * N - 1, "fwd", torch.from_numpy(beta).cuda(), g)
    cols = sorted({a % M for a in absm} | {(-a) % M for a in absm})
    gs = g[list(fields)][:, :, cols].cpu().numpy()
    pos = {c: i for i, c in enumerate(cols)}
    del g
    for i, b in enumerate(fields):
        ref = oracle.alt_forward_orders(N, beta[b], absm)
        got = np.stack([np.stack([gs[i][:, pos[a % M]], gs[i][:, pos[(-a) % M]]]) for a in absm])
        e = rel_l2(got, ref)
        print(f"field {b}: forward rel l2 {e:.2e}", flush=True)
        assert e <= tol
    # weighted transposed ALT of a seeded grid living on the sampled orders
    rng = np.random.default_rng(7021)
    gin = {b: (rng.standard_normal((len(absm), 2, 2 * N)) + 1j * rng.standard_normal((len(absm), 2, 2 * N))) / np.sqrt(2)
           for b in fields}
    gdev = torch.zeros((batch, 2 * N, M), dtype=torch.complex128, device="cuda")
    for b in fields:
        for i, a in enumerate(absm):
            gdev[b, :, a % M] = torch.from_numpy(gin[b][i, 0]).cuda()
            if a:
                gdev[b, :, (-a) % M] = torch.from_numpy(gin[b][i, 1]).cuda()
    bo = torch.zeros((batch, 4 * N * N), dtype=torch.complex128, device="cuda")
    p.alt(0, 2 * N - 1, "inv", gdev, bo)
    bo = bo[list(fields)].cpu().numpy()
    k_of, m_of = inputs.layout(N)
    for i, b in enumerate(fields):
        gi = gin[b].copy()
        gi[0, 1] = 0.0  # m = 0 has a single column
        bref = oracle.alt_transpose_orders(N, gi, absm, weights=True)
        worst = 0.0
        for q, a in enumerate(absm):
            for sgn, m in enumerate((a, -a) if a else (0,)):
                worst = max(worst, rel_l2(bo[i][m_of == m], bref[q, sgn, : 2 * N - a]))
        print(f"field {b}: transposed worst order rel l2 {worst:.2e}", flush=True)
        assert worst <= tol


@pytest.mark.parametrize("f32_mode,name", [(0, "fp32 storage, FP64 matrix cores"), (2, "split-BF16 six products")])
def test_n1024_32_fields_fp32_fast_forms(f32_mode, name):
    """The FP32 fast forms at the benchmark's configuration against the FP64
    oracle (on the FP32-rounded coefficients) at sampled orders, held to the
    FP32 bar 2e-6: FP32 storage with FP64 products, and the split-BF16 form
    with six products (stored factors on the BF16 matrix cores, regenerated
    blocks on the FP64 matrix cores)."""
    from paper_2004_11346_amd.sht import Plan
    N, batch = 1024, 32
    M = 4 * N - 1
    print(f"FP32 {name} N=1024 batch 32 (plan build)", flush=True)
    p = Plan(N, batch, dtype=torch.complex64, method="idbf", f32_mode=f32_mode)
    beta = inputs.make_beta(N, batch, 2, dist="decay").astype(np.complex64)
    absm = sorted({0, 1, N // 2, N, 3 * N // 2, 2 * N - 1} | {int(a) for a in inputs.sample_indices(2 * N, 6, 22)})
    g = torch.zeros((batch, 2 * N, M), dtype=torch.complex64, device="cuda")
    p.alt(0, 2 * N - 1, "fwd", torch.from_numpy(beta).cuda(), g)
    for b in (0, 31):
        ref = oracle.alt_forward_orders(N, beta[b].astype(np.complex128), absm)
        gb = g[b].cpu().numpy().astype(np.complex128)
        got = np.stack([np.stack([gb[:, a % M], gb[:, (-a) % M]]) for a in absm])
        e = rel_l2(got, ref)
        print(f"field {b}: forward rel l2 {e:.2e}", flush=True)
        assert e <= 2e-6
    p.close()
