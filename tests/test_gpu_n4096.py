"""N = 4096 (grid 8192 x 16383), 8 fields, variance (k+1)^-2: the fast ALT of
one GPU's share of the orders (a plan restricted to an order range, applied
with sht_alt_apply), in FP64 and in FP32 on the BF16 matrix cores, against the
oracle at sampled orders.  The full N = 4096 plan is not built here (the
share is what one GPU holds when the orders are distributed)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs

pytestmark = pytest.mark.gpu

N, BATCH = 4096, 8
M_LO, M_HI = 0, 31


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def fields():
    return inputs.make_beta(N, BATCH, 3, dist="decay")


@pytest.mark.parametrize("dtype,mode,tol", [(torch.complex128, 0, 1e-11), (torch.complex64, 2, 2e-6)])
def test_share_forward_and_inverse(fields, dtype, mode, tol):
    from paper_2004_11346_amd.sht import Plan
    print(f"N=4096 share [{M_LO}, {M_HI}] {dtype} mode {mode}: plan build", flush=True)
    p = Plan(N, BATCH, dtype=dtype, method="idbf", m_lo=M_LO, m_hi=M_HI, f32_mode=mode)
    print("plan", p.stats(), flush=True)
    beta_np = fields if dtype == torch.complex128 else fields.astype(np.complex64).astype(np.complex128)
    beta = torch.from_numpy(beta_np).to(dtype).cuda()
    M = 4 * N - 1
    g = torch.zeros((BATCH, 2 * N, M), dtype=dtype, device="cuda")
    p.alt(M_LO, M_HI, "fwd", beta, g)
    absm = [0, 1, 17, 31]
    worst = 0.0
    for b in (0, BATCH - 1):
        ref = oracle.alt_forward_orders(N, beta_np[b], absm)
        gb = g[b]
        got = np.stack([np.stack([gb[:, a % M].cpu().numpy(), gb[:, (-a) % M].cpu().numpy()]) for a in absm])
        worst = max(worst, rel_l2(got, ref))
    print(f"forward rel l2 at sampled orders: {worst:.3e}", flush=True)
    assert worst <= tol
    # transposed with weights, inputs = the oracle's g at the sampled orders
    ref = oracle.alt_forward_orders(N, beta_np[0], absm)
    gin = torch.zeros((BATCH, 2 * N, M), dtype=dtype, device="cuda")
    for i, a in enumerate(absm):
        gin[0, :, a % M] = torch.from_numpy(ref[i, 0]).to(dtype)
        gin[0, :, (-a) % M] = torch.from_numpy(ref[i, 1]).to(dtype)
    bo = torch.zeros((BATCH, 4 * N * N), dtype=dtype, device="cuda")
    p.alt(M_LO, M_HI, "inv", gin, bo)
    bref = oracle.alt_transpose_orders(N, ref, absm, weights=True)
    k_of, m_of = inputs.layout(N)
    bo0 = bo[0].cpu().numpy()
    worst = 0.0
    for i, a in enumerate(absm):
        for s, m in enumerate((a, -a) if a else (0,)):
            sel = np.nonzero(m_of == m)[0]
            worst = max(worst, rel_l2(bo0[sel], bref[i, s, : 2 * N - a]))
    print(f"inverse rel l2 at sampled orders: {worst:.3e}", flush=True)
    assert worst <= tol
    with pytest.raises(Exception):
        p.alt(0, M_HI + 1, "fwd", beta, g)  # outside the plan's orders
    p.close()
