"""N = 4096 (grid 8192 x 16383), 8 fields, variance (k+1)^-2: the fast ALT of
windows of 16 orders spread over the whole order range (plans restricted to
an order range, applied with sht_alt_apply), in FP64 and in FP32 on the BF16
matrix cores (six products), against the oracle at sampled orders of fields 0
and 7, forward and weighted transpose.  The windows reach the high orders
where the recurrence starts far below the binary64 range, many blocks are
dropped as negligible and turning-point blocks dominate (Section 3.2)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs

pytestmark = pytest.mark.gpu

N, BATCH = 4096, 8
WINDOWS = [(0, 15), (2048, 2063), (4096, 4111), (6144, 6159), (8176, 8191)]


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def fields():
    return inputs.make_beta(N, BATCH, 3, dist="decay")


@pytest.mark.parametrize("window", WINDOWS)
@pytest.mark.parametrize("dtype,mode,tol", [(torch.complex128, 0, 1e-11), (torch.complex64, 2, 2e-6)])
def test_window_forward_and_inverse(fields, window, dtype, mode, tol):
    from paper_2004_11346_amd.sht import Plan
    lo, hi = window
    print(f"N=4096 window [{lo}, {hi}] {dtype} mode {mode}: plan build", flush=True)
    p = Plan(N, BATCH, dtype=dtype, method="idbf", m_lo=lo, m_hi=hi, f32_mode=mode)
    print("plan", p.stats(), flush=True)
    beta_np = fields if dtype == torch.complex128 else fields.astype(np.complex64).astype(np.complex128)
    beta = torch.from_numpy(beta_np).to(dtype).cuda()
    M = 4 * N - 1
    g = torch.zeros((BATCH, 2 * N, M), dtype=dtype, device="cuda")
    p.alt(lo, hi, "fwd", beta, g)
    absm = sorted({lo, lo + 1, lo + 7, hi})
    worst = 0.0
    refs = {}
    for b in (0, BATCH - 1):
        ref = oracle.alt_forward_orders(N, beta_np[b], absm)
        refs[b] = ref
        gb = g[b]
        got = np.stack([np.stack([gb[:, a % M].cpu().numpy(), gb[:, (-a) % M].cpu().numpy()]) for a in absm])
        worst = max(worst, rel_l2(got, ref))
    print(f"forward rel l2 at orders {absm}: {worst:.3e}", flush=True)
    assert worst <= tol
    # transposed with weights, inputs = the oracle's g at the sampled orders of fields 0 and 7
    gin = torch.zeros((BATCH, 2 * N, M), dtype=dtype, device="cuda")
    for b, ref in refs.items():
        for i, a in enumerate(absm):
            gin[b, :, a % M] = torch.from_numpy(ref[i, 0]).to(dtype)
            gin[b, :, (-a) % M] = torch.from_numpy(ref[i, 1]).to(dtype)
    bo = torch.zeros((BATCH, 4 * N * N), dtype=dtype, device="cuda")
    p.alt(lo, hi, "inv", gin, bo)
    k_of, m_of = inputs.layout(N)
    worst = 0.0
    for b, ref in refs.items():
        gref = ref if dtype == torch.complex128 else ref.astype(np.complex64).astype(np.complex128)
        bref = oracle.alt_transpose_orders(N, gref, absm, weights=True)
        bob = bo[b].cpu().numpy()
        for i, a in enumerate(absm):
            for s, m in enumerate((a, -a) if a else (0,)):
                sel = np.nonzero(m_of == m)[0]
                worst = max(worst, rel_l2(bob[sel], bref[i, s, : 2 * N - a]))
    print(f"inverse rel l2 at orders {absm}: {worst:.3e}", flush=True)
    assert worst <= tol
    outside = (lo, hi + 1) if hi + 1 < 2 * N else (lo - 1, hi)
    with pytest.raises(Exception):
        p.alt(outside[0], outside[1], "fwd", beta, g)  # orders the plan does not hold
    p.close()
