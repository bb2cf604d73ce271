"""Non-finite inputs (the C ABI's promise: kernels never abort, NaN and Inf
propagate).  Every step of the path keeps right-hand sides apart (each real
part, imaginary part, field and sign of m is its own column of the per-order
products), so a NaN or Inf placed in one coefficient of order m0 of one field
must reach some outputs of that order and field, and must leave every other
order and field bitwise as in a clean run.  The phi DFT then mixes the orders
of a grid row: the full transform turns the touched rows of that field
non-finite and leaves the other fields bitwise unchanged."""
import numpy as np
import pytest
import torch

from paper_2004_11346_amd import inputs

pytestmark = pytest.mark.gpu

PLANS = [
    ("dense", 2, {}),
    ("dense", 4, {}),
    ("idbf", 2, dict(n0=32, leaf=8, rsvd_r=4)),
    ("idbf", 8, dict(n0=32, leaf=8, rsvd_r=4)),
]


def _plan(N, batch, method, dtype, kw):
    from paper_2004_11346_amd.sht import Plan
    return Plan(N, batch, dtype=dtype, method=method, **kw)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("method,batch,kw", PLANS)
def test_nonfinite_forward_stays_in_its_order(method, batch, kw, dtype):
    N = 64
    M = 4 * N - 1
    print(f"nonfinite fwd {method} batch={batch} {dtype}", flush=True)
    p = _plan(N, batch, method, dtype, kw)
    beta = inputs.make_beta(N, batch, 7)
    bad = beta.copy()
    m0, m1 = 5, -17
    bad[0, inputs.slot(N, 20, m0)] = complex(np.nan, 0.0)
    bad[batch - 1, inputs.slot(N, 40, m1)] = complex(0.0, np.inf)
    bc = torch.from_numpy(beta).to(dtype).cuda()
    bb = torch.from_numpy(bad).to(dtype).cuda()
    g_clean = torch.zeros((batch, 2 * N, M), dtype=dtype, device="cuda")
    g_bad = torch.zeros_like(g_clean)
    p.alt(0, 2 * N - 1, "fwd", bc, g_clean)
    p.alt(0, 2 * N - 1, "fwd", bb, g_bad)
    gc, gb = g_clean.cpu().numpy(), g_bad.cpu().numpy()
    touched = {(0, m0 % M), (batch - 1, m1 % M)}
    for b, c in touched:
        assert not np.all(np.isfinite(gb[b][:, c])), (b, c)
    mask = np.ones(gc.shape, bool)
    for b, c in touched:
        mask[b][:, c] = False
    assert np.array_equal(gb[mask], gc[mask])
    # full transform: the rows of the touched fields become non-finite, other fields unchanged
    f_clean = p.forward(bc).cpu().numpy()
    f_bad = p.forward(bb).cpu().numpy()
    for b in {0, batch - 1}:
        assert not np.all(np.isfinite(f_bad[b]))
    for b in range(1, batch - 1):
        assert np.array_equal(f_bad[b], f_clean[b])


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("method,batch,kw", PLANS)
def test_nonfinite_transposed_stays_in_its_order(method, batch, kw, dtype):
    N = 64
    M = 4 * N - 1
    print(f"nonfinite inv {method} batch={batch} {dtype}", flush=True)
    p = _plan(N, batch, method, dtype, kw)
    grid = inputs.make_grid(N, batch, 8)
    bad = grid.copy()
    m0 = 9
    bad[batch - 1, 30, m0] = complex(np.inf, 1.0)
    gc = torch.from_numpy(grid).to(dtype).cuda()
    gb = torch.from_numpy(bad).to(dtype).cuda()
    b_clean = torch.zeros((batch, 4 * N * N), dtype=dtype, device="cuda")
    b_bad = torch.zeros_like(b_clean)
    p.alt(0, 2 * N - 1, "inv", gc, b_clean)
    p.alt(0, 2 * N - 1, "inv", gb, b_bad)
    bc, bb = b_clean.cpu().numpy(), b_bad.cpu().numpy()
    _, m_of = inputs.layout(N)
    sel = m_of == m0
    assert not np.all(np.isfinite(bb[batch - 1][sel]))
    mask = np.ones(bc.shape, bool)
    mask[batch - 1][sel] = False
    assert np.array_equal(bb[mask], bc[mask])
