"""Fused butterfly levels (sht_plan_opts.level_schedule): all non-final
levels of a block (Section 2.2, the column IDs level by level, the middle
couplings and the row IDs; Section 2.3, V^T of a low-rank block) in one
workgroup with the intermediate rows in LDS, against the staged schedule (one
launch per level, rows through HBM) and the oracle, through the C ABI.  The
plans use small partitions so that butterflies of several levels, low-rank
blocks (rsvd_r = 4) and blocks whose levels exceed the LDS buffers (staged
rows inside the fused launch) occur; batches of 4 and 5 fields give 16 and
20 right-hand sides (the matrix-core executor; 20 leaves a ragged 16-column
slab).  Bars: FP64 fused equals staged bitwise (the same products in the same
order) and the oracle to 1e-11; FP32 to 2e-6."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11346_amd import inputs
from paper_2004_11346_amd import lib as L

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


CASES = [
    (64, 4, dict(n0=32, leaf=8, rsvd_r=4)),
    (128, 5, dict(n0=64, leaf=8, rsvd_r=4)),
    (96, 4, dict(n0=32, leaf=8)),
    (256, 4, dict(n0=128, leaf=16)),
]


def _run(p, beta, grid, dtype):
    f = p.forward(torch.from_numpy(beta).to(dtype).cuda())
    bi = p.inverse(torch.from_numpy(grid).to(dtype).cuda())
    ba = p.backward(torch.from_numpy(grid).to(dtype).cuda())
    torch.cuda.synchronize()
    return f.cpu().numpy(), bi.cpu().numpy(), ba.cpu().numpy()


@pytest.mark.parametrize("N,batch,kw", CASES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_fused_levels_vs_staged_and_oracle(N, batch, kw, dtype):
    from paper_2004_11346_amd.sht import Plan
    print(f"fused levels N={N} batch={batch} {kw} {dtype}", flush=True)
    pf = Plan(N, batch, dtype=dtype, method="idbf", level_schedule=L.SHT_LEVELS_FUSED, **kw)
    ps = Plan(N, batch, dtype=dtype, method="idbf", level_schedule=L.SHT_LEVELS_STAGED, **kw)
    st = pf.stats()["program"]
    assert st["fwd_fused_ok"] == 1 and st["adj_fused_ok"] == 1
    assert st["blocks_butterfly"] > 0
    if kw.get("rsvd_r") == 4:
        assert st["blocks_lowrank"] > 0
    if N == 256:  # some blocks' levels exceed the LDS buffers
        assert st["fwd_fused_max_lds_rows"] > 512
    beta = inputs.make_beta(N, batch, 31)
    grid = inputs.make_grid(N, batch, 32)
    pf.profile(True)
    out_f = _run(pf, beta, grid, dtype)
    rep = pf.profile_report()
    pf.profile(False)
    assert "k_ops_fused" in rep, "the fused kernel must run"
    ps.profile(True)
    out_s = _run(ps, beta, grid, dtype)
    assert "k_ops_fused" not in ps.profile_report()
    ps.profile(False)
    tol = 1e-11 if dtype == torch.complex128 else 2e-6
    if dtype == torch.complex64:
        beta = beta.astype(np.complex64).astype(np.complex128)
        grid = grid.astype(np.complex64).astype(np.complex128)
    for which, (a, b) in enumerate(zip(out_f, out_s)):
        if dtype == torch.complex128:
            assert np.array_equal(a, b), ("fused and staged differ", which)
        else:
            assert rel_l2(a, b) <= 1e-6, which
    for b in range(batch):
        assert rel_l2(out_f[0][b], oracle.sht_forward(N, beta[b])) <= tol
        assert rel_l2(out_f[1][b], oracle.sht_inverse(N, grid[b])) <= tol
        assert rel_l2(out_f[2][b], oracle.sht_adjoint(N, grid[b])) <= tol
    pf.close()
    ps.close()


def test_fused_levels_need_the_matrix_core_executor():
    """Batch 1 (4 right-hand sides) runs the VALU executor: a forced fused
    schedule is refused; the default falls back to the staged one."""
    from paper_2004_11346_amd.sht import Plan
    with pytest.raises(L.ShtError, match="unsupported|fused"):
        Plan(64, 1, method="idbf", level_schedule=L.SHT_LEVELS_FUSED, n0=32, leaf=8)
    p = Plan(64, 1, method="idbf", n0=32, leaf=8)
    p.profile(True)
    p.forward(torch.from_numpy(inputs.make_beta(64, 1, 33)).cuda())
    assert "k_ops_fused" not in p.profile_report()
    p.close()
