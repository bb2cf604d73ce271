"""Grouped transforms (persistent kernels over a longest-first work queue)
against the CPU oracle, through the C-ABI: a small mixed group compared in
full, and the uneven workload (64 transforms, N drawn from {128, 256, 512,
1024}, 1-4 fields, seed 4000): every transform's forward compared at two
seeded rows of its first and last field, the inverse by round trip, in FP64
and FP32, eagerly, after autotuning and as hipGraph replays."""
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


def _group(Ns, fields, dtype):
    from paper_2004_11346_amd.sht import Group
    return Group(Ns, fields, dtype=dtype)


def _tensors(Ns, fields, dtype, seed0):
    betas, fs, betas_np = [], [], []
    for i, (N, f) in enumerate(zip(Ns, fields)):
        b = inputs.make_beta(N, f, seed0 + i)
        if dtype == torch.complex64:
            b = b.astype(np.complex64).astype(np.complex128)
        betas_np.append(b)
        betas.append(torch.from_numpy(b).to(dtype).cuda())
        fs.append(torch.zeros((f, 2 * N, 4 * N - 1), dtype=dtype, device="cuda"))
    return betas, fs, betas_np


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_small_group_vs_oracle(dtype, tol):
    Ns = [1, 3, 16, 33, 64, 40, 5]
    fields = [1, 2, 3, 4, 1, 2, 4]
    print(f"group small {dtype}", flush=True)
    g = _group(Ns, fields, dtype)
    betas, fs, bnp = _tensors(Ns, fields, dtype, 7100)
    g.bind(betas, fs)
    g.forward()
    torch.cuda.synchronize()
    for i, (N, f) in enumerate(zip(Ns, fields)):
        got = fs[i].cpu().numpy()
        for b in range(f):
            assert rel_l2(got[b], oracle.sht_forward(N, bnp[i][b])) <= tol, (i, b)
    # inverse of generic grids
    grids = []
    for i, (N, f) in enumerate(zip(Ns, fields)):
        gr = inputs.make_grid(N, f, 7200 + i)
        if dtype == torch.complex64:
            gr = gr.astype(np.complex64).astype(np.complex128)
        grids.append(gr)
        fs[i].copy_(torch.from_numpy(gr).to(dtype))
    g.inverse()
    torch.cuda.synchronize()
    for i, (N, f) in enumerate(zip(Ns, fields)):
        got = betas[i].cpu().numpy()
        for b in range(f):
            assert rel_l2(got[b], oracle.sht_inverse(N, grids[i][b])) <= tol, (i, b)


def _uneven():
    rng = np.random.Generator(np.random.PCG64(4000))
    Ns = [int(v) for v in rng.choice([128, 256, 512, 1024], size=64)]
    fields = [int(v) for v in rng.integers(1, 5, size=64)]
    return Ns, fields


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_uneven_workload(dtype, tol):
    Ns, fields = _uneven()
    print(f"group uneven {dtype}: {sum(fields)} fields", flush=True)
    g = _group(Ns, fields, dtype)
    betas, fs, bnp = _tensors(Ns, fields, dtype, 4100)
    g.bind(betas, fs)
    g.forward()
    torch.cuda.synchronize()
    # every transform against the oracle: two seeded rows of its first and last field
    for i, N in enumerate(Ns):
        rows = list(inputs.sample_indices(2 * N, 2, 500 + i))
        M = 4 * N - 1
        for b in sorted({0, fields[i] - 1}):
            gr = oracle.alt_forward_rows(N, bnp[i][b], rows)
            full = np.zeros((2 * N, M), complex)
            full[rows] = gr
            ref = oracle.dft_synthesis(N, full, rows=rows)
            got = fs[i][b].cpu().numpy()[rows]
            assert rel_l2(got, ref) <= tol, (i, N, b, rel_l2(got, ref))
    f_eager = [t.clone() for t in fs]
    # round trip: inverse(forward(beta)) = beta
    g.inverse()
    torch.cuda.synchronize()
    worst = max(rel_l2(betas[i].cpu().numpy(), bnp[i]) for i in range(len(Ns)))
    assert worst <= (1e-12 if dtype == torch.complex128 else 4e-6), worst
    # autotuned grids give the same results
    for i in range(len(Ns)):
        betas[i].copy_(torch.from_numpy(bnp[i]).to(dtype))
    g.tune()
    st = g.stats()
    assert st["tuned"] and "tuning_ms" in st
    for i in range(len(Ns)):
        betas[i].copy_(torch.from_numpy(bnp[i]).to(dtype))
    g.forward()
    torch.cuda.synchronize()
    for i in range(len(Ns)):
        assert torch.equal(fs[i], f_eager[i]), i
    # hipGraph replays (with eager work in between) reproduce the eager result
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g.capture("fwd", s)
    for rep in range(3):
        for t in fs:
            t.zero_()
        torch.cuda.synchronize()
        g.replay("fwd", s)
        s.synchronize()
        for i in range(len(Ns)):
            assert torch.equal(fs[i], f_eager[i]), (rep, i)
        _ = torch.randn(1000, device="cuda").sum().item()


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_batched_group_vs_oracle(dtype, tol, tmp_path):
    """Batched mode: degrees shared by several transforms (staging copies) and
    single ones (direct), against the oracle; tuning (plain vs fast-form plans
    per degree) keeps the results within the bar, writes its choices to the
    tune file, and a new group reads them back; graph replays equal eager."""
    from paper_2004_11346_amd.sht import Group
    Ns = [16, 64, 16, 33, 64, 5, 64]
    fields = [1, 2, 3, 2, 1, 4, 2]
    tune = str(tmp_path / "tune.json")
    print(f"batched group {dtype}", flush=True)
    g = Group(Ns, fields, dtype=dtype, mode="batched", tune_file=tune)
    betas, fs, bnp = _tensors(Ns, fields, dtype, 7300)

    def check_forward():
        for i, (N, f) in enumerate(zip(Ns, fields)):
            got = fs[i].cpu().numpy()
            for b in range(f):
                assert rel_l2(got[b], oracle.sht_forward(N, bnp[i][b])) <= tol, (i, b)

    g.bind(betas, fs)
    g.forward()
    torch.cuda.synchronize()
    check_forward()
    grids = []
    for i, (N, f) in enumerate(zip(Ns, fields)):
        gr = inputs.make_grid(N, f, 7400 + i)
        if dtype == torch.complex64:
            gr = gr.astype(np.complex64).astype(np.complex128)
        grids.append(gr)
        fs[i].copy_(torch.from_numpy(gr).to(dtype))
    g.inverse()
    torch.cuda.synchronize()
    for i, (N, f) in enumerate(zip(Ns, fields)):
        got = betas[i].cpu().numpy()
        for b in range(f):
            assert rel_l2(got[b], oracle.sht_inverse(N, grids[i][b])) <= tol, (i, b)
    g.tune()
    st = g.stats()
    assert st["mode"] == "batched" and st["tuned"] and len(st["classes"]) == 4
    for i in range(len(Ns)):
        betas[i].copy_(torch.from_numpy(bnp[i]).to(dtype))
    g.forward()
    torch.cuda.synchronize()
    check_forward()
    f_eager = [t.clone() for t in fs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g.capture("fwd", s)
    for rep in range(3):
        for t in fs:
            t.zero_()
        torch.cuda.synchronize()
        g.replay("fwd", s)
        s.synchronize()
        for i in range(len(Ns)):
            assert torch.equal(fs[i], f_eager[i]), (rep, i)
        _ = torch.randn(1000, device="cuda").sum().item()
    chosen = {c["N"]: (c["method"], c["leaf"]) for c in st["classes"]}
    g.close()
    g2 = Group(Ns, fields, dtype=dtype, mode="batched", tune_file=tune)
    st2 = g2.stats()
    assert {c["N"]: (c["method"], c["leaf"]) for c in st2["classes"]} == chosen
    g2.close()
