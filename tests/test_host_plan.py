"""CPU checks of the host side of the library (no GPU): its Gauss-Legendre
rule and Legendre half matrices against the oracle, the exported C-ABI, and
the packed fast-ALT program (the op stream the GPU executes, run by a plain
host loop) against the oracle's dense matrices."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
from paper_2004_11346_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "sht.h")).read()
    names = set(re.findall(r"\b(sht_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 15
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.EXPORTED) <= names


def test_library_gl_rule_matches_oracle():
    for n in [2, 7, 128, 2048]:
        x = np.empty(n)
        w = np.empty(n)
        L.check(L.load().sht_host_gauss_legendre(n, x.ctypes.data, w.ctypes.data), "gl")
        xo, wo = oracle.gauss_legendre(n)
        np.testing.assert_allclose(x, xo, rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, wo, rtol=4e-16, atol=0)


def half_cols(N, a, p):
    return N - (a + 1) // 2 if p else N - a // 2


def oracle_half_matrix(N, a, p, x):
    """Half matrix from the oracle: rows r <-> node 2N-1-r, cols j <-> k = a+p+2j."""
    c = half_cols(N, a, p)
    out = np.empty((N, c))
    for r in range(N):
        col = oracle.plm(a, 2 * N - 1, x[2 * N - 1 - r])
        out[r] = col[p::2][:c]
    return out


class HostPlan:
    def __init__(self, N, method=L.SHT_IDBF, **kw):
        self.lib = L.load()
        o = L.default_opts(**kw)
        self.h = ctypes.c_void_p()
        L.check(self.lib.sht_host_plan_create(N, method, ctypes.byref(o), ctypes.byref(self.h)), "host plan")
        self.N = N

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.sht_host_plan_destroy(self.h)

    def matrix(self, a, p):
        c = half_cols(self.N, a, p)
        A = np.empty((self.N, c))
        L.check(self.lib.sht_host_alt_matrix(self.h, a, p, A.ctypes.data), "matrix")
        return A

    def apply(self, a, p, direction, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        R = x.shape[1]
        c = half_cols(self.N, a, p)
        out = np.empty((self.N if direction == L.SHT_FWD else c, R))
        L.check(self.lib.sht_host_plan_apply(self.h, a, p, direction, R, x.ctypes.data, out.ctypes.data), "apply")
        return out

    def stats(self):
        n = self.lib.sht_host_plan_stats(self.h, None, 0)
        buf = ctypes.create_string_buffer(n)
        self.lib.sht_host_plan_stats(self.h, buf, n)
        return json.loads(buf.value.decode())


@pytest.mark.parametrize("N", [8, 33, 64])
def test_library_half_matrices_match_oracle(N):
    hp = HostPlan(N, method=L.SHT_DENSE)
    x, _ = oracle.gauss_legendre(2 * N)
    for a in sorted({0, 1, 2, N // 2, N, 2 * N - 2, 2 * N - 1}):
        for p in (0, 1):
            if half_cols(N, a, p) <= 0:
                continue
            A = hp.matrix(a, p)
            Ao = oracle_half_matrix(N, a, p, x)
            # binary64 recurrence: rounding error grows like (number of steps) * eps
            np.testing.assert_allclose(A, Ao, rtol=0, atol=2e-15 * 2 * N * max(1.0, np.abs(Ao).max()))


@pytest.mark.parametrize("N,kw", [
    (64, dict(n0=32, leaf=8)),           # butterflies and regenerated dense blocks
    (64, dict(n0=32, leaf=8, rsvd_r=4)),     # also Algorithm 1 low-rank blocks
    (128, dict(n0=64, leaf=8, rsvd_r=4)),
    (64, dict(n0=32, leaf=8, dense_gen=0)),  # dense blocks stored instead
    (40, dict(n0=24, leaf=4)),           # blocks with unaligned first columns
    (96, dict(n0=48, leaf=8, eps=1e-13)),
    (128, dict()),                       # default partition (few butterflies at this size)
])
def test_packed_program_vs_oracle(N, kw):
    """The packed op program (the exact stream the GPU runs) reproduces the
    oracle's half matrices within the factorization tolerance, forward and
    transposed, including the empty odd matrix of the last order."""
    hp = HostPlan(N, **kw)
    st = hp.stats()
    x, _ = oracle.gauss_legendre(2 * N)
    rng = np.random.default_rng(N)
    worst = 0.0
    for a in sorted({0, 1, 3, N // 3, N // 2, N - 1, N, 3 * N // 2, 2 * N - 2, 2 * N - 1}):
        for p in (0, 1):
            c = half_cols(N, a, p)
            if c <= 0:
                continue
            Ao = oracle_half_matrix(N, a, p, x)
            xin = rng.standard_normal((c, 3))
            y = hp.apply(a, p, L.SHT_FWD, xin)
            worst = max(worst, np.linalg.norm(y - Ao @ xin) / np.linalg.norm(Ao @ xin))
            yin = rng.standard_normal((N, 3))
            xt = hp.apply(a, p, L.SHT_ADJ, yin)
            worst = max(worst, np.linalg.norm(xt - Ao.T @ yin) / np.linalg.norm(Ao.T @ yin))
    assert worst <= 1e-11, (worst, st)
    if kw.get("leaf") == 8:
        assert st["blocks_butterfly"] > 0
    if kw.get("rsvd_r") == 4:
        assert st["blocks_lowrank"] > 0 and st["lowrank_stored"] > 0, st
    if kw.get("dense_gen", 1):
        assert st["blocks_generated"] > 0 and st["generated_entries"] > 0
    else:
        assert st["blocks_generated"] == 0


def test_plan_stats_are_consistent():
    hp = HostPlan(64, n0=32, leaf=8)
    st = hp.stats()
    assert st["stored_entries"] == st["dense_stored"] + st["lowrank_stored"] + st["butterfly_stored"]
    assert st["dense_entries"] == 64 * 64 * (2 * 64 + 1)
    area = st["osc"]["area"] + st["nonosc"]["area"] + st["turning"]["area"]
    assert area <= st["dense_entries"]


@pytest.mark.parametrize("N,kw", [(64, dict(n0=32, leaf=8, rsvd_r=4)), (128, dict(n0=64, leaf=8, rsvd_r=4)),
                                  (256, dict(n0=128, leaf=16))])
def test_fused_level_form_equals_staged(N, kw):
    """The fused form of the work stages (every block's levels in one
    workgroup, rows renumbered into two alternating buffers; blocks too large
    for the buffers keep their scratch rows) runs the same products in the
    same order as the staged program: the host executions agree bitwise, and
    the packer's bounds check of the fused form passes."""
    staged = HostPlan(N, level_schedule=L.SHT_LEVELS_STAGED, **kw)
    fused = HostPlan(N, level_schedule=L.SHT_LEVELS_FUSED, **kw)
    st = fused.stats()
    assert st["fwd_fused_ok"] == 1 and st["adj_fused_ok"] == 1
    assert st["fwd_fused_groups"] > 0
    if N == 256:
        assert st["fwd_fused_max_lds_rows"] > 512  # staged rows inside the fused form
    rng = np.random.default_rng(N)
    for a in range(0, 2 * N, max(1, N // 8)):
        for p in (0, 1):
            c = half_cols(N, a, p)
            if c <= 0:
                continue
            for d in (L.SHT_FWD, L.SHT_ADJ):
                x = rng.standard_normal((c if d == L.SHT_FWD else N, 3))
                assert np.array_equal(staged.apply(a, p, d, x), fused.apply(a, p, d, x)), (a, p, d)
