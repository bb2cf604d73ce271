"""Host tables of the phi DFT (Section 1, the phi sums of the SHT), on the CPU.

`sht_host_dft_tables` returns the schedule a length M = 4N - 1 gets and every
table its kernels receive: the passes (radices in order, block lengths, the
slot of each output frequency), the four-step split, and the Rader tables
(input and output slots, spectra) of a prime row or of a last pass.  Here the
algorithm those tables describe is carried out in numpy -- each
decimation-in-frequency pass by its definition
  y[n1 + Ls k2] = w_L^{n1 k2} sum_{n2} x[n1 + Ls n2] w_R^{n2 k2},
a Rader pass as x_0 plus the cyclic convolution of the inputs in slot order
with the phases (through numpy.fft), the four-step composition
X[k1 + M1 k2] = sum_{n2} w_{M2}^{n2 k2} w_M^{n2 k1} sum_{n1} x[M2 n1 + n2] w_{M1}^{n1 k1}
-- and compared with numpy.fft's transform of the same row in both signs.
A wrong radix order, slot table, spectrum slot or sign fails the comparison.
"""
import ctypes
import json

import numpy as np
import pytest

from paper_2004_11346_amd import lib as L


def tables(N, dtype=0, schedule=0):
    lib = L.load()
    n = lib.sht_host_dft_tables(N, dtype, schedule, None, 0)
    assert n > 0
    buf = ctypes.create_string_buffer(n)
    assert lib.sht_host_dft_tables(N, dtype, schedule, buf, n) == n
    return json.loads(buf.value.decode())


def cplx(v):
    a = np.asarray(v, dtype=np.float64)
    return a[0::2] + 1j * a[1::2]


def dif_pass(x, L, R, sgn):
    """One pass of radix R over blocks of length L of every row of x."""
    nseg, L0 = x.shape
    Ls = L // R
    y = x.reshape(nseg, L0 // L, R, Ls)
    n2 = np.arange(R)
    W = np.exp(sgn * 2j * np.pi * np.outer(n2, n2) / R)       # [k2, n2]
    z = np.einsum("kn,sbnj->sbkj", W, y)
    tw = np.exp(sgn * 2j * np.pi * np.outer(np.arange(R), np.arange(Ls)) / L)  # [k2, n1]
    return (z * tw).reshape(nseg, L0)


def rader_blocks(x, R, rl, sgn):
    """Length-R DFT of every contiguous block of R points of every row, from
    the Rader tables (x_0 plus the cyclic convolution through numpy.fft)."""
    Lc = R - 1
    inslot, outslot = np.asarray(rl["inslot"]), np.asarray(rl["outslot"])
    sp = np.asarray(rl["src_pos"])
    bs = cplx(rl["bspec"]).reshape(2, Lc)[0 if sgn > 0 else 1]
    B = bs[sp]  # natural frequency order
    blocks = x.reshape(-1, R)
    a = np.zeros((blocks.shape[0], Lc), dtype=complex)
    a[:, inslot[1:]] = blocks[:, 1:]
    A = np.fft.fft(a, axis=1)
    conv = np.fft.ifft(A * B, axis=1) * Lc
    out = np.empty_like(blocks)
    out[:, 0] = blocks[:, 0] + A[:, 0]
    out[:, 1:] = blocks[:, :1] + conv[:, outslot[1:]]
    return out.reshape(x.shape)


def run_list(x, radix, blen, src_pos, rl, sgn):
    """Every pass of one list over the rows of x (the last one by Rader's
    convolution when rl names a prime), outputs in natural order."""
    for i, (R, Lb) in enumerate(zip(radix, blen)):
        if i == len(radix) - 1 and rl["R"]:
            assert R == rl["R"] and Lb == R
            x = rader_blocks(x, R, rl, sgn)
        else:
            x = dif_pass(x, Lb, R, sgn)
    return x[:, np.asarray(src_pos)]


def transform(t, x, sgn):
    M = t["M"]
    if t["kind"] == "rows":
        return run_list(x[None], t["radix"], t["blen"], t["src_pos"], t["rader_last"][0], sgn)[0]
    if t["kind"] == "rader":
        rl = {"R": M, "inslot": t["inslot"], "outslot": t["outslot"], "bspec": t["bspec"], "src_pos": t["src_pos"]}
        return rader_blocks(x[None], M, rl, sgn)[0]
    assert t["kind"] == "four_step"
    M1, M2 = t["M1"], t["M2"]
    seg = x.reshape(M1, M2).T  # [n2][n1] = x[M2 n1 + n2]
    y = run_list(seg, t["radix"], t["blen"], t["src_pos"], t["rader_last"][0], sgn)  # [n2][k1]
    y = y * np.exp(sgn * 2j * np.pi * np.outer(np.arange(M2), np.arange(M1)) / M)
    z = run_list(y.T.copy(), t["radix2"], t["blen2"], t["src_pos2"], t["rader_last"][1], sgn)  # [k1][k2]
    return z.T.reshape(M)  # X[k1 + M1 k2]


@pytest.mark.parametrize("N,dtype,schedule,kind,rl", [
    (64, 0, 0, "rows", [0, 0]),            # 255 = 5 3 17: 17 as a direct sum
    (67, 0, 1, "rows", [89, 0]),           # 267 = 3 89: 89 by Rader's convolution
    (512, 0, 0, "rows", [89, 0]),          # 2047 = 23 89
    (1024, 0, 0, "rows", [0, 0]),          # 4095 = 13 9 7 5
    (128, 0, 3, "four_step", [73, 0]),     # 511 = 73 x 7
    (441, 0, 3, "four_step", [43, 41]),    # 1763 = 43 x 41
    (4096, 0, 0, "four_step", [43, 127]),  # 16383 = 129 x 127
    (4096, 1, 0, "four_step", [43, 127]),  # FP32 rows would keep 127 and 43 as sums
    (5, 0, 2, "rader", [0, 0]),            # 19 prime
    (2048, 0, 0, "rader", [0, 0]),         # 8191 prime
])
def test_dft_tables_reproduce_the_dft(N, dtype, schedule, kind, rl):
    t = tables(N, dtype, schedule)
    M = 4 * N - 1
    assert t["kind"] == kind and t["M"] == M
    assert [r["R"] for r in t["rader_last"]] == rl
    # every slot table is a permutation
    for key, length in (("src_pos", t["M1"] if kind == "four_step" else (M - 1 if kind == "rader" else M)),
                        ("src_pos2", t["M2"] if kind == "four_step" else 0)):
        assert sorted(t[key]) == list(range(length)), key
    for r in t["rader_last"]:
        if r["R"]:
            assert sorted(r["src_pos"]) == list(range(r["R"] - 1))
            assert sorted(r["inslot"][1:]) == list(range(r["R"] - 1))
            assert max(r["radix"]) <= 13
    rng = np.random.default_rng(N)
    x = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    for sgn, ref in ((1, np.fft.ifft(x) * M), (-1, np.fft.fft(x))):
        got = transform(t, x, sgn)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (sgn, err)


def test_dft_tables_rejects_bad_arguments():
    lib = L.load()
    assert lib.sht_host_dft_tables(0, 0, 0, None, 0) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_host_dft_tables(16, 2, 0, None, 0) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_host_dft_tables(16, 0, 9, None, 0) == L.SHT_ERR_INVALID_ARG
