"""The on-disk plan cache (sht_plan_opts.cache_dir), through the host-plan
entry points of the C ABI (no GPU): a first build writes the file, a second
plan with the same options loads it and applies exactly the same packed
program, other options use another file, and a damaged file is reported as
corrupt by sht_plan_cache_verify and rebuilt by the next plan."""
import ctypes
import os

import numpy as np
import pytest

from paper_2004_11346_amd import lib as L

from test_host_plan import HostPlan, half_cols

KW = dict(n0=32, leaf=8, rsvd_r=4)  # butterflies, low-rank and regenerated blocks


def cache_file(N, d, **kw):
    o = L.default_opts(cache_dir=str(d), **kw)
    buf = ctypes.create_string_buffer(4096)
    n = L.check(L.load().sht_plan_cache_path(N, ctypes.byref(o), buf, 4096), "cache path")
    assert n <= 4096
    return buf.value.decode()


def verify(path):
    return L.load().sht_plan_cache_verify(path.encode())


def outputs(hp, N):
    rng = np.random.default_rng(7)
    outs = []
    for a in (0, 1, N // 2, N, 2 * N - 2):
        for p in (0, 1):
            c = half_cols(N, a, p)
            if c <= 0:
                continue
            outs.append(hp.apply(a, p, L.SHT_FWD, rng.standard_normal((c, 3))))
            outs.append(hp.apply(a, p, L.SHT_ADJ, rng.standard_normal((N, 3))))
    return outs


def test_build_then_load_gives_the_same_program(tmp_path):
    N = 64
    path = cache_file(N, tmp_path, **KW)
    assert not os.path.exists(path)
    built = HostPlan(N, cache_dir=str(tmp_path), **KW)
    assert built.stats()["plan_cache"] == "miss"
    assert os.path.exists(path) and verify(path) == L.SHT_OK
    loaded = HostPlan(N, cache_dir=str(tmp_path), **KW)
    st = loaded.stats()
    assert st["plan_cache"] == "hit"
    ref = built.stats()
    for k in ("stored_entries", "generated_entries", "blocks_butterfly", "blocks_lowrank", "fwd_values"):
        assert st[k] == ref[k], k
    for x, y in zip(outputs(built, N), outputs(loaded, N)):
        assert np.array_equal(x, y)
    plain = HostPlan(N, **KW)
    assert plain.stats()["plan_cache"] == "off"
    for x, y in zip(outputs(plain, N), outputs(loaded, N)):
        assert np.array_equal(x, y)


def test_other_options_use_another_file(tmp_path):
    N = 48
    a = cache_file(N, tmp_path, n0=24, leaf=8)
    b = cache_file(N, tmp_path, n0=24, leaf=8, eps=1e-13)
    c = cache_file(N, tmp_path, n0=24, leaf=8, seed=5)
    assert len({a, b, c}) == 3
    # batch, dtype and the DFT schedule do not change the factors
    assert cache_file(N, tmp_path, n0=24, leaf=8, dft_schedule=L.SHT_DFT_ROWS) == a
    HostPlan(N, cache_dir=str(tmp_path), n0=24, leaf=8)
    assert HostPlan(N, cache_dir=str(tmp_path), n0=24, leaf=8, eps=1e-13).stats()["plan_cache"] == "miss"


@pytest.mark.parametrize("damage", ["flip_payload", "truncate", "bad_magic", "empty"])
def test_corrupt_file_is_detected_and_rebuilt(tmp_path, damage):
    N = 48
    kw = dict(n0=24, leaf=8)
    path = cache_file(N, tmp_path, **kw)
    good = HostPlan(N, cache_dir=str(tmp_path), **kw)
    raw = bytearray(open(path, "rb").read())
    if damage == "flip_payload":
        raw[len(raw) - 100] ^= 0x10
    elif damage == "truncate":
        raw = raw[: len(raw) // 2]
    elif damage == "bad_magic":
        raw[0] ^= 0xFF
    else:
        raw = bytearray()
    open(path, "wb").write(bytes(raw))
    assert verify(path) == L.SHT_ERR_PLAN_CORRUPT
    again = HostPlan(N, cache_dir=str(tmp_path), **kw)
    assert again.stats()["plan_cache"] == "corrupt_rebuilt"
    assert verify(path) == L.SHT_OK
    for x, y in zip(outputs(good, N), outputs(again, N)):
        assert np.array_equal(x, y)
    assert HostPlan(N, cache_dir=str(tmp_path), **kw).stats()["plan_cache"] == "hit"


def test_missing_file_and_unwritable_dir(tmp_path):
    assert verify(str(tmp_path / "nothing.bin")) == L.SHT_ERR_INVALID_ARG
    hp = HostPlan(40, cache_dir=str(tmp_path / "no" / "such" / "dir"), n0=24, leaf=8)
    assert hp.stats()["plan_cache"] == "off"  # built, not stored
