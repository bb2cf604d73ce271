#!/usr/bin/env python3
"""Benchmark of the SHT hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic fields: a
forward SHT (ALT for every order m + length-(4N-1) phi DFT) and an inverse
SHT (phi analysis + transposed ALT) of every field.  `value` is SHT/s over the
timed steps, counting each forward and each inverse of a field as one SHT.
The headline workload is N = 1024 (grid 2048 x 4095), FP64, 32 fields, with
the fast (IDBF) ALT; the plain (dense) ALT and batch 1 are measured beside it
and reported under "details".

Prints ONE JSON line.  `--gpus` above 1 is refused: the transform runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector and matrix, TFLOP/s
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 MFMA


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--method", choices=["idbf", "dense"], default=None)
    ap.add_argument("--no-details", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--profile-target", action="store_true",
                    help="only a 1 GiB device copy (counter scale) and a few ALT calls, for rocprofv3 runs")
    ap.add_argument("--profile-dirs", default="fwd",
                    help="calls run by --profile-target (comma separated: fwd, inv = ALT only; sht_fwd, "
                         "sht_inv = full transforms)")
    ap.add_argument("--orders", default=None,
                    help="plan-build: order range LO:HI of the windows built (default: every order)")
    ap.add_argument("--workload", choices=["default", "n4096-orders", "n4096-every-order", "uneven", "rank-study",
                                           "levels", "plan-build", "dft"],
                    default="default",
                    help="n4096-orders: N=4096, 8 fields, fast vs plain ALT on 64-order windows across the "
                         "order range; uneven: the grouped 64-transform workload; rank-study: ID sampling "
                         "(mock-Chebyshev vs random rows), adaptive rank r_k and tolerance sweeps at m = N; "
                         "levels: staged vs fused butterfly levels at leaf 32/64/128; n4096-every-order: the "
                         "fast ALT of every order at N=4096 in 16 shares vs the plain form; plan-build: host "
                         "construction of the fast-form plan of every order of --N, window by window; dft: the "
                         "phi DFT alone for the schedules of several lengths, against the HBM roofline")
    return ap.parse_args()


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_max(a, b):
    import numpy as np
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


class Timer:
    """HIP events on torch's current stream, which is the stream every library
    call is enqueued on."""

    def __init__(self):
        import torch
        self.torch = torch

    def time(self, fn, reps: int, warmup: int = 1) -> float:
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3  # seconds per call


def cpu_baseline(N: int):
    """The oracle (plain CPU FP64 definition: dense ALT of every order, direct
    phi sums) timed on one full forward and one full inverse SHT of one field
    of the same workload (batch 1 of the headline configuration)."""
    import numpy as np

    import oracle
    from paper_2004_11346_amd import inputs

    beta = inputs.make_beta(N, 1, 2, dist="decay")[0]
    t0 = time.perf_counter()
    f = oracle.sht_forward(N, beta)
    t1 = time.perf_counter()
    back = oracle.sht_inverse(N, f)
    t2 = time.perf_counter()
    return {
        "value": 2.0 / (t2 - t0),
        "unit": "SHT/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"N={N}, one field (batch 1 of the workload): one full forward and one full inverse SHT "
                   f"(dense ALT of all {4 * N - 1} orders, direct phi sums over all {2 * N} rows), "
                   f"measured {t2 - t0:.1f} s, not extrapolated"),
        "seconds_measured": t2 - t0,
        "fwd_s_per_field": t1 - t0,
        "inv_s_per_field": t2 - t1,
        "round_trip_rel_l2": rel_l2(back, beta),
    }


# HBM bytes per call of each kernel family (all its dispatches): rocprofv3
# FETCH_SIZE and WRITE_SIZE runs (separate runs, two calls each, see
# profiles/), scaled by what the counters read for a 1 GiB device copy in the
# same run (fetch x 2.0, write x 1.0).  Each entry is keyed on the SHA-256 of
# the kernel sources it was measured with; a changed source makes the figure
# stale and it is reported as null.
TRAFFIC = {
    ("dense", 1024, 32, "f64", "k_dense_fwd_mfma"): {"bytes_per_call": 24.06e9, "sha": "21a5dbab89ebbe02",
                                                     "profile": "profiles/alt_fwd_dense_n1024_b32_f64.md"},
    ("dense", 1024, 1, "f64", "k_dense_fwd_valu"): {"bytes_per_call": 0.7513e9, "sha": "21a5dbab89ebbe02",
                                                    "profile": "profiles/alt_fwd_dense_n1024_b1_f64.md"},
    ("idbf", 1024, 32, "f64", "k_gen_adj"): {"bytes_per_call": 22.709e9, "sha": "a95bef2d30025b5a",
                                              "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_gen_fwd_mfma"): {"bytes_per_call": 12.625e9, "sha": "a95bef2d30025b5a",
                                                   "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_pack"): {"bytes_per_call": 4.403e9, "sha": "a900dd7b71176d56",
                                          "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_combine"): {"bytes_per_call": 8.659e9, "sha": "a900dd7b71176d56",
                                             "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_fold"): {"bytes_per_call": 9.046e9, "sha": "a900dd7b71176d56",
                                          "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_scatter"): {"bytes_per_call": 4.306e9, "sha": "a900dd7b71176d56",
                                             "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_dft_synthesis"): {"bytes_per_call": 8.779e9, "sha": "24a9a20d9d621217",
                                                    "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_dft_analysis"): {"bytes_per_call": 8.779e9, "sha": "24a9a20d9d621217",
                                                   "profile": "profiles/traffic_sht_idbf_n1024_b32_f64.md"},
}

# the sources each kernel family is built from
FAMILY_SOURCES = {
    "k_dense": ["kernels_dense.hip", "dense_device.h"],
    "k_gen": ["idbf_kernels.hip", "idbf_pack.cpp"],
    "k_ops": ["idbf_kernels.hip", "idbf_pack.cpp"],
    "k_dft": ["kernels_dft.hip", "dft_device.h"],
    "k_pack": ["kernels_panels.hip"],
    "k_scatter": ["kernels_panels.hip"],
    "k_combine": ["kernels_panels.hip"],
    "k_fold": ["kernels_panels.hip"],
}


def kernel_source_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2004_11346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TFLOPS = ("TFLOP/s", PEAK_FP64_TFLOPS)
GBS = ("GB/s", PEAK_HBM_GBS)


def family(name):
    """Kernel family of a recorder label ("k_ops_mfma[L2]" -> "k_ops_mfma");
    the fused levels and the final stage of the op program on the matrix
    cores form one family."""
    f = name.split("[", 1)[0]
    return "k_ops_mfma" if f == "k_ops_fused" else f


def kernel_work(fam, method, N, batch, dtype, prog):
    """Algorithmic work of one call of a kernel family over all orders of one
    batch: (bound, work, unit_peak, dispatches per call, what).

    R = 4 batch real right-hand sides, s bytes per stored value and panel
    entry, E = N^2 (2N + 1) entries of the half matrices of all orders.
      products with regenerated entries (plain form, regenerated blocks of the
        fast form): (2 R + 3) flops per entry -- the product with every
        right-hand side and about 3 flops to generate the entry;
      op program (stored factors): on the matrix cores (R >= 16) 2 R flops
        per stored value; else values s + index bytes + the vector rows one
        call must move once (distinct input-panel rows read, output rows
        written) R s, with the rows the level-by-level schedule moves beyond
        that reported as "schedule_bytes";
      panel moves and phi DFTs: one read and one write of the data they move.
    """
    R = 4 * batch
    sb = 8 if dtype == "f64" else 4
    E = float(N) * N * (2 * N + 1)
    grid = 2.0 * N * (4 * N - 1) * batch * 2 * sb  # complex grid bytes
    coefs = 4.0 * N * N * batch * 2 * sb             # complex coefficient bytes
    pb = 8 if method == "dense" else sb              # the plain form's panels are FP64
    xpan = float(N) * (2 * N + 1) * R * pb
    ypan = 4.0 * N * N * R * pb
    gen_disp = (R + 31) // 32
    if fam in ("k_dense_fwd_mfma", "k_dense_adj_ck"):
        return "mfma", (2.0 * R + 3) * E, TFLOPS, 1, "(2R+3) N^2(2N+1) flops"
    if fam in ("k_dense_fwd_valu", "k_dense_adj_valu"):
        return "alu", (2.0 * R + 3) * E, TFLOPS, 1, "(2R+3) N^2(2N+1) flops"
    if fam == "k_dense_ckpt":
        return "alu", 3.0 * E, TFLOPS, 1, "3 N^2(2N+1) flops (recurrence walk)"
    ng = float(prog.get("generated_entries", 0))
    if fam == "k_gen_fwd_mfma":
        return "mfma", (2.0 * R + 3) * ng, TFLOPS, gen_disp, "(2R+3) x regenerated entries flops"
    if fam == "k_gen_fwd":
        rc = 4 if R <= 4 else 8 if R <= 8 else 16
        return "alu", (2.0 * R + 3) * ng, TFLOPS, (R + rc - 1) // rc, "(2R+3) x regenerated entries flops"
    if fam == "k_gen_adj":
        return "mfma", (2.0 * R + 3) * ng, TFLOPS, 1 if R <= 16 else gen_disp, "(2R+3) x regenerated entries flops"
    if fam.startswith("k_ops"):
        d = "adj" if fam.endswith("@inv") else "fwd"
        nv = float(prog.get(d + "_values", 0))
        if fam.startswith("k_ops_mfma") and R >= 16:
            # many right-hand sides: 2 R flops per stored value (above the
            # FP64 ridge from R = 40)
            return "mfma", 2.0 * R * nv, TFLOPS, None, "2R x stored values flops"
        vals = nv * sb
        idx = float(prog.get(d + "_index_bytes", 0))
        vec = (float(prog.get(d + "_vector_in_rows", 0)) + float(prog.get(d + "_vector_out_rows", 0))) * R * sb
        return "hbm", vals + idx + vec, GBS, None, "values s + index + distinct vector rows R s"
    if fam in ("k_pack", "k_scatter"):
        return "hbm", coefs + xpan, GBS, 1, "coefficients + X panels"
    if fam in ("k_combine", "k_fold"):
        return "hbm", grid + ypan, GBS, 1, "grid + Y panels"
    if fam in ("k_dft_synthesis", "k_dft_analysis"):
        return "hbm", 2.0 * grid, GBS, 1, "grid read + written"
    return None


def plan_shape(stats):
    """How the fast form's work splits: entries stored as IDBF / low-rank /
    dense factors, entries regenerated by the recurrence, and the share of the
    dense matrices dropped as negligible (Section 3.3)."""
    prog = stats.get("program")
    if not prog:
        return None
    dense = float(prog["dense_entries"])
    keys = ("blocks_butterfly", "blocks_lowrank", "blocks_dense", "blocks_generated", "blocks_dropped",
            "butterfly_stored", "lowrank_stored", "dense_stored", "stored_entries", "generated_entries",
            "dense_entries", "leaf", "max_rank")
    out = {k: prog.get(k) for k in keys}
    out["stored_over_dense"] = prog["stored_entries"] / dense
    out["generated_over_dense"] = prog["generated_entries"] / dense
    osc = prog.get("osc", {})
    out["oscillatory_area_over_dense"] = osc.get("area", 0) / dense
    return out


def step_roofline(method, N, batch, dtype, prog, kern_fwd, kern_inv, reps):
    """Per-kernel-family time and roofline fraction over one step (forward +
    inverse SHT), from HIP events recorded on the launch stream; `roofline`
    is the family with the largest time per step."""
    fams = {}
    for tag, kern in (("fwd", kern_fwd), ("inv", kern_inv)):
        for name, v in kern.items():
            fam = family(name)
            key = fam + ("@inv" if fam.startswith("k_ops") and tag == "inv" else "")
            f = fams.setdefault(key, {"ms_per_step": 0.0, "launches_per_step": 0.0})
            f["ms_per_step"] += v["total_ms"] / reps
            f["launches_per_step"] += v["launches"] / reps
    rows = {}
    for key, f in fams.items():
        w = kernel_work(key, method, N, batch, dtype, prog)
        r = {"ms_per_step": f["ms_per_step"], "launches_per_step": f["launches_per_step"]}
        if w:
            bound, work, (unit, peak), disp, what = w
            # every family runs once per step (ops stages split by direction),
            # whatever number of launches that call makes
            per_call_s = f["ms_per_step"] / 1e3
            ach = work / per_call_s / (1e12 if unit == "TFLOP/s" else 1e9)
            r.update({"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                      "work_per_call": work, "work": what})
            if disp:
                r["dispatches_per_call"] = disp
                r["avg_dispatch_ms"] = per_call_s * 1e3 / disp
        if key.startswith("k_ops"):
            d = "adj" if key.endswith("@inv") else "fwd"
            sb = 8 if dtype == "f64" else 4
            r["schedule_bytes"] = ((float(prog.get(d + "_gather_rows", 0)) + float(prog.get(d + "_out_rows", 0)))
                                   * 4 * batch * sb)
        t = traffic_of(method, N, batch, dtype, key)
        if t["traffic"] is not None:
            r["traffic"] = t["traffic"]
        rows[key] = r
    dom = max((k for k in rows if "frac" in rows[k]), key=lambda k: rows[k]["ms_per_step"])
    d = rows[dom]
    roof = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
            "frac": d["frac"], "kernel": dom, "work": d["work"], "work_per_call": d["work_per_call"],
            "kernel_ms_per_call": d["ms_per_step"],
            "kernel_share_of_step_kernels": d["ms_per_step"] / sum(r["ms_per_step"] for r in rows.values())}
    if "dispatches_per_call" in d:
        roof["dispatches_per_call"] = d["dispatches_per_call"]
        roof["avg_dispatch_ms"] = d["avg_dispatch_ms"]
    roof.update(traffic_of(method, N, batch, dtype, dom))
    return roof, rows


def traffic_of(method, N, batch, dtype, fam):
    """Measured HBM bytes per call of a kernel family (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, scaled), with the profile it comes from; null when the kernel
    sources changed since the counters were taken."""
    files = next((v for k, v in FAMILY_SOURCES.items() if fam.startswith(k)), None)
    if files is None:
        return {"traffic": None, "traffic_profile": None, "kernel_src_sha": None}
    sha = kernel_source_sha(files)
    t = TRAFFIC.get((method, N, batch, dtype, fam))
    ok = bool(t) and t["sha"] == sha
    return {"traffic": t["bytes_per_call"] if ok else None,
            "traffic_profile": t["profile"] if ok else None, "kernel_src_sha": sha}


def profile_target(args):
    """What the rocprofv3 counter runs measure: a plain 1 GiB device copy
    (the counter scale), then `steps` forward ALT calls of the workload."""
    import torch

    import paper_2004_11346_amd.sht as S
    from paper_2004_11346_amd import inputs
    torch.cuda.init()
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    cdt = torch.complex128 if args.dtype == "f64" else torch.complex64
    method = args.method or "idbf"
    N, batch = args.N, args.batch
    beta = torch.from_numpy(inputs.make_beta(N, batch, 2, dist="decay")).to(cdt).cuda()
    plan = S.Plan(N, batch, dtype=cdt, method=method)
    g = plan.empty_grid()
    bo = plan.empty_coefs()
    for d in args.profile_dirs.split(","):
        for _ in range(args.steps):
            if d == "fwd":
                plan.alt(0, 2 * N - 1, "fwd", beta, g)
            elif d == "inv":
                plan.alt(0, 2 * N - 1, "inv", g, bo)
            elif d == "sht_fwd":
                plan.forward(beta, out=g)
            elif d == "sht_inv":
                plan.inverse(g, out=bo)
            else:
                raise SystemExit(f"unknown profile direction {d}")
    torch.cuda.synchronize()
    print(json.dumps({"profile_target": True, "N": N, "batch": batch, "method": method, "dtype": args.dtype,
                      "alt_calls": args.steps, "copy_bytes": 2 * a.numel() * 8}), flush=True)


def n4096_full(S, inputs, timer, no_check):
    """N = 4096 (grid 8192 x 16383), 8 fields, FP64, plain form: full forward
    and inverse SHT (the phi DFT rows exceed LDS and run as two four-step
    kernels), with the error at sampled orders and rows against the oracle."""
    import numpy as np
    import torch
    N, B = 4096, 8
    M = 4 * N - 1
    t0 = time.perf_counter()
    p = S.Plan(N, B, dtype=torch.complex128, method="dense")
    tb = time.perf_counter() - t0
    beta_np = inputs.make_beta(N, B, 3, dist="decay")
    beta = torch.from_numpy(beta_np).cuda()
    f = p.forward(beta)
    bo = p.inverse(f)
    tf = timer.time(lambda: p.forward(beta, out=f), reps=2)
    ti = timer.time(lambda: p.inverse(f, out=bo), reps=2)
    r = {"fwd_ms": tf * 1e3, "inv_ms": ti * 1e3, "sht_per_s": 2 * B / (tf + ti), "plan_build_s": tb,
         "alt_gcoef_per_s_fwd_incl_dft": B * 4 * N * N / tf / 1e9}
    if not no_check:
        import oracle
        rows = [0, 4095, 8191]
        g = oracle.alt_forward_rows(N, beta_np[0], rows)
        gg = np.zeros((2 * N, M), complex)
        gg[rows] = g
        ref = oracle.dft_synthesis(N, gg, rows=rows)
        r["fwd_sampled_rows_rel_l2"] = rel_l2(f[0, rows].cpu().numpy(), ref)
        r["round_trip_rel_l2"] = rel_l2(bo.cpu().numpy(), beta_np)
    p.close()
    del beta, f, bo
    torch.cuda.empty_cache()
    return r


def n4096_window(S, inputs, timer, no_check):
    """N = 4096 (grid 8192 x 16383), 8 fields, FP64, fast form on one
    64-order window (orders 4096..4159, the unit of per-GPU sharding) against
    the plain form on the same orders, with the errors of the forward and the
    weighted transposed ALT at three orders of fields 0 and 7 against the
    oracle."""
    import numpy as np
    import torch
    N, B, lo, hi = 4096, 8, 4096, 4159
    M = 4 * N - 1
    t0 = time.perf_counter()
    p = S.Plan(N, B, dtype=torch.complex128, method="idbf", m_lo=lo, m_hi=hi)
    tb = time.perf_counter() - t0
    dense = S.Plan(N, B, dtype=torch.complex128, method="dense")
    beta_np = inputs.make_beta(N, B, 3, dist="decay")
    beta = torch.from_numpy(beta_np).cuda()
    g = torch.zeros((B, 2 * N, M), dtype=torch.complex128, device="cuda")
    bo = torch.zeros_like(beta)
    st = p.stats()["program"]
    r = {"orders": [lo, hi], "plan_build_s": tb, "stored_over_dense": st["stored_entries"] / st["dense_entries"],
         "generated_over_dense": st["generated_entries"] / st["dense_entries"]}
    for name, pl in (("fast", p), ("plain", dense)):
        r[name + "_fwd_ms"] = 1e3 * timer.time(lambda: pl.alt(lo, hi, "fwd", beta, g), reps=3)
        r[name + "_inv_ms"] = 1e3 * timer.time(lambda: pl.alt(lo, hi, "inv", g, bo), reps=3)
    r["fast_over_plain_fwd"] = r["plain_fwd_ms"] / r["fast_fwd_ms"]
    r["fast_over_plain_inv"] = r["plain_inv_ms"] / r["fast_inv_ms"]
    if not no_check:
        import oracle
        k_of, m_of = inputs.layout(N)
        absm = [lo, lo + 31, hi]
        g.zero_()
        p.alt(lo, hi, "fwd", beta, g)
        gin = torch.zeros_like(g)
        ef = ei = 0.0
        for b in (0, B - 1):
            ref = oracle.alt_forward_orders(N, beta_np[b], absm)
            gb = g[b]
            got = np.stack([np.stack([gb[:, a % M].cpu().numpy(), gb[:, (-a) % M].cpu().numpy()]) for a in absm])
            ef = max(ef, rel_l2(got, ref))
            for i, a in enumerate(absm):
                gin[b, :, a % M] = torch.from_numpy(ref[i, 0])
                gin[b, :, (-a) % M] = torch.from_numpy(ref[i, 1])
            refs = ref
            bref = oracle.alt_transpose_orders(N, refs, absm, weights=True)
            bo.zero_()
            p.alt(lo, hi, "inv", gin, bo)
            bob = bo[b].cpu().numpy()
            for i, a in enumerate(absm):
                for sgn, m in enumerate((a, -a)):
                    sel = np.nonzero(m_of == m)[0]
                    ei = max(ei, rel_l2(bob[sel], bref[i, sgn, : 2 * N - a]))
        r["fwd_sampled_orders_rel_l2"] = ef
        r["inv_sampled_orders_rel_l2"] = ei
        r["sampled_orders"] = absm
    p.close()
    dense.close()
    del beta, g, bo
    torch.cuda.empty_cache()
    return r


def n4096_orders(args):
    """N = 4096 (grid 8192 x 16383), 8 fields, FP64: the fast form (plans
    restricted to 64-order windows, the unit of per-GPU sharding) against the
    plain form on the same orders, windows spread over the whole order range.
    The full transform time is the sum over 128 windows, estimated from the
    measured ones by the trapezoid rule in the window start."""
    import torch

    import paper_2004_11346_amd.sht as S
    torch.cuda.init()
    N, B, W = 4096, 8, 64
    M = 4 * N - 1
    starts = [0, 1024, 2048, 3072, 4096, 5120, 6144, 7168, 8128]
    beta = torch.randn((B, 4 * N * N), dtype=torch.complex128, device="cuda")
    g = torch.zeros((B, 2 * N, M), dtype=torch.complex128, device="cuda")
    bo = torch.zeros_like(beta)
    timer = Timer()
    dense = S.Plan(N, B, dtype=torch.complex128, method="dense")
    rows = []
    for a0 in starts:
        lo, hi = a0, min(2 * N - 1, a0 + W - 1)
        t0 = time.perf_counter()
        p = S.Plan(N, B, dtype=torch.complex128, method="idbf", m_lo=lo, m_hi=hi)
        tb = time.perf_counter() - t0
        st = p.stats()["program"]
        r = {"orders": [lo, hi], "plan_build_s": tb, "dense_entries": st["dense_entries"],
             "stored_entries": st["stored_entries"], "generated_entries": st["generated_entries"]}
        for name, pl in (("fast", p), ("plain", dense)):
            r[name + "_fwd_ms"] = 1e3 * timer.time(lambda: pl.alt(lo, hi, "fwd", beta, g), reps=3)
            r[name + "_inv_ms"] = 1e3 * timer.time(lambda: pl.alt(lo, hi, "inv", g, bo), reps=3)
        rows.append(r)
        print(json.dumps({"window": r}), flush=True)
        p.close()
        torch.cuda.empty_cache()
    # trapezoid estimate of the whole transform (128 windows of 64 orders)
    def total(key):
        xs = [r["orders"][0] for r in rows]
        ys = [r[key] for r in rows]
        acc = 0.0
        for i in range(len(xs) - 1):
            acc += 0.5 * (ys[i] + ys[i + 1]) * (xs[i + 1] - xs[i]) / W
        return acc + ys[-1]
    est = {k: total(k) for k in ("fast_fwd_ms", "fast_inv_ms", "plain_fwd_ms", "plain_inv_ms")}
    del g, bo
    torch.cuda.empty_cache()
    fp32 = n4096_fp32_windows(S, N, B, W)
    coefs = B * 4 * N * N
    print(json.dumps({"metric": "ALT Gcoef/s at N=4096, fast vs plain, FP64, 8 fields (estimated from windows)",
                      "unit": "Gcoef/s", "n_gpus": 1, "data": "synthetic", "dtype": "f64",
                      "config": {"workload": "ALT N=4096 (grid 8192x16383), 8 fields, 64-order windows", "N": N,
                                 "batch": B, "windows": starts},
                      "estimated_full_ms": est,
                      "alt_gcoef_per_s": {k.replace("_ms", ""): coefs / (v / 1e3) / 1e9 for k, v in est.items()},
                      "fast_over_plain": {"fwd": est["plain_fwd_ms"] / est["fast_fwd_ms"],
                                          "inv": est["plain_inv_ms"] / est["fast_inv_ms"]},
                      "fp32_windows": fp32}), flush=True)


def n4096_every_order(args):
    """N = 4096 (grid 8192 x 16383), 8 fields, FP64 (or FP32 with --dtype f32:
    the fast form in split-BF16 with six products), every order: the fast ALT
    built and applied share by share (16 plans of 512 orders, the shares a
    sharded run gives each GPU: the full FP64 plan, 269 GB of factors, does not
    fit one GPU beside its grids), against the plain form (one plan of all
    orders) on the same data.  The phi DFTs, timed inside the plain form's
    SHT, complete both SHTs.  Errors against the oracle at two orders of every
    share, fields 0 and 7, forward and weighted transpose."""
    import numpy as np
    import torch

    import oracle
    import paper_2004_11346_amd.sht as S
    from paper_2004_11346_amd import inputs
    torch.cuda.init()
    N, B, W = 4096, 8, 512
    M = 4 * N - 1
    timer = Timer()
    k_of, m_of = inputs.layout(N)
    f32 = args.dtype == "f32"
    cdt = torch.complex64 if f32 else torch.complex128
    extra = {"f32_mode": 2} if f32 else {}  # FP32: split-BF16 with six products
    beta_np = inputs.make_beta(N, B, 3, dist="decay")
    if f32:
        beta_np = beta_np.astype(np.complex64).astype(np.complex128)
    beta = torch.from_numpy(beta_np).to(cdt).cuda()
    g = torch.zeros((B, 2 * N, M), dtype=cdt, device="cuda")
    bo = torch.zeros_like(beta)
    t0 = time.perf_counter()
    dense = S.Plan(N, B, dtype=cdt, method="dense")
    out = {"plain": {"plan_build_s": time.perf_counter() - t0}}
    out["plain"]["alt_fwd_ms"] = 1e3 * timer.time(lambda: dense.alt(0, 2 * N - 1, "fwd", beta, g), reps=2)
    out["plain"]["alt_inv_ms"] = 1e3 * timer.time(lambda: dense.alt(0, 2 * N - 1, "inv", g, bo), reps=2)
    f = dense.forward(beta)
    dense.profile(True)
    for _ in range(2):
        dense.forward(beta, out=f)
        dense.inverse(f, out=bo)
    torch.cuda.synchronize()
    rep = dense.profile_report()
    dense.profile(False)
    dft_ms = sum(v["total_ms"] for k, v in rep.items() if k.startswith("k_dft")) / 2
    out["plain"]["sht_fwd_ms"] = 1e3 * timer.time(lambda: dense.forward(beta, out=f), reps=2)
    out["plain"]["sht_inv_ms"] = 1e3 * timer.time(lambda: dense.inverse(f, out=bo), reps=2)
    out["dft_ms_fwd_plus_inv"] = dft_ms
    print(json.dumps({"plain": out["plain"], "dft_ms_fwd_plus_inv": dft_ms}), flush=True)
    del f
    dense.close()
    torch.cuda.empty_cache()
    shares = []
    for lo in range(0, 2 * N, W):
        hi = lo + W - 1
        t0 = time.perf_counter()
        p = S.Plan(N, B, dtype=cdt, method="idbf", m_lo=lo, m_hi=hi, **extra)
        r = {"orders": [lo, hi], "plan_build_s": time.perf_counter() - t0}
        st = p.stats()["program"]
        r["stored_entries"] = st["stored_entries"]
        r["generated_entries"] = st["generated_entries"]
        r["fwd_ms"] = 1e3 * timer.time(lambda: p.alt(lo, hi, "fwd", beta, g), reps=2)
        r["inv_ms"] = 1e3 * timer.time(lambda: p.alt(lo, hi, "inv", g, bo), reps=2)
        if not args.no_check:
            absm = [lo + 1, hi - 3]
            p.alt(lo, hi, "fwd", beta, g)
            gs = {b: g[b] for b in (0, B - 1)}
            ef = ei = 0.0
            refs = {}
            for b in (0, B - 1):
                ref = oracle.alt_forward_orders(N, beta_np[b], absm)
                if f32:  # the transposed input as the FP32 plan receives it
                    ref = ref.astype(np.complex64).astype(np.complex128)
                refs[b] = ref
                got = np.stack([np.stack([gs[b][:, a % M].cpu().numpy(), gs[b][:, (-a) % M].cpu().numpy()])
                                for a in absm]).astype(np.complex128)
                ef = max(ef, rel_l2(got, ref))
            g.zero_()
            for b, ref in refs.items():
                for i, a in enumerate(absm):
                    g[b, :, a % M] = torch.from_numpy(ref[i, 0]).to(cdt)
                    g[b, :, (-a) % M] = torch.from_numpy(ref[i, 1]).to(cdt)
            p.alt(lo, hi, "inv", g, bo)
            for b, ref in refs.items():
                bref = oracle.alt_transpose_orders(N, ref, absm, weights=True)
                bob = bo[b].cpu().numpy().astype(np.complex128)
                for i, a in enumerate(absm):
                    for sg, m in enumerate((a, -a)):
                        sel = np.nonzero(m_of == m)[0]
                        ei = max(ei, rel_l2(bob[sel], bref[i, sg, : 2 * N - a]))
            r["fwd_rel_l2"] = ef
            r["inv_rel_l2"] = ei
        shares.append(r)
        print(json.dumps({"share": r}), flush=True)
        p.close()
        torch.cuda.empty_cache()
    fast = {k: sum(r[k] for r in shares) for k in ("plan_build_s", "fwd_ms", "inv_ms", "stored_entries",
                                                     "generated_entries")}
    if not args.no_check:
        fast["fwd_rel_l2_max"] = max(r["fwd_rel_l2"] for r in shares)
        fast["inv_rel_l2_max"] = max(r["inv_rel_l2"] for r in shares)
    coefs = B * 4 * N * N
    res = {"metric": f"ALT Gcoef/s and SHT/s at N=4096, every order, fast (16 shares) vs plain, {args.dtype}, 8 fields",
           "n_gpus": 1, "data": "synthetic", "dtype": args.dtype,
           "fast_form": "split-BF16, six products" if f32 else "FP64",
           "config": {"workload": "ALT/SHT N=4096 (grid 8192x16383), 8 fields, every order", "N": N, "batch": B,
                      "shares": len(shares)},
           "fast": fast, "plain": out["plain"], "dft_ms_fwd_plus_inv": dft_ms,
           "alt_gcoef_per_s": {"fast_fwd": coefs / fast["fwd_ms"] / 1e6, "fast_inv": coefs / fast["inv_ms"] / 1e6,
                               "plain_fwd": coefs / out["plain"]["alt_fwd_ms"] / 1e6,
                               "plain_inv": coefs / out["plain"]["alt_inv_ms"] / 1e6},
           "fast_over_plain_alt": {"fwd": out["plain"]["alt_fwd_ms"] / fast["fwd_ms"],
                                   "inv": out["plain"]["alt_inv_ms"] / fast["inv_ms"]},
           "sht_per_s": {"fast": 2 * B / ((fast["fwd_ms"] + fast["inv_ms"] + dft_ms) / 1e3),
                         "plain": 2 * B / ((out["plain"]["sht_fwd_ms"] + out["plain"]["sht_inv_ms"]) / 1e3)},
           "shares": shares}
    print(json.dumps(res), flush=True)


def n4096_fp32_windows(S, N, B, W):
    """FP32 fast-form plans on two 64-order windows at N = 4096 (8 fields):
    split-BF16 with six products and FP32 storage on the FP64 matrix cores,
    timed, with the forward ALT error against the FP64 oracle at three orders
    of the window (fields 0 and 7)."""
    import numpy as np
    import torch

    import oracle
    from paper_2004_11346_amd import inputs
    from paper_2004_11346_amd import lib as L
    M = 4 * N - 1
    timer = Timer()
    beta_np = inputs.make_beta(N, B, 3, dist="decay").astype(np.complex64)
    beta = torch.from_numpy(beta_np).cuda()
    g = torch.zeros((B, 2 * N, M), dtype=torch.complex64, device="cuda")
    bo = torch.zeros_like(beta)
    out = []
    for a0 in (0, 4096):
        lo, hi = a0, a0 + W - 1
        absm = [lo, lo + W // 2, hi]
        refs = {b: oracle.alt_forward_orders(N, beta_np[b].astype(np.complex128), absm) for b in (0, B - 1)}
        for name, mode in (("split_bf16x6", L.SHT_F32_SPLIT_BF16_6), ("f32_storage_fp64_mfma", L.SHT_F32_VALU)):
            p = S.Plan(N, B, dtype=torch.complex64, method="idbf", m_lo=lo, m_hi=hi, f32_mode=mode)
            r = {"orders": [lo, hi], "form": name,
                 "fwd_ms": 1e3 * timer.time(lambda: p.alt(lo, hi, "fwd", beta, g), reps=3),
                 "inv_ms": 1e3 * timer.time(lambda: p.alt(lo, hi, "inv", g, bo), reps=3)}
            p.alt(lo, hi, "fwd", beta, g)
            errs = []
            for b in (0, B - 1):
                cols = [c for a in absm for c in (a % M, (-a) % M)]
                gh = g[b][:, cols].cpu().numpy().astype(np.complex128)
                got = np.stack([np.stack([gh[:, 2 * i], gh[:, 2 * i + 1]]) for i in range(len(absm))])
                errs.append(rel_l2(got, refs[b]))
            r["alt_fwd_sampled_orders_rel_l2"] = max(errs)
            out.append(r)
            print(json.dumps({"fp32_window": r}), flush=True)
            p.close()
            torch.cuda.empty_cache()
    return out


def uneven(args):
    """The grouped workload: 64 transforms, N drawn from {128, 256, 512, 1024}
    and 1-4 fields each (seed 4000), FP64 and FP32, each direction replayed
    from a hipGraph: the persistent mode (one persistent launch per phase,
    grid autotuned) and the batched mode (one plan per degree over all its
    fields, plain or fast form and leaf chosen by the tuner)."""
    import tempfile

    import numpy as np
    import torch

    from paper_2004_11346_amd import inputs
    from paper_2004_11346_amd.sht import Group
    torch.cuda.init()
    rng = np.random.Generator(np.random.PCG64(4000))
    Ns = [int(v) for v in rng.choice([128, 256, 512, 1024], size=64)]
    fields = [int(v) for v in rng.integers(1, 5, size=64)]
    timer = Timer()
    out = {}
    tmp = tempfile.mkdtemp(prefix="sht_group_")
    for dname, dt in (("f64", torch.complex128), ("f32", torch.complex64)):
        for mode in ("persistent", "batched"):
            kw = {} if mode == "persistent" else {"tune_file": os.path.join(tmp, f"tune_{dname}.json"),
                                                  "plan_cache_dir": tmp}
            grp = Group(Ns, fields, dtype=dt, mode=mode, **kw)
            betas = [torch.from_numpy(inputs.make_beta(N, f, 4100 + i)).to(dt).cuda()
                     for i, (N, f) in enumerate(zip(Ns, fields))]
            fs = [torch.zeros((f, 2 * N, 4 * N - 1), dtype=dt, device="cuda") for N, f in zip(Ns, fields)]
            grp.bind(betas, fs)
            t0 = time.perf_counter()
            grp.tune()
            t_tune = time.perf_counter() - t0
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                grp.capture("fwd", s)
                grp.capture("inv", s)
                tf = timer.time(lambda: grp.replay("fwd", s), reps=max(3, args.steps))
                ti = timer.time(lambda: grp.replay("inv", s), reps=max(3, args.steps))
            st = grp.stats()
            out[f"{dname}_{mode}"] = {"fwd_ms": tf * 1e3, "inv_ms": ti * 1e3,
                                      "sht_per_s": 2 * sum(fields) / (tf + ti), "tune_s": t_tune,
                                      "choices": st.get("classes", st.get("grid"))}
            print(json.dumps({"uneven": {f"{dname}_{mode}": out[f"{dname}_{mode}"]}}), flush=True)
            grp.close()
            del betas, fs
            torch.cuda.empty_cache()
    print(json.dumps({"metric": "SHT/s, uneven batch of 64 transforms", "unit": "SHT/s", "n_gpus": 1,
                      "data": "synthetic",
                      "config": {"workload": "64 transforms, N in {128,256,512,1024}, 1-4 fields (seed 4000)",
                                 "fields": sum(fields)}, "results": out}), flush=True)


def rank_study(args):
    """Sampling and rank study (Section 5, Fig. `point`): the forward and
    inverse ALT of one order (m = N where the partition yields butterflies)
    with IDs from mock-Chebyshev or random rows and
    adaptive rank r_k in {50, 100, 150}, IDs as written in Section 2.1 (no
    verification, truncated butterflies kept), plus a tolerance sweep; errors
    eps_fwd / eps_inv on 256 sampled rows against the oracle's direct
    products (Section 5), and on all rows; plan shape and apply time."""
    import numpy as np
    import torch

    import oracle
    import paper_2004_11346_amd.sht as S
    from paper_2004_11346_amd import inputs
    from paper_2004_11346_amd import lib as L
    torch.cuda.init()
    timer = Timer()
    out = []
    # (N, m): m = N as in Section 5 where butterflies exist (from N = 2048 with
    # n0 = 512), and m = N / 2 at N = 1024
    cases = [(1024, 512), (2048, 2048), (4096, 4096)]
    variants = []
    for rk in (50, 100, 150):
        for smp in ("cheb", "rand"):
            variants.append({"rk": rk, "sampling": smp, "eps": 1e-10, "id_check": 0})
    for eps in (1e-6, 1e-8, 1e-12):
        variants.append({"rk": 150, "sampling": "cheb", "eps": eps, "id_check": 0})
    for eps in (1e-10, 1e-12):
        variants.append({"rk": 150, "sampling": "cheb", "eps": eps, "id_check": 1})
    for N, m in cases:
        M = 4 * N - 1
        beta_np = inputs.make_beta(N, 1, 6, dist="half")
        beta = torch.from_numpy(beta_np).cuda()
        ref = oracle.alt_forward_orders(N, beta_np[0], [m])
        rng = np.random.Generator(np.random.PCG64(6000 + N))
        rows = np.sort(rng.choice(2 * N, size=min(256, 2 * N), replace=False))
        gin_np = inputs.make_grid(N, 1, 7)[0][:, [m % M, (-m) % M]].T.copy()
        refi = oracle.alt_transpose_orders(N, gin_np[None], [m], weights=True)[0]
        kidx = np.sort(rng.choice(2 * N - m, size=min(256, 2 * N - m), replace=False))
        gin = torch.zeros((1, 2 * N, M), dtype=torch.complex128, device="cuda")
        gin[0, :, m % M] = torch.from_numpy(gin_np[0]).cuda()
        gin[0, :, (-m) % M] = torch.from_numpy(gin_np[1]).cuda()
        for v in variants:
            smp = L.SHT_SAMPLE_MOCK_CHEB if v["sampling"] == "cheb" else L.SHT_SAMPLE_RANDOM
            t0 = time.perf_counter()
            p = S.Plan(N, 1, method="idbf", m_lo=m, m_hi=m, eps=v["eps"], rk=v["rk"], sampling=smp,
                       id_check=v["id_check"], leaf=32, n0=512)
            tb = time.perf_counter() - t0
            g = torch.zeros((1, 2 * N, M), dtype=torch.complex128, device="cuda")
            bo = torch.zeros((1, 4 * N * N), dtype=torch.complex128, device="cuda")
            tf = timer.time(lambda: p.alt(m, m, "fwd", beta, g), reps=3)
            ti = timer.time(lambda: p.alt(m, m, "inv", gin, bo), reps=3)
            gh = g[0].cpu().numpy()
            got = np.stack([gh[:, m % M], gh[:, (-m) % M]])
            k_of, m_of = inputs.layout(N)
            boh = bo[0].cpu().numpy()
            goti = np.stack([boh[m_of == m], boh[m_of == -m]])
            st = p.stats()["program"]
            r = dict(v, N=N, m=m, plan_build_s=tb, alt_fwd_ms=tf * 1e3, alt_inv_ms=ti * 1e3,
                     eps_fwd_256=rel_l2(got[:, rows], ref[0][:, rows]), eps_fwd_all=rel_l2(got, ref[0]),
                     eps_inv_256=rel_l2(goti[:, kidx], refi[:, kidx]),
                     eps_inv_all=rel_l2(goti, refi[:, : 2 * N - m]),
                     stored_entries=st["stored_entries"], generated_entries=st["generated_entries"],
                     dense_entries=st["dense_entries"], blocks_butterfly=st["blocks_butterfly"],
                     max_rank=st["max_rank"])
            out.append(r)
            print(json.dumps({"rank_study": r}), flush=True)
            p.close()
    print(json.dumps({"metric": "ALT error vs ID sampling, adaptive rank and tolerance",
                      "unit": "relative l2", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "single order, leaf 32, n0 512, IDs as in Section 2.1",
                                 "cases": cases}, "results": out}), flush=True)


def level_schedules(args):
    """The butterfly levels of the fast form at N = 1024, 32 fields, FP64, with
    butterflies from 128, 256 and 512 columns (leaf 32, 64, 128): staged
    schedule (one launch per level) against the fused one (every block's
    levels in one workgroup, rows in LDS), per kernel family of one forward and
    one inverse SHT (HIP events on the launch stream), and the step time."""
    import torch

    import paper_2004_11346_amd.sht as S
    from paper_2004_11346_amd import inputs
    from paper_2004_11346_amd import lib as L
    torch.cuda.init()
    N, batch = args.N, args.batch
    beta = torch.from_numpy(inputs.make_beta(N, batch, 2, dist="decay")).cuda()
    out = {}
    for leaf in (32, 64, 128):
        for name, ls in (("staged", L.SHT_LEVELS_STAGED), ("fused", L.SHT_LEVELS_FUSED)):
            plan = S.Plan(N, batch, method="idbf", leaf=leaf, level_schedule=ls)
            f = plan.empty_grid()
            bo = plan.empty_coefs()
            for _ in range(2):
                plan.forward(beta, out=f)
                plan.inverse(f, out=bo)
            torch.cuda.synchronize()
            rec = {}
            for d in ("fwd", "inv"):
                plan.profile(True)
                for _ in range(args.steps):
                    if d == "fwd":
                        plan.forward(beta, out=f)
                    else:
                        plan.inverse(f, out=bo)
                torch.cuda.synchronize()
                rep = plan.profile_report()
                fam = {}
                for k, v in rep.items():
                    fk = k.split("[", 1)[0] + ("[final]" if k.endswith("[final]") else "")
                    fam[fk] = fam.get(fk, 0.0) + v["total_ms"] / args.steps
                rec[d] = {k: round(v, 4) for k, v in fam.items()}
            plan.profile(False)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                plan.forward(beta, out=f)
                plan.inverse(f, out=bo)
            e1.record()
            torch.cuda.synchronize()
            rec["step_ms"] = e0.elapsed_time(e1) / args.steps
            st = plan.stats()["program"]
            rec["stored_values"] = st["fwd_values"]
            rec["generated_entries"] = st["generated_entries"]
            out[f"leaf{leaf}_{name}"] = rec
            print(json.dumps({f"leaf{leaf}_{name}": rec}), flush=True)
            plan.close()
    print(json.dumps({"metric": "level schedules of the fast form", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"SHT N={N}, {batch} fields, f64, idbf leaf 32/64/128",
                                 "N": N, "batch": batch}, "results": out}))


def plan_build(args):
    """Plan construction of the fast form for every order of one N, window by
    window (64 orders per plan, the share a GPU builds and holds when the
    transform is sharded by order): host build time (the Legendre tables,
    partition, IDs, low-rank factors, packing; all host threads) and the plan's
    size, per window and in total.  Runs on the host only."""
    import ctypes

    from paper_2004_11346_amd import lib as L
    lib = L.load()
    N, W = args.N, 64
    rows = []
    tot = {"build_s": 0.0, "wall_s": 0.0, "stored_entries": 0, "generated_entries": 0, "dense_entries": 0,
           "value_bytes_f64": 0}
    first, last = 0, 2 * N - 1
    if args.orders:
        first, last = (int(v) for v in args.orders.split(":"))
    for a0 in range(first - first % W, min(last, 2 * N - 1) + 1, W):
        lo, hi = a0, min(2 * N - 1, a0 + W - 1)
        o = L.default_opts(m_lo=lo, m_hi=hi)
        h = ctypes.c_void_p()
        t0 = time.perf_counter()
        L.check(lib.sht_host_plan_create(N, L.SHT_IDBF, ctypes.byref(o), ctypes.byref(h)), "host plan")
        wall = time.perf_counter() - t0
        n = lib.sht_host_plan_stats(h, None, 0)
        buf = ctypes.create_string_buffer(n)
        lib.sht_host_plan_stats(h, buf, n)
        st = json.loads(buf.value.decode())
        lib.sht_host_plan_destroy(h)
        r = {"orders": [lo, hi], "build_s": st["build_seconds"], "wall_s": wall,
             "stored_entries": st["stored_entries"], "generated_entries": st["generated_entries"],
             "dense_entries": st["dense_entries"],
             "value_bytes_f64": 8 * (st["fwd_values"] + st["adj_values"])}
        for k in tot:
            tot[k] += r.get(k, 0)
        rows.append(r)
        print(json.dumps({"window": r}), flush=True)
    print(json.dumps({"metric": f"fast-form plan construction, N={N}, orders {first}:{last} in {len(rows)} windows "
                                f"of {W}",
                      "n_gpus": 0, "data": "synthetic", "config": {"workload": f"plan build N={N}", "N": N,
                                                                    "windows": len(rows)},
                      "threads": os.cpu_count(), "totals": tot}), flush=True)


def fp32_legs(S, inputs, timer, N, batch, beta_np, no_check):
    """FP32 plans at the same workload: plain form, fast form on the VALU and
    fast form on the BF16 matrix cores (split-BF16, three and six products),
    with the ALT error against the FP64 oracle at sampled orders (field 0)."""
    import numpy as np
    import torch

    from paper_2004_11346_amd import lib as L
    M = 4 * N - 1
    beta32 = torch.from_numpy(beta_np.astype(np.complex64)).cuda()
    absm = [0, 1, N // 2, N, 3 * N // 2, 2 * N - 1] + list(inputs.sample_indices(2 * N, 10, 11))
    ref = None
    if not no_check:
        import oracle
        ref = oracle.alt_forward_orders(N, beta_np[0].astype(np.complex64).astype(np.complex128), absm)
    legs = {}
    for name, meth, mode in (("dense_f32", "dense", L.SHT_F32_VALU), ("idbf_f32", "idbf", L.SHT_F32_VALU),
                             ("idbf_split_bf16x3", "idbf", L.SHT_F32_SPLIT_BF16),
                             ("idbf_split_bf16x6", "idbf", L.SHT_F32_SPLIT_BF16_6)):
        kw = {} if meth == "dense" else {"f32_mode": mode}
        p = S.Plan(N, batch, dtype=torch.complex64, method=meth, **kw)
        g = p.empty_grid()
        ob = p.empty_coefs()
        taf = timer.time(lambda: p.alt(0, 2 * N - 1, "fwd", beta32, g), reps=3)
        tai = timer.time(lambda: p.alt(0, 2 * N - 1, "inv", g, ob), reps=3)
        leg = {"batch": batch, "alt_fwd_ms": taf * 1e3, "alt_inv_ms": tai * 1e3,
               "alt_fwd_gcoef_s": batch * 4 * N * N / taf / 1e9, "alt_inv_gcoef_s": batch * 4 * N * N / tai / 1e9}
        if ref is not None:
            p.alt(0, 2 * N - 1, "fwd", beta32, g)
            gh = g[0].cpu().numpy().astype(np.complex128)
            got = np.stack([np.stack([gh[:, a % M], gh[:, (-a) % M]]) for a in absm])
            leg["alt_fwd_sampled_orders_rel_l2"] = rel_l2(got, ref)
            leg["alt_fwd_sampled_orders_rel_max"] = rel_max(got, ref)
        legs[name] = leg
        p.close()
        torch.cuda.empty_cache()
    return legs


def dft_lengths(args):
    """The phi DFT alone (Section 1, the phi sums of the SHT) for lengths that
    take each schedule: rows in LDS with register radices (N = 1024), rows with
    a Rader last pass (N = 512, 2047 = 23 x 89), a prime row by Rader's
    convolution (N = 2048, 8191), four-step with Rader last passes (N = 4096,
    16383 = 129 x 127, FP64 and FP32).  Plain-form plans (the DFT does not
    depend on the ALT form); synthesis and analysis timed with the library's
    HIP events over 3 calls each.  Algorithmic bytes: one read and one write of
    the grid per pass through HBM (one for rows and Rader, two for four-step)."""
    import torch

    import paper_2004_11346_amd.sht as S
    from paper_2004_11346_amd import inputs

    torch.cuda.init()
    cases = [(1024, 32, "f64"), (512, 32, "f64"), (2048, 16, "f64"), (4096, 8, "f64"), (4096, 8, "f32")]
    out = []
    for N, B, dt in cases:
        cdt = torch.complex128 if dt == "f64" else torch.complex64
        elt = 16 if dt == "f64" else 8
        M = 4 * N - 1
        plan = S.Plan(N, B, dtype=cdt, method="dense")
        st = plan.stats()
        beta = torch.from_numpy(inputs.make_beta(N, B, 2, dist="decay")).to(cdt).cuda()
        f = plan.empty_grid()
        bo = plan.empty_coefs()
        plan.forward(beta, out=f)
        plan.inverse(f, out=bo)
        torch.cuda.synchronize()
        rt = rel_l2(bo.cpu().numpy().astype("complex128"), beta.cpu().numpy().astype("complex128"))
        plan.profile(True)
        for _ in range(3):
            plan.forward(beta, out=f)
            plan.inverse(f, out=bo)
        torch.cuda.synchronize()
        rep = plan.profile_report()
        plan.profile(False)
        grid_bytes = elt * B * 2 * N * M
        passes = 2 if st["dft"] == "four_step" else 1
        r = {"N": N, "batch": B, "dtype": dt, "M": M, "schedule": st["dft"], "rader_last": st["dft_rader_last"],
             "grid_bytes": grid_bytes, "round_trip_rel_l2": rt}
        for d in ("synthesis", "analysis"):
            ms = rep["k_dft_" + d]["total_ms"] / 3
            gbs = 2 * passes * grid_bytes / (ms / 1e3) / 1e9
            r[d] = {"ms": ms, "GB_s": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        print(json.dumps(r), flush=True)
        out.append(r)
        del f, bo, beta
        plan.close()
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "phi DFT per direction, GB/s of one read and one write of the grid per HBM pass",
                      "n_gpus": 1, "data": "synthetic", "cases": out}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (the path would shard by order across "
                                   "GPUs; only one GPU's share is implemented)"}))
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("one GPU only: launch without torch.distributed", file=sys.stderr)
        sys.exit(2)

    if args.profile_target:
        profile_target(args)
        return
    if args.workload == "n4096-orders":
        n4096_orders(args)
        return
    if args.workload == "n4096-every-order":
        n4096_every_order(args)
        return
    if args.workload == "uneven":
        uneven(args)
        return
    if args.workload == "rank-study":
        rank_study(args)
        return
    if args.workload == "levels":
        level_schedules(args)
        return
    if args.workload == "plan-build":
        plan_build(args)
        return
    if args.workload == "dft":
        dft_lengths(args)
        return

    import numpy as np
    import torch

    import paper_2004_11346_amd.sht as S
    from paper_2004_11346_amd import inputs

    torch.cuda.init()
    N, batch = args.N, args.batch
    cdt = torch.complex128 if args.dtype == "f64" else torch.complex64
    M = 4 * N - 1
    method = args.method or "idbf"
    timer = Timer()

    beta_np = inputs.make_beta(N, batch, 2, dist="decay")
    beta = torch.from_numpy(beta_np).to(cdt).cuda()
    t_build0 = time.perf_counter()
    plan = S.Plan(N, batch, dtype=cdt, method=method)
    t_build = time.perf_counter() - t_build0
    f = plan.empty_grid()
    bout = plan.empty_coefs()

    def step():
        plan.forward(beta, out=f)
        plan.inverse(f, out=bout)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_per_step = e0.elapsed_time(e1) / args.steps
    value = 2.0 * batch / (ms_per_step / 1e3)

    # ALT rates, then the kernels of one step (forward SHT, then inverse SHT),
    # each bracketed by HIP events that the library records on the stream the
    # kernel is launched on
    g = plan.empty_grid()
    reps = max(3, args.steps)
    t_alt_fwd = timer.time(lambda: plan.alt(0, 2 * N - 1, "fwd", beta, g), reps=reps)
    t_alt_inv = timer.time(lambda: plan.alt(0, 2 * N - 1, "inv", g, bout), reps=reps)
    plan.profile(True)
    for _ in range(reps):
        plan.forward(beta, out=f)
    kern_fwd = plan.profile_report()
    plan.profile(True)
    for _ in range(reps):
        plan.inverse(f, out=bout)
    kern_inv = plan.profile_report()
    plan.profile(False)
    stats = plan.stats()
    roof, step_kern = step_roofline(method, N, batch, args.dtype, stats.get("program", {}), kern_fwd, kern_inv,
                                    reps)

    out = {
        "metric": "SHT/s + ALT Gcoef/s at N=1024/4096, IDBF vs dense, FP64 & FP32, vs FP64 oracle",
        "value": value,
        "unit": "SHT/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"SHT N={N} (grid {2 * N}x{M}), {batch} fields, {method} ALT, "
                               f"{args.dtype}, forward+inverse per step",
                   "N": N, "batch": batch, "method": method},
        "alt_gcoef_per_s_fwd": batch * 4 * N * N / t_alt_fwd / 1e9,
        "alt_gcoef_per_s_inv": batch * 4 * N * N / t_alt_inv / 1e9,
        "plan_build_s": t_build,
        "roofline": roof,
        "step_kernels": step_kern,
        "plan_shape": plan_shape(stats),
    }

    if not args.no_check:
        # errors against the oracle at sampled orders (ALT) and rows (full SHT)
        import oracle
        absm = [0, 1, N // 2, N, 3 * N // 2, 2 * N - 1] + list(inputs.sample_indices(2 * N, 10, 11))
        gh = g.cpu().numpy()
        plan.alt(0, 2 * N - 1, "fwd", beta, g)
        gh = g.cpu().numpy()
        errs = []
        for b in sorted({0, batch - 1}):
            ref = oracle.alt_forward_orders(N, beta_np[b], absm)
            got = np.stack([np.stack([gh[b][:, a % M], gh[b][:, (-a) % M]]) for a in absm])
            errs.append((rel_l2(got, ref), rel_max(got, ref)))
        plan.forward(beta, out=f)
        plan.inverse(f, out=bout)
        rt = rel_l2(bout.cpu().numpy(), beta_np)
        out["errors_vs_oracle"] = {"alt_fwd_sampled_orders_rel_l2": max(e[0] for e in errs),
                                   "alt_fwd_sampled_orders_rel_max": max(e[1] for e in errs),
                                   "round_trip_rel_l2": rt, "orders_checked": len(absm)}

    if not args.no_details:
        det = {}
        for meth in (["dense", "idbf"] if method == "idbf" else ["dense"]):
            for bb in (1, batch):
                p = plan if (meth == method and bb == batch) else S.Plan(N, bb, dtype=cdt, method=meth)
                bt = beta[:bb].contiguous()
                ff = p.empty_grid()
                ob = p.empty_coefs()
                tf = timer.time(lambda: p.forward(bt, out=ff), reps=3)
                ti = timer.time(lambda: p.inverse(ff, out=ob), reps=3)
                ga = p.empty_grid()
                taf = timer.time(lambda: p.alt(0, 2 * N - 1, "fwd", bt, ga), reps=3)
                tai = timer.time(lambda: p.alt(0, 2 * N - 1, "inv", ga, ob), reps=3)
                det[f"{meth}_b{bb}"] = {"fwd_sht_per_s": bb / tf, "inv_sht_per_s": bb / ti,
                                        "alt_fwd_ms": taf * 1e3, "alt_inv_ms": tai * 1e3,
                                        "alt_fwd_gcoef_s": bb * 4 * N * N / taf / 1e9,
                                        "alt_inv_gcoef_s": bb * 4 * N * N / tai / 1e9,
                                        "sht_fwd_ms": tf * 1e3, "sht_inv_ms": ti * 1e3}
                if p is not plan:
                    p.close()
        if "dense_b%d" % batch in det and "idbf_b%d" % batch in det:
            for bb in (1, batch):
                for d in ("fwd", "inv"):
                    det[f"idbf_speedup_alt_{d}_b{bb}"] = (det[f"dense_b{bb}"][f"alt_{d}_ms"] /
                                                          det[f"idbf_b{bb}"][f"alt_{d}_ms"])
        if method == "idbf":
            # butterflies from 128 columns (leaf 32, the paper's placement at
            # this size) beside the size-chosen default plan
            t0 = time.perf_counter()
            p = S.Plan(N, batch, dtype=cdt, method="idbf", leaf=32)
            tb = time.perf_counter() - t0
            ga = p.empty_grid()
            ob = p.empty_coefs()
            taf = timer.time(lambda: p.alt(0, 2 * N - 1, "fwd", beta, ga), reps=3)
            tai = timer.time(lambda: p.alt(0, 2 * N - 1, "inv", ga, ob), reps=3)
            det[f"idbf_leaf32_b{batch}"] = {"alt_fwd_ms": taf * 1e3, "alt_inv_ms": tai * 1e3, "plan_build_s": tb,
                                            "plan_shape": plan_shape(p.stats())}
            p.close()
            torch.cuda.empty_cache()
        if args.dtype == "f64" and method == "idbf":
            det.update(fp32_legs(S, inputs, timer, N, batch, beta_np, args.no_check))
        # real fields: 2 batch real fields on the same plan (two per complex
        # transform), forward and inverse
        nreal = 2 * batch
        half = torch.from_numpy(inputs.make_beta(N, nreal, 8, dist="decay")[:, : N * (2 * N + 1)].copy()).to(cdt).cuda()
        fr = plan.forward_real(half)
        hb = plan.inverse_real(fr)
        tfr = timer.time(lambda: plan.forward_real(half, out=fr), reps=3)
        tir = timer.time(lambda: plan.inverse_real(fr, out=hb), reps=3)
        det[f"real_fields_{nreal}"] = {"fwd_ms": tfr * 1e3, "inv_ms": tir * 1e3,
                                       "sht_per_s": 2 * nreal / (tfr + tir),
                                       "note": f"{nreal} real fields on the {batch}-field plan"}
        del half, fr, hb
        torch.cuda.empty_cache()
        if N == 1024 and args.dtype == "f64":
            det["n4096_plain_b8"] = n4096_full(S, inputs, timer, args.no_check)
            det["n4096_window_b8"] = n4096_window(S, inputs, timer, args.no_check)
        out["details"] = det

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
