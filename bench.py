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
                    help="ALT directions run by --profile-target (comma separated: fwd, inv)")
    ap.add_argument("--workload", choices=["default", "n4096-orders", "uneven"], default="default",
                    help="n4096-orders: N=4096, 8 fields, fast vs plain ALT on 64-order windows across the "
                         "order range; uneven: the grouped 64-transform workload")
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
    """The oracle (plain CPU FP64 definition) on a bounded sample of the same
    workload, extrapolated to one forward + one inverse SHT of one field."""
    import numpy as np

    import oracle
    from paper_2004_11346_amd import inputs

    beta = inputs.make_beta(N, 1, 2, dist="decay")[0]
    n = 2 * N
    step = max(1, n // 512)
    absm = list(range(0, n, step))
    rows = list(range(0, n, max(1, n // 128)))
    work_all = sum(n - a for a in range(n))
    work_s = sum(n - a for a in absm)
    t0 = time.perf_counter()
    gfw = oracle.alt_forward_orders(N, beta, absm)
    t1 = time.perf_counter()
    oracle.alt_transpose_orders(N, gfw, absm, weights=True)
    t2 = time.perf_counter()
    g = np.zeros((n, 4 * N - 1), complex)
    fr = oracle.dft_synthesis(N, g, rows=rows)
    t3 = time.perf_counter()
    oracle.dft_analysis(N, fr)
    t4 = time.perf_counter()
    scale_alt = work_all / work_s
    scale_dft = n / len(rows)
    t_fwd = (t1 - t0) * scale_alt + (t3 - t2) * scale_dft
    t_inv = (t2 - t1) * scale_alt + (t4 - t3) * scale_dft
    return {
        "value": 2.0 / (t_fwd + t_inv),
        "unit": "SHT/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"N={N}, one field: forward and transposed ALT for {len(absm)} of {n} orders |m| "
                   f"(both signs), phi synthesis and analysis for {len(rows)} of {n} latitude rows; "
                   f"measured {t4 - t0:.1f} s, extrapolated by work to full forward+inverse SHTs"),
        "seconds_measured": t4 - t0,
        "fwd_s_per_field": t_fwd,
        "inv_s_per_field": t_inv,
    }


# HBM bytes per ALT call read from rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE in separate runs, see profiles/), scaled by the ratio that the
# same counters give for a 1 GiB device copy.  Each entry is keyed on the
# SHA-256 of the kernel sources it was measured with; a changed source makes
# the figure stale and it is reported as null.
TRAFFIC = {
    # HBM bytes per forward ALT call of each kernel family: rocprofv3 FETCH_SIZE
    # and WRITE_SIZE runs (two calls each), scaled by what the counters read
    # for a 1 GiB copy in the same run; valid for the kernel sources of "sha"
    ("dense", 1024, 32, "f64", "k_dense_fwd_mfma"): {"bytes_per_call": 24.06e9, "sha": "21a5dbab89ebbe02",
                                                     "profile": "profiles/alt_fwd_dense_n1024_b32_f64.md"},
    ("dense", 1024, 1, "f64", "k_dense_fwd_valu"): {"bytes_per_call": 0.7513e9, "sha": "21a5dbab89ebbe02",
                                                    "profile": "profiles/alt_fwd_dense_n1024_b1_f64.md"},
    ("idbf", 1024, 32, "f64", "k_gen_fwd_mfma"): {"bytes_per_call": 15.37e9, "sha": "d9dc951b5db97d43",
                                                   "profile": "profiles/alt_fwd_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 32, "f64", "k_ops_mfma"): {"bytes_per_call": 4.346e9, "sha": "d9dc951b5db97d43",
                                               "profile": "profiles/alt_fwd_idbf_n1024_b32_f64.md"},
    ("idbf", 1024, 1, "f64", "k_ops"): {"bytes_per_call": 0.1472e9, "sha": "d9dc951b5db97d43",
                                         "profile": "profiles/alt_fwd_idbf_n1024_b1_f64.md"},
    ("idbf", 1024, 1, "f64", "k_gen_fwd"): {"bytes_per_call": 0.811e9, "sha": "d9dc951b5db97d43",
                                             "profile": "profiles/alt_fwd_idbf_n1024_b1_f64.md"},
}


def kernel_source_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2004_11346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _kernel_sum(kern, names):
    parts = [v for name, v in kern.items() if any(name == n or name.startswith(n + "[") for n in names)]
    return (sum(v["launches"] for v in parts) if parts else 0,
            sum(v["total_ms"] for v in parts) if parts else float("nan"))


def _roof(bound, work, per_call_s, unit_peak):
    unit, peak = unit_peak
    ach = work / per_call_s / (1e12 if unit == "TFLOP/s" else 1e9)
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}


TFLOPS = ("TFLOP/s", PEAK_FP64_TFLOPS)
GBS = ("GB/s", PEAK_HBM_GBS)


def roofline(method, N, batch, dtype, stats, kern, reps):
    """Roofline objects of the forward ALT: the dominant kernel, and (fast
    form) the other kernel family beside it.

    Algorithmic work per ALT call (all orders, one batch, R = 4 batch real
    right-hand sides, s bytes per stored value and vector entry):
      plain form (k_dense_fwd_*): flops = 2 R N^2 (2N + 1), every entry of
        every half matrix once per right-hand side (regeneration not counted);
      regenerated blocks (k_gen_fwd*): flops = (2 R + 6) (regenerated entries):
        the product, and the two-step recurrence and scaling of each entry;
      op stages (k_ops*, one launch per program stage): bytes = stored values
        s + index bytes + (gathered rows + written rows) R s, the rows that the
        level-by-level schedule moves through HBM.
    The dominant family (`roofline`) is the one with the larger measured time
    per call; the other is `roofline_other`.  "launch" = every launch of that
    kernel family per call."""
    R = 4 * batch
    sb = 8 if dtype == "f64" else 4
    if method == "dense":
        mf = any(n.startswith("k_dense_fwd_mfma") for n in kern)
        name = "k_dense_fwd_mfma" if mf else "k_dense_fwd_valu"
        launches, ms = _kernel_sum(kern, [name])
        per = ms / reps / 1e3
        flops = 2.0 * R * N * N * (2 * N + 1)
        prim = _roof("mfma" if mf else "alu", flops, per, TFLOPS)
        prim.update({"kernel": name, "launches_per_call": launches / reps, "kernel_ms_per_call": per * 1e3,
                     "dispatches_per_call": launches / reps, "algorithmic_flops_per_call": flops})
        files = ["kernels_dense.hip", "dense_device.h"]
        return _traffic(prim, method, N, batch, dtype, name, files), None
    prog = stats.get("program", {})
    mf = any(n.startswith("k_ops_mfma") for n in kern)
    ops_name, gen_name = ("k_ops_mfma", "k_gen_fwd_mfma") if mf else ("k_ops", "k_gen_fwd")
    files = ["idbf_kernels.hip", "idbf_pack.cpp"]
    gl, gms = _kernel_sum(kern, [gen_name])
    gper = gms / reps / 1e3
    gflops = (2.0 * R + 6.0) * float(prog.get("generated_entries", 0))
    gen = _roof("mfma" if mf else "alu", gflops, gper, TFLOPS)
    rc_valu = 4 if R <= 4 else 8 if R <= 8 else 16
    gen.update({"kernel": gen_name, "launches_per_call": gl / reps, "kernel_ms_per_call": gper * 1e3,
                "dispatches_per_call": (R + 31) // 32 if mf else (R + rc_valu - 1) // rc_valu,
                "algorithmic_flops_per_call": gflops})
    ol, oms = _kernel_sum(kern, [ops_name])
    oper = oms / reps / 1e3
    obytes = (float(prog.get("stored_entries", 0)) * sb + float(prog.get("fwd_index_bytes", 0))
              + (float(prog.get("fwd_gather_rows", 0)) + float(prog.get("fwd_out_rows", 0))) * R * sb)
    ops = _roof("hbm", obytes, oper, GBS)
    ops.update({"kernel": ops_name + " (all program stages)", "launches_per_call": ol / reps,
                "dispatches_per_call": ol / reps,
                "kernel_ms_per_call": oper * 1e3, "algorithmic_bytes_per_call": obytes,
                "algorithmic_flops_per_call": 2.0 * R * float(prog.get("stored_entries", 0))})
    gen = _traffic(gen, method, N, batch, dtype, gen_name, files)
    ops = _traffic(ops, method, N, batch, dtype, ops_name, files)
    return (gen, ops) if not (oper > gper) else (ops, gen)


def _traffic(r, method, N, batch, dtype, name, files):
    sha = kernel_source_sha(files)
    t = TRAFFIC.get((method, N, batch, dtype, name))
    r["traffic"] = t["bytes_per_call"] if t and t["sha"] == sha else None
    r["kernel_src_sha"] = sha
    return r


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
            else:
                plan.alt(0, 2 * N - 1, "inv", g, bo)
    torch.cuda.synchronize()
    print(json.dumps({"profile_target": True, "N": N, "batch": batch, "method": method, "dtype": args.dtype,
                      "alt_calls": args.steps, "copy_bytes": 2 * a.numel() * 8}), flush=True)


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
    and 1-4 fields each (seed 4000), one persistent launch per phase,
    autotuned, replayed from a hipGraph; FP64 and FP32."""
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
    for dname, dt in (("f64", torch.complex128), ("f32", torch.complex64)):
        grp = Group(Ns, fields, dtype=dt)
        betas = [torch.from_numpy(inputs.make_beta(N, f, 4100 + i)).to(dt).cuda()
                 for i, (N, f) in enumerate(zip(Ns, fields))]
        fs = [torch.zeros((f, 2 * N, 4 * N - 1), dtype=dt, device="cuda") for N, f in zip(Ns, fields)]
        grp.bind(betas, fs)
        grp.tune()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            grp.capture("fwd", s)
            grp.capture("inv", s)
            tf = timer.time(lambda: grp.replay("fwd", s), reps=max(3, args.steps))
            ti = timer.time(lambda: grp.replay("inv", s), reps=max(3, args.steps))
        out[dname] = {"fwd_ms": tf * 1e3, "inv_ms": ti * 1e3, "sht_per_s": 2 * sum(fields) / (tf + ti),
                      "grid": grp.stats()["grid"]}
        grp.close()
    print(json.dumps({"metric": "SHT/s, uneven batch of 64 transforms in one persistent launch per phase",
                      "unit": "SHT/s", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "64 transforms, N in {128,256,512,1024}, 1-4 fields (seed 4000)",
                                 "fields": sum(fields)}, "results": out}), flush=True)


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
    if args.workload == "uneven":
        uneven(args)
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

    # dominant kernel: timed alone, per launch, with HIP events that the
    # library records on the stream the kernel runs on
    g = plan.empty_grid()
    t_alt_fwd = timer.time(lambda: plan.alt(0, 2 * N - 1, "fwd", beta, g), reps=max(3, args.steps))
    t_alt_inv = timer.time(lambda: plan.alt(0, 2 * N - 1, "inv", g, bout), reps=max(3, args.steps))
    reps = max(3, args.steps)
    plan.profile(True)
    for _ in range(reps):
        plan.alt(0, 2 * N - 1, "fwd", beta, g)
    kern = plan.profile_report()
    plan.profile(False)
    stats = plan.stats()
    roof, roof2 = roofline(method, N, batch, args.dtype, stats, kern, reps)

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
        "roofline_other": roof2,
        "alt_kernels_fwd": kern,
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
        if args.dtype == "f64" and method == "idbf":
            det.update(fp32_legs(S, inputs, timer, N, batch, beta_np, args.no_check))
        out["details"] = det

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
