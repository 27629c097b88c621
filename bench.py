#!/usr/bin/env python3
"""Benchmark: GLUP/s of the temporally blocked stencil scheme on one MI355X.

Workload (the one the blocked-vs-naive target is stated for): the 25-point
8th-order variable-coefficient axis-symmetric stencil (Fig. 1d of the paper),
480^3 interior, halo 4, 13 FP32 coefficient arrays, 100 time steps, seeded
synthetic inputs.  One benchmark "step" is one complete stencil_run of all
100 time steps with the blocked scheme (diamond rows in y, wavefront in z),
inputs resident in HBM.  value = lattice-site updates per second, counting
only the algorithmic 480^3 * 100 updates (never recomputed halos).

Beside it the same run is timed with the naive scheme (the baseline of the
2x target), with BF16 coefficients, and the leapfrog adjoint workload
(256^3, 200 steps) is timed forward and backward.  The FP64 CPU oracle is
timed on a bounded sample of the same workload on the host cores.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dw", type=int, default=16)
    ap.add_argument("--no-extras", action="store_true", help="skip naive/BF16/adjoint legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--n", type=int, default=None, help="override the grid size (testing only)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint leg (forward with checkpoints, then the adjoint)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the device-to-device copy probe and print its bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); the path "
              "would shard along y with whole diamonds per GPU, which is not built here.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1410_3060_amd as st
    import workloads
    from paper_1410_3060_amd import model

    st.load()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    probe = copy_probe(torch)
    if args.copy_probe:
        print(json.dumps({"copy_probe": probe}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(st, workloads, torch, np, stream, args)}),
              flush=True)
        return

    t_gen = time.time()
    wl = workloads.make(4, n=args.n)
    log(f"[bench] generated {wl.name} n={wl.n3} in {time.time() - t_gen:.1f}s")
    h, nt = wl.halo, wl.nt
    nx, ny, nz = wl.n3
    lups = nx * ny * nz * nt

    def upload_fields():
        a = st.alloc_field(wl.n3, h)
        a.copy_(torch.from_numpy(wl.u0))
        b = st.alloc_field(wl.n3, h)
        return a, b

    coef32 = st.alloc_field(wl.n3, h, count=13)
    coef32.copy_(torch.from_numpy(wl.coef))
    u_a, u_b = upload_fields()
    u0_dev = u_a.clone()

    def timed(ctx, coef, steps, warmup):
        """Run warmup + steps full runs; returns per-run seconds (HIP events on the stream)."""
        times = []
        for i in range(warmup + steps):
            u_a.copy_(u0_dev)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.run(st.KIND_25PT_VAR, u_a, u_b, nt, halo=h, coef=coef)
            e1.record(stream)
            torch.cuda.synchronize()
            if i >= warmup:
                times.append(e0.elapsed_time(e1) / 1e3)
        return times

    R, K = 4, 13
    H = args.dw // (2 * R)
    n_rows = len(st.plan_rows(3, args.dw, ny, nt))

    log(f"[bench] blocked dw={args.dw}: {n_rows} row launches per run")
    ctx_b = st.Context(st.BLOCKED, dw=args.dw, stream=stream)
    tb = timed(ctx_b, coef32, args.steps, args.warmup)
    t_step = float(np.median(tb))
    value = lups / t_step / 1e9
    log(f"[bench] blocked: {t_step * 1e3:.2f} ms per run, {value:.1f} GLUP/s")

    bpl_b = model.blocked_bytes_per_lup(st.KIND_25PT_VAR, args.dw)
    # average row-launch duration from the same HIP events (launch gaps included)
    avg_launch = t_step / n_rows
    achieved = bpl_b * lups / n_rows / avg_launch / 1e9
    traffic = measured_traffic(wl.name, args.dw)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 3),
                "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                "algorithmic_per_launch_GB": round(bpl_b * lups / n_rows / 1e9, 3),
                "copy_probe_GBps": probe["GBps"],
                "kernel": "blocked_row_kernel<3,float,H=%d>" % H,
                "bytes_per_lup": round(bpl_b, 3), "avg_launch_ms": round(avg_launch * 1e3, 4)}

    extras = {}
    if not args.no_extras:
        ctx_n = st.Context(st.NAIVE, stream=stream)
        tn = timed(ctx_n, coef32, max(2, args.steps // 2), 1)
        tn_s = float(np.median(tn))
        bpl_n = model.naive_code_balance(st.KIND_25PT_VAR)
        extras["naive"] = {"glups": round(lups / tn_s / 1e9, 2), "ms_per_run": round(tn_s * 1e3, 3),
                           "bytes_per_lup": bpl_n,
                           "achieved_GBps": round(bpl_n * lups / tn_s / 1e9, 1)}
        extras["blocked_over_naive"] = round(tn_s / t_step, 3)
        log(f"[bench] naive: {tn_s * 1e3:.2f} ms per run ({extras['naive']['glups']} GLUP/s)")
        # BF16 coefficient storage
        bits = workloads.to_bf16_bits(wl.coef)
        coef16 = st.alloc_field(wl.n3, h, count=13, dtype=torch.bfloat16)
        coef16.copy_(torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16))
        del bits
        tb16 = float(np.median(timed(ctx_b, coef16, max(2, args.steps // 2), 1)))
        tn16 = float(np.median(timed(ctx_n, coef16, max(2, args.steps // 2), 1)))
        extras["bf16"] = {"blocked_glups": round(lups / tb16 / 1e9, 2),
                          "naive_glups": round(lups / tn16 / 1e9, 2),
                          "blocked_over_naive": round(tn16 / tb16, 3)}
        log(f"[bench] bf16: blocked {lups / tb16 / 1e9:.1f}, naive {lups / tn16 / 1e9:.1f} GLUP/s")
        del coef16
        ctx_n.close()
        try:
            extras["adjoint"] = adjoint_leg(st, workloads, torch, np, stream, args)
        except Exception as e:  # the adjoint leg reports, it does not sink the line
            extras["adjoint"] = {"error": str(e)[:200]}
    ctx_b.close()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_leg(wl, args.cpu_seconds)

    line = {
        "metric": "GLUP/s (blocked 25pt var-coef 480^3, 100 steps) + HBM GB/s; blocked vs naive",
        "value": round(value, 2),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "kind": "25pt-var", "n": list(wl.n3), "halo": h, "nt": nt,
                   "scheme": "blocked", "dw": args.dw, "coef_dtype": "f32",
                   "seed": [workloads.SEED_BASE, 4]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


KERNEL_SOURCES = ["paper_1410_3060_amd/csrc/blocked.hip", "paper_1410_3060_amd/csrc/blocked.h",
                  "paper_1410_3060_amd/csrc/point_ops.h", "paper_1410_3060_amd/csrc/common.h",
                  "paper_1410_3060_amd/csrc/kernels.h"]


def measured_traffic(workload, dw):
    """HBM bytes per launch of the blocked kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since the
    counters were taken (or they were taken on another workload)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))["blocked_row_kernel"]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", KERNEL_SOURCES):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("source_sha256") or rec.get("workload") != workload or \
            rec.get("dw") != dw:
        return None
    return float(rec["hbm_bytes_per_launch"])


def copy_probe(torch, nbytes=1 << 32, reps=10):
    """Attainable HBM bandwidth: a plain device-to-device copy of 4 GiB (the
    analogue of the STREAM COPY figure b_S the paper's roofline uses).
    Counts read + write bytes.  Also the known-size kernel that calibrates
    rocprof's FETCH_SIZE / WRITE_SIZE counters."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return {"bytes_per_copy": 2 * nbytes, "GBps": round(2 * nbytes / sec / 1e9, 1),
            "ms": round(sec * 1e3, 3)}


def adjoint_leg(st, workloads, torch, np, stream, args):
    """Workload 5: forward (recording checkpoints) and adjoint, GLUP/s each."""
    wl = workloads.make(5)
    h, nt = wl.halo, wl.nt
    lups = wl.lups
    up = st.alloc_field(wl.n3, h)
    u0 = st.alloc_field(wl.n3, h)
    c = st.alloc_field(wl.n3, h, count=1)
    up.copy_(torch.from_numpy(wl.u_prev))
    u0.copy_(torch.from_numpy(wl.u0))
    c.copy_(torch.from_numpy(wl.coef))
    d = st.alloc_field(wl.n3, h)
    d.copy_(torch.from_numpy(wl.target))
    k = workloads.CKPT_EVERY
    out = {}
    for scheme, name in ((st.NAIVE, "naive"), (st.BLOCKED, "blocked")):
        ctx = st.Context(scheme, ckpt_every=k, stream=stream)
        a, b = st.field_like(up, h), st.field_like(u0, h)
        ts_f, ts_a = [], []
        for i in range(1 + max(1, args.steps // 2)):
            a.copy_(up)
            b.copy_(u0)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            slot = ctx.run(5, a, b, nt, halo=h, coef=c, w=st.L8_WEIGHTS)
            e1.record(stream)
            uT = (a, b)[slot]
            seed = st.alloc_field(wl.n3, h)
            seed.copy_(uT - d)
            g0 = st.alloc_field(wl.n3, h)
            gm1 = st.alloc_field(wl.n3, h)
            gc = st.alloc_field(wl.n3, h, dtype=torch.float64)
            torch.cuda.synchronize()
            e1b = torch.cuda.Event(enable_timing=True)
            e1b.record(stream)
            ctx.adjoint(up, u0, nt, halo=h, coef=c, w=st.L8_WEIGHTS, seed=seed, grad_u0=g0,
                        grad_um1=gm1, grad_c=gc)
            e2.record(stream)
            torch.cuda.synchronize()
            if i >= 1:
                ts_f.append(e0.elapsed_time(e1) / 1e3)
                ts_a.append(e1b.elapsed_time(e2) / 1e3)
        tf, ta = float(np.median(ts_f)), float(np.median(ts_a))
        out[name] = {"fwd_glups": round(lups / tf / 1e9, 2), "adj_glups": round(lups / ta / 1e9, 2),
                     "adj_over_fwd": round(tf / ta, 3)}
        ctx.close()
    out["workload"] = wl.name
    return out


def cpu_leg(wl, seconds):
    """The FP64 oracle on a bounded sample of the workload, on all host cores.

    The sample is the full seeded grid run for as many of the workload's time
    steps as fit in about `seconds` (one calibration step first); if a single
    step already takes longer, the leading planes of the grid instead."""
    import numpy as np

    import oracle
    h = wl.halo
    nx, ny, nz = wl.n3
    u = np.asarray(wl.u0, dtype=np.float64)
    cf = np.asarray(wl.coef, dtype=np.float64)
    t = []
    oracle.run(wl.kind, u, h, 1, coef=cf, timing=t)
    per_step = max(t[0], 1e-3)
    nz_s = nz
    if per_step > seconds / 4:
        nz_s = max(2 * h, int(nz * seconds / 4 / per_step))
        sl = slice(0, nz_s + 2 * h)
        u = np.ascontiguousarray(u[sl])
        cf = np.ascontiguousarray(cf[:, sl])
        per_step *= nz_s / nz
    nt_s = int(max(1, min(wl.nt, seconds / per_step)))
    t = []
    oracle.run(wl.kind, u, h, nt_s, coef=cf, timing=t)
    secs = t[0]
    glups = nx * ny * nz_s * nt_s / secs / 1e9
    return {"value": round(glups, 4), "unit": "GLUP/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{nx}x{ny}x{nz_s} of the same seeded grid, {nt_s} of {wl.nt} steps, FP64, "
                      f"{secs:.1f} s", "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
