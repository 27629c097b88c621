#!/usr/bin/env python3
"""Benchmark: GLUP/s of the temporally blocked stencil scheme on one MI355X.

Workload: the 25-point 8th-order variable-coefficient axis-symmetric stencil
(Fig. 1d of the paper), 480^3 interior, halo 4, 13 FP32 coefficient arrays,
100 time steps, seeded synthetic inputs.  One benchmark "step" is one complete
stencil_run of all 100 time steps with the blocked scheme (diamond rows in y,
wavefront in z; --scheme naive times the one-sweep-per-step scheme instead),
inputs resident in HBM.  value = lattice-site updates per second, counting
only the algorithmic 480^3 * 100 updates (never recomputed halos).

Beside it the other scheme is timed on the same run, both with BF16
coefficients; every other workload at full size with both schemes (7-point
constant 64^3 x 10, 25-point leapfrog 512^3 x 100, 7-point variable 512^3 x
100, leapfrog with c(x) 256^3 x 200), each with the error of its level nt
against the FP64 oracle over the whole interior (for the 25-point
variable-coefficient workload with BF16 coefficients: against the oracle on
the BF16-rounded values, and the storage error against the oracle on the
FP32 values); and the adjoints, forward (recording) and backward: the
leapfrog with c(x) (256^3, 200 steps; checkpoints every 14 steps and every
level) and the 7- and 25-point variable-coefficient Jacobi workloads (every
level recorded).  The FP64 CPU oracle is timed on the full 25-point
workload on the host cores (its result is the reference of the error above)
and on the 7-point constant workload in seconds, on all cores and on one.

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
    ap.add_argument("--scheme", choices=("blocked", "naive"), default="blocked",
                    help="scheme of the timed run (the other one is timed among the extras)")
    ap.add_argument("--workload", type=int, default=4, choices=(1, 2, 3, 4, 5),
                    help="workload of the timed run (4: 25-point variable coefficients, 480^3)")
    ap.add_argument("--dw", type=int, default=0, help="diamond width (0: the library's choice)")
    ap.add_argument("--no-extras", action="store_true", help="skip naive/BF16/adjoint legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--n", type=int, default=None, help="override the grid size (testing only)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line: grid-size sweep (cubes, multiples of 64) of "
                         "the naive and blocked schemes with every provided diamond width, and the "
                         "copy bandwidth by working set (one JSON line)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint legs (forward with checkpoints, then the adjoint)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the device-to-device copy probe and print its bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the multi-GPU path (y bands of "
              "whole diamonds per GPU) is not implemented.", file=sys.stderr)
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
    if args.sweep:
        print(json.dumps(sweep_leg(torch, args)), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(st, workloads, torch, np, stream, args),
                          "adjoint_jacobi": {workloads.NAMES[i]: jacobi_adjoint_leg(
                              st, workloads, torch, np, stream, i, args) for i in (3, 4)}}),
              flush=True)
        return

    t_gen = time.time()
    wl = workloads.make(args.workload, n=args.n)
    log(f"[bench] generated {wl.name} n={wl.n3} in {time.time() - t_gen:.1f}s")
    h, nt, kind = wl.halo, wl.nt, wl.kind
    nx, ny, nz = wl.n3
    lups = nx * ny * nz * nt
    leapfrog = kind in (4, 5)
    w = wl.w if kind == 1 else (st.L8_WEIGHTS if leapfrog else ())
    dw = args.dw or st.default_dw(kind, wl.n3)

    def upload(a):
        t = st.alloc_field(wl.n3, h)
        t.copy_(torch.from_numpy(a))
        return t

    def upload_coef(arr, dtype):
        if arr is None:
            return None
        t = st.alloc_field(wl.n3, h, count=arr.shape[0], dtype=dtype)
        src = torch.from_numpy(arr)
        t.copy_(src.view(torch.bfloat16) if dtype == torch.bfloat16 else src)
        return t

    coef32 = upload_coef(wl.coef, torch.float32)
    init_a = upload(wl.u_prev if leapfrog else wl.u0)
    init_b = upload(wl.u0 if leapfrog else np.zeros_like(wl.u0))
    u_a, u_b = st.field_like(init_a, h), st.field_like(init_b, h)

    def timed(ctx, coef, steps, warmup):
        """Run warmup + steps full runs; returns per-run seconds (HIP events on the stream)."""
        times = []
        for i in range(warmup + steps):
            u_a.copy_(init_a)
            u_b.copy_(init_b)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.run(kind, u_a, u_b, nt, halo=h, coef=coef, w=w, alpha=wl.alpha)
            e1.record(stream)
            torch.cuda.synchronize()
            if i >= warmup:
                times.append(e0.elapsed_time(e1) / 1e3)
        return times

    blocked = args.scheme == "blocked"
    if blocked:
        n_launch = len(st.plan_rows(kind, dw, ny, nt))
        bpl = model.blocked_bytes_per_lup(kind, dw)
        H = dw // (2 * model.RADIUS[kind])
        if model.RADIUS[kind] == 4:
            # multi-workgroup diamonds (one launch per diamond row)
            kname = "mwd_row_kernel<%d, float, H=%d>" % (kind, H)
            tkey = "mwd_row_kernel"
        else:
            kname = "blocked_row_kernel<%d, float, H=%d>" % (kind, H)
            tkey = "blocked_row_kernel"
    else:
        n_launch = nt
        bpl = model.naive_code_balance(kind)
        kname = "naive_step_kernel<%d, float>" % kind
        tkey = "naive_step_kernel"
    log(f"[bench] {args.scheme}: {n_launch} kernel launches per run")
    ctx_b = st.Context(st.BLOCKED, dw=dw, stream=stream)
    ctx_n = st.Context(st.NAIVE, stream=stream)
    tb = timed(ctx_b if blocked else ctx_n, coef32, args.steps, args.warmup)
    t_step = float(np.median(tb))
    value = lups / t_step / 1e9
    log(f"[bench] {args.scheme}: {t_step * 1e3:.2f} ms per run, {value:.1f} GLUP/s")

    # average launch duration of the dominant kernel from the same HIP events
    # (launch gaps and the few small copies of a run included)
    avg_launch = t_step / n_launch
    achieved = bpl * lups / n_launch / avg_launch / 1e9
    traffic = measured_traffic(tkey, wl.name, dw if blocked else 0)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 3),
                "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                "algorithmic_per_launch_GB": round(bpl * lups / n_launch / 1e9, 3),
                "copy_probe_GBps": probe["GBps"], "kernel": kname,
                "bytes_per_lup": round(bpl, 3), "avg_launch_ms": round(avg_launch * 1e3, 4)}
    if traffic is not None:
        # the rate of the bytes the counters saw (L2 misses), beside the
        # algorithmic rate that `achieved` reports
        roofline["traffic_GBps"] = round(traffic / avg_launch / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / avg_launch / 1e9 / PEAK_HBM_GBS, 4)

    extras = {}
    if not args.no_extras:
        other = max(2, args.steps // 2)
        tn_s = t_step if not blocked else float(np.median(timed(ctx_n, coef32, other, 1)))
        tb_s = t_step if blocked else float(np.median(timed(ctx_b, coef32, other, 1)))
        for name, t, b in (("naive", tn_s, model.naive_code_balance(kind)),
                           ("blocked", tb_s, model.blocked_bytes_per_lup(kind, dw))):
            extras[name] = {"glups": round(lups / t / 1e9, 2), "ms_per_run": round(t * 1e3, 3),
                            "bytes_per_lup": round(b, 3),
                            "algorithmic_GBps": round(b * lups / t / 1e9, 1)}
        extras["blocked_over_naive"] = round(tn_s / tb_s, 3)
        log(f"[bench] naive {extras['naive']['glups']}, blocked {extras['blocked']['glups']} GLUP/s")
        # level nt of both schemes (FP32 coefficients), for the error legs
        fin = {}
        for name, cx in (("naive", ctx_n), ("blocked", ctx_b)):
            u_a.copy_(init_a)
            u_b.copy_(init_b)
            slot = cx.run(kind, u_a, u_b, nt, halo=h, coef=coef32, w=w, alpha=wl.alpha)
            fin[name] = (u_a, u_b)[slot].cpu().numpy()
        extras["blocked_equals_naive"] = bool(np.array_equal(fin["naive"], fin["blocked"]))
        gpu_final = {"f32": fin["blocked"]}
        del fin
        if wl.coef is not None:
            # BF16 coefficient storage
            coef16 = upload_coef(workloads.to_bf16_bits(wl.coef).view(np.int16), torch.bfloat16)
            tb16 = float(np.median(timed(ctx_b, coef16, other, 1)))
            tn16 = float(np.median(timed(ctx_n, coef16, other, 1)))
            extras["bf16"] = {"blocked_glups": round(lups / tb16 / 1e9, 2),
                              "naive_glups": round(lups / tn16 / 1e9, 2),
                              "blocked_over_naive": round(tn16 / tb16, 3)}
            log(f"[bench] bf16: blocked {lups / tb16 / 1e9:.1f}, naive {lups / tn16 / 1e9:.1f} GLUP/s")
            fin = {}
            for name, cx in (("naive", ctx_n), ("blocked", ctx_b)):
                u_a.copy_(init_a)
                u_b.copy_(init_b)
                slot = cx.run(kind, u_a, u_b, nt, halo=h, coef=coef16, w=w, alpha=wl.alpha)
                fin[name] = (u_a, u_b)[slot].cpu().numpy()
            extras["bf16"]["blocked_equals_naive"] = bool(np.array_equal(fin["naive"],
                                                                         fin["blocked"]))
            gpu_final["bf16"] = fin["blocked"]
            del coef16, fin
        if args.n is None:
            configs = {}
            for i in (1, 2, 3, 5):
                if i == args.workload:
                    continue
                try:
                    configs[workloads.NAMES[i]] = config_leg(st, workloads, model, torch, np,
                                                             stream, i, args.cpu_seconds)
                except Exception as e:  # a failing leg reports, it does not sink the line
                    configs[workloads.NAMES[i]] = {"error": str(e)[:200]}
            extras["configs"] = configs
        try:
            extras["adjoint"] = adjoint_leg(st, workloads, torch, np, stream, args)
        except Exception as e:  # the adjoint legs report, they do not sink the line
            extras["adjoint"] = {"error": str(e)[:200]}
        for i in (3, 4):
            try:
                extras.setdefault("adjoint_jacobi", {})[workloads.NAMES[i]] = \
                    jacobi_adjoint_leg(st, workloads, torch, np, stream, i, args)
            except Exception as e:
                extras.setdefault("adjoint_jacobi", {})[workloads.NAMES[i]] = \
                    {"error": str(e)[:200]}
    ctx_b.close()
    ctx_n.close()

    cpu = None
    ref = None
    if not args.no_cpu:
        cpu, ref = cpu_leg(wl, args.cpu_seconds)
        if args.n is None and not args.no_extras:
            extras["c1_oracle_seconds"] = c1_oracle_seconds(workloads)
    if not args.no_extras and args.n is None:
        # error of level nt against the FP64 oracle over the whole interior
        err = {}
        for name, c in extras.get("configs", {}).items():
            if "error_vs_oracle" in c:
                err[name] = c["error_vs_oracle"]
        err[wl.name] = error_stats(np, gpu_final["f32"], ref if ref is not None else
                                   oracle_final(np, wl, wl.coef), h)
        if "bf16" in gpu_final:
            rounded = workloads.bf16_bits_to_f32(workloads.to_bf16_bits(wl.coef))
            parity = error_stats(np, gpu_final["bf16"], oracle_final(np, wl, rounded), h)
            del rounded
            storage = error_stats(np, gpu_final["bf16"], ref if ref is not None else
                                  oracle_final(np, wl, wl.coef), h)
            err[wl.name + "-bf16"] = {
                "vs_oracle_on_bf16_values": parity,
                "storage_error_vs_oracle_on_f32_values": storage,
                "storage_target_rel_l2": 1e-3,
                "storage_target_met": storage["rel_l2"] <= 1e-3}
        extras["error"] = err
        log("[bench] error vs FP64 oracle: " + json.dumps(err))

    line = {
        "metric": "GLUP/s (%s) + HBM GB/s; blocked vs naive" % wl.name,
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
        "config": {"workload": wl.name, "kind": kind, "n": list(wl.n3), "halo": h, "nt": nt,
                   "scheme": args.scheme, "dw": dw if blocked else None, "coef_dtype": "f32",
                   "seed": [workloads.SEED_BASE, args.workload]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


def measured_traffic(key, workload, dw):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None when the kernel's sources changed since the counters were
    taken (or they were taken on another workload)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[f"{key}@{workload}"]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("source_sha256") or rec.get("dw", 0) != dw:
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


def timed_pair(torch, stream, first, second):
    """HIP-event seconds of first() and of second(), with a sync in between."""
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    e0.record(stream)
    first()
    e1.record(stream)
    torch.cuda.synchronize()
    e2.record(stream)
    second()
    e3.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, e2.elapsed_time(e3) / 1e3


def adjoint_leg(st, workloads, torch, np, stream, args):
    """Workload 5: plain forward, then forward (recording) and adjoint with
    checkpoints every 14 steps (naive and blocked forward) and with every
    level recorded; GLUP/s each."""
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
    reps = max(1, args.steps // 2)
    a, b = st.field_like(up, h), st.field_like(u0, h)
    seed = st.alloc_field(wl.n3, h)
    g0 = st.alloc_field(wl.n3, h)
    gm1 = st.alloc_field(wl.n3, h)
    gc = st.alloc_field(wl.n3, h, dtype=torch.float64)
    out = {"workload": wl.name}
    ctx0 = st.Context(st.NAIVE, stream=stream)
    ts = []
    for i in range(1 + reps):
        a.copy_(up)
        b.copy_(u0)
        t, _ = timed_pair(torch, stream, lambda: ctx0.run(5, a, b, nt, halo=h, coef=c,
                                                          w=st.L8_WEIGHTS), lambda: None)
        ts.append(t)
    ctx0.close()
    tp = float(np.median(ts[1:]))
    out["plain_fwd_glups"] = round(lups / tp / 1e9, 2)
    for scheme, k, name in ((st.NAIVE, workloads.CKPT_EVERY, "naive_ckpt14"),
                            (st.BLOCKED, workloads.CKPT_EVERY, "blocked_ckpt14"),
                            (st.NAIVE, 1, "every_level")):
        ctx = st.Context(scheme, ckpt_every=k, stream=stream)
        ts_f, ts_a = [], []
        for i in range(1 + reps):
            a.copy_(up)
            b.copy_(u0)
            slot = [0]

            def fwd():
                slot[0] = ctx.run(5, a, b, nt, halo=h, coef=c, w=st.L8_WEIGHTS)
                seed.copy_((a, b)[slot[0]] - d)

            tf, ta = timed_pair(torch, stream, fwd, lambda: ctx.adjoint(
                up, u0, nt, halo=h, coef=c, w=st.L8_WEIGHTS, seed=seed, grad_u0=g0,
                grad_um1=gm1, grad_c=gc))
            if i >= 1:
                ts_f.append(tf)
                ts_a.append(ta)
        ctx.close()
        tf, ta = float(np.median(ts_f)), float(np.median(ts_a))
        out[name] = {"ckpt_every": k, "fwd_glups": round(lups / tf / 1e9, 2),
                     "adj_glups": round(lups / ta / 1e9, 2),
                     "adj_over_plain_fwd": round(tp / ta, 3)}
    log(f"[bench] leapfrog adjoint: every level {out['every_level']['adj_glups']} GLUP/s "
        f"({out['every_level']['adj_over_plain_fwd']} of the plain forward)")
    return out


def jacobi_adjoint_leg(st, workloads, torch, np, stream, index, args):
    """Workload 3 (7-point) or 4 (25-point variable coefficients): plain
    forward, forward recording every level, and the adjoint with the
    gradients of all K coefficient arrays; GLUP/s each."""
    wl = workloads.make(index)
    h, nt, kind = wl.halo, wl.nt, wl.kind
    lups = wl.lups
    K = wl.coef.shape[0]
    u0 = st.alloc_field(wl.n3, h)
    u0.copy_(torch.from_numpy(wl.u0))
    cf = st.alloc_field(wl.n3, h, count=K)
    cf.copy_(torch.from_numpy(wl.coef))
    wl.coef = None
    a, b = st.field_like(u0, h), st.field_like(u0, h)
    seed = st.alloc_field(wl.n3, h)
    gen = torch.Generator(device=seed.device)
    gen.manual_seed(1410 + index)
    seed[h:-h, h:-h, h:-h].uniform_(-1, 1, generator=gen)
    g0 = st.alloc_field(wl.n3, h)
    gc = st.alloc_field(wl.n3, h, count=K, dtype=torch.float64)
    reps = max(1, args.steps // 2)
    out = {"workload": wl.name, "ckpt_every": 1}
    ctx0 = st.Context(st.NAIVE, stream=stream)
    ctx = st.Context(st.NAIVE, ckpt_every=1, stream=stream)
    tp, tf, ta = [], [], []
    for i in range(1 + reps):
        a.copy_(u0)
        b.copy_(u0)
        t, _ = timed_pair(torch, stream, lambda: ctx0.run(kind, a, b, nt, halo=h, coef=cf),
                          lambda: None)
        a.copy_(u0)
        b.copy_(u0)
        f, g = timed_pair(torch, stream, lambda: ctx.run(kind, a, b, nt, halo=h, coef=cf),
                          lambda: ctx.adjoint_jacobi(kind, a, b, nt, halo=h, coef=cf, seed=seed,
                                                     grad_u0=g0, grad_c=gc))
        if i >= 1:
            tp.append(t)
            tf.append(f)
            ta.append(g)
    ctx.close()
    ctx0.close()
    tp, tf, ta = (float(np.median(x)) for x in (tp, tf, ta))
    out.update({"plain_fwd_glups": round(lups / tp / 1e9, 2),
                "rec_fwd_glups": round(lups / tf / 1e9, 2),
                "adj_glups": round(lups / ta / 1e9, 2),
                "adj_over_plain_fwd": round(tp / ta, 3)})
    log(f"[bench] {wl.name} adjoint: {out['adj_glups']} GLUP/s ({out['adj_over_plain_fwd']} of "
        f"the plain forward)")
    return out


def sweep_leg(torch, args):
    """Copy bandwidth by working set (the in-cache and HBM roofs), then for the
    7-point constant, 7-point and 25-point variable-coefficient stencils at
    cubes of 64 .. 512 (100 steps) the GLUP/s of the naive sweep and of the
    blocked scheme at every provided diamond width."""
    from paper_1410_3060_amd import model, tune
    out = {"roofs": tune.memory_roofs()}
    log("[sweep] copy roofs " + ", ".join(f"{r['working_set_MiB']} MiB {r['GBps']:.0f} GB/s"
                                          for r in out["roofs"]))
    rows = []
    nt = 100
    for kind in (1, 2, 3):
        for n in range(64, 513, 64):
            r = tune.autotune(kind, (n, n, n), nt, reps=1)
            naive = next(x for x in r["results"] if x["scheme"] == "naive")
            blk = {str(x["dw"]): round(x["glups"], 2) for x in r["results"] if x["scheme"] == "blocked"}
            bpl = model.naive_code_balance(kind)
            # bytes the naive sweep touches per step: fields and coefficients
            ws = (2 + model.NCOEF[kind]) * (n + 2 * model.RADIUS[kind]) ** 3 * 4 / 2 ** 20
            row = {"kind": kind, "n": n, "nt": nt, "working_set_MiB": round(ws, 1),
                   "naive_glups": round(naive["glups"], 2),
                   "naive_alg_GBps": round(naive["glups"] * bpl, 1),
                   "blocked_glups_by_dw": blk,
                   "best": {"scheme": r["best"]["scheme"], "dw": r["best"]["dw"],
                            "glups": round(r["best"]["glups"], 2)}}
            rows.append(row)
            log(f"[sweep] kind {kind} {n}^3: naive {row['naive_glups']}, blocked {blk}")
    out["rows"] = rows
    return out


def error_stats(np, got, want, h):
    """rel-L2 and max-norm error of a level against the oracle's, interior only."""
    g = got[h:-h, h:-h, h:-h].astype(np.float64)
    w = want[h:-h, h:-h, h:-h]
    d = g - w
    return {"rel_l2": float(np.linalg.norm(d.ravel()) / np.linalg.norm(w.ravel())),
            "max_rel": float(np.abs(d).max() / np.abs(w).max())}


def oracle_final(np, wl, coef):
    """The FP64 oracle's level nt of the workload with the given coefficient values."""
    import oracle
    h = wl.halo
    w = wl.w if wl.kind == 1 else (oracle.l8_weights_3d() if wl.kind in (4, 5) else ())
    cf = None if coef is None else np.asarray(coef, dtype=np.float64)
    if wl.kind in (4, 5):
        return oracle.run(wl.kind, wl.u0.astype(np.float64), h, wl.nt,
                          u_prev=wl.u_prev.astype(np.float64), coef=cf, w=w, alpha=wl.alpha)[1]
    return oracle.run(wl.kind, wl.u0.astype(np.float64), h, wl.nt, coef=cf, w=w)


def config_leg(st, workloads, model, torch, np, stream, index, cpu_seconds, reps=3):
    """One workload at full size: naive and blocked GLUP/s (default diamond
    width), whether blocked equals naive bit for bit, and the error of level
    nt against the FP64 oracle over the whole interior."""
    wl = workloads.make(index)
    h, kind, nt = wl.halo, wl.kind, wl.nt
    lf = kind in (4, 5)
    w = wl.w if kind == 1 else (st.L8_WEIGHTS if lf else ())
    a0 = st.alloc_field(wl.n3, h)
    a0.copy_(torch.from_numpy(wl.u_prev if lf else wl.u0))
    b0 = st.alloc_field(wl.n3, h)
    b0.copy_(torch.from_numpy(wl.u0 if lf else np.zeros_like(wl.u0)))
    cf = None
    if wl.coef is not None:
        cf = st.alloc_field(wl.n3, h, count=wl.coef.shape[0])
        cf.copy_(torch.from_numpy(wl.coef))
    a, b = st.field_like(a0, h), st.field_like(b0, h)
    dw = st.default_dw(kind, wl.n3)
    out = {"workload": wl.name, "dw": dw}
    fin = {}
    for scheme, name in ((st.NAIVE, "naive"), (st.BLOCKED, "blocked")):
        ctx = st.Context(scheme, stream=stream)
        ts = []
        for i in range(reps + 1):
            a.copy_(a0)
            b.copy_(b0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            slot = ctx.run(kind, a, b, nt, halo=h, coef=cf, w=w, alpha=wl.alpha)
            e1.record(stream)
            torch.cuda.synchronize()
            if i:
                ts.append(e0.elapsed_time(e1) / 1e3)
        ctx.close()
        t = float(np.median(ts))
        fin[name] = (a, b)[slot].cpu().numpy()
        bpl = model.naive_code_balance(kind) if scheme == st.NAIVE else \
            model.blocked_bytes_per_lup(kind, dw)
        out[name] = {"glups": round(wl.lups / t / 1e9, 2), "ms_per_run": round(t * 1e3, 3),
                     "bytes_per_lup": round(bpl, 3),
                     "algorithmic_GBps": round(bpl * wl.lups / t / 1e9, 1)}
    out["blocked_over_naive"] = round(out["blocked"]["glups"] / out["naive"]["glups"], 3)
    out["blocked_equals_naive"] = bool(np.array_equal(fin["naive"], fin["blocked"]))
    del a, b, a0, b0, cf
    torch.cuda.empty_cache()
    out["error_vs_oracle"] = error_stats(np, fin["blocked"], oracle_final(np, wl, wl.coef), h)
    log(f"[bench] {wl.name}: naive {out['naive']['glups']}, blocked {out['blocked']['glups']} "
        f"GLUP/s; error {out['error_vs_oracle']}")
    return out


def c1_oracle_seconds(workloads):
    """Seconds of the FP64 oracle on the 7-point constant workload (64^3, 10
    steps), time-step loop only: on all host cores and on one thread."""
    import numpy as np

    import oracle
    wl = workloads.make(1)
    out = {"workload": wl.name}
    for key, nth in (("all_cores", 0), ("one_thread", 1)):
        best = None
        for _ in range(3):
            t = []
            oracle.run(1, wl.u0.astype(np.float64), wl.halo, wl.nt, w=wl.w, nthreads=nth,
                       timing=t)
            best = t[0] if best is None else min(best, t[0])
        out[key] = {"seconds": round(best, 5),
                    "threads": oracle.max_threads() if nth == 0 else 1}
    return out


def cpu_leg(wl, seconds):
    """The FP64 oracle on a bounded sample of the workload, on all host cores.

    The sample is the full seeded grid run for as many of the workload's time
    steps as fit in about `seconds` (one calibration step first); if a single
    step already takes longer, the leading planes of the grid instead.
    Returns the record and, when the sample was the whole run, the oracle's
    level nt (else None)."""
    import numpy as np

    import oracle
    h = wl.halo
    nx, ny, nz = wl.n3
    lf = wl.kind in (4, 5)
    w = wl.w if wl.kind == 1 else (oracle.l8_weights_3d() if lf else ())
    u = np.asarray(wl.u0, dtype=np.float64)
    up = np.asarray(wl.u_prev, dtype=np.float64) if lf else None
    cf = None if wl.coef is None else np.asarray(wl.coef, dtype=np.float64)

    def run(nsteps, t):
        r = oracle.run(wl.kind, u, h, nsteps, u_prev=up, coef=cf, w=w, alpha=wl.alpha, timing=t)
        return r[1] if lf else r

    t = []
    run(1, t)
    per_step = max(t[0], 1e-3)
    nz_s = nz
    if per_step > seconds / 4:
        nz_s = max(2 * h, int(nz * seconds / 4 / per_step))
        sl = slice(0, nz_s + 2 * h)
        u = np.ascontiguousarray(u[sl])
        up = None if up is None else np.ascontiguousarray(up[sl])
        cf = None if cf is None else np.ascontiguousarray(cf[:, sl])
        per_step *= nz_s / nz
    nt_s = int(max(1, min(wl.nt, seconds / per_step)))
    t = []
    res = run(nt_s, t)
    secs = t[0]
    glups = nx * ny * nz_s * nt_s / secs / 1e9
    full = nz_s == nz and nt_s == wl.nt
    return ({"value": round(glups, 4), "unit": "GLUP/s", "cores": oracle.max_threads(),
             "kind": "oracle",
             "sample": f"{nx}x{ny}x{nz_s} of the same seeded grid, {nt_s} of {wl.nt} steps, FP64, "
                       f"{secs:.1f} s", "host_cpus": os.cpu_count()},
            res if full else None)


if __name__ == "__main__":
    main()
