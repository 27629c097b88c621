"""Measured choice of the scheme and the diamond width for one problem size.

The paper auto-tunes the diamond width and the number of wavefront
frontlines, searching only tiles whose cache block (Sect. 5.3) fits a cache
size range (Sect. 5.1).  On MI355X the on-chip block of each diamond width is
fixed by the compiled kernel configurations, so the choice left is which
scheme to run and, for the blocked one, which of the provided widths;
``autotune`` times every candidate through the library on synthetic inputs of
the caller's sizes and returns the fastest.  Only the library runs here:
nothing in this module computes stencil values.

``memory_roofs`` measures the attainable bandwidth of a plain device copy as a
function of its working set: the in-cache roofs (L2, Infinity Cache) and the
HBM roof that bound the naive sweep's GLUP/s at each grid size.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional

from . import (BLOCKED, blocked_slices, KIND_25PT_WAVE, KIND_7PT_CONST, L8_WEIGHTS, LEAPFROG, NAIVE, NCOEF,
               RADIUS, Context, alloc_field, default_dw, field_like)

# diamond widths the blocked kernel is compiled for, per stencil radius
PROVIDED_DW = {1: (4, 6, 8, 10, 12), 2: (4, 6, 8, 10, 12), 3: (16, 24), 4: (16, 24, 32),
               5: (16, 24, 32)}


def _inputs(kind, n3, h, coef_dtype, seed):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    a = alloc_field(n3, h)
    inner = (slice(h, -h),) * 3
    a[inner].uniform_(-1.0, 1.0, generator=gen)
    b = alloc_field(n3, h)
    if kind in LEAPFROG:
        b.copy_(a)
    K = NCOEF[kind]
    cf = None
    if K:
        dt = torch.bfloat16 if coef_dtype == "bf16" else torch.float32
        cf = alloc_field(n3, h, count=K, dtype=dt)
        # bounded, stable values: row sums below one (Jacobi) or a small c(x)
        scale = 0.05 if kind in LEAPFROG else 0.99 / (K if kind == 2 else 2 * K)
        tmp = torch.empty(cf.shape, device="cuda").uniform_(0.0, scale, generator=gen)
        cf.copy_(tmp.to(dt))
        del tmp
    return a, b, cf


def _weights(kind):
    if kind == KIND_7PT_CONST:
        return (0.4, 0.1), 0.0
    if kind in LEAPFROG:
        return L8_WEIGHTS, (0.1 if kind == KIND_25PT_WAVE else 0.0)
    return (), 0.0


def time_run(kind, scheme, n3, nt, *, dw=0, halo=None, coef_dtype="f32", reps=2, seed=1410,
             inputs=None, xtile=0) -> float:
    """Median seconds of one complete ``nt``-step run (after one warm-up run),
    HIP events on the current stream."""
    import torch
    h = halo or RADIUS[kind]
    a0, b0, cf = inputs if inputs is not None else _inputs(kind, n3, h, coef_dtype, seed)
    a, b = field_like(a0, h), field_like(b0, h)
    w, alpha = _weights(kind)
    stream = torch.cuda.current_stream()
    ts: List[float] = []
    with Context(scheme, dw=dw, xtile=xtile, stream=stream) as ctx:
        for i in range(reps + 1):
            a.copy_(a0)
            b.copy_(b0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.run(kind, a, b, nt, halo=h, coef=cf, w=w, alpha=alpha)
            e1.record(stream)
            torch.cuda.synchronize()
            if i:
                ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def autotune(kind: int, n3, nt: int, *, halo: Optional[int] = None, coef_dtype: str = "f32",
             reps: int = 2, dws: Optional[Iterable[int]] = None, seed: int = 1410,
             xtiles: Iterable[int] = (0,)) -> Dict:
    """Time the naive sweep and the blocked scheme at every provided diamond
    width (or ``dws``) and, for the radius-4 kinds, every slice width in
    ``xtiles`` (0 = the library's choice; 16 and 32 set the workgroups per
    diamond, ``blocked_slices``) for this kind, size and step count; returns
    ``{"best": {...}, "results": [...]}`` with GLUP/s per candidate.  Pass the
    best ``dw`` and ``xtile`` to ``Context(BLOCKED, dw=..., xtile=...)``."""
    h = halo or RADIUS[kind]
    nx, ny, nz = n3
    lups = nx * ny * nz * nt
    inputs = _inputs(kind, n3, h, coef_dtype, seed)
    xts = list(xtiles) if RADIUS[kind] == 4 else [0]
    cands = [(NAIVE, 0, 0)] + [(BLOCKED, d, x) for d in (dws or PROVIDED_DW[kind]) for x in xts
                               if blocked_slices(kind, d, x, nx) > 0]
    results = []
    for scheme, d, x in cands:
        t = time_run(kind, scheme, n3, nt, dw=d, halo=h, reps=reps, inputs=inputs, xtile=x)
        results.append({"scheme": "naive" if scheme == NAIVE else "blocked",
                        "dw": d if scheme == BLOCKED else None,
                        "xtile": x if scheme == BLOCKED else None,
                        "workgroups_per_diamond": blocked_slices(kind, d, x, nx)
                        if scheme == BLOCKED else None,
                        "seconds": t, "glups": lups / t / 1e9})
    best = max(results, key=lambda r: r["glups"])
    return {"kind": kind, "n": list(n3), "nt": nt, "coef_dtype": coef_dtype,
            "library_default_dw": default_dw(kind, n3, coef_dtype), "best": best, "results": results}


def memory_roofs(sizes_mib: Iterable[float] = (2, 8, 32, 64, 128, 256, 512, 1024, 4096),
                 reps: int = 20) -> List[Dict]:
    """GB/s (read + write bytes) of a device-to-device copy whose source and
    destination together span each working set; small sets stay in L2 or the
    Infinity Cache across repetitions, large ones stream from HBM."""
    import torch
    out = []
    for mib in sizes_mib:
        n = max(1, int(mib * 2 ** 20 / 8))  # two float32 buffers of n elements
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        out.append({"working_set_MiB": mib, "GBps": 8 * n / sec / 1e9})
        del a, b
    return out
