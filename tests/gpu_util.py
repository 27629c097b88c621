"""Helpers for the GPU tests: move seeded workloads to the device, run the
library through its C ABI, and run the oracle on the very same stored values."""
from __future__ import annotations

import numpy as np

import oracle
import paper_1410_3060_amd as st
import workloads


def torch():
    import torch as _t
    return _t


def to_dev(a: np.ndarray, h: int, aligned: bool = True):
    """Padded float32 numpy field -> CUDA tensor view (aligned layout or contiguous)."""
    T = torch()
    pz, py, px = a.shape
    n3 = (px - 2 * h, py - 2 * h, pz - 2 * h)
    if aligned:
        t = st.alloc_field(n3, h)
        t.copy_(T.from_numpy(np.ascontiguousarray(a, dtype=np.float32)))
        return t
    return T.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def coef_to_dev(wl: workloads.Workload, aligned: bool = True):
    T = torch()
    if wl.coef is None:
        return None
    K = wl.coef.shape[0]
    h = wl.halo
    if wl.coef_bf16 is not None:
        host = T.from_numpy(np.ascontiguousarray(wl.coef_bf16).view(np.int16)).view(T.bfloat16)
        dt = T.bfloat16
    else:
        host = T.from_numpy(np.ascontiguousarray(wl.coef))
        dt = T.float32
    if aligned:
        t = st.alloc_field(wl.n3, h, count=K, dtype=dt)
        t.copy_(host)
        return t
    return host.cuda()


def from_dev(t) -> np.ndarray:
    return t.detach().cpu().contiguous().numpy().astype(np.float64)


def gpu_weights(wl):
    if wl.kind == 1:
        return wl.w
    if wl.kind in (4, 5):
        return st.L8_WEIGHTS
    return ()


def oracle_weights(wl):
    if wl.kind == 1:
        return wl.w
    if wl.kind in (4, 5):
        return oracle.l8_weights_3d()
    return ()


def run_gpu(wl, scheme=st.NAIVE, nt=None, aligned=True, **ctx_kw):
    """Run the library on the workload; returns (level nt, level nt-1 or None) as float64."""
    T = torch()
    nt = wl.nt if nt is None else nt
    h = wl.halo
    if wl.kind in (4, 5):
        a = to_dev(wl.u_prev, h, aligned)
        b = to_dev(wl.u0, h, aligned)
    else:
        a = to_dev(wl.u0, h, aligned)
        b = to_dev(np.zeros_like(wl.u0), h, aligned)  # same (zero) boundary shell
    cf = coef_to_dev(wl, aligned)
    with st.Context(scheme, **ctx_kw) as ctx:
        slot = ctx.run(wl.kind, a, b, nt, halo=h, coef=cf, w=gpu_weights(wl), alpha=wl.alpha)
        ctx.sync()
    T.cuda.synchronize()
    bufs = (a, b)
    last = from_dev(bufs[slot])
    other = from_dev(bufs[1 - slot]) if wl.kind in (4, 5) else None
    return last, other


def run_oracle(wl, nt=None, coef_override=None):
    """FP64 oracle on the stored (FP32 or BF16-rounded) inputs."""
    nt = wl.nt if nt is None else nt
    cf = None
    if wl.coef is not None:
        cf = wl.coef_values_f32() if coef_override is None else coef_override
        cf = cf.astype(np.float64)
    if wl.kind in (4, 5):
        up, u = oracle.run(wl.kind, wl.u0.astype(np.float64), wl.halo, nt,
                           u_prev=wl.u_prev.astype(np.float64), coef=cf, w=oracle_weights(wl),
                           alpha=wl.alpha)
        return u, up
    return oracle.run(wl.kind, wl.u0.astype(np.float64), wl.halo, nt, coef=cf,
                      w=oracle_weights(wl)), None


def rel_l2(got, want, h):
    g = oracle.interior(got, h)
    w = oracle.interior(want, h)
    return float(np.linalg.norm((g - w).ravel()) / max(np.linalg.norm(w.ravel()), 1e-300))


def max_rel(got, want, h):
    g = oracle.interior(got, h)
    w = oracle.interior(want, h)
    return float(np.abs(g - w).max() / max(np.abs(w).max(), 1e-300))
