"""The allocation-free entry point (stencil_run_noalloc) against stencil_run.

Two calls in a row on one GPU, the second with a smaller grid, each compared
bit for bit with stencil_run of the blocked scheme on the same inputs: the
scratch array keeps the first call's contents, so the second shows that
nothing stale is read.  Every kind, through the C ABI.
"""
import numpy as np
import pytest

import paper_1410_3060_amd as st
import workloads

from gpu_util import coef_to_dev, gpu_weights, to_dev

pytestmark = pytest.mark.gpu

INDEX = {1: 1, 2: 3, 3: 4, 4: 2, 5: 5}


def run_both(index, n3, nt, coef_dtype="f32"):
    import torch
    wl = workloads.make(index, n=n3, nt=nt, coef_dtype=coef_dtype)
    h = wl.halo
    lf = wl.kind in (4, 5)
    first = wl.u_prev if lf else wl.u0
    second = wl.u0 if lf else np.zeros_like(wl.u0)
    cf = coef_to_dev(wl)
    out = []
    for noalloc in (False, True):
        a, b = to_dev(first, h), to_dev(second, h)
        with st.Context(st.BLOCKED) as ctx:
            fn = ctx.run_noalloc if noalloc else ctx.run
            slot = fn(wl.kind, a, b, nt, halo=h, coef=cf, w=gpu_weights(wl), alpha=wl.alpha)
            ctx.sync()
        torch.cuda.synchronize()
        out.append((slot, a.cpu().numpy(), b.cpu().numpy()))
    return out


@pytest.mark.parametrize("kind", [1, 2, 3, 4, 5])
def test_noalloc_equals_run_twice_second_smaller(kind):
    idx = INDEX[kind]
    for n3, nt in (((70, 45, 33), 9), ((37, 22, 19), 5)):
        print(f"noalloc kind {kind} n={n3} nt={nt}", flush=True)
        (s0, a0, b0), (s1, a1, b1) = run_both(idx, n3, nt)
        assert s0 == s1
        assert np.array_equal(a0, a1) and np.array_equal(b0, b1), (kind, n3)


def test_noalloc_bf16_coefficients():
    (s0, a0, b0), (s1, a1, b1) = run_both(4, (66, 40, 25), 7, coef_dtype="bf16")
    assert s0 == s1 and np.array_equal(a0, a1) and np.array_equal(b0, b1)
