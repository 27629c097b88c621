"""GPU adjoint of the leapfrog with c(x) (workload 5) against the FP64 oracle.

* gradients (dJ/du_{-1}, dJ/du_0, dJ/dc) element by element against the
  oracle adjoint run on the same stored inputs, at sizes spanning several
  tiles with ragged tails;
* the checkpoint interval only changes the schedule: every interval, with or
  without a forward recording, naive or blocked forward, gives bit-identical
  gradients for u_{-1} and u_0 (the recomputation reproduces the forward bit
  for bit) and FP64 coefficient gradients that differ only in the grouping of
  their additions;
* the torch.autograd binding returns the same gradients;
* nt = 0 and nt = 1 edge cases.
"""
import numpy as np
import pytest

import oracle
import paper_1410_3060_amd as st
import workloads

from gpu_util import from_dev, to_dev

pytestmark = pytest.mark.gpu

N3 = (70, 37, 29)


def grads_gpu(wl, nt, scheme=st.NAIVE, k=0, record=True):
    import torch
    h = wl.halo
    up = to_dev(wl.u_prev, h)
    u0 = to_dev(wl.u0, h)
    c = st.alloc_field(wl.n3, h, count=1)
    c.copy_(torch.from_numpy(wl.coef))
    d = to_dev(wl.target, h)
    a, b = st.field_like(up, h), st.field_like(u0, h)
    with st.Context(scheme, ckpt_every=(k if record else 0)) as ctx:
        slot = ctx.run(5, a, b, nt, halo=h, coef=c, w=st.L8_WEIGHTS)
        ctx.sync()
        seed = st.alloc_field(wl.n3, h)
        seed.copy_((a, b)[slot] - d)
        g0 = st.alloc_field(wl.n3, h)
        gm1 = st.alloc_field(wl.n3, h)
        gc = st.alloc_field(wl.n3, h, dtype=torch.float64)
        if not record:
            # no recording in this context: the adjoint recomputes from (up, u0)
            ctx2 = st.Context(scheme, ckpt_every=k)
            ctx2.adjoint(up, u0, nt, halo=h, coef=c, w=st.L8_WEIGHTS, seed=seed, grad_u0=g0,
                         grad_um1=gm1, grad_c=gc)
            ctx2.sync()
            ctx2.close()
        else:
            ctx.adjoint(up, u0, nt, halo=h, coef=c, w=st.L8_WEIGHTS, seed=seed, grad_u0=g0,
                        grad_um1=gm1, grad_c=gc)
            ctx.sync()
    torch.cuda.synchronize()
    return (from_dev(gm1), from_dev(g0), gc.cpu().contiguous().numpy(),
            from_dev(seed))


def grads_oracle(wl, nt, seed):
    h = wl.halo
    c = wl.coef[0].astype(np.float64)
    return oracle.adjoint_wave_varc(wl.u_prev.astype(np.float64), wl.u0.astype(np.float64), c, h,
                                    nt, seed, oracle.l8_weights_3d())


def rel(got, want, h):
    g, w = oracle.interior(got, h), oracle.interior(want, h)
    return float(np.linalg.norm((g - w).ravel()) / np.linalg.norm(w.ravel()))


# Element-wise bound beside the norm: the largest point error relative to the
# largest gradient magnitude.  A mistake confined to a few points barely moves
# the rel-L2 norm but gives O(1) here.
MAXN_TOL = 1e-4


def maxn(got, want, h):
    g, w = oracle.interior(got, h), oracle.interior(want, h)
    return float(np.abs(g - w).max() / np.abs(w).max())


@pytest.mark.parametrize("nt,k", [(20, 4), (13, 5), (7, 7)])
def test_adjoint_matches_oracle(nt, k):
    wl = workloads.make(5, n=N3, nt=nt)
    gm1, g0, gc, seed = grads_gpu(wl, nt, k=k)
    om1, o0, oc = grads_oracle(wl, nt, seed)
    h = wl.halo
    e = {n: rel(a, b, h) for n, a, b in (("um1", gm1, om1), ("u0", g0, o0), ("c", gc, oc))}
    m = {n: maxn(a, b, h) for n, a, b in (("um1", gm1, om1), ("u0", g0, o0), ("c", gc, oc))}
    print(f"adjoint nt={nt} k={k}: rel-L2 {e}; max-norm {m}")
    # FP32 state and lambda against FP64: each is within 1e-5 (the forward
    # target); the coefficient gradient multiplies L8(u_n) by lambda_{n+1}
    for name, v in e.items():
        assert v <= 1e-5, (name, v)
    for name, v in m.items():
        assert v <= MAXN_TOL, (name, v)


def test_adjoint_schedule_is_bitwise_invariant():
    nt = 15
    wl = workloads.make(5, n=N3, nt=nt)
    ref = grads_gpu(wl, nt, k=4)
    for kw in (dict(k=1), dict(k=1, record=False), dict(k=1, scheme=st.BLOCKED), dict(k=7),
               dict(k=15), dict(k=4, record=False),
               dict(k=5, scheme=st.BLOCKED), dict(k=3, scheme=st.BLOCKED, record=False)):
        got = grads_gpu(wl, nt, **kw)
        for a, b, name in zip(got[:2], ref[:2], ("um1", "u0")):
            assert np.array_equal(a, b), (kw, name)
        # the FP64 gradient sums the same FP32-exact terms; only the grouping
        # of the additions follows the checkpoint segments
        diff = np.abs(got[2] - ref[2]).max() / np.abs(ref[2]).max()
        assert diff <= 1e-13, (kw, diff)


def test_adjoint_nt_zero_and_one():
    wl = workloads.make(5, n=(40, 20, 12), nt=1)
    h = wl.halo
    for nt in (0, 1):
        gm1, g0, gc, seed = grads_gpu(wl, nt, k=1)
        om1, o0, oc = grads_oracle(wl, nt, seed)
        if nt == 0:
            np.testing.assert_array_equal(oracle.interior(g0, h), oracle.interior(seed, h))
            assert not gm1.any() and not gc.any()
        else:
            assert rel(g0, o0, h) <= 1e-5 and rel(gc, oc, h) <= 1e-5
            # lambda_1 = seed; the scaled form returns (c * seed) / c, one
            # rounding of the product and one of the quotient away from it
            np.testing.assert_allclose(oracle.interior(gm1, h), -oracle.interior(seed, h),
                                       rtol=2.0 ** -22, atol=0)


def test_adjoint_with_zero_coefficients():
    """c = 0 on a slab: the scaled form (mu = c lambda) cannot be divided back
    there, so the library takes the unscaled recurrence; the gradients still
    match the oracle."""
    nt = 11
    wl = workloads.make(5, n=(56, 29, 23), nt=nt)
    h = wl.halo
    wl.coef[0][h + 5:h + 9, :, :] = 0.0
    gm1, g0, gc, seed = grads_gpu(wl, nt, k=4)
    om1, o0, oc = grads_oracle(wl, nt, seed)
    e = {n: rel(a, b, h) for n, a, b in (("um1", gm1, om1), ("u0", g0, o0), ("c", gc, oc))}
    m = {n: maxn(a, b, h) for n, a, b in (("um1", gm1, om1), ("u0", g0, o0), ("c", gc, oc))}
    print(f"adjoint with zero slab: rel-L2 {e}; max-norm {m}")
    for name, v in e.items():
        assert v <= 1e-5, (name, v)
    for name, v in m.items():
        assert v <= MAXN_TOL, (name, v)


def test_autograd_function_matches_adjoint():
    import torch
    from paper_1410_3060_amd.autograd import wave_varc
    nt = 10
    wl = workloads.make(5, n=(48, 33, 21), nt=nt)
    h = wl.halo
    up = torch.from_numpy(wl.u_prev).cuda().requires_grad_(True)
    u0 = torch.from_numpy(wl.u0).cuda().requires_grad_(True)
    c = torch.from_numpy(wl.coef[0]).cuda().requires_grad_(True)
    d = torch.from_numpy(wl.target).cuda()
    uT = wave_varc(up, u0, c, nt, halo=h, ckpt_every=3)
    inner = (slice(h, -h),) * 3
    loss = 0.5 * ((uT - d)[inner] ** 2).sum()
    loss.backward()
    gm1, g0, gc, seed = grads_gpu(wl, nt, k=3)
    np.testing.assert_array_equal(oracle.interior(up.grad.double().cpu().numpy(), h),
                                  oracle.interior(gm1, h))
    np.testing.assert_array_equal(oracle.interior(u0.grad.double().cpu().numpy(), h),
                                  oracle.interior(g0, h))
    np.testing.assert_allclose(oracle.interior(c.grad.double().cpu().numpy(), h),
                               oracle.interior(gc, h), rtol=1e-6, atol=0)


def test_autograd_default_interval_and_fp64_gradient():
    """ckpt_every = 0 checkpoints every round(sqrt(nt)) steps: the gradients
    equal those of that explicit interval, bit for bit; the FP64 coefficient
    gradient handed to grad_c64 is the adjoint's own."""
    import torch
    from paper_1410_3060_amd.autograd import wave_varc
    nt = 6
    wl = workloads.make(5, n=(40, 27, 19), nt=nt)
    h = wl.halo
    grads = []
    sink = {}
    for k in (0, 2):
        up = torch.from_numpy(wl.u_prev).cuda().requires_grad_(True)
        u0 = torch.from_numpy(wl.u0).cuda().requires_grad_(True)
        c = torch.from_numpy(wl.coef[0]).cuda().requires_grad_(True)
        uT = wave_varc(up, u0, c, nt, halo=h, ckpt_every=k, grad_c64=sink if k == 0 else None)
        (uT * torch.from_numpy(wl.target).cuda()).sum().backward()
        grads.append((up.grad.clone(), u0.grad.clone(), c.grad.clone()))
    for a, b in zip(*grads):
        assert torch.equal(a, b)
    g64 = sink["grad_c"]
    assert g64.dtype == torch.float64
    assert torch.equal(g64.float(), grads[0][2])
