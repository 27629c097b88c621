"""GPU adjoint of the variable-coefficient Jacobi stencils (kinds 2 and 3,
workloads 3 and 4) against the FP64 oracle.

* dJ/du_0 and every coefficient gradient dJ/dW_k, element by element against
  the oracle adjoint on the same stored inputs, at sizes spanning several
  tiles with ragged tails, FP32 and BF16 coefficient storage;
* nt = 1: the coefficient gradient is one product of FP32 values per tap
  (two-term sums for the 25-point pairs), exact in FP64, so it equals the
  oracle's bit for bit;
* the schedule only regroups FP64 additions: every checkpoint interval, with
  or without a recording, naive or blocked forward, gives the same dJ/du_0
  bit for bit (the reverse recurrence does not depend on the schedule) and
  coefficient gradients equal up to the grouping of their additions;
* nt = 0.
"""
import numpy as np
import pytest

import oracle
import paper_1410_3060_amd as st
import workloads

from gpu_util import coef_to_dev, from_dev, to_dev

pytestmark = pytest.mark.gpu

WL = {2: 3, 3: 4}  # kind -> workload index


def seed_field(wl, tag):
    rng = np.random.default_rng([1410, 97, wl.kind, tag])
    h = wl.halo
    s = np.zeros_like(wl.u0)
    inner = (slice(h, -h),) * 3
    s[inner] = rng.uniform(-1, 1, s[inner].shape).astype(np.float32)
    return s


def grads_gpu(wl, nt, seed, scheme=st.NAIVE, k=3, record=True):
    import torch
    h = wl.halo
    cf = coef_to_dev(wl)
    a, b = to_dev(wl.u0, h), to_dev(wl.u0, h)
    sd = to_dev(seed, h)
    g0 = st.alloc_field(wl.n3, h)
    gc = st.alloc_field(wl.n3, h, count=cf.shape[0], dtype=torch.float64)
    with st.Context(scheme, ckpt_every=(k if record else 0)) as ctx:
        if record:
            ctx.run(wl.kind, a, b, nt, halo=h, coef=cf)
            ctx.adjoint_jacobi(wl.kind, a, b, nt, halo=h, coef=cf, seed=sd, grad_u0=g0,
                               grad_c=gc)
            ctx.sync()
        else:
            with st.Context(scheme, ckpt_every=k) as ctx2:
                ctx2.adjoint_jacobi(wl.kind, a, b, nt, halo=h, coef=cf, seed=sd, grad_u0=g0,
                                    grad_c=gc)
                ctx2.sync()
    torch.cuda.synchronize()
    return from_dev(g0), gc.cpu().numpy()


def grads_oracle(wl, nt, seed):
    c = wl.coef_values_f32().astype(np.float64)
    return oracle.adjoint_jacobi_var(wl.kind, wl.u0.astype(np.float64), c, wl.halo, nt,
                                     seed.astype(np.float64))


def rel(got, want, h):
    g, w = oracle.interior(got, h), oracle.interior(want, h)
    return float(np.linalg.norm((g - w).ravel()) / max(np.linalg.norm(w.ravel()), 1e-300))


# Element-wise bound beside the norm: the largest point error relative to the
# largest gradient magnitude.  A mistake confined to a few points (a wrong
# tap at a tile edge) barely moves the rel-L2 norm but gives O(1) here.
MAXN_TOL = 1e-4


def maxn(got, want, h):
    g, w = oracle.interior(got, h), oracle.interior(want, h)
    return float(np.abs(g - w).max() / max(np.abs(w).max(), 1e-300))


@pytest.mark.parametrize("kind,n3,nt,k", [(2, (70, 37, 29), 12, 5), (2, (131, 45, 17), 9, 9),
                                          (3, (70, 37, 29), 10, 4), (3, (75, 19, 23), 7, 7)])
@pytest.mark.parametrize("coef_dtype", ["f32", "bf16"])
def test_adjoint_jacobi_matches_oracle(kind, n3, nt, k, coef_dtype):
    wl = workloads.make(WL[kind], n=n3, nt=nt, coef_dtype=coef_dtype)
    h = wl.halo
    s = seed_field(wl, 0)
    g0, gc = grads_gpu(wl, nt, s, k=k)
    o0, oc = grads_oracle(wl, nt, s)
    e0 = rel(g0, o0, h)
    ec = [rel(gc[i], oc[i], h) for i in range(gc.shape[0])]
    m0 = maxn(g0, o0, h)
    mc = [maxn(gc[i], oc[i], h) for i in range(gc.shape[0])]
    print(f"kind {kind} {n3} nt={nt} k={k} {coef_dtype}: rel-L2 u0 {e0:.2e}, max coef "
          f"{max(ec):.2e}; max-norm u0 {m0:.2e}, max coef {max(mc):.2e}")
    # FP32 lambda against FP64: within the forward target; the coefficient
    # gradients sum FP64 products of FP32 lambda and u values
    assert e0 <= 1e-5
    assert max(ec) <= 1e-5, ec
    assert m0 <= MAXN_TOL and max(mc) <= MAXN_TOL, (m0, mc)
    # the shells of the outputs are not written
    assert not (g0 - np.pad(oracle.interior(g0, h), h)).any()
    for i in range(gc.shape[0]):
        assert not (gc[i] - np.pad(oracle.interior(gc[i], h), h)).any()


@pytest.mark.parametrize("kind", [2, 3])
def test_adjoint_jacobi_one_step_exact(kind):
    wl = workloads.make(WL[kind], n=(67, 21, 13), nt=1)
    h = wl.halo
    s = seed_field(wl, 1)
    g0, gc = grads_gpu(wl, 1, s, k=1)
    o0, oc = grads_oracle(wl, 1, s)
    np.testing.assert_array_equal(gc, oc)
    assert rel(g0, o0, h) <= 1e-6


@pytest.mark.parametrize("kind", [2, 3])
def test_adjoint_jacobi_schedule_invariance(kind):
    nt = 11
    wl = workloads.make(WL[kind], n=(70, 33, 21), nt=nt)
    s = seed_field(wl, 2)
    ref0, refc = grads_gpu(wl, nt, s, k=4)
    for kw in (dict(k=1), dict(k=1, record=False), dict(k=1, scheme=st.BLOCKED), dict(k=6),
               dict(k=11), dict(k=3, record=False),
               dict(k=5, scheme=st.BLOCKED), dict(k=2, scheme=st.BLOCKED, record=False)):
        g0, gc = grads_gpu(wl, nt, s, **kw)
        assert np.array_equal(g0, ref0), kw
        diff = np.abs(gc - refc).max() / np.abs(refc).max()
        assert diff <= 1e-13, (kw, diff)


@pytest.mark.parametrize("kind", [2, 3])
def test_adjoint_jacobi_nt_zero(kind):
    wl = workloads.make(WL[kind], n=(40, 20, 12), nt=1)
    h = wl.halo
    s = seed_field(wl, 3)
    g0, gc = grads_gpu(wl, 0, s, k=1)
    np.testing.assert_array_equal(oracle.interior(g0, h), oracle.interior(s, h))
    assert not gc.any()


@pytest.mark.parametrize("kind,k", [(2, 1), (2, 3), (3, 1), (3, 4)])
def test_adjoint_jacobi_nonzero_shell(kind, k):
    """A non-zero boundary shell on u_0 enters the coefficient gradients of
    the boundary points (their taps read it); the checkpoints and the
    recomputed levels carry the level-0 shell."""
    nt = 6
    wl = workloads.make(WL[kind], n=(66, 35, 19), nt=nt)
    h = wl.halo
    rng = np.random.default_rng([1410, 95, kind])
    shell = rng.uniform(-1, 1, wl.u0.shape).astype(np.float32)
    inner = (slice(h, -h),) * 3
    shell[inner] = wl.u0[inner]
    wl.u0 = shell
    s = seed_field(wl, 4)
    g0, gc = grads_gpu(wl, nt, s, k=k)
    o0, oc = grads_oracle(wl, nt, s)
    assert rel(g0, o0, h) <= 1e-5
    assert max(rel(gc[i], oc[i], h) for i in range(gc.shape[0])) <= 1e-5
    assert maxn(g0, o0, h) <= MAXN_TOL
    assert max(maxn(gc[i], oc[i], h) for i in range(gc.shape[0])) <= MAXN_TOL


@pytest.mark.parametrize("kind,k", [(2, 3), (3, 1)])
def test_autograd_jacobi_matches_adjoint(kind, k):
    import torch
    from paper_1410_3060_amd.autograd import jacobi_var
    nt = 7
    wl = workloads.make(WL[kind], n=(48, 33, 21), nt=nt)
    h = wl.halo
    u0 = torch.from_numpy(wl.u0).cuda().requires_grad_(True)
    cf = torch.from_numpy(wl.coef).cuda().requires_grad_(True)
    s = seed_field(wl, 5)
    uT = jacobi_var(u0, cf, nt, kind=kind, ckpt_every=k)
    # loss = <u_T, s>: its gradient with respect to u_T is the seed
    loss = (uT * torch.from_numpy(s).cuda()).sum()
    loss.backward()
    g0, gc = grads_gpu(wl, nt, s, k=k)
    np.testing.assert_array_equal(oracle.interior(u0.grad.double().cpu().numpy(), h),
                                  oracle.interior(g0, h))
    # the library's FP64 gradient rounded once to the coefficients' FP32
    np.testing.assert_array_equal(cf.grad.cpu().numpy(), gc.astype(np.float32))


@pytest.mark.parametrize("kind", [2, 3])
def test_adjoint_jacobi_contiguous_layout(kind):
    """Plain contiguous tensors (no 256-byte alignment of the rows): the
    library's workspace follows the caller's alignment; same gradients as the
    aligned layout, bit for bit for dJ/du_0."""
    import torch
    nt = 6
    wl = workloads.make(WL[kind], n=(61, 27, 19), nt=nt)
    h = wl.halo
    s = seed_field(wl, 6)
    ref0, refc = grads_gpu(wl, nt, s, k=2)
    u = torch.from_numpy(wl.u0).cuda()
    a, b = u.clone(), u.clone()
    cf = torch.from_numpy(wl.coef).cuda()
    sd = torch.from_numpy(s).cuda()
    g0 = torch.zeros_like(a)
    gc = torch.zeros(cf.shape, dtype=torch.float64, device="cuda")
    with st.Context(st.NAIVE, ckpt_every=2) as ctx:
        ctx.run(wl.kind, a, b, nt, halo=h, coef=cf)
        ctx.adjoint_jacobi(wl.kind, a, b, nt, halo=h, coef=cf, seed=sd, grad_u0=g0, grad_c=gc)
        ctx.sync()
    assert np.array_equal(from_dev(g0), ref0)
    diff = np.abs(gc.cpu().numpy() - refc).max() / np.abs(refc).max()
    assert diff <= 1e-13
