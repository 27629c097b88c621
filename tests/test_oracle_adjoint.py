"""Pins of the oracle adjoint (reverse time stepping of the leapfrog with c(x)).

* dot-product test: for fixed c the map (u_{-1}, u_0) -> u_T is linear, so
  <J d, s> must equal <d, J^T s> for the adjoint seeded with s;
* T = 1 closed form: dJ/du_0 = (2I + L diag(c)) s, dJ/dc = s * L(u_0);
* central finite differences on a 32^3 grid (the workload-5 check) and a
  smaller one, for c, u_0 and u_{-1}, in FP64.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from oracle.weights import l8_weights_3d

RNG = np.random.default_rng(31415)
W = l8_weights_3d()


def padded(n3, h):
    nx, ny, nz = n3
    return np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h))


def rand(n3, h, lo=-1.0, hi=1.0):
    a = padded(n3, h)
    oracle.interior(a, h)[...] = RNG.uniform(lo, hi, size=oracle.interior(a, h).shape)
    return a


def forward(um1, u0, c, h, nt):
    return oracle.run(5, u0, h, nt, u_prev=um1, coef=c[None], w=W)[1]


def loss(um1, u0, c, d, h, nt):
    uT = forward(um1, u0, c, h, nt)
    r = oracle.interior(uT - d, h)
    return 0.5 * float((r * r).sum())


def grads(um1, u0, c, d, h, nt):
    uT = forward(um1, u0, c, h, nt)
    seed = uT - d
    oracle.interior(seed, h)  # shell of uT - d is zero already
    return oracle.adjoint_wave_varc(um1, u0, c, h, nt, seed, W)


@pytest.mark.parametrize("nt", [1, 2, 7])
def test_dot_product(nt):
    n3, h = (9, 8, 10), 4
    c = rand(n3, h, 0.05, 0.1)
    d_m1, d_0, s = rand(n3, h), rand(n3, h), rand(n3, h)
    out = forward(d_m1, d_0, c, h, nt)
    g_m1, g_0, _ = oracle.adjoint_wave_varc(d_m1, d_0, c, h, nt, s, W)
    lhs = float((oracle.interior(out, h) * oracle.interior(s, h)).sum())
    rhs = float((g_0 * d_0).sum() + (g_m1 * d_m1).sum())
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_t1_closed_form():
    n3, h = (8, 9, 7), 4
    nx, ny, nz = n3
    c = rand(n3, h, 0.05, 0.1)
    u0, um1, s = rand(n3, h), rand(n3, h), rand(n3, h)
    g_m1, g_0, g_c = oracle.adjoint_wave_varc(um1, u0, c, h, 1, s, W)
    L = brute.operator(5, nx, ny, nz, w=W)
    sv = oracle.interior(s, h).reshape(-1)
    cv = oracle.interior(c, h).reshape(-1)
    want_u0 = 2 * sv + L @ (cv * sv)
    want_c = sv * (L @ oracle.interior(u0, h).reshape(-1))
    np.testing.assert_allclose(oracle.interior(g_0, h).reshape(-1), want_u0, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.interior(g_c, h).reshape(-1), want_c, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.interior(g_m1, h), -oracle.interior(s, h), rtol=0, atol=0)
    # nt = 0: u_T = u_0
    g_m1, g_0, g_c = oracle.adjoint_wave_varc(um1, u0, c, h, 0, s, W)
    np.testing.assert_array_equal(oracle.interior(g_0, h), oracle.interior(s, h))
    assert not g_m1.any() and not g_c.any()


@pytest.mark.parametrize("n3,nt", [((8, 7, 9), 7), ((32, 32, 32), 12)])
def test_finite_differences(n3, nt):
    h = 4
    c = padded(n3, h)
    oracle.interior(c, h)[...] = 0.08 * (1 + 0.3 * RNG.uniform(-1, 1, size=oracle.interior(c, h).shape))
    u0 = rand(n3, h, -0.5, 0.5)
    um1 = u0.copy()
    oracle.interior(um1, h)[...] += RNG.uniform(-0.01, 0.01, size=oracle.interior(um1, h).shape)
    d = rand(n3, h)
    g_m1, g_0, g_c = grads(um1, u0, c, d, h, nt)
    # J(+) - J(-) = 0.5 * <u_T(+) - u_T(-), r(+) + r(-)>: differencing the
    # states instead of the losses avoids cancelling two O(1e3) sums
    for name, base, g, eps in (("c", c, g_c, 1e-7), ("u0", u0, g_0, 1e-4),
                               ("um1", um1, g_m1, 1e-4)):
        # one random direction and three single points
        dirs = [rand(n3, h)]
        for _ in range(3):
            e = padded(n3, h)
            z, y, x = (RNG.integers(0, s) + h for s in reversed(n3))
            e[z, y, x] = 1.0
            dirs.append(e)
        for e in dirs:
            args = {"c": c, "u0": u0, "um1": um1}
            plus = dict(args)
            minus = dict(args)
            plus[name] = base + eps * e
            minus[name] = base - eps * e
            up = forward(plus["um1"], plus["u0"], plus["c"], h, nt)
            um = forward(minus["um1"], minus["u0"], minus["c"], h, nt)
            du = oracle.interior(up - um, h)
            rs = oracle.interior(up + um - 2 * d, h)
            fd = 0.5 * float((du * rs).sum()) / (2 * eps)
            an = float((g * e).sum())
            assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3), (name, fd, an)
