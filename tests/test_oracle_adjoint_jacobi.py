"""Pins of the oracle adjoint of the variable-coefficient Jacobi kinds 2 and 3
(Fig. 1c, 1d), u_{t+1} = A(W) u_t with a fixed (Dirichlet) shell.

* dense closed form: dJ/du_0 = (A^T)^nt s with A assembled by the brute-force
  Kronecker formulation and transposed by scipy (the oracle gathers the
  transpose point by point, a different statement of it);
* dot-product identity <A^nt d, s> = <d, dJ/du_0> for a zero shell;
* nt = 1 closed form of every coefficient gradient: dJ/dW_k = s * (the value
  W_k multiplies), including a non-zero shell;
* central finite differences on single coefficient entries and a random
  direction, with a non-zero shell, for several steps;
* nt = 0: dJ/du_0 = s, dJ/dW = 0.
"""
import numpy as np
import pytest

import oracle
from oracle import brute

RNG = np.random.default_rng(31416)


def padded(n3, h, k=None):
    nx, ny, nz = n3
    shape = (nz + 2 * h, ny + 2 * h, nx + 2 * h)
    return np.zeros(shape if k is None else (k,) + shape)


def rand(n3, h, lo=-1.0, hi=1.0, shell=False):
    a = padded(n3, h)
    if shell:
        a[...] = RNG.uniform(lo, hi, size=a.shape)
    else:
        oracle.interior(a, h)[...] = RNG.uniform(lo, hi, size=oracle.interior(a, h).shape)
    return a


def coefs(kind, n3, h):
    K = oracle.NCOEF[kind]
    c = RNG.uniform(-0.3, 0.3, size=padded(n3, h, K).shape)
    c[0] += 0.2
    return c / (1.5 if kind == 2 else 4.0)


def inner_coef(c, h):
    return np.stack([oracle.interior(ck, h) for ck in c])


def forward(kind, u0, c, h, nt):
    return oracle.run(kind, u0, h, nt, coef=c)


@pytest.mark.parametrize("kind,n3,nt", [(2, (5, 4, 6), 3), (3, (9, 10, 9), 2), (2, (6, 6, 5), 1)])
def test_dense_transpose_power(kind, n3, nt):
    h = oracle.RADIUS[kind]
    c = coefs(kind, n3, h)
    u0, s = rand(n3, h), rand(n3, h)
    g0, _ = oracle.adjoint_jacobi_var(kind, u0, c, h, nt, s)
    A = brute.operator(kind, *n3, coef=inner_coef(c, h)).toarray()
    want = np.linalg.matrix_power(A.T, nt) @ oracle.interior(s, h).reshape(-1)
    np.testing.assert_allclose(oracle.interior(g0, h).reshape(-1), want, rtol=1e-12, atol=1e-13)
    # shell of the input gradient stays zero
    assert not (g0 - np.pad(oracle.interior(g0, h), h)).any()


@pytest.mark.parametrize("kind", [2, 3])
def test_dot_product(kind):
    n3, nt = (11, 9, 10), 5
    h = oracle.RADIUS[kind]
    c = coefs(kind, n3, h)
    d, s = rand(n3, h), rand(n3, h)
    out = forward(kind, d, c, h, nt)
    g0, _ = oracle.adjoint_jacobi_var(kind, d, c, h, nt, s)
    lhs = float((oracle.interior(out, h) * oracle.interior(s, h)).sum())
    rhs = float((g0 * d).sum())
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("kind", [2, 3])
def test_t1_coefficient_gradients(kind):
    n3 = (7, 8, 9)
    h = oracle.RADIUS[kind]
    c = coefs(kind, n3, h)
    u0, s = rand(n3, h, shell=True), rand(n3, h)
    _, gc = oracle.adjoint_jacobi_var(kind, u0, c, h, 1, s)
    nx, ny, nz = n3
    si = oracle.interior(s, h)

    def sh(dx, dy, dz):
        # u0 at p + (dx, dy, dz) for interior p, shell values included
        return u0[h + dz:h + dz + nz, h + dy:h + dy + ny, h + dx:h + dx + nx]

    if kind == 2:
        taps = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
        want = [si * sh(*t) for t in taps]
    else:
        want = [si * sh(0, 0, 0)]
        for r in range(1, 5):
            want += [si * (sh(-r, 0, 0) + sh(r, 0, 0)), si * (sh(0, -r, 0) + sh(0, r, 0)),
                     si * (sh(0, 0, -r) + sh(0, 0, r))]
    for k in range(oracle.NCOEF[kind]):
        np.testing.assert_allclose(oracle.interior(gc[k], h), want[k], rtol=1e-14, atol=1e-15)
        # gradients live on interior points only
        assert not (gc[k] - np.pad(oracle.interior(gc[k], h), h)).any()


@pytest.mark.parametrize("kind,nt", [(2, 6), (3, 4)])
def test_finite_differences(kind, nt):
    n3 = (8, 7, 9)
    h = oracle.RADIUS[kind]
    K = oracle.NCOEF[kind]
    c = coefs(kind, n3, h)
    u0 = rand(n3, h, shell=True)
    d = rand(n3, h)
    uT = forward(kind, u0, c, h, nt)
    g0, gc = oracle.adjoint_jacobi_var(kind, u0, c, h, nt, uT - d)

    def loss_diff(cp, cm, up, um):
        a, b = forward(kind, up, cp, h, nt), forward(kind, um, cm, h, nt)
        du = oracle.interior(a - b, h)
        rs = oracle.interior(a + b - 2 * d, h)
        return 0.5 * float((du * rs).sum())

    eps = 1e-6
    checks = []
    for _ in range(6):
        e = padded(n3, h, K)
        k = int(RNG.integers(0, K))
        z, y, x = (int(RNG.integers(0, s)) + h for s in reversed(n3))
        e[k, z, y, x] = 1.0
        checks.append(e)
    e = padded(n3, h, K)
    for k in range(K):
        oracle.interior(e[k], h)[...] = RNG.uniform(-1, 1, size=oracle.interior(e[k], h).shape)
    checks.append(e)
    for e in checks:
        fd = loss_diff(c + eps * e, c - eps * e, u0, u0) / (2 * eps)
        an = float((gc * e).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)
    e = rand(n3, h)
    fd = loss_diff(c, c, u0 + eps * e, u0 - eps * e) / (2 * eps)
    an = float((g0 * e).sum())
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)


@pytest.mark.parametrize("kind", [2, 3])
def test_nt_zero(kind):
    n3 = (5, 6, 7)
    h = oracle.RADIUS[kind]
    c = coefs(kind, n3, h)
    u0, s = rand(n3, h, shell=True), rand(n3, h)
    g0, gc = oracle.adjoint_jacobi_var(kind, u0, c, h, 0, s)
    np.testing.assert_array_equal(g0, s)
    assert not gc.any()
