"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test would fail on a plausible slip in oracle.c (a dropped term, a wrong
sign, a swapped neighbour, a transposed coefficient index):

* 8th-order weights: moment conditions, textbook values, exactness on
  polynomials of degree <= 9 and the exact degree-10 residual (Fig. 1e);
* constant preservation (Fig. 1b, Fig. 1e) and row-sum decay (Fig. 1c, 1d);
* single-coefficient special cases that reduce Fig. 1c / 1d to pure shifts,
  which pins every coefficient index to its neighbour;
* brute force: A^nt u0 from an independently assembled sparse matrix;
* leapfrog energy conservation.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle.weights import l8_weights_1d, l8_weights_3d, l8_weights_3d_exact

RNG = np.random.default_rng(20141011)


def padded(n3, h, fill=0.0):
    nx, ny, nz = n3
    return np.full((nz + 2 * h, ny + 2 * h, nx + 2 * h), fill, dtype=np.float64)


def inner(a, h):
    return oracle.interior(a, h)


def rand_interior(n3, h, lo=-1.0, hi=1.0):
    a = padded(n3, h)
    inner(a, h)[...] = RNG.uniform(lo, hi, size=inner(a, h).shape)
    return a


# ---------------------------------------------------------------- weights


def test_l8_moments_exact():
    a = l8_weights_1d()
    for m in range(6):
        mom = a[0] * (1 if m == 0 else 0) + sum(2 * a[k] * k ** (2 * m) for k in range(1, 5))
        if m == 1:
            assert mom == 2
        elif m <= 4:
            assert mom == 0
        else:  # first non-vanishing error moment: sum a_k k^10 = 2*10!/(−3150*...)
            assert mom != 0


def test_l8_textbook_values():
    # Fornberg's table of central second-derivative weights, 8th order
    assert l8_weights_1d() == (Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5),
                               Fraction(8, 315), Fraction(-1, 560))
    assert l8_weights_3d_exact()[0] == Fraction(-205, 24)


def _poly_field(n3, h, coeffs, shift):
    """p(x,y,z) = sum c_abc x^a y^b z^c sampled on every padded point, with
    integer coordinates shifted so that the grid is centred near 0."""
    nx, ny, nz = n3
    z = np.arange(-h, nz + h, dtype=np.float64) - shift[2]
    y = np.arange(-h, ny + h, dtype=np.float64) - shift[1]
    x = np.arange(-h, nx + h, dtype=np.float64) - shift[0]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    p = np.zeros_like(X)
    lap = np.zeros_like(X)
    for (ea, eb, ec), c in coeffs.items():
        p += c * X ** ea * Y ** eb * Z ** ec
        if ea >= 2:
            lap += c * ea * (ea - 1) * X ** (ea - 2) * Y ** eb * Z ** ec
        if eb >= 2:
            lap += c * eb * (eb - 1) * X ** ea * Y ** (eb - 2) * Z ** ec
        if ec >= 2:
            lap += c * ec * (ec - 1) * X ** ea * Y ** eb * Z ** (ec - 2)
    return p, lap


def _apply_l8(u, h, w):
    # kind 4 with alpha = 1 and u_{-1} = 2 u gives u_1 = L8(u)
    up, un = oracle.run(oracle.KIND_WAVE, u, h, 1, u_prev=2.0 * u, w=w, alpha=1.0)
    return un


@pytest.mark.parametrize("deg", [2, 5, 9])
def test_l8_exact_on_polynomials(deg):
    n3, h = (7, 6, 5), 4
    coeffs = {}
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                coeffs[(a, b, c)] = RNG.uniform(-1, 1) / (1 + a + b + c) ** 2
    p, lap = _poly_field(n3, h, coeffs, shift=(3, 2.5, 2))
    got = inner(_apply_l8(p, h, l8_weights_3d()), h)
    want = inner(lap, h)
    scale = np.abs(want).max() + np.abs(inner(p, h)).max()
    assert np.abs(got - want).max() <= 1e-11 * scale


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_l8_degree10_residual(axis):
    # D8(t^10) - 90 t^8 = -h^8 f^(10)/3150 = -10!/3150 = -1152 at every point
    n3, h = (5, 5, 5), 4
    e = [0, 0, 0]
    e[axis] = 10
    p, lap = _poly_field(n3, h, {tuple(e): 1.0}, shift=(2, 2, 2))
    got = inner(_apply_l8(p, h, l8_weights_3d()), h) - inner(lap, h)
    np.testing.assert_allclose(got, -1152.0, rtol=0, atol=1e-5)


# ---------------------------------------------------------------- invariants


def test_7pt_const_preserves_constant():
    n3, h, c = (9, 8, 7), 1, 0.75
    u = padded(n3, h, fill=c)
    out = oracle.run(oracle.KIND_7PT_CONST, u, h, 20, w=(0.4, 0.1))
    np.testing.assert_allclose(inner(out, h), c, rtol=0, atol=20 * 1e-15)


@pytest.mark.parametrize("kind", [oracle.KIND_WAVE, oracle.KIND_WAVE_VARC])
def test_leapfrog_preserves_constant(kind):
    n3, h, c = (9, 10, 11), 4, -0.3
    u = padded(n3, h, fill=c)
    coef = None
    if kind == oracle.KIND_WAVE_VARC:
        coef = RNG.uniform(0.05, 0.1, size=(1,) + u.shape)
    up, un = oracle.run(kind, u, h, 15, u_prev=u.copy(), coef=coef,
                        w=l8_weights_3d(), alpha=0.1)
    np.testing.assert_allclose(inner(un, h), c, rtol=0, atol=1e-13)
    np.testing.assert_allclose(inner(up, h), c, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind,K,R,pw", [(oracle.KIND_7PT_VAR, 7, 1, [1] * 7),
                                          (oracle.KIND_25PT_VAR, 13, 4, [1] + [2] * 12)])
def test_row_sum_decay(kind, K, R, pw):
    # constant field, zero boundary, per-point row sum s: points farther than
    # R*t from the boundary hold s^t * c after t steps
    n3, h, c, s, nt = (20, 21, 22), R, 1.0, 0.99, 2
    u = padded(n3, h)
    inner(u, h)[...] = c
    coef = RNG.uniform(0, 1, size=(K,) + u.shape)
    tot = sum(pw[k] * coef[k] for k in range(K))
    coef = coef * (s / tot)
    out = oracle.run(kind, u, h, nt, coef=coef)
    m = R * nt
    core = inner(out, h)[m:-m, m:-m, m:-m]
    np.testing.assert_allclose(core, s ** nt * c, rtol=1e-14)
    # and the boundary layer has lost mass (the zero shell is felt)
    assert inner(out, h)[0, 0, 0] < s ** nt * c


# ---------------------------------------------------------------- special cases


SHIFTS_7 = [(None, 0), (0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)]


def _shifted(u, h, axis, r):
    """u(p + r e_axis) on the interior (reads the shell)."""
    nz, ny, nx = (s - 2 * h for s in u.shape)
    sl = [slice(h, h + nz), slice(h, h + ny), slice(h, h + nx)]
    ax = 2 - axis  # numpy axis for x is 2
    sl[ax] = slice(h + r, h + r + [nz, ny, nx][ax])
    return u[tuple(sl)]


@pytest.mark.parametrize("k", range(7))
def test_7pt_var_single_coefficient_is_a_shift(k):
    n3, h = (6, 7, 8), 1
    u = rand_interior(n3, h)
    u[0, :, :] = 5.0  # nonzero shell so that boundary reads are visible
    u[:, :, -1] = -3.0
    coef = np.zeros((7,) + u.shape)
    coef[k] = 1.0
    out = oracle.run(oracle.KIND_7PT_VAR, u, h, 1, coef=coef)
    axis, r = SHIFTS_7[k]
    want = inner(u, h) if axis is None else _shifted(u, h, axis, r)
    np.testing.assert_array_equal(inner(out, h), want)


@pytest.mark.parametrize("k", range(13))
def test_25pt_var_single_coefficient_is_a_pair(k):
    n3, h = (9, 10, 11), 4
    u = rand_interior(n3, h)
    u[1, :, :] = 2.0
    u[:, -2, :] = -1.5
    coef = np.zeros((13,) + u.shape)
    coef[k] = 1.0
    out = oracle.run(oracle.KIND_25PT_VAR, u, h, 1, coef=coef)
    if k == 0:
        want = inner(u, h)
    else:
        r, axis = (k - 1) // 3 + 1, (k - 1) % 3  # Fig. 1d: W1 x r1, W2 y r1, W3 z r1, W4 x r2 ...
        want = _shifted(u, h, axis, -r) + _shifted(u, h, axis, r)
    np.testing.assert_array_equal(inner(out, h), want)


def test_7pt_const_weights_roles():
    # w0 multiplies the centre, w1 the neighbour sum
    n3, h = (5, 5, 5), 1
    u = rand_interior(n3, h)
    a = oracle.run(oracle.KIND_7PT_CONST, u, h, 1, w=(1.0, 0.0))
    np.testing.assert_array_equal(inner(a, h), inner(u, h))
    b = oracle.run(oracle.KIND_7PT_CONST, u, h, 1, w=(0.0, 1.0))
    want = sum(_shifted(u, h, ax, r) for ax in range(3) for r in (-1, 1))
    np.testing.assert_allclose(inner(b, h), want, rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------- brute force


def _vec(a, h):
    return inner(a, h).reshape(-1).copy()


@pytest.mark.parametrize("n3", [(8, 8, 8), (8, 8, 12), (6, 7, 9)])
@pytest.mark.parametrize("kind", [1, 2, 3])
def test_brute_force_first_order(kind, n3):
    h, nt = oracle.RADIUS[kind], 6
    u = rand_interior(n3, h)
    nx, ny, nz = n3
    coef = None
    w = (0.4, 0.1)
    if kind > 1:
        K = oracle.NCOEF[kind]
        coef = np.zeros((K,) + u.shape)
        for k in range(K):
            inner(coef[k], h)[...] = RNG.uniform(0, 0.3, size=(nz, ny, nx))
    out = oracle.run(kind, u, h, nt, coef=coef, w=w)
    A = brute.operator(kind, nx, ny, nz,
                       coef=None if coef is None else inner(coef, h), w=w)
    want = brute.power_apply(A, _vec(u, h), nt)
    got = _vec(out, h)
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("n3", [(8, 8, 8), (8, 8, 12)])
@pytest.mark.parametrize("kind", [4, 5])
def test_brute_force_leapfrog(kind, n3):
    h, nt = 4, 9
    nx, ny, nz = n3
    w = l8_weights_3d()
    u0 = rand_interior(n3, h)
    um1 = rand_interior(n3, h)
    coef, alpha = None, 0.1
    if kind == 5:
        coef = padded(n3, h)[None].copy()
        inner(coef[0], h)[...] = RNG.uniform(0.05, 0.1, size=(nz, ny, nx))
        alpha_vec = inner(coef[0], h)
    else:
        alpha_vec = alpha
    up, un = oracle.run(kind, u0, h, nt, u_prev=um1, coef=coef, w=w, alpha=alpha)
    L = brute.operator(kind, nx, ny, nz, w=w)
    C = brute.leapfrog_companion(L, alpha_vec)
    state = np.concatenate([_vec(u0, h), _vec(um1, h)])
    want = brute.power_apply(C, state, nt)
    n = nx * ny * nz
    scale = max(1.0, np.abs(want).max())
    assert np.abs(_vec(un, h) - want[:n]).max() <= 1e-12 * scale
    assert np.abs(_vec(up, h) - want[n:]).max() <= 1e-12 * scale


def test_nt_zero_is_identity_and_negative_rejected():
    n3, h = (4, 4, 4), 1
    u = rand_interior(n3, h)
    out = oracle.run(1, u, h, 0, w=(0.4, 0.1))
    np.testing.assert_array_equal(out, u)
    with pytest.raises(ValueError):
        oracle.run(1, u, h, -1, w=(0.4, 0.1))


# ---------------------------------------------------------------- energy


def test_leapfrog_energy_conserved():
    n3, h, nt = (10, 11, 12), 4, 200
    nx, ny, nz = n3
    w = l8_weights_3d()
    u0 = rand_interior(n3, h, -0.1, 0.1)
    um1 = u0.copy()
    inner(um1, h)[...] += RNG.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    coef = padded(n3, h)[None].copy()
    inner(coef[0], h)[...] = RNG.uniform(0.06, 0.1, size=(nz, ny, nx))
    c = _vec(coef[0], h)
    L = brute.operator(5, nx, ny, nz, w=w)

    def energy(u_next, u_cur):
        d = u_next - u_cur
        return d @ (d / c) - u_next @ (L @ u_cur)

    prev, cur = um1, u0
    E = []
    for _ in range(nt):
        nxt_prev, nxt = oracle.run(5, cur, h, 1, u_prev=prev, coef=coef, w=w)
        E.append(energy(_vec(nxt, h), _vec(cur, h)))
        prev, cur = nxt_prev, nxt
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-11 * np.abs(E[0])
