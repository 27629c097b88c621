"""Exact weights of the 8th-order central second derivative (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The leapfrog operator of Fig. 1e is a radius-4 star with one weight per
radius, w_0 .. w_4.  For an 8th-order accurate second derivative on a unit
grid the 1D weights a_0 .. a_4 (symmetric, a_{-k} = a_k) must satisfy the
moment conditions

    sum_{k=-4..4} a_|k| * k^(2m) = 2 if m == 1 else 0,   m = 0..4,

i.e. the stencil reproduces d^2/dx^2 exactly on every polynomial of degree
<= 9 (odd moments vanish by symmetry).  This module solves that 5x5 system
in exact rational arithmetic.  In 3D the same 1D weights act along each axis,
so the centre weight is 3*a_0 and the radius-r weight is a_r.
"""
from __future__ import annotations

from fractions import Fraction


def _solve(mat, rhs):
    """Gauss-Jordan elimination over the rationals."""
    n = len(rhs)
    a = [list(row) + [rhs[i]] for i, row in enumerate(mat)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        pv = a[col][col]
        a[col] = [v / pv for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[col])]
    return [a[i][n] for i in range(n)]


def l8_weights_1d():
    """Exact 1D weights (a_0, a_1, a_2, a_3, a_4) as Fractions."""
    # unknowns a_0..a_4; moment m: a_0*[m==0] + sum_{k>=1} 2*a_k*k^(2m)
    mat, rhs = [], []
    for m in range(5):
        row = [Fraction(1 if m == 0 else 0)]
        row += [Fraction(2 * k ** (2 * m)) for k in range(1, 5)]
        mat.append(row)
        rhs.append(Fraction(2 if m == 1 else 0))
    return tuple(_solve(mat, rhs))


def l8_weights_3d_exact():
    a = l8_weights_1d()
    return (3 * a[0],) + tuple(a[1:])


def l8_weights_3d():
    """3D weights (w_0 .. w_4) as floats."""
    return tuple(float(v) for v in l8_weights_3d_exact())
