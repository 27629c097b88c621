"""Brute-force matrix formulation of the stencils (oracle side, tiny grids).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A second, structurally different statement of Fig. 1b-1e used to pin the loop
oracle: every operator is assembled as a sparse matrix over the interior
unknowns (C order, x fastest) from Kronecker products of 1D shift matrices,

    S_a^{(r)} u (p) = u(p + r e_a)          (zero outside the interior),

scaled row-wise by diag(W) for domain-sized coefficients.  The time loop is
then a plain matrix power: u_nt = A^nt u_0 for the first-order kinds, and the
companion form [u_{n+1}; u_n] = [[2I + diag(alpha) L, -I], [I, 0]] [u_n; u_{n-1}]
for the leapfrog.  Boundary values are zero (homogeneous Dirichlet): a zero
shell contributes nothing, which is what truncating the shifts encodes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _shift1d(n, r):
    # (E u)[i] = u[i + r]; ones on diagonal r
    return sp.eye(n, n, k=r, format="csr")


def shift3d(nx, ny, nz, axis, r):
    """Sparse S with (S u)(x,y,z) = u(point + r along axis), zero outside."""
    ix, iy, iz = sp.eye(nx, format="csr"), sp.eye(ny, format="csr"), sp.eye(nz, format="csr")
    ex = _shift1d(nx, r) if axis == 0 else ix
    ey = _shift1d(ny, r) if axis == 1 else iy
    ez = _shift1d(nz, r) if axis == 2 else iz
    # index = (z*ny + y)*nx + x  ->  z is the slowest factor
    return sp.kron(ez, sp.kron(ey, ex, format="csr"), format="csr")


def operator(kind, nx, ny, nz, coef=None, w=None):
    """Sparse matrix of one sweep (kinds 1-3) or of L8 (kinds 4-5).

    coef: interior-only arrays of shape (K, nz, ny, nx) for kinds 2 and 3.
    """
    n = nx * ny * nz
    S = lambda a, r: shift3d(nx, ny, nz, a, r)  # noqa: E731
    D = lambda arr: sp.diags(np.asarray(arr, dtype=np.float64).reshape(-1))  # noqa: E731
    if kind == 1:
        nb = sum(S(a, s) for a in range(3) for s in (-1, 1))
        return w[0] * sp.eye(n) + w[1] * nb
    if kind == 2:
        offs = [(None, 0), (0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)]
        A = D(coef[0])
        for k, (a, r) in enumerate(offs[1:], start=1):
            A = A + D(coef[k]) @ S(a, r)
        return A.tocsr()
    if kind == 3:
        A = D(coef[0])
        for r in range(1, 5):
            for a in range(3):
                A = A + D(coef[3 * (r - 1) + a + 1]) @ (S(a, -r) + S(a, r))
        return A.tocsr()
    if kind in (4, 5):
        L = w[0] * sp.eye(n)
        for r in range(1, 5):
            L = L + w[r] * sum(S(a, -r) + S(a, r) for a in range(3))
        return L.tocsr()
    raise ValueError(kind)


def power_apply(A, v, nt):
    """A^nt v as a dense matrix power (tiny n only)."""
    Ad = A.toarray()
    return np.linalg.matrix_power(Ad, int(nt)) @ v


def leapfrog_companion(L, alpha):
    """Block matrix advancing (u_n, u_{n-1}) -> (u_{n+1}, u_n)."""
    n = L.shape[0]
    a = np.broadcast_to(np.asarray(alpha, dtype=np.float64).reshape(-1), (n,))
    M = 2.0 * sp.eye(n) + sp.diags(a) @ L
    top = sp.hstack([M, -sp.eye(n)])
    bot = sp.hstack([sp.eye(n), sp.csr_matrix((n, n))])
    return sp.vstack([top, bot]).tocsr()
