"""Pin of the oracle's single-update evaluator (``oracle.step_points``).

``step_points`` restates the five updates of Fig. 1b-1e (Sect. 3.1) a second
time so that single sweeps of very large grids can be checked on sampled
points.  It is pinned here against one sweep of ``oracle.run``, which the
other oracle tests pin to matrix powers, closed forms and invariants: at every
interior point of small grids, every kind, with a non-zero boundary shell
(the shell is read by the stencil, so a wrong neighbour offset that lands in
the shell is caught too) and random coefficients.  The two evaluate the sums
in different orders, so they agree to rounding, not bit for bit.
"""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(1410_3060)


def _field(n3, h):
    nx, ny, nz = n3
    # non-zero everywhere, the shell included
    return RNG.uniform(-1.0, 1.0, size=(nz + 2 * h, ny + 2 * h, nx + 2 * h))


@pytest.mark.parametrize("kind", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n3", [(5, 6, 7), (9, 4, 6)])
def test_step_points_equals_one_sweep(kind, n3):
    R = oracle.RADIUS[kind]
    h = R + 1  # a shell wider than the radius: values beyond R must not be read
    u = _field(n3, h)
    up = _field(n3, h) if kind >= 4 else None
    K = oracle.NCOEF[kind]
    coef = RNG.uniform(-1.0, 1.0, size=(K,) + u.shape) if K else None
    w = (0.4, 0.1) if kind == 1 else tuple(RNG.uniform(-1.0, 1.0, size=5))
    alpha = 0.37
    if kind >= 4:
        _, want = oracle.run(kind, u, h, 1, u_prev=up, coef=coef, w=w, alpha=alpha)
    else:
        want = oracle.run(kind, u, h, 1, coef=coef, w=w)
    nx, ny, nz = n3
    pts = np.array([(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)],
                   dtype=np.int64)
    got = oracle.step_points(kind, u, h, pts, u_prev=up, coef=coef, w=w, alpha=alpha)
    ref = np.array([want[z + h, y + h, x + h] for x, y, z in pts])
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale


def test_step_points_reads_float32_fields():
    """The sampled check of the full-size tests hands float32 fields over; the
    gathered neighbourhoods are upcast exactly."""
    kind, n3, h = 3, (6, 5, 9), 4
    u = _field(n3, h).astype(np.float32)
    coef = RNG.uniform(0.0, 1.0, size=(13,) + u.shape).astype(np.float32)
    want = oracle.run(kind, u.astype(np.float64), h, 1, coef=coef.astype(np.float64))
    pts = np.array([[0, 0, 0], [5, 4, 8], [2, 3, 4]], dtype=np.int64)
    got = oracle.step_points(kind, u, h, pts, coef=coef)
    ref = np.array([want[z + h, y + h, x + h] for x, y, z in pts])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_step_points_rejects_points_outside():
    u = _field((4, 4, 4), 1)
    with pytest.raises(ValueError):
        oracle.step_points(1, u, 1, np.array([[4, 0, 0]]), w=(0.4, 0.1))
