"""FP64 CPU oracle for time-stepped 3D star stencils.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and the library never calls it.

The arithmetic lives in ``oracle.c`` (plain loops, one sweep per time step, in
double precision; Sect. 3.1 and Fig. 1 of the paper); this module builds it
with gcc and marshals numpy arrays.  ``weights.py`` derives the 8th-order
second-derivative weights exactly; ``brute.py`` is an independent
matrix-power formulation used to pin the loops on tiny grids.

Array convention: every field is a C-contiguous float64 numpy array of shape
(nz+2h, ny+2h, nx+2h) (x fastest, Sect. 3.1); the h-wide shell is a fixed
boundary that is read and never written.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .weights import l8_weights_3d  # noqa: F401  (re-exported)

KIND_7PT_CONST = 1
KIND_7PT_VAR = 2
KIND_25PT_VAR = 3
KIND_WAVE = 4
KIND_WAVE_VARC = 5

RADIUS = {1: 1, 2: 1, 3: 4, 4: 4, 5: 4}
NCOEF = {1: 0, 2: 7, 3: 13, 4: 0, 5: 1}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-std=c11", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    D = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_run.argtypes = [ctypes.c_int, i64, i64, i64, i64, D, D, D, D,
                               ctypes.c_double, i64, ctypes.c_int, D]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_adjoint_wave_varc.argtypes = [i64, i64, i64, i64, D, D, D, D, i64, D,
                                             D, D, D, ctypes.c_int]
    lib.oracle_adjoint_wave_varc.restype = ctypes.c_int
    lib.oracle_adjoint_jacobi_var.argtypes = [ctypes.c_int, i64, i64, i64, i64, D, D, i64, D,
                                              D, D, ctypes.c_int]
    lib.oracle_adjoint_jacobi_var.restype = ctypes.c_int
    lib.oracle_step_points.argtypes = [ctypes.c_int, i64, i64, i64, i64, D, D, D, D,
                                       ctypes.c_double, i64, ctypes.POINTER(i64), D]
    lib.oracle_step_points.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(u, h):
    pz, py, px = u.shape
    return px - 2 * h, py - 2 * h, pz - 2 * h


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def run(kind, u, h, nt, *, u_prev=None, coef=None, w=(0.0,) * 5, alpha=0.0,
        nthreads=0, timing=None):
    """Advance nt steps; returns the final level(s) as new arrays.

    kind 1-3: returns u_nt.  kind 4-5: returns (u_{nt-1}, u_nt), starting from
    (u_prev, u) = (u_{-1}, u_0).  ``coef`` is a (K, nz+2h, ny+2h, nx+2h) array
    (K = 7, 13, 1 for kinds 2, 3, 5).  ``timing`` (a list) receives the wall
    seconds of the time-step loop.
    """
    lib = _load()
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    nx, ny, nz = _dims(u, h)
    up = None
    if kind >= KIND_WAVE:
        up = np.array(u_prev, dtype=np.float64, order="C", copy=True)
        assert up.shape == u.shape
    cf = None
    if NCOEF[kind]:
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        assert cf.shape == (NCOEF[kind],) + u.shape, cf.shape
    wv = np.zeros(5, dtype=np.float64)
    wv[: len(w)] = np.asarray(w, dtype=np.float64)
    secs = ctypes.c_double(0.0)
    rc = lib.oracle_run(kind, nx, ny, nz, h, _p(up), _p(u), _p(cf), _p(wv), float(alpha),
                        int(nt), int(nthreads), ctypes.byref(secs))
    if rc != 0:
        raise ValueError("oracle_run rejected its arguments")
    if timing is not None:
        timing.append(secs.value)
    return (up, u) if kind >= KIND_WAVE else u


def step_points(kind, u, h, pts, *, u_prev=None, coef=None, w=(0.0,) * 5, alpha=0.0):
    """One update evaluated at interior points pts (an (n, 3) array of x, y, z).

    Works on arrays of any size: only the neighbourhoods of the points are read.
    ``u``, ``u_prev`` and ``coef`` may be float32 arrays; they are read as
    float64 one point at a time via a gathered copy of the needed values.
    """
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    n = pts.shape[0]
    R = RADIUS[kind]
    nx, ny, nz = _dims(u, h)
    if h < R or pts.ndim != 2 or pts.shape[1] != 3:
        raise ValueError("step_points: bad boundary width or point array")
    if n and ((pts < 0).any() or (pts >= np.array([nx, ny, nz])).any()):
        raise ValueError("step_points: a point lies outside the interior")
    # gather the (2R+1)^3 neighbourhood boxes into a small padded array per
    # point so that huge float32 fields need not be converted whole
    side = 2 * R + 1
    out = np.empty(n, dtype=np.float64)
    K = NCOEF[kind]
    wv = np.zeros(5, dtype=np.float64)
    wv[: len(w)] = np.asarray(w, dtype=np.float64)
    offs = np.arange(-R, R + 1)
    for i in range(n):
        x, y, z = (int(v) for v in pts[i])
        zs, ys, xs = z + h + offs, y + h + offs, x + h + offs
        sub = np.ascontiguousarray(u[np.ix_(zs, ys, xs)], dtype=np.float64)
        sp_ = None
        if kind >= KIND_WAVE:
            sp_ = np.ascontiguousarray(u_prev[np.ix_(zs, ys, xs)], dtype=np.float64)
        cf = None
        if K:
            cf = np.ascontiguousarray(coef[(slice(None),) + np.ix_(zs, ys, xs)], dtype=np.float64)
        one = np.array([[0, 0, 0]], dtype=np.int64)
        res = np.empty(1, dtype=np.float64)
        rc = lib.oracle_step_points(kind, 1, 1, 1, R, _p(sp_), _p(sub), _p(cf), _p(wv),
                                    float(alpha), 1,
                                    one.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(res))
        if rc != 0:
            raise ValueError("oracle_step_points rejected its arguments")
        out[i] = res[0]
    return out


def adjoint_wave_varc(um1, u0, c, h, nt, seed, w, nthreads=0):
    """Gradients (dJ/du_{-1}, dJ/du_0, dJ/dc) of a loss with dJ/du_nt = seed."""
    lib = _load()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (um1, u0, c, seed)]
    um1, u0, c, seed = arrs
    nx, ny, nz = _dims(u0, h)
    wv = np.ascontiguousarray(w, dtype=np.float64)
    g_um1 = np.zeros_like(u0)
    g_u0 = np.zeros_like(u0)
    g_c = np.zeros_like(u0)
    rc = lib.oracle_adjoint_wave_varc(nx, ny, nz, h, _p(um1), _p(u0), _p(c), _p(wv), int(nt),
                                      _p(seed), _p(g_um1), _p(g_u0), _p(g_c), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_adjoint_wave_varc rejected its arguments")
    return g_um1, g_u0, g_c


def adjoint_jacobi_var(kind, u0, coef, h, nt, seed, nthreads=0):
    """Gradients (dJ/du_0, dJ/dW) of a loss with dJ/du_nt = seed for the
    variable-coefficient kinds 2 (Fig. 1c) and 3 (Fig. 1d); dJ/dW has the
    shape of coef (K arrays)."""
    lib = _load()
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    cf = np.ascontiguousarray(coef, dtype=np.float64)
    sd = np.ascontiguousarray(seed, dtype=np.float64)
    nx, ny, nz = _dims(u0, h)
    g_u0 = np.zeros_like(u0)
    g_c = np.zeros_like(cf)
    rc = lib.oracle_adjoint_jacobi_var(int(kind), nx, ny, nz, h, _p(u0), _p(cf), int(nt), _p(sd),
                                       _p(g_u0), _p(g_c), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_adjoint_jacobi_var rejected its arguments")
    return g_u0, g_c


def interior(a, h):
    """View of the interior of a padded field (last three axes)."""
    return a[..., h:a.shape[-3] - h, h:a.shape[-2] - h, h:a.shape[-1] - h]
