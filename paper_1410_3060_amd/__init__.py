"""MI355X-native time-stepped 3D star stencils (naive, diamond/wavefront
temporally blocked, and the leapfrog adjoint) -- Python binding.

This module only marshals arguments to the C ABI of ``libstencil.so``
(declared in ``include/stencil.h``); every lattice update runs in the HIP
kernels of that library.  PyTorch supplies device memory and streams.  If the
library is missing the import of any entry point raises: there is no CPU
fallback.

Fields are torch float32 CUDA tensors of shape (nz+2h, ny+2h, nx+2h) (a view
is fine) with x contiguous, addressing the padded origin; coefficient arrays
are (K, nz+2h, ny+2h, nx+2h) float32 or bfloat16 tensors with the same row
and plane strides.  ``alloc_field`` builds such views with the interior x = 0
aligned to 256 bytes and 256-byte row pitch.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstencil.so")

# stencil_kind
KIND_7PT_CONST = 1
KIND_7PT_VAR = 2
KIND_25PT_VAR = 3
KIND_25PT_WAVE = 4
KIND_25PT_WAVE_VARC = 5
# stencil_scheme
NAIVE = 0
BLOCKED = 1
# stencil_dtype
F32 = 0
BF16 = 1

RADIUS = {1: 1, 2: 1, 3: 4, 4: 4, 5: 4}
NCOEF = {1: 0, 2: 7, 3: 13, 4: 0, 5: 1}
LEAPFROG = {4, 5}

# Weights of the 8th-order central second difference along one axis are
# (-205/72, 8/5, -1/5, 8/315, -1/560); the 3D operator L8 of Fig. 1e takes
# the centre weight three times.
L8_WEIGHTS = (3.0 * (-205.0 / 72.0), 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)


class StencilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("sy", ctypes.c_int64), ("sz", ctypes.c_int64),
                ("u", ctypes.c_void_p * 2)]


class _Coeffs(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("arrays", ctypes.c_void_p), ("sk", ctypes.c_int64),
                ("w", ctypes.c_double * 5), ("alpha", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("dw", ctypes.c_int32), ("xtile", ctypes.c_int32), ("zchunk", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("workspace_limit", ctypes.c_int64)]


EXPORTS = ("stencil_create", "stencil_run", "stencil_run_noalloc", "stencil_adjoint",
           "stencil_sync", "stencil_destroy", "stencil_last_error", "stencil_plan_rows",
           "stencil_default_dw", "stencil_blocked_slices")

_lib = None


def load(path: Optional[str] = None):
    """Load libstencil.so (built by ``paper_1410_3060_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_1410_3060_amd.build`")
    # torch ships its own HIP runtime; importing it first lets the library
    # bind to the runtime already in the process.  Opened before torch, the
    # library's later HIP calls found no device once torch had initialised
    # its own.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.stencil_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(_Tuning), vp]
    lib.stencil_create.restype = ctypes.c_int
    lib.stencil_run.argtypes = [vp, ctypes.c_int, ctypes.POINTER(_Grid), ctypes.POINTER(_Coeffs),
                                i64, ctypes.POINTER(ctypes.c_int)]
    lib.stencil_run.restype = ctypes.c_int
    lib.stencil_run_noalloc.argtypes = lib.stencil_run.argtypes
    lib.stencil_run_noalloc.restype = ctypes.c_int
    lib.stencil_adjoint.argtypes = [vp, ctypes.c_int, ctypes.POINTER(_Grid),
                                    ctypes.POINTER(_Coeffs), i64, vp, vp, vp, vp]
    lib.stencil_adjoint.restype = ctypes.c_int
    lib.stencil_sync.argtypes = [vp]
    lib.stencil_sync.restype = ctypes.c_int
    lib.stencil_destroy.argtypes = [vp]
    lib.stencil_destroy.restype = None
    lib.stencil_last_error.argtypes = []
    lib.stencil_last_error.restype = ctypes.c_char_p
    lib.stencil_plan_rows.argtypes = [ctypes.c_int, i32, i32, i64, ctypes.POINTER(i64), i32]
    lib.stencil_plan_rows.restype = ctypes.c_int
    lib.stencil_default_dw.argtypes = [ctypes.c_int, i32, i32, i32, ctypes.c_int]
    lib.stencil_default_dw.restype = ctypes.c_int32
    lib.stencil_blocked_slices.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32]
    lib.stencil_blocked_slices.restype = ctypes.c_int32
    if path is None:
        _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = load().stencil_last_error().decode(errors="replace")
        raise StencilError(rc, msg)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _strides3(t):
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("fields must be 3D with contiguous x")
    return t.stride(1), t.stride(0)


def grid_struct(u0, u1, halo: int) -> _Grid:
    import torch
    for t in (u0, u1):
        if t.dtype != torch.float32 or not t.is_cuda:
            raise ValueError("fields must be float32 CUDA tensors")
    if u0.shape != u1.shape or _strides3(u0) != _strides3(u1):
        raise ValueError("u0 and u1 must have the same shape and strides")
    sy, sz = _strides3(u0)
    pz, py, px = u0.shape
    g = _Grid()
    g.nx, g.ny, g.nz, g.halo = px - 2 * halo, py - 2 * halo, pz - 2 * halo, halo
    g.sy, g.sz = sy, sz
    g.u[0], g.u[1] = _ptr(u0), _ptr(u1)
    return g


def coeff_struct(kind: int, ref, coef=None, w: Sequence[float] = (), alpha: float = 0.0) -> _Coeffs:
    import torch
    c = _Coeffs()
    c.dtype = F32
    c.arrays = None
    c.sk = 0
    if coef is not None:
        if coef.dim() != 4 or coef.stride(3) != 1:
            raise ValueError("coefficients must be (K, z, y, x) with contiguous x")
        if (coef.stride(2), coef.stride(1)) != _strides3(ref):
            raise ValueError("coefficient row/plane strides must match the fields")
        if coef.dtype == torch.bfloat16:
            c.dtype = BF16
        elif coef.dtype != torch.float32:
            raise ValueError("coefficients must be float32 or bfloat16")
        c.arrays = _ptr(coef)
        c.sk = coef.stride(0)
    ws = list(w) + [0.0] * (5 - len(w))
    for i in range(5):
        c.w[i] = float(ws[i])
    c.alpha = float(alpha)
    return c


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Context:
    """A library context: one scheme, tuning knobs, a borrowed HIP stream."""

    def __init__(self, scheme: int = NAIVE, *, dw: int = 0, zchunk: int = 0, ckpt_every: int = 0,
                 workspace_limit: int = 0, stream=None, xtile: int = 0):
        lib = load()
        t = _Tuning(dw, xtile, zchunk, ckpt_every, workspace_limit)
        h = ctypes.c_void_p()
        _check(lib.stencil_create(ctypes.byref(h), scheme, ctypes.byref(t),
                                  ctypes.c_void_p(_stream_handle(stream))))
        self._h = h
        self.scheme = scheme

    def close(self):
        if getattr(self, "_h", None):
            load().stencil_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def run(self, kind: int, u0, u1, nt: int, *, halo: int, coef=None, w=(), alpha: float = 0.0) -> int:
        """Advance nt steps in place; returns the slot (0 or 1) holding level nt."""
        g = grid_struct(u0, u1, halo)
        c = coeff_struct(kind, u0, coef, w, alpha)
        slot = ctypes.c_int(-1)
        _check(load().stencil_run(self._h, kind, ctypes.byref(g), ctypes.byref(c), int(nt),
                                  ctypes.byref(slot)))
        return slot.value

    def run_noalloc(self, kind: int, u0, u1, nt: int, *, halo: int, coef=None, w=(),
                    alpha: float = 0.0) -> int:
        """As run() on a BLOCKED context, allocating nothing (the library's
        static scratch holds the second frontier pair); see
        stencil_run_noalloc in include/stencil.h."""
        g = grid_struct(u0, u1, halo)
        c = coeff_struct(kind, u0, coef, w, alpha)
        slot = ctypes.c_int(-1)
        _check(load().stencil_run_noalloc(self._h, kind, ctypes.byref(g), ctypes.byref(c),
                                          int(nt), ctypes.byref(slot)))
        return slot.value

    def adjoint(self, u_prev, u0, nt: int, *, halo: int, coef, w, seed, grad_u0, grad_um1, grad_c):
        """Reverse time stepping of kind 5; see stencil_adjoint in include/stencil.h."""
        import torch
        g = grid_struct(u_prev, u0, halo)
        c = coeff_struct(KIND_25PT_WAVE_VARC, u0, coef, w, 0.0)
        for t in (seed, grad_u0, grad_um1):
            if t.dtype != torch.float32 or _strides3(t) != _strides3(u0) or t.shape != u0.shape:
                raise ValueError("adjoint fields must match the grid")
        if grad_c.dtype != torch.float64 or _strides3(grad_c) != _strides3(u0):
            raise ValueError("grad_c must be float64 with the grid's strides")
        _check(load().stencil_adjoint(self._h, KIND_25PT_WAVE_VARC, ctypes.byref(g), ctypes.byref(c),
                                      int(nt), _ptr(seed), _ptr(grad_u0), _ptr(grad_um1),
                                      _ptr(grad_c)))

    def adjoint_jacobi(self, kind: int, u0, u1, nt: int, *, halo: int, coef, seed, grad_u0,
                       grad_c):
        """Reverse time stepping of the Jacobi kinds 2 and 3; see stencil_adjoint
        in include/stencil.h.  (u0, u1) is the forward's grid (u0 holds level 0
        unless this context recorded the forward); grad_c is a float64
        (K, z, y, x) tensor with the coefficients' element strides."""
        import torch
        if kind not in (KIND_7PT_VAR, KIND_25PT_VAR):
            raise ValueError("adjoint_jacobi takes kinds 2 and 3")
        g = grid_struct(u0, u1, halo)
        c = coeff_struct(kind, u0, coef, (), 0.0)
        for t in (seed, grad_u0):
            if t.dtype != torch.float32 or _strides3(t) != _strides3(u0) or t.shape != u0.shape:
                raise ValueError("adjoint fields must match the grid")
        if (grad_c.dtype != torch.float64 or grad_c.shape != coef.shape or
                grad_c.stride() != coef.stride()):
            raise ValueError("grad_c must be float64 with the coefficients' shape and strides")
        _check(load().stencil_adjoint(self._h, kind, ctypes.byref(g), ctypes.byref(c), int(nt),
                                      _ptr(seed), _ptr(grad_u0), None, _ptr(grad_c)))

    def sync(self):
        _check(load().stencil_sync(self._h))


def default_dw(kind: int, n3=(0, 0, 0), coef_dtype: str = "f32") -> int:
    """Diamond width the blocked scheme uses for `kind` when none is given, on a
    grid of interior size n3 = (nx, ny, nz) with coefficients stored as
    ``coef_dtype`` ("f32" or "bf16"; ``stencil_default_dw``)."""
    if coef_dtype not in ("f32", "bf16"):
        raise ValueError(f"coef_dtype must be 'f32' or 'bf16', not {coef_dtype!r}")
    nx, ny, nz = (int(v) for v in n3)
    dw = load().stencil_default_dw(kind, nx, ny, nz, 1 if coef_dtype == "bf16" else 0)
    if dw <= 0:
        raise ValueError(load().stencil_last_error().decode(errors="replace"))
    return dw


def blocked_slices(kind: int, dw: int = 0, xtile: int = 0, nx: int = 1) -> int:
    """Workgroups sharing one diamond of the blocked scheme (``stencil_blocked_slices``):
    ceil(nx / slice width) for the radius-4 kinds, 1 for radius 1, 0 if not provided."""
    return int(load().stencil_blocked_slices(kind, dw, xtile, nx))


def plan_rows(kind: int, dw: int, ny: int, nt: int):
    """Diamond rows (r, t0, n_diamonds, first_centre) of the blocked scheme."""
    lib = load()
    n = lib.stencil_plan_rows(kind, dw, ny, nt, None, 0)
    if n < 0:
        raise ValueError("invalid plan arguments")
    buf = (ctypes.c_int64 * (4 * max(n, 1)))()
    lib.stencil_plan_rows(kind, dw, ny, nt, buf, n)
    return [tuple(buf[4 * i: 4 * i + 4]) for i in range(n)]


def field_like(t, halo: int):
    """A new aligned field (see alloc_field) holding a copy of the 3D field t."""
    pz, py, px = t.shape
    out = alloc_field((px - 2 * halo, py - 2 * halo, pz - 2 * halo), halo, dtype=t.dtype,
                      device=t.device)
    out.copy_(t)
    return out


def alloc_field(n3, halo: int, *, count: Optional[int] = None, dtype=None, device="cuda"):
    """Zeroed padded field(s) laid out for coalesced access.

    Returns a view of shape (nz+2h, ny+2h, nx+2h) -- or (count, ...) when
    ``count`` is given -- whose interior x = 0 sits on a 64-element boundary
    and whose row pitch is a multiple of 64 elements.
    """
    import torch
    dtype = dtype or torch.float32
    nx, ny, nz = n3
    lead = (64 - halo % 64) % 64
    pitch = -(-(lead + nx + 2 * halo) // 64) * 64
    py, pz = ny + 2 * halo, nz + 2 * halo
    plane = pitch * py
    vol = plane * pz
    k = 1 if count is None else count
    base = torch.zeros(k * vol + 64, dtype=dtype, device=device)
    if count is None:
        return base.as_strided((pz, py, nx + 2 * halo), (plane, pitch, 1), lead)
    return base.as_strided((k, pz, py, nx + 2 * halo), (vol, plane, pitch, 1), lead)
