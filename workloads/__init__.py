"""Seeded synthetic workloads for the stencil library and its oracle.

This module only draws and shapes input data.  It holds none of the stencil
arithmetic, so that both the GPU path and the CPU oracle can consume the very
same stored values without sharing any of the method's code.

Five workloads (sizes are the full ones; every generator takes a smaller
``n`` and ``nt`` for parity tests):

  1  7-point constant Jacobi (Fig. 1b), 64^3, halo 1, u0 ~ U[-1, 1],
     w = (0.4, 0.1), 10 steps.
  2  25-point 8th-order leapfrog, scalar alpha = 0.1 (Fig. 1e), 512^3, halo 4,
     u0 = u_{-1} = Gaussian blob (amplitude 1, sigma 8 cells, centred at the
     interior centre) + U[-1e-3, 1e-3] noise, 100 steps.
  3  7-point variable (Fig. 1c), 512^3, halo 1, u0 ~ U[-1, 1], 7 arrays
     U[0, 1] normalised per point to sum 0.99, 100 steps.
  4  25-point variable axis-symmetric (Fig. 1d), 480^3, halo 4,
     u0 ~ U[-1, 1], 13 arrays U[0, 1] scaled per point so that the effective
     row sum W0 + 2*sum_{k>=1} Wk is 0.99; FP32 or BF16 (round to nearest
     even) coefficient storage; 100 steps.
  5  leapfrog with alpha = c(x) = 0.08*(1 + 0.3*s), s a Gaussian-filtered
     (sigma 6 cells, periodic, truncate 4) N(0, 1) field scaled to max|s| = 1;
     256^3, halo 4, u0 = u_{-1} = blob + noise as in 2; target d ~ U[-1, 1];
     loss 0.5*||u_T - d||^2; 200 steps, checkpoint interval 14.

Random streams: numpy PCG64 seeded with [1410, workload, array id], drawn in
float64 and stored as float32 (BF16 by rounding the float32 value).  Every
boundary shell is zero.  Fields are numpy arrays of shape (nz+2h, ny+2h,
nx+2h), x fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 1410

# (kind, n, halo, nt) of the five workloads at full size
FULL = {
    1: dict(kind=1, n=64, halo=1, nt=10),
    2: dict(kind=4, n=512, halo=4, nt=100),
    3: dict(kind=2, n=512, halo=1, nt=100),
    4: dict(kind=3, n=480, halo=4, nt=100),
    5: dict(kind=5, n=256, halo=4, nt=200),
}
NAMES = {
    1: "7pt-const-jacobi-64^3-nt10",
    2: "25pt-leapfrog-const-512^3-nt100",
    3: "7pt-var-512^3-nt100",
    4: "25pt-var-480^3-nt100",
    5: "25pt-leapfrog-varc-256^3-nt200-adjoint",
}
CKPT_EVERY = 14


def rng(workload: int, array_id: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, workload, array_id])


def _padded(n3, h, dtype=np.float32):
    nx, ny, nz = n3
    return np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h), dtype=dtype)


def _inner(a, h):
    return a[..., h:a.shape[-3] - h, h:a.shape[-2] - h, h:a.shape[-1] - h]


def _shape3(n):
    if isinstance(n, int):
        return (n, n, n)
    nx, ny, nz = n
    return (int(nx), int(ny), int(nz))


def uniform_field(workload, array_id, n3, h, lo=-1.0, hi=1.0):
    nx, ny, nz = n3
    a = _padded(n3, h)
    _inner(a, h)[...] = rng(workload, array_id).uniform(lo, hi, size=(nz, ny, nx))
    return a


def blob_field(workload, array_id, n3, h, sigma=8.0, noise=1e-3):
    """Gaussian blob of amplitude 1 at the interior centre plus uniform noise."""
    nx, ny, nz = n3
    z = np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0
    y = np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0
    x = np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0
    gz = np.exp(-z * z / (2 * sigma * sigma))[:, None, None]
    gy = np.exp(-y * y / (2 * sigma * sigma))[None, :, None]
    gx = np.exp(-x * x / (2 * sigma * sigma))[None, None, :]
    a = _padded(n3, h)
    g = rng(workload, array_id)
    blk = 64  # fill z-slabs to bound the float64 temporaries
    inner = _inner(a, h)
    for z0 in range(0, nz, blk):
        z1 = min(nz, z0 + blk)
        v = gz[z0:z1] * gy * gx + g.uniform(-noise, noise, size=(z1 - z0, ny, nx))
        inner[z0:z1] = v
    return a


def to_bf16_bits(a32: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (nearest, ties to even); returns uint16 bits."""
    b = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    lsb = (b >> 16) & 1
    r = (b + np.uint32(0x7FFF) + lsb) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def normalised_coefficients(workload, K, n3, h, row_sum, pair_weight):
    """K arrays U[0, 1], scaled per point so that
    pair_weight[0]*W0 + sum_k pair_weight[k]*Wk == row_sum (in float64),
    then stored as float32.  Drawn twice (sum pass, scale pass) to bound memory."""
    nx, ny, nz = n3
    total = np.zeros((nz, ny, nx), dtype=np.float64)
    for k in range(K):
        total += pair_weight[k] * rng(workload, 1 + k).uniform(0.0, 1.0, size=(nz, ny, nx))
    scale = row_sum / total
    del total
    out = np.zeros((K,) + (nz + 2 * h, ny + 2 * h, nx + 2 * h), dtype=np.float32)
    for k in range(K):
        v = rng(workload, 1 + k).uniform(0.0, 1.0, size=(nz, ny, nx))
        _inner(out[k], h)[...] = v * scale
    return out


def smooth_coefficient(workload, array_id, n3, h, base=0.08, amp=0.3, sigma=6.0):
    from scipy.ndimage import gaussian_filter
    nx, ny, nz = n3
    s = rng(workload, array_id).standard_normal(size=(nz, ny, nx))
    s = gaussian_filter(s, sigma=sigma, mode="wrap", truncate=4.0)
    s /= np.abs(s).max()
    a = _padded(n3, h)
    _inner(a, h)[...] = base * (1.0 + amp * s)
    return a


@dataclasses.dataclass
class Workload:
    """One seeded instance.  Arrays are numpy, padded, float32 unless noted."""
    index: int
    kind: int
    n3: tuple
    halo: int
    nt: int
    u0: np.ndarray                    # level 0
    u_prev: Optional[np.ndarray]      # level -1 (leapfrog kinds)
    coef: Optional[np.ndarray]        # (K, ...) float32 values as stored
    coef_bf16: Optional[np.ndarray]   # (K, ...) uint16 bits, if BF16 storage
    w: tuple                          # scalar weights (kind 1: w0, w1; leapfrog: none)
    alpha: float                      # scalar alpha (kind 4)
    target: Optional[np.ndarray]      # d for the workload-5 loss
    name: str

    @property
    def lups(self) -> int:
        nx, ny, nz = self.n3
        return nx * ny * nz * self.nt

    def coef_values_f32(self):
        """The coefficient values the stencil actually sees, as float32."""
        if self.coef_bf16 is not None:
            return bf16_bits_to_f32(self.coef_bf16)
        return self.coef


def make(index: int, n=None, nt: Optional[int] = None, coef_dtype: str = "f32") -> Workload:
    spec = FULL[index]
    n3 = _shape3(spec["n"] if n is None else n)
    h = spec["halo"]
    nt = spec["nt"] if nt is None else int(nt)
    kind = spec["kind"]
    u_prev = coef = bf = target = None
    w = ()
    alpha = 0.0
    if index == 1:
        u0 = uniform_field(1, 0, n3, h)
        w = (0.4, 0.1)
    elif index == 2:
        u0 = blob_field(2, 0, n3, h)
        u_prev = u0.copy()
        alpha = 0.1
    elif index == 3:
        u0 = uniform_field(3, 0, n3, h)
        coef = normalised_coefficients(3, 7, n3, h, 0.99, [1.0] * 7)
    elif index == 4:
        u0 = uniform_field(4, 0, n3, h)
        coef = normalised_coefficients(4, 13, n3, h, 0.99, [1.0] + [2.0] * 12)
    elif index == 5:
        u0 = blob_field(5, 0, n3, h)
        u_prev = u0.copy()
        coef = smooth_coefficient(5, 1, n3, h)[None]
        target = uniform_field(5, 2, n3, h)
    else:
        raise ValueError(index)
    if coef_dtype == "bf16":
        if coef is None or index not in (3, 4, 5):
            raise ValueError("BF16 storage applies to variable-coefficient workloads")
        bf = to_bf16_bits(coef)
    elif coef_dtype != "f32":
        raise ValueError(coef_dtype)
    return Workload(index=index, kind=kind, n3=n3, halo=h, nt=nt, u0=u0, u_prev=u_prev,
                    coef=coef, coef_bf16=bf, w=w, alpha=alpha, target=target,
                    name=NAMES[index])


def ckpt_interval(nt: int) -> int:
    """Checkpoint interval ~ sqrt(nt) (14 for 200 steps)."""
    return max(1, int(round(math.sqrt(nt))))
