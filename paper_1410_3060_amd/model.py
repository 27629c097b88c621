"""Traffic and capacity models used to read the measurements.

Host-side arithmetic only (no device code):

* algorithmic bytes per lattice-site update of the naive sweep (the code
  balance of Sect. 3.3, with or without the write-allocate transfer of a CPU
  cache) and of the blocked scheme (one diamond per (x, z) column);
* the wavefront width and the cache-block size of a wavefront diamond block
  (Sect. 5.3), which on the GPU is the on-chip state (registers + LDS) one
  workgroup needs to keep every coefficient and level of its diamond resident.
"""
from __future__ import annotations

RADIUS = {1: 1, 2: 1, 3: 4, 4: 4, 5: 4}
NCOEF = {1: 0, 2: 7, 3: 13, 4: 0, 5: 1}
LEAPFROG = {1: False, 2: False, 3: False, 4: True, 5: True}


def naive_code_balance(kind: int, value_bytes: int = 4, coef_bytes: int | None = None,
                       write_allocate: bool = False) -> float:
    """Bytes per update of one sweep with ideal spatial blocking (every value
    read from memory once per sweep).

    Jacobi kinds read the old level and write the new one into a second array
    (plus a write-allocate read of that array on a cache-based CPU); the
    leapfrog kinds read u_n and u_{n-1} and overwrite u_{n-1} in place, so
    there is no write-allocate transfer.  Coefficient arrays are read once.
    """
    cb = value_bytes if coef_bytes is None else coef_bytes
    if LEAPFROG[kind]:
        fields = 3 * value_bytes
    else:
        fields = (3 if write_allocate else 2) * value_bytes
    return float(fields + NCOEF[kind] * cb)


def blocked_bytes_per_lup(kind: int, dw: int, value_bytes: int = 4,
                          coef_bytes: int | None = None) -> float:
    """Bytes per update of the blocked scheme, per diamond and (x, z) column:
    the old two-level frontier read on dw + 2R cells, the coefficients on dw
    cells, the new frontier written on dw cells, for dw * H updates."""
    R = RADIUS[kind]
    H = dw // (2 * R)
    cb = value_bytes if coef_bytes is None else coef_bytes
    read = 2 * (dw + 2 * R) * value_bytes
    coef = NCOEF[kind] * dw * cb
    write = 2 * dw * value_bytes
    return (read + coef + write) / float(dw * H)


def wavefront_width(R: int, dw: int, n_f: int) -> int:
    """Wavefront width W_w (Sect. 5.3): dw + N_F - 1 for R = 1, in general
    dw - 2R + N_F + 1."""
    return dw - 2 * R + n_f + 1


def cache_block_bytes(R: int, dw: int, n_f: int, n_d: int, n_xb: int) -> int:
    """Cache block of one wavefront diamond (Sect. 5.3): N_D streams over the
    diamond's area in the y-z plane plus the perimeter of the enclosing
    rectangle (2R wide), times the bytes of the untiled x extent N_xb."""
    w = wavefront_width(R, dw, n_f)
    if R == 1:
        area = dw * dw // 2 + dw * n_f
        return n_xb * (n_d * area + 2 * (dw + w))
    return n_xb * (n_d * dw * (dw // 2 - R + n_f + 1) + 2 * R * (dw + w))
