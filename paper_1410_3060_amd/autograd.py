"""torch.autograd bindings of the stencils that have an adjoint.

``wave_varc(u_prev, u0, c, nt)`` returns u_nt of
    u_{n+1} = 2 u_n - u_{n-1} + c * L8(u_n)        (Fig. 1e, alpha = c(x));
``jacobi_var(u0, coef, nt, kind=2|3)`` returns u_nt of u_{t+1} = A(W) u_t
(Fig. 1c, 1d).  Both are computed by libstencil.so; their backward runs the
library's adjoint (reverse time stepping from checkpoints recorded during the
forward, every ``ckpt_every`` steps -- about sqrt(nt) by default -- with
recomputation in between; 1 records every level) and returns the gradients
with respect to the initial state and the coefficients.  The coefficient
gradient is accumulated in FP64; autograd returns it in the coefficients'
dtype, and the FP64 arrays themselves are handed to a caller-supplied dict
(``grad_c64``).  Only the marshalling lives here.

The boundary shell of the fields is a fixed Dirichlet boundary: gradients
with respect to shell entries are reported as zero.
"""
from __future__ import annotations

import math

import torch

from . import (BLOCKED, KIND_7PT_VAR, KIND_25PT_VAR, KIND_25PT_WAVE_VARC, L8_WEIGHTS, NAIVE,
               Context, alloc_field)


def _default_k(nt, ckpt_every):
    """Checkpoint interval: the caller's, else about sqrt(nt) (the library
    recomputes each segment of the forward in the backward).  1 records every
    level: no recomputation, nt + 1 fields of workspace, and the recording
    forward is the naive sweep whatever the scheme."""
    if ckpt_every > 0:
        return ckpt_every
    return max(1, int(round(math.sqrt(max(nt, 1)))))


def _aligned_copy(t, halo):
    pz, py, px = t.shape[-3:]
    out = alloc_field((px - 2 * halo, py - 2 * halo, pz - 2 * halo), halo)
    out.copy_(t.reshape(pz, py, px))
    return out


class WaveFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_prev, u0, c, nt: int, halo: int, ckpt_every: int, scheme: int,
                grad_c64):
        if not (u_prev.is_cuda and u0.is_cuda and c.is_cuda):
            raise ValueError("wave_varc needs CUDA tensors")
        k = _default_k(nt, ckpt_every)
        a = _aligned_copy(u_prev.detach().float(), halo)
        b = _aligned_copy(u0.detach().float(), halo)
        cc = _aligned_copy(c.detach().float(), halo)
        c4 = cc.unsqueeze(0)
        sctx = Context(scheme, ckpt_every=k)
        slot = sctx.run(KIND_25PT_WAVE_VARC, a, b, nt, halo=halo, coef=c4, w=L8_WEIGHTS)
        out = (a, b)[slot]
        # the initial state, for a backward without a usable recording
        ctx.sctx = sctx
        ctx.nt, ctx.halo = nt, halo
        ctx.c4 = c4
        ctx.init = (_aligned_copy(u_prev.detach().float(), halo),
                    _aligned_copy(u0.detach().float(), halo))
        ctx.shape = u0.shape
        ctx.c_dtype = c.dtype
        ctx.c_shape = c.shape
        ctx.grad_c64 = grad_c64
        return out.clone().reshape(u0.shape)

    @staticmethod
    def backward(ctx, grad_out):
        halo = ctx.halo
        seed = _aligned_copy(grad_out.detach().float(), halo)
        # the boundary shell is not a state variable: its seed is dropped
        shell = torch.ones_like(seed, dtype=torch.bool)
        shell[halo:seed.shape[0] - halo, halo:seed.shape[1] - halo, halo:seed.shape[2] - halo] = False
        seed.masked_fill_(shell, 0.0)
        n3 = (seed.shape[2] - 2 * halo, seed.shape[1] - 2 * halo, seed.shape[0] - 2 * halo)
        g0 = alloc_field(n3, halo)
        gm1 = alloc_field(n3, halo)
        gc = alloc_field(n3, halo, dtype=torch.float64)
        up, u0 = ctx.init
        ctx.sctx.adjoint(up, u0, ctx.nt, halo=halo, coef=ctx.c4, w=L8_WEIGHTS, seed=seed,
                         grad_u0=g0, grad_um1=gm1, grad_c=gc)
        ctx.sctx.close()
        if ctx.grad_c64 is not None:
            ctx.grad_c64["grad_c"] = gc.reshape(ctx.c_shape)
        gc_out = gc.to(ctx.c_dtype).reshape(ctx.c_shape)
        return (gm1.clone().reshape(ctx.shape), g0.clone().reshape(ctx.shape), gc_out, None, None,
                None, None, None)


def wave_varc(u_prev, u0, c, nt: int, *, halo: int = 4, ckpt_every: int = 0,
              scheme: int = NAIVE, grad_c64=None):
    """u_nt of the leapfrog with c(x); differentiable in u_prev, u0 and c.

    Fields are (nz+2h, ny+2h, nx+2h) CUDA tensors (padded, x fastest).  Pass
    the same tensor as u_prev and u0 for a start from rest; autograd then adds
    the two gradients.  ``scheme`` is NAIVE or BLOCKED for the forward (with
    ``ckpt_every`` = 1 the recording forward is the naive sweep either way).
    ``ckpt_every`` = 0 checkpoints every ~sqrt(nt) steps.  The gradient of c
    comes back in c's dtype; if ``grad_c64`` is a dict, the backward also
    stores the FP64 accumulation there under "grad_c".
    """
    if scheme not in (NAIVE, BLOCKED):
        raise ValueError("scheme must be NAIVE or BLOCKED")
    return WaveFunction.apply(u_prev, u0, c, int(nt), int(halo), int(ckpt_every), int(scheme),
                              grad_c64)


class JacobiFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, coef, nt: int, kind: int, halo: int, ckpt_every: int, scheme: int,
                grad_c64):
        if not (u0.is_cuda and coef.is_cuda):
            raise ValueError("jacobi_var needs CUDA tensors")
        K = coef.shape[0]
        pz, py, px = u0.shape
        n3 = (px - 2 * halo, py - 2 * halo, pz - 2 * halo)
        a = _aligned_copy(u0.detach().float(), halo)
        b = _aligned_copy(u0.detach().float(), halo)
        cdt = torch.bfloat16 if coef.dtype == torch.bfloat16 else torch.float32
        cf = alloc_field(n3, halo, count=K, dtype=cdt)
        cf.copy_(coef.detach().to(cdt))
        sctx = Context(scheme, ckpt_every=_default_k(nt, ckpt_every))
        slot = sctx.run(kind, a, b, nt, halo=halo, coef=cf)
        out = (a, b)[slot].clone().reshape(u0.shape)
        ctx.sctx, ctx.nt, ctx.kind, ctx.halo, ctx.cf, ctx.n3 = sctx, nt, kind, halo, cf, n3
        # the initial state, for a backward without a usable recording
        ctx.init = (_aligned_copy(u0.detach().float(), halo), _aligned_copy(u0.detach().float(), halo))
        ctx.shape, ctx.c_dtype, ctx.c_shape = u0.shape, coef.dtype, coef.shape
        ctx.grad_c64 = grad_c64
        return out

    @staticmethod
    def backward(ctx, grad_out):
        halo = ctx.halo
        seed = _aligned_copy(grad_out.detach().float(), halo)
        # the boundary shell is not a state variable: its seed is dropped
        shell = torch.ones_like(seed, dtype=torch.bool)
        shell[halo:seed.shape[0] - halo, halo:seed.shape[1] - halo, halo:seed.shape[2] - halo] = False
        seed.masked_fill_(shell, 0.0)
        g0 = alloc_field(ctx.n3, halo)
        gc = alloc_field(ctx.n3, halo, count=ctx.cf.shape[0], dtype=torch.float64)
        a, b = ctx.init
        ctx.sctx.adjoint_jacobi(ctx.kind, a, b, ctx.nt, halo=halo, coef=ctx.cf, seed=seed,
                                grad_u0=g0, grad_c=gc)
        ctx.sctx.close()
        if ctx.grad_c64 is not None:
            ctx.grad_c64["grad_c"] = gc.reshape(ctx.c_shape)
        return (g0.clone().reshape(ctx.shape), gc.to(ctx.c_dtype).reshape(ctx.c_shape), None, None,
                None, None, None, None)


def jacobi_var(u0, coef, nt: int, *, kind: int, halo: int = 0, ckpt_every: int = 0,
               scheme: int = NAIVE, grad_c64=None):
    """u_nt of the variable-coefficient Jacobi stencil of Fig. 1c (kind 2, K = 7)
    or Fig. 1d (kind 3, K = 13); differentiable in u0 and coef.

    u0 is a (nz+2h, ny+2h, nx+2h) CUDA tensor, coef (K, nz+2h, ny+2h, nx+2h)
    float32 or bfloat16 (BF16 is differentiated at its FP32 expansion; the
    gradient is returned in the coefficients' dtype; ``grad_c64`` receives the
    FP64 accumulation as for ``wave_varc``).  halo defaults to the stencil
    radius; ``ckpt_every`` and ``scheme`` as for ``wave_varc``.
    """
    if kind not in (KIND_7PT_VAR, KIND_25PT_VAR):
        raise ValueError("kind must be 2 or 3")
    if scheme not in (NAIVE, BLOCKED):
        raise ValueError("scheme must be NAIVE or BLOCKED")
    h = halo if halo > 0 else (1 if kind == KIND_7PT_VAR else 4)
    return JacobiFunction.apply(u0, coef, int(nt), int(kind), int(h), int(ckpt_every), int(scheme),
                                grad_c64)
