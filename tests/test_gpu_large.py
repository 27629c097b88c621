"""Fields larger than 2 GiB: the blocked kernel addresses each z-chunk through
a window of 32-bit offsets from a base of its own, so it must still equal the
naive sweep bit for bit (FP32 and BF16 coefficients, radius 1 and 4; the
BF16 cases of radius 4 take the word-aligned coefficient loads)."""
import pytest

import paper_1410_3060_amd as st

pytestmark = pytest.mark.gpu


def inputs(kind, n3, h, coef_dtype):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1410 + kind)
    inner = (slice(h, -h),) * 3
    a = st.alloc_field(n3, h)
    a[inner].uniform_(-1.0, 1.0, generator=gen)
    b = st.alloc_field(n3, h)
    if kind in st.LEAPFROG:
        b.copy_(a)
    K = st.NCOEF[kind]
    dt = torch.bfloat16 if coef_dtype == "bf16" else torch.float32
    cf = st.alloc_field(n3, h, count=K, dtype=dt)
    scale = 0.05 if kind in st.LEAPFROG else 0.99 / K
    for k in range(K):
        cf[k].copy_(torch.empty(cf.shape[1:], device="cuda").uniform_(0.0, scale, generator=gen).to(dt))
    return a, b, cf


@pytest.mark.parametrize("kind,n3,nt,coef_dtype", [(2, (1000, 1000, 560), 7, "f32"),
                                                    (2, (1000, 1000, 560), 4, "bf16"),
                                                    (5, (832, 832, 800), 5, "f32"),
                                                    (3, (832, 832, 800), 3, "bf16"),
                                                    (5, (832, 832, 800), 4, "bf16")])
def test_blocked_beyond_2gib(kind, n3, nt, coef_dtype):
    import torch
    h = st.RADIUS[kind]
    a0, b0, cf = inputs(kind, n3, h, coef_dtype)
    span = (a0.shape[0] - 1) * a0.stride(0) + (a0.shape[1] - 1) * a0.stride(1) + a0.shape[2]
    assert span * 4 > 2 ** 31
    w = st.L8_WEIGHTS if kind in st.LEAPFROG else ()
    out = {}
    for scheme in (st.NAIVE, st.BLOCKED):
        a, b = st.field_like(a0, h), st.field_like(b0, h)
        with st.Context(scheme) as ctx:
            slot = ctx.run(kind, a, b, nt, halo=h, coef=cf, w=w)
            ctx.sync()
        out[scheme] = ((a, b)[slot], (a, b)[1 - slot])
    assert torch.equal(out[st.NAIVE][0], out[st.BLOCKED][0]), "level nt differs"
    if kind in st.LEAPFROG:
        assert torch.equal(out[st.NAIVE][1], out[st.BLOCKED][1]), "level nt-1 differs"
