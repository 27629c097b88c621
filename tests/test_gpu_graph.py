"""stencil_run captured into a HIP graph (through torch.cuda.graph on the
context's stream): a run makes only kernel launches and device copies once
the context has run once, so its replays must equal the eager run bit for
bit.  Each replay is checked, with eager work and synchronisations between
the replays."""
import pytest

import paper_1410_3060_amd as st
from paper_1410_3060_amd import tune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,n3,nt,scheme", [(1, (64, 64, 64), 10, st.NAIVE),
                                               (2, (70, 41, 29), 9, st.BLOCKED),
                                               (3, (66, 37, 21), 5, st.BLOCKED)])
def test_run_graph_replays_match_eager(kind, n3, nt, scheme):
    import torch
    h = st.RADIUS[kind]
    a0, b0, cf = tune._inputs(kind, n3, h, "f32", 1410)
    w, alpha = tune._weights(kind)
    side = torch.cuda.Stream()
    a, b = st.field_like(a0, h), st.field_like(b0, h)
    with torch.cuda.stream(side):
        ctx = st.Context(scheme, stream=side)
        # eager reference (also allocates the context's workspace)
        slot = ctx.run(kind, a, b, nt, halo=h, coef=cf, w=w, alpha=alpha)
        ctx.sync()
        want = (a, b)[slot].clone()
        g = torch.cuda.CUDAGraph()
        a.copy_(a0)
        b.copy_(b0)
        side.synchronize()
        with torch.cuda.graph(g, stream=side):
            ctx.run(kind, a, b, nt, halo=h, coef=cf, w=w, alpha=alpha)
    for i in range(3):
        a.copy_(a0)
        b.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal((a, b)[slot], want), f"replay {i}"
        # eager work between replays
        other = st.field_like(a0, h)
        other.mul_(2.0)
        torch.cuda.synchronize()
    ctx.close()
