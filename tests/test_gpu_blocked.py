"""GPU parity of the temporally blocked scheme.

The blocked scheme reorders the naive updates (diamond rows, wavefront along
z) but evaluates every point with the same FMA order, so it must equal the
naive scheme bit for bit -- on every interior point and without touching the
boundary shell -- and both must match the FP64 oracle.  Cases cover both
parities of the number of diamond rows, nt below, at and above the diamond
half-height H, odd sizes with ragged x/y/z tiles, forced small z-chunks (so
overlapping workgroups recompute halos) and BF16 coefficients."""
import numpy as np
import pytest

import paper_1410_3060_amd as st
import workloads

from gpu_util import coef_to_dev, from_dev, gpu_weights, max_rel, rel_l2, run_gpu, run_oracle, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5
SIZES = {1: (150, 45, 23), 2: (70, 37, 19), 3: (130, 41, 29), 4: (131, 39, 26), 5: (97, 35, 27)}
# diamond widths per workload: R = 1 for workloads 1 and 3, R = 4 for 2, 4 and 5
DWS = {1: [8, 4, 12], 2: [32, 24, 16], 3: [8, 4, 12, 10, 6], 4: [16, 24], 5: [16, 24, 32]}


def both(wl, dw, nt, **kw):
    nb, nb_prev = run_gpu(wl, st.NAIVE, nt=nt)
    bl, bl_prev = run_gpu(wl, st.BLOCKED, nt=nt, dw=dw, **kw)
    return nb, nb_prev, bl, bl_prev


def assert_bitwise(a, b, what):
    if not np.array_equal(a, b):
        d = np.argwhere(a != b)
        raise AssertionError(f"{what}: {len(d)} points differ, first at (z,y,x)={tuple(d[0])}: "
                             f"{a[tuple(d[0])]!r} vs {b[tuple(d[0])]!r}")


@pytest.mark.parametrize("index", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nt", [1, 2, 3, 4, 5, 9])
def test_blocked_equals_naive_bitwise(index, nt):
    wl = workloads.make(index, n=SIZES[index], nt=nt)
    dw = DWS[index][0]
    nb, nb_prev, bl, bl_prev = both(wl, dw, nt, zchunk=9)
    assert_bitwise(bl, nb, f"workload {index} dw {dw} nt {nt}")
    if nb_prev is not None:
        assert_bitwise(bl_prev, nb_prev, f"workload {index} dw {dw} nt {nt} (level nt-1)")


@pytest.mark.parametrize("index", [1, 3])
@pytest.mark.parametrize("dw", [4, 6, 10, 12])
def test_blocked_other_diamond_widths(index, dw):
    for nt in (5, 6, 13):
        wl = workloads.make(index, n=SIZES[index], nt=nt)
        nb, _, bl, _ = both(wl, dw, nt)
        assert_bitwise(bl, nb, f"workload {index} dw {dw} nt {nt}")


@pytest.mark.parametrize("index", [1, 2, 3, 4, 5])
def test_blocked_matches_oracle(index):
    wl = workloads.make(index, n=SIZES[index], nt=10)
    got, got_prev = run_gpu(wl, st.BLOCKED, dw=DWS[index][0])
    want, want_prev = run_oracle(wl)
    for g, w in ((got, want), (got_prev, want_prev)):
        if g is None:
            continue
        e2, em = rel_l2(g, w, wl.halo), max_rel(g, w, wl.halo)
        print(f"workload {index}: blocked rel-L2 {e2:.3e} max-rel {em:.3e}")
        assert e2 <= TOL and em <= TOL


@pytest.mark.parametrize("index", [3, 4, 5])
def test_blocked_bf16_bitwise(index):
    for dw in DWS[index]:
        wl = workloads.make(index, n=SIZES[index], nt=7, coef_dtype="bf16")
        nb, nb_prev, bl, bl_prev = both(wl, dw, 7, zchunk=13)
        assert_bitwise(bl, nb, f"workload {index} bf16 dw {dw}")


@pytest.mark.parametrize("index", [2, 4, 5])
@pytest.mark.parametrize("nt", [3, 6, 9])
def test_blocked_radius4_every_width_zchunks(index, nt):
    """Every provided width of the radius-4 stencils (16-column slices at
    H = 3 of the 25-point variable stencil, 32-column slices elsewhere) with
    forced small z-chunks."""
    for dw in DWS[index][1:]:
        wl = workloads.make(index, n=SIZES[index], nt=nt)
        nb, nb_prev, bl, bl_prev = both(wl, dw, nt, zchunk=9)
        assert_bitwise(bl, nb, f"workload {index} dw {dw} nt {nt}")
        if nb_prev is not None:
            assert_bitwise(bl_prev, nb_prev, f"workload {index} dw {dw} nt {nt} (level nt-1)")


@pytest.mark.parametrize("index", [1, 4])
def test_blocked_contiguous_layout(index):
    wl = workloads.make(index, n=(77, 50, 33), nt=6)
    nb, _ = run_gpu(wl, st.NAIVE, aligned=False)
    bl, _ = run_gpu(wl, st.BLOCKED, aligned=False, dw=DWS[index][0])
    assert_bitwise(bl, nb, f"workload {index} contiguous")


@pytest.mark.parametrize("index", [3, 4, 5])
def test_blocked_bf16_unaligned_coefficients(index):
    """BF16 coefficient arrays that do not all start on 4-byte boundaries
    (odd plane and array strides of a contiguous layout, and a base 2 bytes
    past an allocation) take the general loads; aligned arrays of the 25-point
    and leapfrog kinds take word loads and a per-column selector.  All three equal the naive scheme bit for
    bit."""
    import torch
    wl = workloads.make(index, n=(77, 51, 33), nt=6, coef_dtype="bf16")
    h = wl.halo
    assert ((77 + 2 * h) * (51 + 2 * h)) % 2 == 1  # odd sz and sk
    dw = DWS[index][0]
    ref, _ = run_gpu(wl, st.NAIVE)
    outs = {"aligned": run_gpu(wl, st.BLOCKED, dw=dw)[0],
            "contiguous": run_gpu(wl, st.BLOCKED, aligned=False, dw=dw)[0]}
    # the same arrays 2 bytes past a 256-byte aligned allocation
    cf = coef_to_dev(wl, aligned=False)
    buf = torch.empty(cf.numel() + 1, dtype=cf.dtype, device="cuda")
    shifted = buf[1:].view(cf.shape)
    shifted.copy_(cf)
    assert shifted.data_ptr() % 4 == 2
    a = to_dev(wl.u_prev if index == 5 else wl.u0, h, False)
    b = to_dev(wl.u0 if index == 5 else np.zeros_like(wl.u0), h, False)
    with st.Context(st.BLOCKED, dw=dw) as ctx:
        slot = ctx.run(wl.kind, a, b, 6, halo=h, coef=shifted, w=gpu_weights(wl), alpha=wl.alpha)
        ctx.sync()
    outs["shifted base"] = from_dev((a, b)[slot])
    for what, got in outs.items():
        assert_bitwise(got, ref, f"workload {index} bf16 {what}")


def test_blocked_thin_and_tiny():
    for n in [(1, 1, 1), (3, 70, 2), (64, 8, 1), (200, 3, 5)]:
        wl = workloads.make(3, n=n, nt=5)
        nb, _ = run_gpu(wl, st.NAIVE)
        bl, _ = run_gpu(wl, st.BLOCKED, dw=8)
        assert_bitwise(bl, nb, f"7pt var n={n}")


@pytest.mark.parametrize("index", [2, 4, 5])
def test_blocked_radius4_other_widths_and_shapes(index):
    """The multi-workgroup diamonds of the radius-4 stencils at every provided
    width, on one slice (nx <= 16), many slices with a ragged last one, thin
    grids and nt around the diamond half-heights."""
    shapes = [(16, 30, 21), (9, 11, 40), (53, 7, 3), (1, 1, 1), (40, 66, 9)]
    for dw in DWS[index]:
        for n3 in shapes:
            for nt in (2, 7):
                print(f"workload {index} dw {dw} n {n3} nt {nt}", flush=True)
                wl = workloads.make(index, n=n3, nt=nt)
                nb, nb_prev, bl, bl_prev = both(wl, dw, nt)
                assert_bitwise(bl, nb, f"workload {index} dw {dw} n {n3} nt {nt}")
                if nb_prev is not None:
                    assert_bitwise(bl_prev, nb_prev, f"workload {index} dw {dw} n {n3} nt {nt} prev")


@pytest.mark.parametrize("index", [2, 4, 5])
def test_blocked_radius4_slice_widths(index):
    """Both slice widths (16 and 32 columns per workgroup, i.e. the
    workgroups that share a diamond) at every provided diamond width, several
    slices with a ragged last one, bit-identical to the naive scheme."""
    n3 = (77, 30, 21)
    for dw in DWS[index]:
        for xtile in (16, 32):
            if st.blocked_slices(workloads.FULL[index]["kind"], dw, xtile, n3[0]) == 0:
                continue
            for nt in (3, 7):
                wl = workloads.make(index, n=n3, nt=nt)
                nb, nb_prev, bl, bl_prev = both(wl, dw, nt, xtile=xtile)
                assert_bitwise(bl, nb, f"workload {index} dw {dw} xtile {xtile} nt {nt}")
                if nb_prev is not None:
                    assert_bitwise(bl_prev, nb_prev, f"workload {index} dw {dw} xtile {xtile} prev")


def test_blocked_radius4_seeded_random_cases():
    """Seeded random configurations of the radius-4 kernel: shape (1..90 per
    axis), nt 1..9, every provided width and slice width, FP32 or BF16
    coefficients, default or forced z-chunks; each bit-identical to naive."""
    rng = np.random.default_rng([1410, 3060, 7])
    kinds = {2: 4, 4: 3, 5: 5}
    done = 0
    while done < 24:
        index = int(rng.choice([2, 4, 5]))
        dw = int(rng.choice(DWS[index]))
        xtile = int(rng.choice([0, 16, 32]))
        n3 = tuple(int(v) for v in rng.integers(1, 91, size=3))
        if st.blocked_slices(kinds[index], dw, xtile, n3[0]) == 0:
            continue
        nt = int(rng.integers(1, 10))
        dtype = "bf16" if index != 2 and rng.random() < 0.4 else "f32"
        zchunk = int(rng.choice([0, 5, 17]))
        what = f"workload {index} dw {dw} xtile {xtile} n {n3} nt {nt} {dtype} zchunk {zchunk}"
        print(what, flush=True)
        wl = workloads.make(index, n=n3, nt=nt, coef_dtype=dtype)
        nb, nb_prev, bl, bl_prev = both(wl, dw, nt, xtile=xtile, zchunk=zchunk)
        assert_bitwise(bl, nb, what)
        if nb_prev is not None:
            assert_bitwise(bl_prev, nb_prev, what + " prev")
        done += 1


def test_blocked_radius1_seeded_random_cases():
    """Seeded random configurations of the radius-1 kernel: shape (x up to 200
    so that interior x-tiles occur beside boundary ones, y up to 60, z up to
    90 so that the steady-state steps occur in some z-chunks and not in
    others), nt 1..13, every provided width, FP32 or BF16 coefficients for the
    variable stencil, padded or contiguous layout, default or forced
    z-chunks; each bit-identical to naive."""
    rng = np.random.default_rng([1410, 3060, 1])
    for _ in range(24):
        index = int(rng.choice([1, 3]))
        dw = int(rng.choice([4, 6, 8, 10, 12]))
        n3 = (int(rng.integers(1, 201)), int(rng.integers(1, 61)), int(rng.integers(1, 91)))
        nt = int(rng.integers(1, 14))
        dtype = "bf16" if index == 3 and rng.random() < 0.4 else "f32"
        aligned = bool(rng.random() < 0.7)
        zchunk = int(rng.choice([0, 5, 17, 40]))
        what = (f"workload {index} dw {dw} n {n3} nt {nt} {dtype} "
                f"{'padded' if aligned else 'contiguous'} zchunk {zchunk}")
        print(what, flush=True)
        wl = workloads.make(index, n=n3, nt=nt, coef_dtype=dtype)
        nb, _ = run_gpu(wl, st.NAIVE, nt=nt, aligned=aligned)
        bl, _ = run_gpu(wl, st.BLOCKED, nt=nt, aligned=aligned, dw=dw, zchunk=zchunk)
        assert_bitwise(bl, nb, what)


@pytest.mark.parametrize("index,dw,nx", [(2, 32, 1100), (4, 24, 1100), (5, 16, 2100)])
def test_blocked_radius4_team_across_xcds(index, dw, nx):
    """A team larger than one XCD holds (33 to 69 slices against 32 or 64
    resident workgroups per XCD): its slices exchange halos across XCDs
    through device-coherent stores and loads.  Bit-identical to naive, and
    no halo waited for in vain (the context reports that as an error)."""
    print(f"workload {index} dw {dw} nx {nx}", flush=True)
    wl = workloads.make(index, n=(nx, 20, 12), nt=5)
    nb, nb_prev, bl, bl_prev = both(wl, dw, 5)
    assert_bitwise(bl, nb, f"workload {index} dw {dw} nx {nx}")


@pytest.mark.parametrize("index", [3, 4, 5])
def test_blocked_nonzero_shell(index):
    """A non-zero Dirichlet shell held only by the buffer of level 0 (u[0] for
    the Jacobi kinds, u[1] for the leapfrog): both schemes copy it into the
    other buffer before the first step, so each equals the naive scheme run
    with that shell in both buffers, bit for bit."""
    import torch
    from gpu_util import coef_to_dev, gpu_weights, oracle_weights, to_dev
    import oracle
    nt = 7
    wl = workloads.make(index, n=SIZES[index], nt=nt)
    h = wl.halo
    rng = np.random.default_rng([1410, 96, index])
    shell = rng.uniform(-1, 1, wl.u0.shape).astype(np.float32)
    inner = (slice(h, -h),) * 3

    def with_shell(a):
        b = shell.copy()
        b[inner] = a[inner]
        return b

    lf = wl.kind in (4, 5)
    lv0 = with_shell(wl.u0)
    other = wl.u_prev if lf else np.zeros_like(wl.u0)
    cf = coef_to_dev(wl)
    out = {}
    cases = (("ref", st.NAIVE, with_shell(other)), ("naive", st.NAIVE, other),
             ("blocked", st.BLOCKED, other))
    for name, scheme, oth in cases:
        bufs = (to_dev(oth, h), to_dev(lv0, h)) if lf else (to_dev(lv0, h), to_dev(oth, h))
        with st.Context(scheme) as ctx:
            slot = ctx.run(wl.kind, bufs[0], bufs[1], nt, halo=h, coef=cf, w=gpu_weights(wl),
                           alpha=wl.alpha)
            ctx.sync()
        torch.cuda.synchronize()
        out[name] = (bufs[slot].cpu().numpy(), bufs[1 - slot].cpu().numpy())
    for name in ("naive", "blocked"):
        assert_bitwise(out["ref"][0][inner], out[name][0][inner], name + " level nt")
        if lf:
            assert_bitwise(out["ref"][1][inner], out[name][1][inner], name + " level nt-1")
        # the scheme gave the other buffer the level-0 shell
        for a in out[name]:
            b = a.copy()
            b[inner] = shell[inner]
            assert np.array_equal(b, shell), name
    cfo = wl.coef_values_f32().astype(np.float64) if wl.coef is not None else None
    if lf:
        want = oracle.run(wl.kind, lv0.astype(np.float64), h, nt,
                          u_prev=with_shell(other).astype(np.float64), coef=cfo,
                          w=oracle_weights(wl), alpha=wl.alpha)[1]
    else:
        want = oracle.run(wl.kind, lv0.astype(np.float64), h, nt, coef=cfo, w=oracle_weights(wl))
    assert rel_l2(out["blocked"][0].astype(np.float64), want, h) <= TOL
