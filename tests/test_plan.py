"""CPU checks of the diamond schedule the blocked scheme runs (Sect. 4.2).

The library reports its rows (stencil_plan_rows); this test rebuilds each
diamond's level ranges from the geometry documented in csrc/plan.h and
simulates the schedule on the (y, t) plane:

* every (y, t), 0 <= y < ny, 1 <= t <= nt, is updated exactly once;
* every dependency of an update -- (y', t-1) for |y' - y| <= R, and (y, t-2)
  for the leapfrog -- is either an initial level (t' <= 0), an update of an
  earlier row, or an update of the same diamond (rows are launched in order,
  diamonds of one row are independent: Sect. 4.2);
* what a diamond reads from outside itself is exactly its old frontier (the
  two newest levels per column below it), and its new frontier is the two
  newest levels after it -- the storage invariant of the frontier buffers;
* the widths and tiles-per-row numbers the paper prints.
"""
import itertools

import pytest

import paper_1410_3060_amd as st


def diamonds(R, dw, ny, nt):
    H = dw // (2 * R)
    rows = st.plan_rows(1 if R == 1 else 3, dw, ny, nt)
    out = []
    for r, t0, n, first in rows:
        row = []
        for i in range(n):
            yc = first + i * dw
            cells = set()
            for j in range(1, 2 * H):
                t = t0 + j
                if t < 1 or t > nt:
                    continue
                m = min(j, 2 * H - j)
                for y in range(max(0, yc - R * m), min(ny, yc + R * m)):
                    cells.add((y, t))
            row.append(cells)
        out.append((r, t0, row))
    return out


CASES = [(1, 4, 17, 9), (1, 8, 33, 20), (1, 12, 50, 13), (4, 16, 45, 7), (4, 16, 64, 10),
         (4, 24, 70, 9), (1, 8, 1, 5), (4, 16, 3, 1)]


@pytest.mark.parametrize("R,dw,ny,nt", CASES)
@pytest.mark.parametrize("leapfrog", [False, True])
def test_schedule_exactly_once_and_ordered(R, dw, ny, nt, leapfrog):
    plan = diamonds(R, dw, ny, nt)
    owner = {}
    for q, (r, t0, row) in enumerate(plan):
        for i, cells in enumerate(row):
            for c in cells:
                assert c not in owner, f"{c} updated twice"
                owner[c] = (q, i)
    assert set(owner) == {(y, t) for y in range(ny) for t in range(1, nt + 1)}
    for (y, t), (q, i) in owner.items():
        deps = [(yy, t - 1) for yy in range(y - R, y + R + 1)]
        if leapfrog:
            deps.append((y, t - 2))
        for (yy, tt) in deps:
            if tt <= 0 or yy < 0 or yy >= ny:
                continue  # initial levels and the boundary shell
            oq, oi = owner[(yy, tt)]
            assert oq < q or (oq == q and oi == i), f"({y},{t}) needs ({yy},{tt}) too late"


@pytest.mark.parametrize("R,dw,ny,nt", CASES)
def test_frontier_invariant(R, dw, ny, nt):
    """A diamond reads from outside itself only the two newest levels of the
    columns it touches (the old frontier), so two frontier buffers suffice."""
    plan = diamonds(R, dw, ny, nt)
    top = {y: 0 for y in range(ny)}  # newest level per column so far
    for r, t0, row in plan:
        for cells in row:
            for (y, t) in cells:
                for yy in range(y - R, y + R + 1):
                    if 0 <= yy < ny and (yy, t - 1) not in cells:
                        assert top[yy] - 1 <= t - 1 <= top[yy], (y, t, yy, top[yy])
                if (y, t - 2) not in cells and t - 2 >= 0:
                    assert top[y] - 1 <= t - 2 <= top[y]
        for cells in row:
            for (y, t) in cells:
                top[y] = max(top[y], t)
    assert all(v == nt for v in top.values())


def test_diamond_shape_numbers_from_the_paper():
    # R = 1, D_w = 8: seven levels of widths 2,4,6,8,6,4,2, area D_w^2/2 = 32
    # and wavefront width W_w = D_w - 2R + N_F + 1 = 7 (Sect. 5.3 example)
    R, dw = 1, 8
    H = dw // (2 * R)
    widths = [2 * R * min(j, 2 * H - j) for j in range(1, 2 * H)]
    assert widths == [2, 4, 6, 8, 6, 4, 2] and sum(widths) == dw * dw // 2
    assert len(widths) == dw - 2 * R + 0 + 1
    # R = 4, D_w = 16: three levels 8, 16, 8; W_w = 16 - 8 + 1 = 9
    R, dw = 4, 16
    H = dw // (2 * R)
    widths = [2 * R * min(j, 2 * H - j) for j in range(1, 2 * H)]
    assert widths == [8, 16, 8]
    # concurrency: 768 / (4 * 16) = 12 diamonds per row (Sect. 6.3)
    rows = st.plan_rows(3, 64, 768, 40)
    assert all(n in (12, 13) for (_, _, n, _) in rows)


def test_plan_rejects_bad_widths():
    with pytest.raises(ValueError):
        st.plan_rows(3, 12, 100, 10)  # not a multiple of 2R = 8
    with pytest.raises(ValueError):
        st.plan_rows(1, 2, 100, 10)   # below 4R
    assert st.plan_rows(1, 8, 100, 0) == []
