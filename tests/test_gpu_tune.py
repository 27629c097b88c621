"""The measured tuner: every candidate runs through the library and the best
is the fastest measured; the copy-roof probe returns one figure per working
set."""
import pytest

import paper_1410_3060_amd as st
from paper_1410_3060_amd import tune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,n3", [(2, (70, 40, 30)), (3, (66, 36, 20))])
def test_autotune_candidates_and_best(kind, n3):
    r = tune.autotune(kind, n3, 8, reps=1)
    widths = tune.PROVIDED_DW[kind]
    assert len(r["results"]) == 1 + len(widths)
    assert [x["dw"] for x in r["results"][1:]] == list(widths)
    assert all(x["glups"] > 0 for x in r["results"])
    assert r["best"]["glups"] == max(x["glups"] for x in r["results"])
    assert r["library_default_dw"] == st.default_dw(kind, n3)


def test_autotune_slice_widths():
    """The radius-4 candidates at both slice widths: the tuner reports the
    workgroups that share each diamond (ceil(nx / width)); 32-column slices are
    not provided at dw 24 of the 25-point variable stencil."""
    r = tune.autotune(3, (66, 36, 20), 8, reps=1, xtiles=(16, 32))
    got = [(x["dw"], x["xtile"], x["workgroups_per_diamond"]) for x in r["results"][1:]]
    assert got == [(16, 16, 5), (16, 32, 3), (24, 16, 5)]
    assert all(x["glups"] > 0 for x in r["results"])


def test_memory_roofs():
    roofs = tune.memory_roofs((4, 64), reps=3)
    assert [x["working_set_MiB"] for x in roofs] == [4, 64]
    assert all(x["GBps"] > 0 for x in roofs)
