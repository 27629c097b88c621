"""The traffic and capacity models (paper_1410_3060_amd/model.py) against the
numbers the paper prints (tests/golden/paper_numbers.json, each cited)."""
import json
import os

import pytest

from paper_1410_3060_amd import model

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


@pytest.mark.parametrize("case", GOLDEN["code_balance"], ids=lambda c: c["cite"][:40])
def test_code_balance_matches_paper(case):
    got = model.naive_code_balance(case["kind"], value_bytes=case["value_bytes"],
                                   write_allocate=case["write_allocate"])
    assert got == case["bytes_per_lup"], case["cite"]


def test_roofline_example():
    r = GOLDEN["roofline"]
    b = model.naive_code_balance(r["kind"], value_bytes=r["value_bytes"],
                                 write_allocate=r["write_allocate"])
    assert r["bandwidth_GBps"] / b == pytest.approx(r["glups"])


@pytest.mark.parametrize("case", GOLDEN["wavefront_width"], ids=lambda c: c["cite"][:40])
def test_wavefront_width(case):
    assert model.wavefront_width(case["R"], case["dw"], case["n_f"]) == case["w_w"]


@pytest.mark.parametrize("case", GOLDEN["cache_block"], ids=lambda c: c["cite"][:40])
def test_cache_block_examples(case):
    assert model.cache_block_bytes(case["R"], case["dw"], case["n_f"], case["n_d"], 1) == \
        case["bytes_per_n_xb"]


def test_cache_block_1wd_25pt_var():
    c = GOLDEN["cache_block_1wd_25pt_var"]
    per_group = model.cache_block_bytes(c["R"], c["dw"], c["n_f"], c["n_d"], c["nx"] * c["value_bytes"])
    total_mib = c["thread_groups"] * per_group / 2 ** 20
    assert abs(total_mib - c["approx_MiB"]) / c["approx_MiB"] < 0.05


def test_gpu_code_balances():
    # FP32 values, no write-allocate (GPU stores do not read the line first)
    assert [model.naive_code_balance(k) for k in (1, 4, 2, 3, 5)] == [8, 12, 36, 60, 16]
    assert model.naive_code_balance(3, coef_bytes=2) == 34
    # blocked: the diamond widths the library uses
    assert model.blocked_bytes_per_lup(3, 16) == 36.0
    assert model.blocked_bytes_per_lup(2, 8) == 11.5
    # wider diamonds move fewer bytes per update, all below the naive balance
    assert model.blocked_bytes_per_lup(3, 32) < model.blocked_bytes_per_lup(3, 24) < \
        model.blocked_bytes_per_lup(3, 16) < model.naive_code_balance(3)
