"""The traffic/flop model reproduces the numbers the paper prints."""

import json
import os

import pytest

from paper_1104_0737_amd import model

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cost_model.json")))


def test_paper_cost_numbers():
    assert model.paper_flops_per_site(1) == GOLD["wilson_flops_per_site"]["value"]
    assert model.paper_words_per_site(1) == GOLD["wilson_words_per_site_L1"]["value"]
    g = GOLD["flops_per_byte_single_L1"]
    assert model.paper_flops_per_byte(1, 4) == pytest.approx(g["value"], abs=g["tol"])
    g = GOLD["flops_per_byte_double_L1"]
    assert model.paper_flops_per_byte(1, 8) == pytest.approx(g["value"], abs=g["tol"])
    assert model.link_bytes_per_site(4) == GOLD["link_bytes_single"]["value"]
    assert model.link_bytes_per_site(8) == GOLD["link_bytes_double"]["value"]
    for L, key in ((1, "clover_flops_per_byte_single_L1"), (12, "clover_flops_per_byte_single_L12")):
        g = GOLD[key]
        assert model.paper_flops_per_byte(L, 4, clover=True) == pytest.approx(g["value"], abs=g["tol"])


def test_flops_per_byte_grows_with_L():
    fb = [model.paper_flops_per_byte(L, 4) for L in (1, 2, 3, 4, 6, 12)]
    assert all(b > a for a, b in zip(fb, fb[1:]))


def test_compulsory_bytes():
    assert model.dslash_bytes_per_site(12, "fp64") == 5184
    assert model.dslash_bytes_per_site(12, "fp32") == 2592
    assert model.dslash_bytes_per_site(12, "fp16s") == 1392
    assert model.dslash_bytes_per_site(1, "fp64") == 960


def test_table1_gains_consistent():
    t = GOLD["table1"]
    for tm, g in zip(t["time_s"], t["time_gain"]):
        assert t["time_s"][0] / tm == pytest.approx(g, abs=0.06)
    for n, g in zip(t["nmvm"], t["nmvm_gain"]):
        assert t["nmvm"][0] / n == pytest.approx(g, abs=0.06)
