"""Host logic of the learned-precision pipeline (no GPU): the plain precision
rule, the seeded instance sampler, the stored pairs and the trained model
file (shapes, scaling, statistics)."""
import json
import math
import os
from fractions import Fraction

import numpy as np

from paper_0902_0852_amd import learned


def test_plain_bits_rule():
    assert learned.plain_bits(16) == 1024
    assert learned.plain_bits(50) == 1024
    assert learned.plain_bits(400) == 8192
    for N in (51, 123, 250, 399, 777):
        k = learned.plain_bits(N)
        assert k % 64 == 0
        assert k >= 1024 + (8192 - 1024) * (N - 50) / 350.0
        assert k - 64 < 1024 + (8192 - 1024) * (N - 50) / 350.0


def test_sampler_is_seeded_and_in_range():
    a = learned.sample_instances(200, 5, 50, 400)
    b = learned.sample_instances(200, 5, 50, 400)
    assert a == b
    assert a != learned.sample_instances(200, 6, 50, 400)
    for N, (p, q) in a:
        assert 50 <= N <= 400
        assert math.gcd(p, q) == 1 and 1 <= p <= 8 and 1 <= q <= 8
        assert Fraction(1, 2) <= Fraction(p, q) <= 3


def test_groups_cover_everything_once():
    idx = list(range(37))
    g = learned._groups(idx, lambda i: -i, 8)
    flat = [i for grp in g for i in grp]
    assert sorted(flat) == idx and all(len(x) <= 8 for x in g)
    assert flat == sorted(idx, key=lambda i: -i)


def test_pairs_round_trip(tmp_path):
    rows = [{"N": 30, "p": 2, "q": 1, "bits": 448, "ln_lambda": -45.99, "lambda_dec": "1.06e-20"},
            {"N": 224, "p": 5, "q": 2, "bits": 1504, "ln_lambda": -305.7, "lambda_dec": "1.7e-133"}]
    path = str(tmp_path / "pairs.csv")
    learned.save_pairs(rows, path)
    back = learned.load_pairs(path)
    assert [r["N"] for r in back] == [30, 224]
    assert back[1]["lambda_dec"] == "1.7e-133"
    assert abs(back[0]["ln_lambda"] + 45.99) < 1e-12


def test_ln_decimal():
    assert abs(learned.ln_decimal("1.5e-3") - math.log(1.5e-3)) < 1e-12
    assert abs(learned.ln_decimal("4.4e-230") - (math.log(4.4) - 230 * math.log(10))) < 1e-9


def test_stored_pairs_are_consistent():
    rows = learned.load_pairs()
    assert len(rows) >= 2000
    for r in rows:
        assert r["bits"] % learned.GRID == 0 and r["bits"] >= 64
        assert abs(learned.ln_decimal(r["lambda_dec"]) - r["ln_lambda"]) < 1e-6 * (1 + abs(r["ln_lambda"]))
        assert r["ln_lambda"] < 1.0


def test_model_file_shapes_and_statistics():
    m = learned.load_model()
    assert len(m["W"]) == 64 * 3 + 64 + 2 * (64 * 64 + 64) + 2 * 64 + 2
    assert len(m["in_mean"]) == 3 and len(m["in_scale"]) == 3
    assert len(m["out_mean"]) == 2 and len(m["out_scale"]) == 2
    assert m["bits_margin"] >= 1.0 and m["rmse_ln_lambda"] > 0
    assert all(np.isfinite(m["W"]))
    assert m["n_train"] + m["n_val"] == m["pairs"]["count"]
