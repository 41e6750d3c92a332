"""Pins for oracle.precision: Table 1.1 constants and round-to-format against independent
library conversions and hand-worked tie cases."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import precision as P

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table_1_1.json")


def _sig3(x):
    return float(f"{x:.2e}")


@pytest.mark.parametrize("fmt", P.FORMATS)
def test_table_1_1_constants(fmt):
    g = json.load(open(GOLD))["formats"][fmt]
    assert P._BITS[fmt] == (g["t"], g["e"])
    assert _sig3(P.unit_roundoff(fmt)) == pytest.approx(g["u"], rel=6e-3)
    assert _sig3(P.x_min(fmt)) == pytest.approx(g["x_min"], rel=6e-3)
    assert _sig3(P.x_max(fmt)) == pytest.approx(g["x_max"], rel=6e-3)


def test_fp16_matches_ieee_library_and_generic_rounding():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(200000) * np.exp(rng.uniform(-22, 12, 200000))
    with np.errstate(over="ignore"):
        lib = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(P.fl(x, "fp16"), lib)
    gen = P.round_to_format(x, 11, -14, P.x_max("fp16"))
    assert np.array_equal(gen, lib)


def test_bf16_matches_torch_on_binary32_inputs():
    # torch converts binary32 -> bfloat16 with round-to-nearest-even; on binary32 inputs
    # there is no double rounding, so the two must agree bit for bit.
    rng = np.random.default_rng(1)
    x32 = (rng.standard_normal(200000) * np.exp(rng.uniform(-90, 87, 200000))).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = P.fl(x32.astype(np.float64), "bf16")
    assert np.array_equal(got, ref)


def test_bf16_ties_to_even_and_limits():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to the even significand (1).
    assert P.fl(np.array([1 + 2.0 ** -8]), "bf16")[0] == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6: even is 1 + 2^-6.
    assert P.fl(np.array([1 + 3 * 2.0 ** -8]), "bf16")[0] == 1 + 2.0 ** -6
    # just above the tie rounds up
    assert P.fl(np.array([1 + 2.0 ** -8 + 2.0 ** -30]), "bf16")[0] == 1 + 2.0 ** -7
    # subnormal spacing 2^-133 is kept
    assert P.fl(np.array([2.0 ** -133]), "bf16")[0] == 2.0 ** -133
    assert P.fl(np.array([2.0 ** -135]), "bf16")[0] == 0.0
    assert np.isinf(P.fl(np.array([3.5e38]), "bf16")[0])


def test_fp32_rounding_is_ieee():
    x = np.array([1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, 1e39])
    got = P.fl(x, "fp32")
    assert got[0] == 1.0 and got[1] == 1 + 2.0 ** -22 and np.isinf(got[2])


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_rounding_error_within_unit_roundoff(fmt):
    rng = np.random.default_rng(2)
    x = rng.uniform(0.5, 1000.0, 50000)
    rel = np.abs(P.fl(x, fmt) - x) / x
    assert rel.max() <= P.unit_roundoff(fmt) * (1 + 1e-12)


def test_reduced_matmul_accumulates_in_binary32():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((16, 64))
    b = rng.standard_normal((64, 8))
    got = P.matmul(a, b, "fp16")
    ref = (a.astype(np.float16).astype(np.float32) @ b.astype(np.float16).astype(np.float32))
    assert np.array_equal(got, ref.astype(np.float16).astype(np.float64))
