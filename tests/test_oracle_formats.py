"""Pins for the oracle's centring and storage-format encoders (row a0).

Each encoder is checked against an independent library routine (torch's CPU
bfloat16 / float8_e4m3fn conversions) or against exact arithmetic."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O


def test_bf16_round_matches_torch_cpu():
    rng = np.random.default_rng(0)
    v = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-30).astype(np.float32),
        (rng.standard_normal(2000) * 1e30).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e38], np.float32),
    ])
    # exact ties: low 16 bits == 0x8000, both parities of the kept LSB
    mant = rng.integers(0, 128, 500).astype(np.uint32) << 16
    expo = rng.integers(1, 254, 500).astype(np.uint32) << 23
    sign = rng.integers(0, 2, 500).astype(np.uint32) << 31
    ties = sign | expo | mant | np.uint32(0x8000)
    v = np.concatenate([v, ties.view(np.float32)])
    ours = O.bf16_round(v)
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_e4m3_table_known_values():
    t = O.e4m3_table()
    assert t[0x7E] == 448.0
    assert t[0x38] == 1.0
    assert t[0x08] == 2.0 ** -6            # smallest normal
    assert t[0x01] == 2.0 ** -9            # smallest subnormal
    assert t[0x07] == 7 * 2.0 ** -9
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert np.sum(np.isfinite(t)) == 254
    assert t[0xB8] == -1.0


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(1)
    v = np.concatenate([
        (rng.standard_normal(20000) * 50).astype(np.float32),
        (rng.standard_normal(5000) * 1e-2).astype(np.float32),
        (rng.uniform(-448, 448, 5000)).astype(np.float32),
    ])
    # midpoints between neighbouring codes (ties) and the codes themselves
    t = O.e4m3_table()[:0x7F]
    mids = ((t[1:] + t[:-1]) / 2).astype(np.float32)
    v = np.concatenate([v, mids, -mids, t.astype(np.float32)])
    v = v[np.abs(v) <= 448.0]
    ours = O.e4m3_encode(v)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # torch keeps the sign of a value that rounds to zero as well
    assert np.array_equal(ours, ref)


def test_e4m3_encode_saturates():
    v = np.array([448.0, 449.0, 464.0, 500.0, 1e6, -1e6, np.float32(3e38)], np.float32)
    codes = O.e4m3_encode(v)
    assert list(codes) == [0x7E, 0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0x7E]


def test_column_means_exact_sum():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal((301, 7)) * np.array([1, 1e3, 1e-3, 1e8, 1, 1, 1])).astype(np.float32)
    x[:, 4] = 1e8
    x[0, 4] = 1.0          # a value lost by naive float32 accumulation
    mu = O.column_means(x)
    for j in range(x.shape[1]):
        exact = sum(Fraction(float(a)) for a in x[:, j])
        assert mu[j] == float(exact) / x.shape[0] or mu[j] == float(exact / x.shape[0])
        assert abs(Fraction(mu[j]) - exact / x.shape[0]) <= abs(exact / x.shape[0]) * Fraction(2, 2 ** 52)


def test_center_and_scales():
    rng = np.random.default_rng(3)
    x = (rng.standard_normal((100, 5)) + 3.0).astype(np.float32)
    mu = O.column_means(x)
    c = O.center_fp32(x, mu)
    assert c.dtype == np.float32
    assert np.max(np.abs(c.astype(np.float64).mean(axis=0))) < 1e-6
    s = O.fp8_column_scales(c)
    assert np.all(s == (np.max(np.abs(c), axis=0) / np.float32(448)).astype(np.float32))
    q = O.fp8_quantize(c, s)
    # the largest magnitude of each column maps to the top code
    for j in range(5):
        r = np.argmax(np.abs(c[:, j]))
        assert q[r, j] & 0x7F == 0x7E
    deq = O.e4m3_value(q) * s[None, :]
    assert np.max(np.abs(deq - c) / np.max(np.abs(c), axis=0)) <= 2.0 ** -4


def test_zero_column_scale_is_one():
    c = np.zeros((4, 2), np.float32)
    c[:, 1] = [1, -2, 3, 0]
    s = O.fp8_column_scales(c)
    assert s[0] == 1.0 and s[1] == np.float32(3.0 / 448.0)
    assert np.all(O.fp8_quantize(c, s)[:, 0] == 0)
