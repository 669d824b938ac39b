"""Pins for the exact-sum oracle of the precision variant."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import fpsum


# values fixed by the OCP 8-bit floating point definition of E4M3
E4M3_SPEC = {
    0x00: 0.0, 0x80: -0.0, 0x01: 2.0**-9, 0x07: 7 * 2.0**-9, 0x08: 2.0**-6,
    0x38: 1.0, 0x40: 2.0, 0xC0: -2.0, 0x3C: 1.5, 0x7E: 448.0, 0xFE: -448.0,
    0x77: 240.0, 0x30: 0.5,
}


@pytest.mark.parametrize("code,val", sorted(E4M3_SPEC.items()))
def test_e4m3_spec_values(code, val):
    k, nan = fpsum.e4m3_scaled_int(code)
    assert not nan and math.ldexp(k, -9) == val


def test_e4m3_nan_codes():
    t = fpsum.e4m3_table()
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert np.isfinite(np.delete(t, [0x7F, 0xFF])).all()
    assert np.nanmax(t) == 448.0


def test_e4m3_matches_torch_for_all_codes():
    codes = torch.arange(256, dtype=torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = fpsum.decode_e4m3(np.arange(256, dtype=np.uint8))
    both_nan = np.isnan(ref) & np.isnan(got)
    assert (both_nan | (ref == got)).all()


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2**16, 20000, dtype=np.uint16)
    bits = bits[((bits >> 7) & 0xFF) != 0xFF]          # drop inf / NaN
    ref = torch.from_numpy(bits.astype(np.int16)).view(torch.bfloat16)
    assert np.array_equal(fpsum.decode_bf16(bits), ref.to(torch.float64).numpy())


def _wide(rng, n):
    mant = rng.standard_normal(n)
    expo = rng.integers(-60, 30, n)
    return np.ldexp(mant, expo).astype(np.float32).astype(np.float64)


def test_exact_sum_matches_fsum():
    rng = np.random.default_rng(1)
    for n in (1, 2, 1000, 50000):
        x = _wide(rng, n)
        assert fpsum.exact_sum(x, chunk=777) == math.fsum(x.tolist())


def test_exact_sum_matches_fractions():
    rng = np.random.default_rng(2)
    x = _wide(rng, 300)
    assert fpsum.exact_sum_rational(x) == fpsum.exact_sum_fraction(x)


def test_exact_sum_special_cases():
    assert fpsum.exact_sum(np.full(1 << 16, 0.1, dtype=np.float32)) == \
        float(Fraction(float(np.float32(0.1))) * (1 << 16))
    x = np.random.default_rng(3).standard_normal(10001).astype(np.float32)
    assert fpsum.exact_sum(np.concatenate([x, -x])) == 0.0
    assert fpsum.exact_sum(np.array([1e8, 1.0, -1e8], dtype=np.float32)) == 1.0
    assert fpsum.exact_sum(np.array([], dtype=np.float32)) == 0.0
    assert fpsum.exact_sum(np.array([2.0**-149, 2.0**-149])) == 2.0**-148
    with pytest.raises(ValueError):
        fpsum.exact_sum(np.array([1.0, np.inf]))


def test_exact_sum_e4m3():
    rng = np.random.default_rng(4)
    codes = rng.integers(0, 256, 100000, dtype=np.uint8)
    codes = codes[(codes != 0x7F) & (codes != 0xFF)]
    assert fpsum.exact_sum_e4m3(codes) == math.fsum(fpsum.decode_e4m3(codes).tolist())


def test_64_e4m3_values_sum_exactly_in_fp32():
    # any 64 finite e4m3 values are k * 2**-9 with |k| <= 229376, and
    # 64 * 229376 < 2**24, so a float32 running sum never rounds
    rng = np.random.default_rng(5)
    t = fpsum.e4m3_table()
    finite = np.flatnonzero(np.isfinite(t))
    for _ in range(200):
        v = t[rng.choice(finite, 64)].astype(np.float32)
        acc = np.float32(0)
        for e in v:
            acc = np.float32(acc + e)
        assert float(acc) == math.fsum(v.astype(np.float64).tolist())
    worst = np.full(64, np.float32(448.0))
    assert float(np.add.reduce(worst, dtype=np.float32)) == 64 * 448.0


def _sum2_lane_sim(x32):
    """Ogita-Rump-Oishi Sum2 in binary32 (a CPU model of one lane)."""
    s = np.float32(0)
    c = np.float32(0)
    for v in x32:
        t = np.float32(s + v)
        bb = np.float32(t - s)
        e = np.float32(np.float32(s - np.float32(t - bb)) + np.float32(v - bb))
        s = t
        c = np.float32(c + e)
    return float(s) + float(c)


def test_sum2_bound_holds_on_hard_data():
    rng = np.random.default_rng(6)
    for trial in range(20):
        n = int(rng.integers(2, 400))
        x = _wide(rng, n).astype(np.float32)
        x[::7] *= np.float32(2.0**20)
        exact = fpsum.exact_sum_rational(x.astype(np.float64))
        got = _sum2_lane_sim(x)
        err = abs(Fraction(got) - exact)
        bound = fpsum.sum2_bound(float(np.abs(x.astype(np.float64)).sum()), n, 0, 0)
        assert float(err) <= bound


def test_sum2_recovers_what_plain_fp32_loses():
    # ones absorbed by a large running sum are recovered by the c term
    x = np.array([2.0**30] + [1.0] * 1000 + [-(2.0**30)], dtype=np.float32)
    assert _sum2_lane_sim(x) == 1000.0
    plain = np.float32(0)
    for v in x:
        plain = np.float32(plain + v)
    assert float(plain) != 1000.0


# ------------------------------------------- the histogram exact sums
def _finite_f32_bits(rng, n):
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return b[((b >> 23) & 0xFF) != 0xFF]


def test_f32_histogram_sum_matches_the_rational_sum():
    rng = np.random.default_rng(11)
    bits = _finite_f32_bits(rng, 100000)            # every exponent, subnormals too
    want = fpsum.exact_sum_rational(fpsum.decode_f32(bits))
    assert fpsum.exact_sum_f32_bits(bits, chunk=4097, rational=True) == want
    assert fpsum.exact_sum_f32_bits(bits) == float(want)
    x = _wide(rng, 5000).astype(np.float32)
    assert fpsum.exact_sum_f32_bits(x.view(np.uint32)) == math.fsum(x.astype(np.float64).tolist())


def test_bf16_histogram_sum_matches_the_rational_sum():
    rng = np.random.default_rng(12)
    b = rng.integers(0, 2**16, 100000, dtype=np.uint32).astype(np.uint16)
    b = b[((b >> 7) & 0xFF) != 0xFF]
    want = fpsum.exact_sum_rational(fpsum.decode_bf16(b))
    assert fpsum.exact_sum_bf16_bits(b, chunk=1000, rational=True) == want


def test_e4m3_histogram_sum_matches_the_integer_sum():
    rng = np.random.default_rng(13)
    c = rng.integers(0, 256, 300000, dtype=np.uint32).astype(np.uint8)
    c = c[(c != 0x7F) & (c != 0xFF)]
    assert fpsum.exact_sum_e4m3_hist(c, chunk=999) == fpsum.exact_sum_e4m3(c)
    assert fpsum.exact_sum_e4m3_hist(c, rational=True) * 512 == \
        sum(fpsum.e4m3_scaled_int(int(v))[0] for v in c)


def test_histogram_sums_special_cases():
    # constant payloads sum to n * x; +x / -x pairs cancel; signed zeros
    x = np.full(3001, np.float32(0.1))
    assert fpsum.exact_sum_f32_bits(x.view(np.uint32), rational=True) == \
        3001 * Fraction(float(np.float32(0.1)))
    y = np.random.default_rng(14).standard_normal(5000).astype(np.float32)
    both = np.concatenate([y, -y])
    assert fpsum.exact_sum_f32_bits(both.view(np.uint32)) == 0.0
    assert fpsum.exact_sum_f32_bits(np.array([0x80000000, 0], dtype=np.uint32)) == 0.0
    # the smallest subnormals: 2**-149 (binary32) and 2**-133 (BF16)
    assert fpsum.exact_sum_f32_bits(np.array([1, 1], dtype=np.uint32)) == 2.0**-148
    assert fpsum.exact_sum_bf16_bits(np.array([1, 0x8001, 1], dtype=np.uint16)) == 2.0**-133
    assert fpsum.exact_sum_e4m3_hist(np.array([0x7E, 0xFE, 0x01], dtype=np.uint8)) == 2.0**-9
    assert fpsum.exact_sum_f32_bits(np.array([], dtype=np.uint32)) == 0.0
    with pytest.raises(ValueError):
        fpsum.exact_sum_f32_bits(np.array([0x7F800000], dtype=np.uint32))   # +inf
    with pytest.raises(ValueError):
        fpsum.exact_sum_bf16_bits(np.array([0x7FC0], dtype=np.uint16))     # NaN
    with pytest.raises(ValueError):
        fpsum.exact_sum_e4m3_hist(np.array([0x7F], dtype=np.uint8))
