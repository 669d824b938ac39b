"""Exact sums of low-precision payloads and the compensated-sum error bound.

The precision variant of the streaming path sums a payload of FP32, BF16 or
FP8-e4m3 values.  This module gives what that sum must approach: the EXACT
real sum of the stored (decoded) values, rounded once to FP64, plus the
worst-case error bound of the GPU's accumulation scheme.

Decoding, written from the format definitions:

* BF16 is the upper half of an IEEE-754 binary32: value bits << 16.
* FP8 E4M3 ("e4m3fn", OCP 8-bit floating point specification, 2023):
  1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits; exponent field
  0 encodes subnormals m * 2**-9; S.1111.111 is NaN; there are no
  infinities; the largest finite magnitude is 1.75 * 2**8 = 448.  Every
  finite value is an integer multiple of 2**-9.

Exact summation: each value x (a finite binary64 after decoding) is split
as x = (h + r) * 2**-P with h an integer below 2**51 in magnitude and r the
(exact) fractional remainder; sum(h) is accumulated in Python integers and
sum(r) in exact rationals, so no rounding happens until the final
conversion to binary64 (correctly rounded by Python's int/int division).
"""
import math
from fractions import Fraction

import numpy as np

U32 = 2.0 ** -24          # unit roundoff of binary32
U64 = 2.0 ** -53          # unit roundoff of binary64


# ----------------------------------------------------------------- decoding
def e4m3_scaled_int(code):
    """FP8 e4m3 code (0..255) -> (k, is_nan) with value = k * 2**-9."""
    code = int(code) & 0xFF
    sign = -1 if code & 0x80 else 1
    exp = (code >> 3) & 0xF
    man = code & 0x7
    if exp == 0xF and man == 0x7:
        return 0, True
    if exp == 0:
        k = man                                  # subnormal: m * 2**-9
    else:
        k = (8 + man) << (exp - 1)               # (1 + m/8) * 2**(e-7)
    return sign * k, False


def e4m3_table():
    """Decoded value of every FP8 e4m3 code as float64 (NaN for NaN codes)."""
    t = np.empty(256, dtype=np.float64)
    for c in range(256):
        k, nan = e4m3_scaled_int(c)
        t[c] = math.nan if nan else math.ldexp(k, -9)
    return t


def decode_e4m3(codes_u8):
    """Decode a uint8 array of FP8 e4m3 codes to float64."""
    return e4m3_table()[np.asarray(codes_u8, dtype=np.uint8)]


def decode_bf16(bits_u16):
    """Decode a uint16 array of BF16 bit patterns to float64."""
    b = np.asarray(bits_u16, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def decode_f32(bits_u32):
    """Reinterpret a uint32 array of binary32 bit patterns as float64."""
    return np.asarray(bits_u32, dtype=np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------- exact summation
def exact_sum_fraction(values):
    """Exact sum as a Fraction (every finite float is an exact rational)."""
    total = Fraction(0)
    for v in values:
        total += Fraction(float(v))
    return total


def exact_sum(values, chunk=1 << 22):
    """Exact sum of a float array, rounded once to the nearest binary64."""
    return float(exact_sum_rational(values, chunk))


def exact_sum_rational(values, chunk=1 << 22):
    """Exact sum of a float array as a Fraction (see module docstring).

    The input is widened to binary64 chunk by chunk (exactly), so a large
    binary32 payload is never copied whole.
    """
    x = np.asarray(values).ravel()
    if x.size == 0:
        return Fraction(0)
    amax = 0.0
    for s in range(0, x.size, chunk):
        c = x[s:s + chunk].astype(np.float64)
        if not np.all(np.isfinite(c)):
            raise ValueError("payload holds a non-finite value")
        amax = max(amax, float(np.max(np.abs(c))))
    if amax == 0.0:
        return Fraction(0)
    # |x| < 2**e_max, so |x * 2**P| < 2**51 with P = 51 - e_max
    e_max = math.frexp(amax)[1]
    P = 51 - e_max
    hi_total = 0
    rem = []
    for s in range(0, x.size, chunk):
        a = np.ldexp(x[s:s + chunk].astype(np.float64), P)   # exact scaling
        h = np.trunc(a)
        r = a - h                                  # exact fractional part
        hi = h.astype(np.int64)
        # blocks of 2**11 terms below 2**51 each cannot overflow int64
        pad = (-hi.size) % 2048
        blk = np.concatenate([hi, np.zeros(pad, np.int64)]).reshape(-1, 2048)
        hi_total += sum(int(v) for v in blk.sum(axis=1))
        nz = r[r != 0.0]
        if nz.size:
            rem.append(nz)
    total = Fraction(hi_total)
    for nz in rem:
        total += exact_sum_fraction(nz)
    return total * Fraction(1, 2) ** P if P >= 0 else total * (2 ** -P)


def exact_sum_e4m3(codes_u8, chunk=1 << 24):
    """Exact sum of FP8 e4m3 codes via their integer multiples of 2**-9."""
    table = np.empty(256, dtype=np.int64)
    for c in range(256):
        k, nan = e4m3_scaled_int(c)
        table[c] = k
        if nan:
            table[c] = 0
    codes = np.asarray(codes_u8, dtype=np.uint8).ravel()
    for c in (0x7F, 0xFF):
        if np.any(codes == c):
            raise ValueError("payload holds an e4m3 NaN")
    total = 0
    for s in range(0, codes.size, chunk):
        total += int(table[codes[s:s + chunk]].sum())
    return float(Fraction(total, 512))


# -------------------------------------------------------------- error bound
def gamma(n, u=U32):
    """gamma_n = n u / (1 - n u) (Higham's notation)."""
    if n * u >= 1:
        raise ValueError("n too large for gamma_n")
    return n * u / (1 - n * u)


def sum2_bound(abs_sum, n_lane, depth, n_groups, threads=256):
    """Worst-case |S_gpu - S| of the GPU's accumulation, over sum |x|,
    against the exact sum S rounded once to binary64.

    Scheme: every lane runs Sum2 (Ogita, Rump and Oishi, "Accurate sum and
    dot product", 2005): error-free TwoSum into (s, c) over at most
    ``n_lane`` terms, whose value s + c is within gamma_{n-1}^2 sum|x| of
    the lane's exact sum (zero for a single term: TwoSum of 0 and x is
    exact).  Pairs are then merged up a tree of ``depth`` levels (TwoSum of
    the s parts, c = fl(fl(c_a + c_b) + e)), each level adding at most
    gamma_2 (sum|c| + u sum|s|) <= gamma_2 (gamma_{n-1} + (depth + 1) u)
    sum|x| (with a 1.01 safety factor on the c growth).

    The ``n_groups`` workgroup pairs are then widened to binary64 and
    combined by ``threads`` threads: thread t adds fl(s_i + c_i) of pairs
    i = t, t + threads, ... in turn, and the thread totals meet in a
    binary tree.  Every pair so passes through at most h = 1 + ceil(G /
    threads) + ceil(log2 min(G, threads)) binary64 additions, and a sum in
    which every term passes through at most h additions is within
    gamma_h sum|x| of exact (Higham, "Accuracy and Stability of Numerical
    Algorithms", 2002, Section 4.2), with a 1.001 factor for the pairs'
    sum |s| + |c| over sum |x|.  One more binary64 unit roundoff covers the
    rounding of the exact reference itself.
    """
    g = gamma(n_lane - 1) if n_lane >= 2 else 0.0
    lane = g * g
    tree = depth * gamma(2) * 1.01 * (g + (depth + 1) * U32)
    final = U64
    if n_groups > 0:
        chain = -(-n_groups // threads)
        levels = (min(n_groups, threads) - 1).bit_length()
        final += gamma(1 + chain + levels, U64) * 1.001
    return (lane + tree + final) * abs_sum


# ------------------------------------------- exact sums by value histogram
# The same exact sums, computed another way for large payloads: a value
# is sign * significand * 2**scale with an integer significand, so the
# payload's sum is the sum over (sign, exponent) classes of the class's
# significand total times the class's power of two.  Significand totals
# are gathered with NumPy histograms (bincount) in pieces small enough that
# every float64 bin stays an exact integer (below 2**53), then combined in
# Python integers; nothing is rounded until the final conversion.

def _class_totals(tot, keys, sig, sig_split=None):
    """Add the integer significand totals of every class to ``tot`` (a list
    of Python ints indexed by class: sign bit above the exponent bits)."""
    parts = [(sig, 1)] if sig_split is None else \
        [(sig >> sig_split, 1 << sig_split), (sig & ((1 << sig_split) - 1), 1)]
    for s, mul in parts:
        h = np.bincount(keys, weights=s.astype(np.float64), minlength=len(tot))
        for k in np.flatnonzero(h):
            tot[int(k)] += int(h[k]) * mul


def _combine_classes(tot, scale_of):
    """sum over classes of sign * total * 2**scale, exactly, as a Fraction."""
    half = len(tot) // 2
    lo = min(scale_of(k % half) for k, t in enumerate(tot) if t) if any(tot) else 0
    acc = 0
    for k, t in enumerate(tot):
        if t:
            sign = -1 if k >= half else 1
            acc += sign * t << (scale_of(k % half) - lo)
    return Fraction(acc) * Fraction(2) ** lo


def exact_sum_f32_bits(bits_u32, chunk=1 << 20, rational=False):
    """Exact sum of binary32 bit patterns, rounded once to binary64 (or as a
    Fraction with ``rational``).

    binary32: value = (-1)**s * m * 2**(e - 150) with m = 2**23 + fraction
    for exponent field e >= 1, and m = fraction, scale 2**-149, for e = 0.
    Significands are split into 12-bit halves so that a chunk's bin totals
    stay below 2**12 * 2**20 = 2**32."""
    b = np.asarray(bits_u32, dtype=np.uint32).ravel()
    tot = [0] * 512
    for s in range(0, b.size, chunk):
        c = b[s:s + chunk]
        e = (c >> np.uint32(23)) & np.uint32(0xFF)
        if np.any(e == 0xFF):
            raise ValueError("payload holds a non-finite value")
        m = (c & np.uint32(0x7FFFFF)) | ((e != 0).astype(np.uint32) << np.uint32(23))
        _class_totals(tot, (c >> np.uint32(23)).astype(np.int64), m.astype(np.int64), 12)
    r = _combine_classes(tot, lambda k: (k if k else 1) - 150)
    return r if rational else float(r)


def exact_sum_bf16_bits(bits_u16, chunk=1 << 20, rational=False):
    """Exact sum of BF16 bit patterns, rounded once to binary64 (or as a
    Fraction with ``rational``).

    BF16: value = (-1)**s * m * 2**(e - 134) with m = 2**7 + fraction for
    exponent field e >= 1, and m = fraction, scale 2**-133, for e = 0.
    A chunk's bin totals stay below 2**8 * 2**20 = 2**28."""
    b = np.asarray(bits_u16, dtype=np.uint16).ravel()
    tot = [0] * 512
    for s in range(0, b.size, chunk):
        c = b[s:s + chunk].astype(np.int64)
        e = (c >> 7) & 0xFF
        if np.any(e == 0xFF):
            raise ValueError("payload holds a non-finite value")
        _class_totals(tot, c >> 7, (c & 0x7F) | ((e != 0).astype(np.int64) << 7))
    r = _combine_classes(tot, lambda k: (k if k else 1) - 134)
    return r if rational else float(r)


def exact_sum_e4m3_hist(codes_u8, chunk=1 << 22, rational=False):
    """Exact sum of FP8 e4m3 codes from a histogram of the 256 codes:
    sum over codes of count * k * 2**-9, with k from ``e4m3_scaled_int``;
    rounded once to binary64 (or a Fraction with ``rational``)."""
    codes = np.asarray(codes_u8, dtype=np.uint8).ravel()
    counts = [0] * 256
    for s in range(0, codes.size, chunk):
        h = np.bincount(codes[s:s + chunk], minlength=256)
        for c in np.flatnonzero(h):
            counts[int(c)] += int(h[c])
    total = 0
    for c, n in enumerate(counts):
        if n:
            k, nan = e4m3_scaled_int(c)
            if nan:
                raise ValueError("payload holds an e4m3 NaN")
            total += n * k
    r = Fraction(total, 512)
    return r if rational else float(r)
