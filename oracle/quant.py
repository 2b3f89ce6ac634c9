"""Reduced-precision coupling forms, from their definitions.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use this package.

The paper fixes no number format for SB; the library offers forms that
store J in a narrow format while positions, momenta and accumulation stay
FP32 and energies FP64.  This module writes out the 16-bit and FP8 forms:

* IEEE binary16 ("FP16"): 10 stored mantissa bits, exponents -14 .. 15,
  subnormals k * 2^-24; the coupling used is the FP64 J rounded once to the
  nearest binary16 value, ties to the even significand.
* bfloat16 ("BF16"): the upper half of a binary32 (8 exponent bits, 7
  stored mantissa bits); the FP64 J is first rounded to binary32 (the
  kernels' coupling type) and that value rounded to the nearest bfloat16,
  ties to the even significand.

* OCP 8-bit E4M3 ("e4m3fn"): sign bit, 4 exponent bits with bias 7, 3
  mantissa bits; exponent field 0 holds subnormals m/8 * 2^-6; the pattern
  S.1111.111 is NaN and there are no infinities, so the largest finite
  magnitude is 1.75 * 2^8 = 448; rounding is to nearest, ties to even.
* per-row scaling: s_i = fl32(fl32(max_j |J_ij|) / 448) (1 for an all-zero
  row), code_ij = e4m3(min(max(fl32(J_ij / s_i), -448), 448)) and the
  coupling used is J'_ij = fl32(s_i * e4m3_value(code_ij)).  J enters in
  FP32 (the kernels' coupling type).
* per-block scaling: the same with one scale per block of 8 consecutive
  stored couplings of a row, in CSR order (the last block of a row may be
  shorter).
* BF16 pair ("hi + lo"): hi = bf16(J32), lo = bf16(J32 - hi) (the
  difference is exact in binary32), coupling used hi + lo (exact in
  binary32: 16 significant bits).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

E4M3_MAX = 448.0
E4M3_MIN_NORMAL = 2.0 ** -6
E4M3_MIN_SUBNORMAL = 2.0 ** -9


def e4m3_value(code) -> np.ndarray:
    """Value of E4M3 codes (uint8 array); NaN for the two NaN patterns."""
    c = np.asarray(code, dtype=np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    mag = np.where(e == 0, m / 8.0 * E4M3_MIN_NORMAL, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    mag = np.where((e == 15) & (m == 7), np.nan, mag)
    return sign * mag


def e4m3_encode(v) -> np.ndarray:
    """Round finite values with |v| <= 448 to the nearest E4M3 code (ties to
    the even code).  Raises for larger or non-finite inputs."""
    v = np.asarray(v, dtype=np.float64)
    if not np.all(np.isfinite(v)) or np.any(np.abs(v) > E4M3_MAX):
        raise ValueError("e4m3_encode takes finite values with |v| <= 448")
    a = np.abs(v)
    # spacing of representable magnitudes near a: 2^(E - 3) with E the
    # binary exponent of a, floored at the subnormal exponent -6
    with np.errstate(divide="ignore"):
        E = np.where(a > 0, np.floor(np.log2(np.where(a > 0, a, 1.0))), -6.0)
    E = np.maximum(E, -6.0)
    quantum = np.exp2(E - 3.0)
    r = np.rint(a / quantum) * quantum          # exact scaling; rint ties to even
    # code of the rounded magnitude (it may have moved up one binade)
    normal = r >= E4M3_MIN_NORMAL
    with np.errstate(divide="ignore"):
        e = np.where(normal, np.floor(np.log2(np.where(normal, r, 1.0))) + 7.0, 0.0)
    m = np.where(normal, (r / np.exp2(e - 7.0) - 1.0) * 8.0, r / E4M3_MIN_SUBNORMAL)
    code = (e.astype(np.int64) << 3) | np.rint(m).astype(np.int64)
    code = np.where(np.signbit(v) & (r > 0), code | 0x80, code)
    return code.astype(np.uint8)


def _round_to_grid(v, mant_bits, min_exp):
    """Round FP64 values to the nearest value with `mant_bits` stored
    mantissa bits and exponents >= min_exp (subnormals below), ties to the
    even significand, with no upper bound (callers stay in range).  The
    spacing at |v| is 2^(max(E, min_exp) - mant_bits), E = floor(log2|v|);
    v / spacing is exact (a power-of-two scaling) and rint rounds half to
    even."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    with np.errstate(divide="ignore"):
        E = np.where(a > 0, np.floor(np.log2(np.where(a > 0, a, 1.0))), float(min_exp))
    # log2 of a value just below a power of two can round up to it: pull
    # E back where 2^E exceeds a
    E = np.where(np.exp2(E) > a, E - 1.0, E)
    q = np.exp2(np.maximum(E, float(min_exp)) - mant_bits)
    return np.copysign(np.rint(a / q) * q, v)


def fp16_value(v) -> np.ndarray:
    """FP64 values rounded once to the nearest binary16 value (ties to
    even), returned as FP64; |v| must stay below 65520 (no overflow)."""
    v = np.asarray(v, dtype=np.float64)
    if np.any(np.abs(v) >= 65520.0) or not np.all(np.isfinite(v)):
        raise ValueError("fp16_value takes finite |v| < 65520")
    return _round_to_grid(v, 10, -14)


def bf16_value(v) -> np.ndarray:
    """FP64 values rounded to binary32 and then to the nearest bfloat16
    value (ties to even), returned as FP64."""
    v32 = np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)
    if not np.all(np.isfinite(v32)):
        raise ValueError("bf16_value takes values finite in binary32")
    return _round_to_grid(v32, 7, -126)


def fp16_couplings(J: sp.csr_matrix) -> sp.csr_matrix:
    """The FP16 coupling form: every stored J_ij rounded to binary16."""
    J = sp.csr_matrix(J, dtype=np.float64, copy=True)
    J.data = fp16_value(J.data)
    return J


def bf16_couplings(J: sp.csr_matrix) -> sp.csr_matrix:
    """The BF16 coupling form: every stored J_ij rounded to binary32, then
    to bfloat16."""
    J = sp.csr_matrix(J, dtype=np.float64, copy=True)
    J.data = bf16_value(J.data)
    return J


def fp8_rows(J: sp.csr_matrix):
    """Per-row FP8 form of the couplings: (J' as CSR FP64 of FP32 values,
    codes per stored entry, FP32 scale per row)."""
    J = sp.csr_matrix(J)
    J32 = J.data.astype(np.float32)
    n = J.shape[0]
    scale = np.ones(n, dtype=np.float32)
    codes = np.zeros(J32.shape[0], dtype=np.uint8)
    vals = np.zeros(J32.shape[0], dtype=np.float32)
    for i in range(n):
        lo, hi = J.indptr[i], J.indptr[i + 1]
        if hi == lo:
            continue
        mx = np.float32(np.max(np.abs(J32[lo:hi])))
        s = np.float32(mx / np.float32(E4M3_MAX)) if mx > 0 else np.float32(1.0)
        scale[i] = s
        q = np.clip((J32[lo:hi] / s).astype(np.float32), -E4M3_MAX, E4M3_MAX)
        codes[lo:hi] = e4m3_encode(q)
        vals[lo:hi] = (s * e4m3_value(codes[lo:hi]).astype(np.float32)).astype(np.float32)
    Jq = sp.csr_matrix((vals.astype(np.float64), J.indices.copy(), J.indptr.copy()), shape=J.shape)
    return Jq, codes, scale


def fp8_blocks(J: sp.csr_matrix, block: int = 8):
    """Per-block FP8 form: blocks of `block` consecutive stored couplings of
    each row.  Returns (J' as CSR FP64 of FP32 values, codes per stored
    entry, FP32 scale per block in row-major block order)."""
    J = sp.csr_matrix(J)
    J.sort_indices()
    J32 = J.data.astype(np.float32)
    codes = np.zeros(J32.shape[0], dtype=np.uint8)
    vals = np.zeros(J32.shape[0], dtype=np.float32)
    scales = []
    for i in range(J.shape[0]):
        for lo in range(J.indptr[i], J.indptr[i + 1], block):
            hi = min(lo + block, J.indptr[i + 1])
            mx = np.float32(np.max(np.abs(J32[lo:hi])))
            s = np.float32(mx / np.float32(E4M3_MAX)) if mx > 0 else np.float32(1.0)
            scales.append(s)
            q = np.clip((J32[lo:hi] / s).astype(np.float32), -E4M3_MAX, E4M3_MAX)
            codes[lo:hi] = e4m3_encode(q)
            vals[lo:hi] = (s * e4m3_value(codes[lo:hi]).astype(np.float32)).astype(np.float32)
    Jq = sp.csr_matrix((vals.astype(np.float64), J.indices.copy(), J.indptr.copy()), shape=J.shape)
    return Jq, codes, np.array(scales, dtype=np.float32)


def bf16x2_value(v) -> np.ndarray:
    """hi + lo with hi = bf16(fl32(v)), lo = bf16(fl32(v) - hi), as FP64."""
    v32 = np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)
    hi = bf16_value(v32)
    rest = v32 - hi                       # exact: fewer than 24 significant bits
    assert np.array_equal(rest.astype(np.float32).astype(np.float64), rest)
    return hi + bf16_value(rest)          # exact in binary32


def bf16x2_couplings(J: sp.csr_matrix) -> sp.csr_matrix:
    """The BF16-pair coupling form: every stored J_ij as hi + lo."""
    J = sp.csr_matrix(J, dtype=np.float64, copy=True)
    J.data = bf16x2_value(J.data)
    return J
