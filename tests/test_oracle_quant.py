"""Pins of the oracle's FP8 coupling form against torch's own E4M3
(float8_e4m3fn) conversion, a library routine independent of the oracle,
and against closed-form facts of the format."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import quant

torch = pytest.importorskip("torch")


def _torch_value(codes):
    t = torch.from_numpy(np.asarray(codes, dtype=np.uint8)).view(torch.float8_e4m3fn)
    return t.to(torch.float64).numpy()


def _torch_code(v32):
    t = torch.from_numpy(np.asarray(v32, dtype=np.float32)).to(torch.float8_e4m3fn)
    return t.view(torch.uint8).numpy()


def test_every_code_decodes_like_the_library():
    codes = np.arange(256, dtype=np.uint8)
    ours, ref = quant.e4m3_value(codes), _torch_value(codes)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert nan.sum() == 2                     # S.1111.111 only: no infinities
    assert np.array_equal(ours[~nan], ref[~nan])


def test_format_constants():
    v = quant.e4m3_value(np.arange(0x7F, dtype=np.uint8))
    assert v.max() == 448.0
    assert v[1] == 2.0 ** -9                  # smallest subnormal
    assert v[8] == 2.0 ** -6                  # smallest normal
    assert np.all(np.diff(v) > 0)             # codes are monotone in value


def test_encode_matches_library_on_values_midpoints_and_random():
    reps = quant.e4m3_value(np.arange(0x7F, dtype=np.uint8))
    mids = (reps[:-1] + reps[1:]) / 2         # exact ties: even code wins
    rng = np.random.default_rng(7)
    rand = np.concatenate([rng.uniform(-448, 448, 20000),
                           np.exp2(rng.uniform(-12, 8.8, 20000)) * rng.choice([-1, 1], 20000)])
    rand = np.clip(rand, -448, 448)
    for v in (reps, -reps, mids, -mids, np.nextafter(mids, 0), np.nextafter(mids, 1000), rand):
        v32 = np.asarray(v, dtype=np.float32)
        v32 = v32[np.abs(v32) <= 448]
        ours = quant.e4m3_encode(v32)
        ref = _torch_code(v32)
        # the library keeps the sign of values that round to zero; the value is 0 either way
        same = (ours == ref) | ((ours & 0x7F) == 0) & ((ref & 0x7F) == 0)
        assert np.all(same), v32[~same][:5]


def test_ties_go_to_even_code():
    # 1 + 1/16 lies halfway between 1 (code 0x38, mantissa 0) and 1.125 (0x39)
    assert quant.e4m3_encode([1.0625])[0] == 0x38
    # 1.1875 lies halfway between 1.125 (0x39) and 1.25 (0x3A, even)
    assert quant.e4m3_encode([1.1875])[0] == 0x3A
    # halfway between the two smallest subnormals rounds to the even one
    assert quant.e4m3_encode([1.5 * 2.0 ** -9])[0] == 0x02
    with pytest.raises(ValueError):
        quant.e4m3_encode([449.0])


def test_row_form_scales_each_row_to_the_format_maximum():
    rng = np.random.default_rng(3)
    n = 40
    A = sp.random(n, n, density=0.2, random_state=4, data_rvs=lambda k: rng.normal(0, 1, k))
    A = sp.csr_matrix(A + A.T)
    A.sort_indices()
    Jq, codes, scale = quant.fp8_rows(A)
    J32 = A.data.astype(np.float32)
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        if hi == lo:
            assert scale[i] == 1.0
            continue
        k = lo + int(np.argmax(np.abs(J32[lo:hi])))
        # the largest entry of each row maps onto +-448 (code 0x7E / 0xFE)
        assert codes[k] & 0x7F == 0x7E
        # relative error of an E4M3 normal is at most 2^-4
        big = np.abs(J32[lo:hi]) >= scale[i] * 2.0 ** -6
        err = np.abs(Jq.data[lo:hi] - J32[lo:hi])[big] / np.abs(J32[lo:hi])[big]
        assert np.all(err <= 2.0 ** -4 + 1e-6)
    # structure is unchanged
    assert np.array_equal(Jq.indptr, A.indptr) and np.array_equal(Jq.indices, A.indices)


# ------------------------------------------------------- 16-bit forms

def _all_finite_fp16():
    v = np.arange(1 << 16, dtype=np.uint16).view(np.float16)
    return v[np.isfinite(v)].astype(np.float64)


def test_fp16_every_value_midpoint_and_neighbour_matches_numpy():
    """Every finite binary16 value, every midpoint between neighbours
    (exact in FP64) and the FP64 values just below and above each midpoint,
    rounded by the oracle and by NumPy's own float64 -> float16 cast."""
    v = np.unique(_all_finite_fp16())
    mids = (v[:-1] + v[1:]) / 2.0
    cases = np.concatenate([v, mids, np.nextafter(mids, -np.inf), np.nextafter(mids, np.inf)])
    cases = cases[np.abs(cases) < 65504.0]
    ref = cases.astype(np.float16).astype(np.float64)
    assert np.array_equal(quant.fp16_value(cases), ref)


def test_fp16_random_couplings_match_numpy():
    rng = np.random.default_rng(5)
    v = rng.normal(0, 0.3, 200_000) * np.exp2(rng.integers(-30, 4, 200_000))
    assert np.array_equal(quant.fp16_value(v), v.astype(np.float16).astype(np.float64))


def test_fp16_ties_and_subnormals_by_hand():
    one_ulp = 2.0 ** -10
    assert quant.fp16_value(1.0 + one_ulp / 2) == 1.0                 # tie -> even
    assert quant.fp16_value(1.0 + 1.5 * one_ulp) == 1.0 + 2 * one_ulp  # tie -> even
    assert quant.fp16_value(2.0 ** -24) == 2.0 ** -24                  # smallest subnormal
    assert quant.fp16_value(2.0 ** -25) == 0.0                         # tie to zero (even)
    assert quant.fp16_value(3 * 2.0 ** -26) == 2.0 ** -24
    assert quant.fp16_value(-0.25) == -0.25
    with pytest.raises(ValueError):
        quant.fp16_value(70000.0)


def _bf16_grid(lo_exp, hi_exp):
    """Every positive bfloat16 value with exponent in [lo_exp, hi_exp]
    (subnormals included when lo_exp <= -126), as FP64."""
    m = np.arange(128, dtype=np.float64)
    out = [m * 2.0 ** (-126 - 7)] if lo_exp <= -126 else []
    for e in range(max(lo_exp, -126), hi_exp + 1):
        out.append((1.0 + m / 128.0) * 2.0 ** e)
    return np.unique(np.concatenate(out))


def _torch_bf16(v64):
    t = torch.from_numpy(np.asarray(v64, dtype=np.float64)).to(torch.float32)
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_every_midpoint_and_neighbour_matches_torch():
    """bfloat16 values from the subnormals to 2^40, the midpoints between
    neighbours (exact in binary32) and the binary32 values next to each
    midpoint, both signs, against torch's float32 -> bfloat16 cast."""
    v = _bf16_grid(-133, 40)
    mids = (v[:-1] + v[1:]) / 2.0
    m32 = mids.astype(np.float32)
    assert np.array_equal(m32.astype(np.float64), mids)
    cases = np.concatenate([v, mids, np.nextafter(m32, np.float32(-np.inf)).astype(np.float64),
                            np.nextafter(m32, np.float32(np.inf)).astype(np.float64)])
    cases = np.concatenate([cases, -cases])
    assert np.array_equal(quant.bf16_value(cases), _torch_bf16(cases))


def test_bf16_rounds_through_binary32_first():
    """An FP64 value a hair above a bfloat16 midpoint, closer to the
    midpoint than half a binary32 ulp, becomes the midpoint in binary32 and
    then ties to even -- the kernels' two-step conversion (torch's cast of
    the binary32 value agrees)."""
    lo = 1.0
    mid = lo + 2.0 ** -8                       # halfway to 1 + 2^-7
    v = mid + 2.0 ** -30                       # below half a binary32 ulp (2^-24)
    assert np.float64(np.float32(v)) == mid
    assert quant.bf16_value(v) == 1.0           # tie -> even (1.0), not up
    assert _torch_bf16([v])[0] == 1.0
    rng = np.random.default_rng(8)
    r = rng.normal(0, 0.3, 200_000) * np.exp2(rng.integers(-40, 4, 200_000))
    assert np.array_equal(quant.bf16_value(r), _torch_bf16(r))


def test_16bit_coupling_forms_keep_the_sparsity():
    J = sp.random(40, 40, density=0.1, random_state=3, format="csr")
    for f, g in ((quant.fp16_couplings, quant.fp16_value), (quant.bf16_couplings, quant.bf16_value)):
        Jq = f(J)
        assert np.array_equal(Jq.indptr, J.indptr) and np.array_equal(Jq.indices, J.indices)
        assert np.array_equal(Jq.data, g(J.data))


# ------------------------------------------------ FP8 blocks, BF16 pairs

def test_fp8_blocks_partition_rows_in_blocks_of_eight():
    rng = np.random.default_rng(2)
    lens = [0, 1, 7, 8, 9, 16, 23]
    rows, cols, vals = [], [], []
    n = 40
    for i, L in enumerate(lens):
        cs = np.sort(rng.choice(n, L, replace=False))
        rows += [i] * L
        cols += list(cs)
        vals += list(rng.normal(0, 0.2, L) * np.exp2(rng.integers(-6, 3, L)))
    J = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    Jq, codes, scales = quant.fp8_blocks(J)
    assert scales.shape[0] == sum((L + 7) // 8 for L in lens)
    k = 0
    for i in range(len(lens)):
        lo, hi = J.indptr[i], J.indptr[i + 1]
        for b in range(lo, hi, 8):
            e = min(b + 8, hi)
            blk = J.data[b:e].astype(np.float32)
            s = scales[k]
            k += 1
            assert s == np.float32(np.float32(np.abs(blk).max()) / np.float32(448.0))
            # torch's own E4M3 cast of the scaled block, decoded and rescaled
            ref = _torch_code(np.clip(blk / s, -448, 448).astype(np.float32))
            assert np.array_equal(codes[b:e], ref)
            assert np.array_equal(Jq.data[b:e], (s * _torch_value(ref).astype(np.float32)).astype(
                np.float32).astype(np.float64))
            assert np.abs(Jq.data[b:e]).max() == np.float32(s * np.float32(448.0))
            # relative to its block's largest coupling, error <= 2^-4
            assert np.all(np.abs(Jq.data[b:e] - blk) <= 2.0 ** -4 * np.abs(blk).max())


def test_fp8_blocks_beat_rows_on_mixed_scales():
    """A row whose first block of eight couplings is near 1 and second near
    5e-6: per-row scaling puts the small ones among the FP8 subnormals,
    per-block scaling gives them their own scale."""
    vals = np.array([1.0 - 0.05 * k for k in range(8)] + [5e-6 * (1 + 0.1 * k) for k in range(8)])
    J = sp.csr_matrix((vals, ([0] * 16, np.arange(1, 17))), shape=(17, 17))
    small = slice(8, 16)
    er = np.abs(quant.fp8_rows(J)[0].data[small] - vals[small]) / vals[small]
    eb = np.abs(quant.fp8_blocks(J)[0].data[small] - vals[small]) / vals[small]
    assert eb.max() <= 2.0 ** -4 and er.max() > 4 * eb.max()


def test_bf16x2_matches_torch_pair_and_bounds():
    rng = np.random.default_rng(4)
    v = rng.normal(0, 0.3, 100_000) * np.exp2(rng.integers(-30, 4, 100_000))
    v32 = torch.from_numpy(v.astype(np.float32))
    hi = v32.to(torch.bfloat16).to(torch.float32)
    lo = (v32 - hi).to(torch.bfloat16).to(torch.float32)
    ref = (hi + lo).to(torch.float64).numpy()
    got = quant.bf16x2_value(v)
    assert np.array_equal(got, ref)
    x32 = v.astype(np.float32).astype(np.float64)
    # 16 significant bits: relative error <= 2^-16
    assert np.all(np.abs(got - x32) <= 2.0 ** -16 * np.abs(x32))
    assert np.array_equal(got.astype(np.float32).astype(np.float64), got)
    J = sp.random(30, 30, density=0.2, random_state=1, format="csr")
    assert np.array_equal(quant.bf16x2_couplings(J).data, quant.bf16x2_value(J.data))
