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
