"""The FP32 WENO-5 reconstruction scales its three smoothness indicators by
one factor c taken from the bits of the largest, m: c = bits^-1(0x7e800000 -
bits(m)).  For a normal m = (1 + u) 2^(E-127) this encodes c = (2 - u) 2^(125-E),
so c m = (2 - u)(1 + u) / 4 lies in [1/2, 9/16]: the scaled indicators stay
below 1 and their fourth powers (the weights) inside the FP32 range.  Checked
here on the host for every binade of m below 2^125 (differences below about
1e18; from 2^125 on c would fall below the normal range), with the same 32-bit
arithmetic."""
import numpy as np


def _scale(m):
    bits = np.asarray(m, dtype=np.float32).view(np.uint32)
    return (np.uint32(0x7E800000) - bits).astype(np.uint32).view(np.float32)


def test_scaled_largest_indicator_lies_in_half_to_nine_sixteenths():
    rng = np.random.default_rng(7)
    # every binade of the normal range below 2^125, several mantissas each
    exps = np.arange(-126, 125)
    mant = rng.random((exps.size, 64), dtype=np.float64)
    m = np.ldexp(1.0 + mant, exps[:, None]).astype(np.float32).ravel()
    m = np.concatenate([m, np.float32([1.0, 1.5, np.nextafter(np.float32(2), np.float32(0)),
                                       np.finfo(np.float32).tiny,
                                       np.nextafter(np.float32(2.0 ** 125), np.float32(0))])])
    c = _scale(m).astype(np.float64)
    prod = c * m.astype(np.float64)
    assert np.all(prod >= 0.5) and np.all(prod <= 9.0 / 16.0 + 1e-12)
    # the closed form (2 - u) 2^(125 - E), E the biased exponent
    mm, ee = np.frexp(m.astype(np.float64))          # m = mm 2^ee, mm in [1/2, 1)
    u = 2.0 * mm - 1.0                               # m = (1 + u) 2^(ee - 1), E = ee + 126
    np.testing.assert_allclose(c, (2.0 - u) * np.ldexp(1.0, -1 - ee), rtol=0, atol=0)


def test_subnormal_and_zero_largest_indicator():
    # below the normal range the product stays under 1/2 (weights of values that
    # agree far below FP32 rounding); m = 0 gives c = 2^126 and scaled zeros
    sub = np.float32([1e-45, 1e-40, 1.1e-38])
    prod = _scale(sub).astype(np.float64) * sub.astype(np.float64)
    assert np.all(prod > 0.0) and np.all(prod <= 0.5)
    assert _scale(np.float32(0.0)) == np.float32(2.0 ** 126)
