"""Pins of the FP64 closure oracle (oracle/cnn.py) against independent facts.

* conv3x3 equals scipy.ndimage.correlate with periodic wrap, summed over
  input channels (an independent library routine);
* the analytic gradient equals central finite differences of the loss
  (directional derivatives and single parameters, pure float64);
* bf16 rounding equals torch's float32 -> bfloat16 conversion and the
  half-to-even cases worked out by hand;
* Adam's first step and any step under a constant gradient move every
  parameter by lr g / (|g| + eps) (bias correction makes m_hat = g, v_hat = g^2);
* the restriction conserves mass, momentum and energy, reproduces
  block-constant fields, and is local to its blocks;
* the correction gives a distribution whose moments are m + dm exactly (the
  quadrature reproduces the equilibrium's moments), leaves f alone where dm
  = 0, and skips inadmissible nodes.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import olb_inputs as I
import oracle
from oracle import cnn


def _net_inputs(nx=7, ny=5, seed=3):
    params = I.closure_params(seed=seed, last_scale=1.0).astype(np.float64)
    # non-zero biases so that every block of the gradient is exercised
    d = cnn.unpack(params.copy())
    rng_b = I.uniform(seed + 100, 68) - 0.5
    d["b1"][:] = 0.1 * rng_b[:32]
    d["b2"][:] = 0.1 * rng_b[32:64]
    d["b3"][:] = 0.1 * rng_b[64:68]
    params = cnn.pack(d)
    m = I.closure_moments(nx, ny, seed=seed + 1)
    ref = m + 0.01 * (I.closure_moments(nx, ny, seed=seed + 2) - m)
    norm = (m.mean(axis=(1, 2)), m.std(axis=(1, 2)), np.abs(ref - m).std(axis=(1, 2)))
    return params, m, ref, norm


def test_conv3x3_equals_scipy_correlate_with_wrap():
    x = I.closure_moments(9, 6, seed=4)
    W = (I.uniform(5, 3 * 4 * 9).reshape(3, 4, 3, 3) - 0.5)
    b = np.array([0.1, -0.2, 0.3])
    out = cnn.conv3x3(x, W, b)
    for o in range(3):
        ref = b[o] + sum(ndi.correlate(x[c], W[o, c], mode="wrap") for c in range(4))
        np.testing.assert_allclose(out[o], ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_translation_equivariance():
    x = I.closure_moments(8, 5, seed=6)
    W = I.uniform(7, 2 * 4 * 9).reshape(2, 4, 3, 3) - 0.5
    b = np.zeros(2)
    shifted = np.roll(x, (2, 3), axis=(1, 2))
    np.testing.assert_allclose(cnn.conv3x3(shifted, W, b), np.roll(cnn.conv3x3(x, W, b), (2, 3), axis=(1, 2)),
                               rtol=1e-13, atol=1e-14)


def test_gradient_directional_derivatives_match_finite_differences():
    params, m, ref, norm = _net_inputs()
    L0, g = cnn.loss_and_gradient(params, m, ref, norm)
    assert L0 > 0
    for seed in (21, 22, 23):
        d = I.uniform(seed, params.size) - 0.5
        h = 1e-6
        Lp, _ = cnn.loss_and_gradient(params + h * d, m, ref, norm)
        Lm, _ = cnn.loss_and_gradient(params - h * d, m, ref, norm)
        fd = (Lp - Lm) / (2 * h)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12, (fd, an)


@pytest.mark.parametrize("block", ["W1", "b1", "W2", "b2", "W3", "b3"])
def test_gradient_single_parameters_match_finite_differences(block):
    params, m, ref, norm = _net_inputs(nx=6, ny=6, seed=8)
    _, g = cnn.loss_and_gradient(params, m, ref, norm)
    offsets, o = {}, 0
    for name, shape in cnn.BLOCKS:
        offsets[name] = (o, int(np.prod(shape)))
        o += int(np.prod(shape))
    start, size = offsets[block]
    picks = start + (I.uniform(31, 6) * size).astype(int)
    # the loss is piecewise quadratic in any one parameter, so the central
    # difference is exact up to rounding (about 1e-16 L / h) away from ReLU kinks
    for k in picks:
        h = 1e-5
        e = np.zeros_like(params)
        e[k] = h
        fd = (cnn.loss_and_gradient(params + e, m, ref, norm)[0] -
              cnn.loss_and_gradient(params - e, m, ref, norm)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * abs(g[k]) + 1e-10, (block, k, fd, g[k])


def test_bf16_rounding_matches_torch_and_hand_cases():
    import torch
    x = (I.uniform(41, 5000) - 0.5) * 10.0 ** (8 * I.uniform(42, 5000) - 4)
    x32 = x.astype(np.float32).astype(np.float64)   # torch rounds from float32
    ref = torch.tensor(x32, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x32), ref)
    # ties to even around 1 (bf16 spacing 2^-7 there)
    assert cnn.bf16(1.0 + 2.0 ** -8) == 1.0
    assert cnn.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert cnn.bf16(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    assert cnn.bf16(0.0) == 0.0


def test_adam_closed_forms():
    g = np.array([1e-3, -2.0, 5e-9, 0.0, 30.0])
    p0 = np.array([0.5, -0.5, 1.0, 2.0, 0.0])
    lr, eps = 1e-3, 1e-8
    p, m, v = cnn.adam(p0, g, np.zeros(5), np.zeros(5), 1, lr)
    np.testing.assert_allclose(p0 - p, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
    for t in range(2, 40):
        prev = p
        p, m, v = cnn.adam(p, g, m, v, t, lr)
        np.testing.assert_allclose(prev - p, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-18)


def test_restriction_conserves_and_reproduces_block_constants():
    f = I.closure_moments(16, 12, seed=51, amplitude=0.05)
    c = cnn.restrict(f, 4)
    n, ux, uy, T = f
    cn, cux, cuy, cT = c
    r2 = 16.0
    assert np.isclose(cn.sum() * r2, n.sum(), rtol=1e-14)
    assert np.isclose((cn * cux).sum() * r2, (n * ux).sum(), rtol=1e-12)
    assert np.isclose((cn * cuy).sum() * r2, (n * uy).sum(), rtol=1e-12)
    e = (n * (ux * ux + uy * uy + 2 * T)).sum()
    assert np.isclose((cn * (cux * cux + cuy * cuy + 2 * cT)).sum() * r2, e, rtol=1e-13)
    # block-constant fields restrict to their constants
    blocks = I.closure_moments(4, 3, seed=52)
    fine = np.repeat(np.repeat(blocks, 4, axis=1), 4, axis=2)
    np.testing.assert_allclose(cnn.restrict(fine, 4), blocks, rtol=1e-14)
    # locality: changing one fine node changes only its block
    g = f.copy()
    g[0, 5, 9] *= 1.01
    diff = np.any(cnn.restrict(g, 4) != c, axis=0)
    assert diff.sum() == 1 and diff[1, 2]


def test_restriction_of_uniform_drift_keeps_temperature():
    # uniform velocity and temperature with varying density: u and T pass through
    f = I.closure_moments(8, 8, seed=53)
    f[1] = 0.02
    f[2] = -0.01
    f[3] = 0.5
    c = cnn.restrict(f, 4)
    np.testing.assert_allclose(c[1], 0.02, rtol=1e-13)
    np.testing.assert_allclose(c[2], -0.01, rtol=1e-13)
    np.testing.assert_allclose(c[3], 0.5, rtol=1e-13)


def _moments_of(f, params):
    o = oracle.Oracle(params)
    o.set_f(f)
    return np.stack(o.moments())


def test_correction_moves_moments_by_dm_and_skips_inadmissible():
    params = I.coarse_params(I.closure_sample(32, 24, seed=5001).params, precision=0)
    m = I.closure_moments(params["nx"], params["ny"], seed=61)
    o = oracle.Oracle(params)
    o.set_fields(*m)
    o.step(2)                     # a non-equilibrium f
    f = o.get_f()
    m = np.stack(o.moments())
    dm = 0.01 * (I.closure_moments(params["nx"], params["ny"], seed=62) - I.closure_moments(params["nx"], params["ny"], seed=63))
    dm[0, 0, 0] = 20.0            # n + dn > 1/b: skipped
    dm[3, 1, 2] = -5.0            # T + dT < 0: skipped
    g, skipped = cnn.apply_correction(f, m, dm, params["b"], oracle.feq)
    assert skipped.sum() == 2 and skipped[0, 0] and skipped[1, 2]
    np.testing.assert_array_equal(g[:, skipped], f[:, skipped])
    m2 = _moments_of(g, params)
    ok = ~skipped
    target = m + dm
    np.testing.assert_allclose(m2[0][ok], target[0][ok], rtol=1e-13)
    np.testing.assert_allclose(m2[1][ok], target[1][ok], rtol=0, atol=1e-13)
    np.testing.assert_allclose(m2[2][ok], target[2][ok], rtol=0, atol=1e-13)
    np.testing.assert_allclose(m2[3][ok], target[3][ok], rtol=1e-12)
    same, _ = cnn.apply_correction(f, m, np.zeros_like(dm), params["b"], oracle.feq)
    np.testing.assert_allclose(same, f, rtol=1e-15, atol=1e-15)


def test_conservative_projection_zeroes_channel_totals():
    params, m, ref, norm = _net_inputs(nx=6, ny=5, seed=12)
    raw = cnn.correction(params, m, norm)
    for mask in (1, 7, 15):
        dm = cnn.correction(params, m, norm, conserve_mask=mask)
        for c in range(4):
            if (mask >> c) & 1:
                assert abs(dm[c].sum()) <= 1e-12 * np.abs(dm[c]).sum()
                # only the uniform part is removed
                np.testing.assert_allclose(dm[c] - raw[c], (dm[c] - raw[c]).mean(), rtol=0, atol=1e-15)
            else:
                np.testing.assert_array_equal(dm[c], raw[c])
