"""Host-side analysis of the shear-wave sweep (Sec. 6.1): the amplitude
projection (Eq. shear_ut), the decay-rate fit behind eta_app, the trapezoid
L2 norm (Eq. shear_L2) and the power-law exponents, each against a closed
form or an independent library fit."""
import numpy as np
import pytest

import olb_inputs as I
from conftest import golden
from paper_1702_01690_amd import galilei as G

T0, TAU, U0 = 0.8, 5e-4, 1e-3
NU = (2 * np.pi) ** 2 * TAU * T0
TIMES = np.arange(201) * 0.2


@pytest.mark.parametrize("N,V,t", [(20, 0.0, 0.0), (30, 0.7, 3.1), (60, 2.0, 17.3)])
def test_amplitude_of_a_pure_mode_is_its_amplitude(N, V, t):
    c = I.shear_wave(N, V)
    x = c.extra["x"]
    uy = 0.37 * U0 * np.sin(2 * np.pi * (x - V * t))
    assert G.amplitude(uy, x, V, t) == pytest.approx(0.37 * U0, rel=1e-13)
    # the companion cosine mode does not leak into the projection
    assert abs(G.amplitude(np.cos(2 * np.pi * (x - V * t)), x, V, t)) < 1e-13


def test_shear_wave_inputs_follow_the_setup():
    g = golden("shear_galilei.json")["setup"]
    c = I.shear_wave(20, 1.5)
    p = c.params
    assert (p["nx"], p["ny"]) == (20, 1)
    assert p["ds"] == 1 / 20 and p["dt"] == g["dt"] and p["tau"] == g["tau"]
    assert np.all(c.ux == 1.5) and np.all(c.T == g["T0"]) and p["a"] == 0.0
    # x_i = (i - 1/2)/N - 1/2 for i = 1..N
    assert c.extra["x"][0] == pytest.approx(0.5 / 20 - 0.5) and c.extra["x"][-1] == pytest.approx(0.5 - 0.5 / 20)
    assert G.amplitude(c.uy, c.extra["x"], 1.5, 0.0) == pytest.approx(g["u0"], rel=1e-13)


def test_decay_rate_recovers_an_exact_exponential():
    a = U0 * np.exp(-1.0123 * NU * TIMES)
    assert G.decay_rate(a, TIMES, U0) == pytest.approx(1.0123 * NU, rel=1e-13)
    assert G.viscosity_ratio(a, TIMES, U0, TAU, T0) == pytest.approx(1.0123, rel=1e-13)


def test_decay_rate_is_the_least_squares_minimiser():
    from scipy.optimize import curve_fit
    rng = np.random.default_rng(3)
    a = U0 * np.exp(-NU * TIMES) * (1 + 1e-3 * np.sin(5 * TIMES)) + 1e-7 * rng.standard_normal(TIMES.size)
    ours = G.decay_rate(a, TIMES, U0)
    ref = curve_fit(lambda t, v: U0 * np.exp(-v * t), TIMES, a, p0=[NU], xtol=1e-15, ftol=1e-15)[0][0]
    assert ours == pytest.approx(ref, rel=1e-9)
    res = lambda v: np.sum((a - U0 * np.exp(-v * TIMES)) ** 2)
    assert res(ours) <= min(res(ours * (1 + 1e-6)), res(ours * (1 - 1e-6)))


def test_l2_norm_closed_forms():
    lin = U0 * np.exp(-NU * TIMES)
    assert G.l2_norm(lin, TIMES, U0, TAU, T0) == pytest.approx(0.0, abs=1e-15)
    # constant relative error eps: the weights sum to S, so L2 = eps
    assert G.l2_norm(lin * (1 + 2e-4), TIMES, U0, TAU, T0) == pytest.approx(2e-4, rel=1e-9)
    # error only at the last sample (weight 1/2): L2 = eps / sqrt(2 S)
    a = lin.copy()
    a[-1] *= 1 + 1e-3
    assert G.l2_norm(a, TIMES, U0, TAU, T0) == pytest.approx(1e-3 / np.sqrt(400), rel=1e-9)


def test_orders_recover_planted_power_laws():
    sizes, media = (20, 30, 40, 50, 60), ("ideal",)
    speeds = (0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 1.0, 2.0)
    res = {}
    for N in sizes:
        for V in speeds:
            dx = 1.0 / N
            res[("ideal", N, V)] = (1 + 3.0 * dx ** 4.9 + 0.2 * dx * V ** 2.0,
                                    2.0 * dx ** 4.8 + 0.1 * dx * V ** 1.9)
    dxo, vo = G.orders(res, media, sizes)
    # at V = 0 the planted laws are pure powers of dx (eta - 1 of order 1e-9
    # is stored next to 1, which costs it about 8 digits)
    assert dxo["ideal"][0.0] == pytest.approx((4.9, 4.8), abs=1e-6)
    for N in sizes:
        # the V = 0 parts cancel in the departure, leaving pure powers of V
        assert vo["ideal"][N] == pytest.approx((2.0, 1.9), abs=1e-9)


def test_sound_linear_reduces_to_the_ideal_gas_and_matches_printed_limits():
    """Ideal gas (a = b = sigma = 0): c_s = sqrt(2 T), nu_a = nu_t = tau k^2 T
    (the closed forms Sec. 6.2 prints) and S = 0; the vdW liquid has the
    oracle-independent property c_s^2 = dp/dn + T/(1 - b n) + n k^2 sigma."""
    cs, nua, nut, S = G.sound_linear(1.0, 0.8, 5e-4)
    assert cs == pytest.approx(np.sqrt(1.6), rel=1e-15)
    assert nua == pytest.approx(5e-4 * (2 * np.pi) ** 2 * 0.8, rel=1e-14)
    assert nut == pytest.approx(nua, rel=1e-14) and abs(S) < 1e-15
    n, T, a, b, s = 1.932703, 0.8, 9 / 8, 1 / 3, 1e-4
    cs, *_ = G.sound_linear(n, T, 5e-4, a=a, b=b, sigma=s)
    dpdn = T / (1 - b * n) ** 2 - 2 * a * n
    assert cs ** 2 == pytest.approx(dpdn + T / (1 - b * n) + n * (2 * np.pi) ** 2 * s, rel=1e-14)


def test_sound_fit_recovers_a_damped_oscillation():
    t = np.arange(501) * 0.02
    a = 1e-3 * np.exp(-0.017 * t) * (np.cos(1.13 * 2 * np.pi * t) - 2e-4 * np.sin(1.13 * 2 * np.pi * t))
    nu, c, S = G.sound_fit(a, t, 1e-3, 0.02, 1.1, 0.0)
    assert nu == pytest.approx(0.017, rel=1e-9) and c == pytest.approx(1.13, rel=1e-12)
    assert S == pytest.approx(-2e-4, rel=1e-6)
    nu, c, S = G.sound_fit(1e-3 * np.exp(-0.02 * t) * np.cos(1.26 * 2 * np.pi * t), t, 1e-3, 0.015, 1.2)
    assert nu == pytest.approx(0.02, rel=1e-9) and c == pytest.approx(1.26, rel=1e-12) and S == 0.0
