"""The package's coexistence solver (equal pressure and equal chemical
potential of the vdW free energy) against the oracle's equal-area Maxwell
construction and the densities the paper prints (Sec. 5).  CPU only."""
import numpy as np
import pytest

import olb_inputs as I
from conftest import golden
from oracle import analytic
from paper_1702_01690_amd import phase


@pytest.mark.parametrize("T", [0.74, 0.8, 0.85, 0.9, 0.95, 0.99])
def test_coexistence_equals_equal_area_construction(T):
    ng, nl = phase.maxwell_coexistence(T)
    rg, rl = analytic.maxwell(T)
    assert abs(ng - rg) <= 1e-11 * rg and abs(nl - rl) <= 1e-11 * rl


def test_coexistence_reproduces_printed_values_and_other_units():
    g = golden("eos_values.json")
    ng, nl = phase.maxwell_coexistence(0.8)
    m = g["maxwell_T08"]
    assert abs(ng - m["n_g"]) < 5e-7
    assert abs(nl - m["n_l"]) < m["tol_n_l"]
    # a = 9/49, b = 2/21 scales densities by 3.5 and temperatures by 4/7
    ng2, nl2 = phase.maxwell_coexistence(0.9 * I.T_CRIT, I.VDW_A, I.VDW_B)
    ng1, nl1 = phase.maxwell_coexistence(0.9)
    assert abs(ng2 - 3.5 * ng1) < 1e-11 and abs(nl2 - 3.5 * nl1) < 1e-10


def test_coexistence_far_below_the_critical_point():
    # equal pressure and chemical potential hold at the returned pair
    for T in (0.3, 0.5):
        ng, nl = phase.maxwell_coexistence(T)
        assert ng < nl
        p = lambda n: phase._pressure(n, T, 9 / 8, 1 / 3)
        mu = lambda n: phase._chemical_potential(n, T, 9 / 8, 1 / 3)
        assert abs(p(ng) - p(nl)) < 1e-12 and abs(mu(ng) - mu(nl)) < 1e-12
    with pytest.raises(ValueError):
        phase.maxwell_coexistence(1.0)


def test_surface_tension_of_a_tanh_profile():
    """Eq. gamma_int on n = c + b tanh((x - x0)/xi): sigma b^2 (4/3) / xi in
    closed form; the fourth-order rule on a resolved grid (xi = 6.7 ds) lands
    within its truncation error, and the error falls about 16-fold when the
    grid is refined twice."""
    from paper_1702_01690_amd import phase
    sigma, b, c, xi, x0 = 1e-4, 0.85, 1.09, 0.021, 0.25
    exact = sigma * b * b * (4.0 / 3.0) / xi
    errs = []
    for N in (160, 320):
        ds = 0.5 / N
        x = (np.arange(N) + 0.5) * ds
        n = c + b * np.tanh((x - x0) / xi)
        errs.append(abs(phase.surface_tension(n, ds, sigma) / exact - 1.0))
    assert errs[0] < 2e-4
    assert 10.0 < errs[0] / errs[1] < 25.0
    # a flat profile has none
    assert phase.surface_tension(np.full(50, 1.3), 0.01, 1e-4) == 0.0


def test_bubble_profile_pressures_and_laplace_fit():
    """The bubble analysis on a synthetic field with known answers: a tanh
    bubble of radius 0.2 and width 0.02 in R is recovered; the pressures
    inside and outside are those of the two uniform states (up to the tanh
    tails); gamma is the least-squares slope of dp against 1/R through the
    origin."""
    from paper_1702_01690_amd import phase
    N, ds = 160, 1.0 / 320
    c = (np.arange(N) + 0.5) * ds
    R = np.hypot(c[None, :], c[:, None])
    n = 1.1 + 0.8 * np.tanh((R - 0.2) / 0.02)
    rf, xi, nin, nout = phase.bubble_profile(n, ds, 0.22, 0.03)
    assert abs(rf - 0.2) < 1e-10 and abs(xi - 0.02) < 1e-10
    assert abs(nin - 0.3) < 1e-10 and abs(nout - 1.9) < 1e-10
    T = np.full((N, N), 0.8)
    pin, pout = phase.bubble_pressures(n, T, ds, rf, xi)
    ref = lambda q: q * 0.8 / (1 - q / 3) - 9 / 8 * q * q
    # the tanh tails beyond 5 xi still move n by up to 1e-4
    assert abs(pin - ref(0.3)) < 2e-5 and abs(pout - ref(1.9)) < 2e-5
    radii = np.array([0.15, 0.2, 0.3])
    assert phase.laplace_tension(radii, 4.9e-3 / radii) == pytest.approx(4.9e-3, rel=1e-14)
    noisy = 4.9e-3 / radii + np.array([1e-5, -2e-5, 1e-5])
    x = 1 / radii
    assert phase.laplace_tension(radii, noisy) == pytest.approx(np.dot(x, noisy) / np.dot(x, x), rel=1e-14)


def test_interface_width_fit_recovers_a_tanh_profile():
    from paper_1702_01690_amd import phase
    ds = 1.0 / 320
    x = (np.arange(160) + 0.5) * ds
    n = 1.09 + 0.85 * np.tanh((x - 0.2513) / 0.0197)
    xi, xpos = phase.interface_width(n, ds, 0.25, 0.021)
    assert xi == pytest.approx(0.0197, rel=1e-9) and xpos == pytest.approx(0.2513, rel=1e-9)
