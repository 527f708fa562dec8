"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one part of the oracle against something other than itself:
values printed in the paper (tests/golden), closed forms, invariants,
polynomial exactness or brute force.  No test here needs a GPU.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import frac, golden

R, W = oracle.quadrature()
SQ10 = math.sqrt(10.0)


def _expr(s):
    return float(eval(s, {"sqrt": math.sqrt}))


# --------------------------------------------------------------- quadrature --

def test_quadrature_matches_table_trots():
    g = golden("quadrature.json")
    roots = [_expr(s) for s in g["roots"]]
    weights = [_expr(s) for s in g["weights"]]
    np.testing.assert_allclose(R, roots, rtol=0, atol=1e-15)
    # the oracle computes W from Q!/He_6(R)^2; the table prints closed forms
    np.testing.assert_allclose(W, weights, rtol=2e-15, atol=0)
    assert abs(R[4] - g["p_max_printed"]) < 5e-3
    assert abs((W[2] / W[0]) ** 2 / g["weight_ratio_printed"] - 1) < 0.01


def test_roots_are_zeros_of_he5_and_weights_integrate_gaussian_moments():
    for r in R:
        assert abs(oracle.hermite(5, r)) < 1e-12
    assert abs(W.sum() - 1.0) < 1e-15
    # Gauss-Hermite Q = 5 is exact up to degree 9: E[p^2j] = (2j-1)!!
    for j in range(1, 5):
        dfact = float(np.prod(np.arange(2 * j - 1, 0, -2)))
        assert abs(np.sum(W * R ** (2 * j)) - dfact) < 1e-12 * dfact
        assert abs(np.sum(W * R ** (2 * j - 1))) < 1e-14


def test_hermite_recurrence_against_explicit_polynomials():
    # He_0..He_6 written out (Abramowitz & Stegun 22.3.11, probabilists' form)
    explicit = [lambda p: 1.0, lambda p: p, lambda p: p * p - 1, lambda p: p ** 3 - 3 * p,
                lambda p: p ** 4 - 6 * p ** 2 + 3, lambda p: p ** 5 - 10 * p ** 3 + 15 * p,
                lambda p: p ** 6 - 15 * p ** 4 + 45 * p ** 2 - 15]
    for l, fn in enumerate(explicit):
        for p in (-2.3, -0.7, 0.0, 0.4, 1.9):
            assert abs(oracle.hermite(l, p) - fn(p)) < 1e-12
    # orthogonality sum_q W He_l He_l' = l! delta (exact while l + l' <= 9)
    for l in range(5):
        for lp in range(5):
            s = sum(W[q] * oracle.hermite(l, R[q]) * oracle.hermite(lp, R[q]) for q in range(5))
            assert abs(s - (math.factorial(l) if l == lp else 0.0)) < 1e-12


# -------------------------------------------------------------- equilibrium --

def _gauss_moment(a, u, T):
    return [1.0, u, u * u + T, u ** 3 + 3 * u * T, u ** 4 + 6 * u * u * T + 3 * T * T][a]


@pytest.mark.parametrize("n,ux,uy,T", [(1.0, 0.0, 0.0, 1.0), (1.3, 0.02, -0.05, 0.8),
                                       (3.5, 0.3, 0.1, 0.514), (0.24, -0.4, 0.25, 1.6)])
def test_equilibrium_recovers_moments_up_to_fourth_order(n, ux, uy, T):
    fe = oracle.feq(n, ux, uy, T)
    px = np.array([R[k % 5] for k in range(25)])
    py = np.array([R[k // 5] for k in range(25)])
    for a in range(5):
        for b in range(5):
            got = np.sum(fe * px ** a * py ** b)
            want = n * _gauss_moment(a, ux, T) * _gauss_moment(b, uy, T)
            assert abs(got - want) < 1e-13 * max(1.0, abs(want)) * 10


def test_equilibrium_at_rest_unit_temperature_is_the_weights():
    fe = oracle.feq(2.0, 0.0, 0.0, 1.0)
    w = np.array([W[k % 5] * W[k // 5] for k in range(25)])
    np.testing.assert_allclose(fe, 2.0 * w, rtol=1e-15, atol=1e-17)


def test_equilibrium_factor_negative_outer_weight_below_0p6126():
    # g_outer(0, T) = w_1 [1 + (T-1)/2 He_2 + 3(T-1)^2/24 He_4](R_1) changes
    # sign near T = 0.6126 (a property of the truncated expansion).
    assert oracle.g(0, 0.0, 0.62) > 0.0
    assert oracle.g(0, 0.0, 0.60) < 0.0


# ----------------------------------------------------- momentum derivative --

def test_momentum_derivative_moment_identities():
    rng = np.random.default_rng(7)
    f = rng.uniform(0.1, 1.0, 25)
    dx, dy = oracle.dpf(f)
    px = np.array([R[k % 5] for k in range(25)])
    py = np.array([R[k // 5] for k in range(25)])
    n = f.sum()
    assert abs(dx.sum()) < 1e-14 and abs(dy.sum()) < 1e-14
    assert abs(np.sum(px * dx) + n) < 1e-13
    assert abs(np.sum(py * dy) + n) < 1e-13
    assert abs(np.sum(py * dx)) < 1e-13 and abs(np.sum(px * dy)) < 1e-13
    # energy: sum (p^2/2) d_px f = -sum p_x f
    assert abs(np.sum(0.5 * (px ** 2 + py ** 2) * dx) + np.sum(px * f)) < 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_momentum_derivative_product_rule(seed):
    # f = w(p_x) w(p_y) P(p_x) Q(p_y) with deg P, Q <= 4: the Hermite-projected
    # derivative is exact on the nodes, d_px f = w (P' - p P) Q (calculus of
    # the weight function e^{-p^2/2}).
    rng = np.random.default_rng(seed)
    P = np.polynomial.Polynomial(rng.normal(size=5))
    Qp = np.polynomial.Polynomial(rng.normal(size=5))
    f = np.array([W[k % 5] * W[k // 5] * P(R[k % 5]) * Qp(R[k // 5]) for k in range(25)])
    dx, dy = oracle.dpf(f)
    ex = np.array([W[k % 5] * W[k // 5] * (P.deriv()(R[k % 5]) - R[k % 5] * P(R[k % 5])) * Qp(R[k // 5])
                   for k in range(25)])
    ey = np.array([W[k % 5] * W[k // 5] * P(R[k % 5]) * (Qp.deriv()(R[k // 5]) - R[k // 5] * Qp(R[k // 5]))
                   for k in range(25)])
    scale = np.abs(ex).max() + np.abs(ey).max()
    np.testing.assert_allclose(dx, ex, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(dy, ey, rtol=0, atol=1e-13 * scale)


# ---------------------------------------------------------------- stencils --

def test_stencil_tables_match_printed_weights_and_1d_reductions():
    g = golden("stencils.json")
    gw, D = oracle.stencil_tables()
    for key, val in g["grad_weights"].items():
        l, m = (int(t) for t in key.split(","))
        assert gw[l, m] == pytest.approx(frac(val), abs=1e-16)
        assert gw[m, l] == pytest.approx(frac(val), abs=1e-16)
    # 1-D reductions: sum over m of the x-derivative coefficients
    for off, c in zip(g["grad_1d"]["offsets"], g["grad_1d"]["coeffs"]):
        s = sum(off * gw[abs(off), abs(m)] for m in range(-3, 4))
        assert s == pytest.approx(frac(c), abs=1e-15)
    for off, c in zip(g["glap_1d"]["offsets"], g["glap_1d"]["coeffs"]):
        s = sum(D[off + 3, m + 3] for m in range(-3, 4))
        assert s == pytest.approx(frac(c), abs=1e-15)


def test_printed_glap_coefficients_fail_the_1d_reduction():
    # Documents the reading: with the printed c1, c4 the |l| = 3 column of the
    # gradient-of-Laplacian stencil does not sum to the printed 1-D -1/8.
    g = golden("stencils.json")["glap_printed"]
    printed = frac(g["c4"]) + 2 * (frac(g["c3"]) + frac(g["c2"]) + frac(g["c1"]))
    assert abs(printed - (-1.0 / 8.0)) > 0.1
    r = golden("stencils.json")["glap_reading"]
    fixed = frac(r["c4"]) + 2 * (frac(g["c3"]) + frac(g["c2"]) + frac(r["c1"]))
    assert fixed == pytest.approx(-1.0 / 8.0, abs=1e-15)


def _poly_patch(fn, h):
    y, x = np.mgrid[-3:4, -3:4].astype(float) * h
    return fn(x, y)


@pytest.mark.parametrize("a,b", [(a, b) for a in range(7) for b in range(7) if a + b <= 6])
def test_stencils_exact_on_polynomials_up_to_degree_six(a, b):
    h = 0.37
    x0, y0 = 0.3, -0.2
    fn = lambda x, y: (x + x0) ** a * (y + y0) ** b
    patch = _poly_patch(fn, h)
    gx, gy = oracle.grad(patch, h, 3, 3)
    lx, ly = oracle.glap(patch, h, 3, 3)

    def d(p, k, s):  # k-th derivative of s^p
        if k > p:
            return 0.0
        return math.factorial(p) / math.factorial(p - k) * s ** (p - k)

    ex_gx = d(a, 1, x0) * d(b, 0, y0)
    ex_gy = d(a, 0, x0) * d(b, 1, y0)
    ex_lx = d(a, 3, x0) * d(b, 0, y0) + d(a, 1, x0) * d(b, 2, y0)
    ex_ly = d(a, 2, x0) * d(b, 1, y0) + d(a, 0, x0) * d(b, 3, y0)
    tol = 1e-11 * max(1.0, np.abs(patch).max()) / h ** 3
    assert abs(gx - ex_gx) < tol and abs(gy - ex_gy) < tol
    assert abs(lx - ex_lx) < tol and abs(ly - ex_ly) < tol


def test_stencil_orders_on_smooth_periodic_field():
    # gradient: 6th order; gradient of Laplacian: 4th order (Sec. 3.3)
    errs_g, errs_l = [], []
    for r, N in enumerate((24, 48)):
        h = 2 * np.pi / N
        y, x = np.mgrid[0:N, 0:N] * h
        fld = np.sin(x + 0.3) * np.cos(2 * y)
        i, j = 5 * (r + 1), 7 * (r + 1)      # the same physical point
        gx, _ = oracle.grad(fld, h, i, j)
        lx, _ = oracle.glap(fld, h, i, j)
        X, Y = i * h, j * h
        errs_g.append(abs(gx - np.cos(X + 0.3) * np.cos(2 * Y)))
        errs_l.append(abs(lx - (-5.0) * np.cos(X + 0.3) * np.cos(2 * Y)))
    assert math.log2(errs_g[0] / errs_g[1]) > 5.5
    assert math.log2(errs_l[0] / errs_l[1]) > 3.7


# -------------------------------------------------------------------- WENO --

def test_weno_candidates_and_ideal_weights_from_table():
    g = golden("weno_table.json")
    # for data e_j (unit vector), the candidate combination with ideal weights
    # must equal sum_q delta_q c_q[j] (linear scheme in the smooth limit)
    cands = np.array([[frac(c) for c in row] for row in g["candidates"]])
    ideal = np.array(g["ideal"])
    # smooth data: quadratic plus tiny cubic -> weights near ideal
    x = np.arange(-2, 3, dtype=float)
    v = 1.0 + 0.5 * x + 0.1 * x ** 2
    r, w = oracle.weno_recon(v)
    assert r == pytest.approx(float(np.dot(cands @ v, w)), rel=1e-14)
    assert r == pytest.approx(float(np.dot(ideal, cands @ v)), rel=1e-14)


def test_weno_vanishing_indicator_table():
    g = golden("weno_table.json")
    rows = {tuple(r["zero"]): [frac(s) for s in r["w"]] for r in g["rows"]}
    cases = {
        (1, 1, 1): [2.0, 2.0, 2.0, 2.0, 2.0],
        (0, 1, 1): [5.0, 2.0, 2.0, 2.0, 2.0],
        (1, 1, 0): [2.0, 2.0, 2.0, 2.0, 7.0],
        (1, 0, 0): [2.0, 2.0, 2.0, 3.0, 5.0],
        (0, 1, 0): [1.0, 2.0, 2.0, 2.0, 4.0],
        (0, 0, 1): [0.0, 5.0, 2.0, 2.0, 2.0],
    }
    for z, v in cases.items():
        _, w = oracle.weno_recon(np.array(v))
        np.testing.assert_allclose(w, rows[z], rtol=0, atol=1e-15)
    # the row (1, 0, 1) cannot occur: indicators 1 and 3 vanish only when all
    # five values are equal, which also zeroes indicator 2.


def test_weno_flux_difference_exact_for_quadratics():
    for coef in ([0.3, -1.2, 0.7], [2.0, 0.0, -0.05], [1e-3, 4e-4, 2e-5]):
        fn = lambda j: coef[0] + coef[1] * j + coef[2] * j * j
        for i in (-1.0, 0.0, 2.0):
            vp = np.array([fn(i + d) for d in (-2, -1, 0, 1, 2)])
            vm = np.array([fn(i - 1 + d) for d in (-2, -1, 0, 1, 2)])
            diff = oracle.weno_recon(vp)[0] - oracle.weno_recon(vm)[0]
            assert diff == pytest.approx(coef[1] + 2 * coef[2] * i, abs=1e-13)


def test_weno_fifth_order_on_smooth_monotone_data():
    errs = []
    for h in (0.1, 0.05):
        fn = lambda s: math.exp(s)
        vp = np.array([fn((j) * h) for j in (-2, -1, 0, 1, 2)])
        vm = np.array([fn((j - 1) * h) for j in (-2, -1, 0, 1, 2)])
        d = (oracle.weno_recon(vp)[0] - oracle.weno_recon(vm)[0]) / h
        errs.append(abs(d - 1.0))
    assert math.log2(errs[0] / errs[1]) > 4.5


# -------------------------------------------------------------- EOS helpers --

def test_eos_reduced_form_and_maxwell_construction():
    from oracle import analytic
    # general form with a = 9/8, b = 1/3 equals the printed reduced Eq. vdw
    for n, T in ((0.5, 0.8), (1.7, 1.1), (2.5, 0.3)):
        assert oracle.pw(n, T, 9 / 8, 1 / 3) == pytest.approx(3 * n * T / (3 - n) - 9 / 8 * n * n, rel=1e-14)
    g = golden("eos_values.json")
    ng, nl = analytic.maxwell(0.8)
    assert ng == pytest.approx(g["maxwell_T08"]["n_g"], abs=1e-7)
    assert nl == pytest.approx(g["maxwell_T08"]["n_l"], abs=g["maxwell_T08"]["tol_n_l"])
    s = analytic.spinodal(0.8)
    for got, want in zip(s, g["spinodal_T08"]["values"]):
        assert got == pytest.approx(want, abs=6e-4)
    k = 2 * math.pi
    cs = g["sound_speed_T08"]
    assert analytic.sound_coefficients(ng, 0.8, 5e-4, k, sigma=1e-4)[0] == pytest.approx(cs["model_vapour"], abs=6e-4)
    assert analytic.sound_coefficients(nl, 0.8, 5e-4, k, sigma=1e-4)[0] == pytest.approx(cs["model_liquid"], abs=6e-4)
    assert analytic.sound_coefficients(ng, 0.8, 5e-4, k, sigma=1e-4, true_vdw=True)[0] == pytest.approx(cs["vdw_vapour"], abs=6e-5)
    assert analytic.sound_coefficients(nl, 0.8, 5e-4, k, sigma=1e-4, true_vdw=True)[0] == pytest.approx(cs["vdw_liquid"], abs=6e-4)
    lm = g["lmin_T08"]
    assert 2 * math.pi / analytic.k_min(1e-4, 0.8) == pytest.approx(lm["L_min"], abs=6e-5)
    assert analytic.xi_wagner(1e-4, 0.8) == pytest.approx(lm["xi_w"], abs=6e-4)
