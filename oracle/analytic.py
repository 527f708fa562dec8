"""Closed-form helpers used to pin the oracle (test infrastructure).

Every function states the passage it follows.  The van der Waals pressure is
taken from the oracle library itself (``oracle.pw``) wherever the printed
numbers are meant to pin it.
"""
import math

import numpy as np
from scipy import integrate, optimize

from . import pw as _pw


def maxwell(T, a=9.0 / 8.0, b=1.0 / 3.0):
    """Coexisting gas / liquid densities at temperature T by the equal-area
    (Maxwell) construction on p^w(n, T) (Sec. 4, planar interface): equal
    pressure and  int_{v_l}^{v_g} p dv = p_sat (v_g - v_l),  v = 1/n."""
    p = lambda n: _pw(n, T, a, b)
    nmax = 1.0 / b
    # spinodal points bracket the loop
    sp = spinodal(T, a, b)
    if sp is None:
        raise ValueError("T above the critical temperature")
    ns_lo, ns_hi = sp

    def residual(x):
        ng, nl = x
        ps = p(ng)
        area = integrate.quad(lambda v: p(1.0 / v), 1.0 / nl, 1.0 / ng,
                              epsabs=1e-14, epsrel=1e-13, limit=200)[0]
        return [p(nl) - ps, area - ps * (1.0 / ng - 1.0 / nl)]

    guess = [0.5 * ns_lo, min(0.5 * (ns_hi + nmax), nmax * 0.99)]
    sol = optimize.fsolve(residual, guess, xtol=1e-12)
    # the Newton iteration from this guess can collapse onto the trivial
    # solution n_g = n_l far below T_c: refuse rather than return it
    if not (0.0 < sol[0] < ns_lo and ns_hi < sol[1] < nmax):
        raise RuntimeError(f"Maxwell construction did not converge at T = {T}")
    return float(sol[0]), float(sol[1])


def spinodal(T, a=9.0 / 8.0, b=1.0 / 3.0):
    """Densities where d p^w / d n = 0 (the spinodal; Sec. 6.2)."""
    dpdn = lambda n: T / (1.0 - b * n) ** 2 - 2.0 * a * n
    nmax = 1.0 / b
    grid = np.linspace(1e-6, nmax * (1 - 1e-9), 20001)
    vals = np.array([dpdn(n) for n in grid])
    idx = np.nonzero(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    if len(idx) < 2:
        return None
    roots = [optimize.brentq(dpdn, grid[i], grid[i + 1], xtol=1e-15) for i in idx[:2]]
    return roots[0], roots[1]


def sound_coefficients(n0, T0, tau, k, a=9.0 / 8.0, b=1.0 / 3.0, sigma=0.0, m=1.0,
                       true_vdw=False):
    """Speed of sound and damping rates of the linearised model, Eqs. sound_cs
    and long_coeff: P_eta = p^w and P_kappa = p^i = nT for this model
    (P_kappa = p^w when true_vdw).  Returns (c_s, nu_t, nu_a)."""
    dPdn = T0 / (1.0 - b * n0) ** 2 - 2.0 * a * n0
    dPdT = n0 / (1.0 - b * n0)
    Pk = (n0 * T0 / (1.0 - b * n0) - a * n0 * n0) if true_vdw else n0 * T0
    rho0 = m * n0
    eta = tau * n0 * T0
    kap = 2.0 * tau * n0 * T0 / m
    cs2 = dPdn / m + Pk / (n0 * rho0) * dPdT + n0 * k * k * sigma / m
    cs = math.sqrt(cs2)
    nu_t = k * k * kap / (rho0 * cs2) * (dPdn + n0 * k * k * sigma)
    nu_a = k * k * (eta + m * kap) / (2.0 * rho0) - 0.5 * nu_t
    return cs, nu_t, nu_a


def shear_rate(k, tau, T0, m=1.0):
    """nu_an = k^2 eta_0 / rho_0 with eta_0 = tau n_0 T_0 (Eq. shear_sol)."""
    return k * k * tau * T0 / m


def k_min(sigma, T):
    """Smallest unstable wavenumber (Sec. 6.2), reduced vdW units."""
    t3 = T ** (1.0 / 3.0)
    return 3.0 * math.sqrt(3.0) / (2.0 * math.sqrt(sigma)) * math.sqrt((1.0 - t3) / (3.0 - 2.0 * t3))


def xi_wagner(kappa, Tw):
    """Interface width estimate of Eq. xiwagner."""
    return math.sqrt(8.0 * kappa / (9.0 * (1.0 - Tw)))
