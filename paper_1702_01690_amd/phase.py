"""Steady planar interfaces and the solver's liquid-vapour coexistence curve
(Sec. 5 of the paper: half channel between a specular symmetry plane and a
diffuse wall at T_w).

Python only sequences library calls (a batch of half channels stepped in HIP
graphs); the densities are read back at the end of each chunk.
"""
import numpy as np

from . import olb


def relax(batch, chunk=10000, rtol=1e-8, max_steps=600000, log=None):
    """Step every instance of ``batch`` until the largest density change over
    one chunk, relative to the density, is below ``rtol`` (or ``max_steps``).
    Returns (steps taken, last relative change)."""
    prev = [batch.moments(i)[0].copy() for i in range(len(batch))]
    steps, change = 0, np.inf
    while steps < max_steps:
        batch.step(chunk)
        steps += chunk
        change = 0.0
        for i in range(len(batch)):
            n = batch.moments(i)[0]
            change = max(change, float(np.max(np.abs(n - prev[i]) / n)))
            prev[i] = n.copy()
        if log:
            log(f"{steps} steps: relative density change per chunk {change:.3e}")
        if change < rtol:
            break
    return steps, change


def coexistence(n):
    """Gas and liquid densities of a steady half-channel profile, taken where
    the paper takes them: the node at the channel centre (next to the
    symmetry plane) and the node next to the wall."""
    n = np.asarray(n).reshape(-1)
    return float(n[0]), float(n[-1])


def spurious(moments, tw):
    """Largest speed and largest temperature excess T - T_w of a profile."""
    n, ux, uy, T = (np.asarray(a) for a in moments)
    return float(np.max(np.hypot(ux, uy))), float(np.max(T - tw))


def surface_tension(n, ds, sigma):
    """Eq. gamma_int, sigma times the integral of (dn/dx)^2 across one
    interface, for a half-channel profile n (specular plane before the first
    node, wall after the last): fourth-order central differences (the profile
    mirrored across the plane, held constant past the wall) and the
    rectangle rule."""
    n = np.asarray(n, dtype=np.float64).reshape(-1)
    if n.size < 4:
        raise ValueError("profile too short for the five-point derivative")
    ext = np.concatenate([n[2::-1], n, np.full(3, n[-1])])
    m = n.size
    d = (2.0 / 3.0 * (ext[4:4 + m] - ext[2:2 + m]) - 1.0 / 12.0 * (ext[5:5 + m] - ext[1:1 + m])) / ds
    return float(sigma * np.sum(d * d) * ds)


def interface_width(n, ds, x0, xi0):
    """Fit of Eq. tanh, n = c + h tanh((x - x_i)/xi), to a half-channel
    profile n (node centres (j + 1/2) ds from the specular plane): (xi, x_i)
    by least squares over every node."""
    from scipy.optimize import curve_fit
    n = np.asarray(n, dtype=np.float64).reshape(-1)
    x = (np.arange(n.size) + 0.5) * ds
    model = lambda xx, c, h, xi_pos, xi: c + h * np.tanh((xx - xi_pos) / xi)
    p0 = [0.5 * (n.max() + n.min()), 0.5 * (n.max() - n.min()), x0, xi0]
    (c, h, xpos, xi), _ = curve_fit(model, x, n, p0=p0)
    return float(abs(xi)), float(xpos)


def bubble_profile(n, ds, R0, xi0):
    """Fit of Eq. tanh in the distance R from the corner x = y = 0 to a
    bubble's density field n[y][x] (node centres at (i + 1/2) ds): n = c +
    h tanh((R - R_f)/xi) by least squares over every node.  Returns (R_f,
    xi, c - h, c + h), i.e. radius, width, inner and outer densities."""
    from scipy.optimize import curve_fit
    n = np.asarray(n, dtype=np.float64)
    cy = (np.arange(n.shape[0]) + 0.5) * ds
    cx = (np.arange(n.shape[1]) + 0.5) * ds
    R = np.hypot(cx[None, :], cy[:, None]).ravel()
    model = lambda r, c, h, rf, xi: c + h * np.tanh((r - rf) / xi)
    p0 = [0.5 * (n.max() + n.min()), 0.5 * (n.max() - n.min()), R0, xi0]
    (c, h, rf, xi), _ = curve_fit(model, R, n.ravel(), p0=p0)
    return float(rf), float(abs(xi)), float(c - h), float(c + h)


def bubble_pressures(n, T, ds, R_f, xi, a=9.0 / 8.0, b=1.0 / 3.0, margin=5.0):
    """Mean van der Waals pressure p^w (Eq. vdw) of the nodes inside
    (R < R_f - margin xi) and outside (R > R_f + margin xi) a bubble centred
    on the corner."""
    n = np.asarray(n, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    cy = (np.arange(n.shape[0]) + 0.5) * ds
    cx = (np.arange(n.shape[1]) + 0.5) * ds
    R = np.hypot(cx[None, :], cy[:, None])
    p = _pressure(n, T, a, b)
    inner, outer = R < R_f - margin * xi, R > R_f + margin * xi
    if not inner.any() or not outer.any():
        raise ValueError("bubble too small or too large for the pressure regions")
    return float(p[inner].mean()), float(p[outer].mean())


def track_bubble(n, T, x, y, xc0, R0, xi0, period, a=9.0 / 8.0, b=1.0 / 3.0, margin=5.0):
    """A bubble centred on the plane y = 0 of a field n[y][x] periodic in x
    with the given period: least-squares fit of Eq. tanh in the distance
    R = sqrt(dx^2 + y^2) to the centre (x_c, 0), dx taken modulo the period;
    then the mean p^w inside and outside (as bubble_pressures).  Returns
    (x_c, R_f, xi, p_in - p_out); x_c is the continuation nearest xc0."""
    from scipy.optimize import curve_fit
    n = np.asarray(n, dtype=np.float64)
    X, Y = np.meshgrid(np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64))

    def dist(xc):
        dx = np.mod(X - xc + 0.5 * period, period) - 0.5 * period
        return np.hypot(dx, Y)

    import warnings
    from scipy.optimize import OptimizeWarning
    model = lambda _, c, h, rf, xi, xc: (c + h * np.tanh((dist(xc) - rf) / xi)).ravel()
    p0 = [0.5 * (n.max() + n.min()), 0.5 * (n.max() - n.min()), R0, xi0, xc0]
    with warnings.catch_warnings():
        # the covariance is not used (and is singular for a bubble at rest)
        warnings.simplefilter("ignore", OptimizeWarning)
        (c, h, rf, xi, xc), _ = curve_fit(model, None, n.ravel(), p0=p0)
    xi = abs(xi)
    xc = xc0 + (np.mod(xc - xc0 + 0.5 * period, period) - 0.5 * period)
    R = dist(xc)
    p = _pressure(n, np.asarray(T, dtype=np.float64), a, b)
    inner, outer = R < rf - margin * xi, R > rf + margin * xi
    if not inner.any() or not outer.any():
        raise ValueError("bubble too small or too large for the pressure regions")
    return float(xc), float(rf), float(xi), float(p[inner].mean() - p[outer].mean())


def laplace_tension(radii, dp):
    """Eq. Laplace, p_in - p_out = gamma / R_f, fitted through the origin
    by least squares over several bubbles: gamma."""
    x = 1.0 / np.asarray(radii, dtype=np.float64)
    y = np.asarray(dp, dtype=np.float64)
    return float(np.sum(x * y) / np.sum(x * x))


def _pressure(n, T, a, b):
    return n * T / (1.0 - b * n) - a * n * n


def _chemical_potential(n, T, a, b):
    # mu = dF/dn of the free energy density F = n T [ln(n / (1 - b n)) - 1] - a n^2
    # (m = k_B = 1); p = n mu - F reproduces Eq. vdw
    return T * (np.log(n / (1.0 - b * n)) + b * n / (1.0 - b * n)) - 2.0 * a * n


def maxwell_coexistence(T, a=9.0 / 8.0, b=1.0 / 3.0):
    """Gas and liquid densities of the van der Waals fluid (Eq. vdw) at
    T < T_c = 8a / (27b): equal pressure and equal chemical potential (the
    Maxwell construction).  The steady momentum balance of the paper's force,
    grad p^w = sigma n grad lap n, imposes exactly these two conditions
    between the bulk phases of a planar interface."""
    from scipy.optimize import brentq
    nc, nmax = 1.0 / (3.0 * b), 1.0 / b
    if not T < 8.0 * a / (27.0 * b):
        raise ValueError("temperature at or above the critical point")
    eps = 1e-12 * nmax
    # spinodal points: dp/dn = T / (1 - b n)^2 - 2 a n = 0 on either side of n_c
    dp = lambda n: T / (1.0 - b * n) ** 2 - 2.0 * a * n
    s1 = brentq(dp, eps, nc)
    s2 = brentq(dp, nc, nmax - eps)
    p_min = _pressure(s2, T, a, b)
    lo = brentq(lambda n: _pressure(n, T, a, b) - p_min, eps, s1) if p_min > 0.0 else eps

    def liquid(ng):
        pg = _pressure(ng, T, a, b)
        return brentq(lambda n: _pressure(n, T, a, b) - pg, s2, nmax - eps)

    gap = lambda ng: _chemical_potential(ng, T, a, b) - _chemical_potential(liquid(ng), T, a, b)
    ng = brentq(gap, lo * (1.0 + 1e-9) + 1e-300, s1 * (1.0 - 1e-9), xtol=1e-15, rtol=1e-14)
    return float(ng), float(liquid(ng))
