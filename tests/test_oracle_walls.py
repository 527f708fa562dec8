"""Pins of the oracle's wall ghosts (Sec. 3.4) against closed forms: the
quadratic extrapolation of the populations travelling towards a diffuse wall,
the wall density of Eq. nw on a non-uniform state, the wall Maxwellian of the
emitted populations, and the specular mirror (Sec. 3.4.1).  CPU only.

The expected values never come from the oracle's ghost code: the ghosts of a
population that is quadratic in y near the wall are that quadratic's values
at the ghost rows (the three-point extrapolation is exact on quadratics and
is the only three-point rule that is), and for nodal values of a quadratic q
every WENO-5 candidate of Eqs. weno5_flux..weno5_sigma returns
h(y_face) = q(y_face) - q''/24 (h is the quadratic whose cell means are the
nodal values), whatever the weights.  So the outgoing flux through a wall
face, and with it n_w, has a closed form on such states.
"""
import math

import numpy as np
import pytest

import oracle

S10 = math.sqrt(10.0)
# Table trots, exact
RX = np.array([-math.sqrt(5 + S10), -math.sqrt(5 - S10), 0.0, math.sqrt(5 - S10), math.sqrt(5 + S10)])
WX = np.array([(7 - 2 * S10) / 60, (7 + 2 * S10) / 60, 8 / 15, (7 + 2 * S10) / 60, (7 - 2 * S10) / 60])

NX, NY = 5, 9


def _params(**kw):
    p = dict(nx=NX, ny=NY, ds=1 / 32, dt=5e-4, tau=0.01, a=9 / 49, b=2 / 21, sigma=1e-4, bc_y=1,
             tw_lo=1.0, tw_hi=1.0, uw_lo=0.0, uw_hi=0.0)
    p.update(kw)
    return p


def _quadratic_state(seed):
    """f[25][NY][NX] whose rows 0..2 follow, per population and column, a
    quadratic c0 + c1 y + c2 y^2 (lower wall), rows NY-3..NY-1 another one
    (upper wall), and whose middle rows are random; every value positive.
    Returns f and the coefficients [wall][25][NX][3]."""
    rng = np.random.default_rng(seed)
    f = np.empty((25, NY, NX))
    # a uniform equilibrium scale per population (n = 1.2, u = 0, T = 0.9) keeps
    # the state physical; the quadratics are relative departures of a few %
    scale = np.outer(WX * (1 + 0.05 * (RX ** 2 - 1)), WX * (1 + 0.05 * (RX ** 2 - 1))).ravel() * 1.2
    coef = np.empty((2, 25, NX, 3))
    for wall in range(2):
        c = rng.uniform(-1, 1, size=(25, NX, 3)) * np.array([0.05, 0.02, 0.01])
        c[..., 0] += 1.0
        coef[wall] = c * scale[:, None, None]
    y = np.arange(NY, dtype=float)
    for wall, rows in ((0, range(0, 3)), (1, range(NY - 3, NY))):
        for r in rows:
            c = coef[wall]
            f[:, r, :] = c[..., 0] + c[..., 1] * y[r] + c[..., 2] * y[r] ** 2
    mid = range(3, NY - 3)
    for r in mid:
        f[:, r, :] = scale[:, None] * (1 + 0.05 * rng.uniform(-1, 1, size=(25, NX)))
    return f, coef


def _q(c, y):
    return c[..., 0] + c[..., 1] * y + c[..., 2] * y * y


def _ghosts(params, f):
    o = oracle.Oracle(params)
    o.set_f(f)
    o.rhs(f)          # refreshes the ghosts of f
    glo, ghi = o.wall_ghosts()
    nlo, nhi = o.wall_density()
    return glo, ghi, nlo, nhi


def test_towards_wall_ghosts_extend_the_quadratic():
    """Sec. 3.4.2: two ghost layers of every population moving towards the
    wall (and of p_y = 0) continue the quadratic through the three nearest
    rows; the third layer, which no WENO stencil of these populations reads,
    continues it too."""
    f, coef = _quadratic_state(1)
    glo, ghi, _, _ = _ghosts(_params(), f)
    for k in range(25):
        ky = k // 5
        for j in range(3):
            if ky <= 2:    # lower wall: p_y <= 0 travels towards it
                want = _q(coef[0, k], -1.0 - j)
                np.testing.assert_allclose(glo[k, j], want, rtol=1e-13, atol=1e-16)
            if ky >= 2:    # upper wall: p_y >= 0
                want = _q(coef[1, k], float(NY + j))
                np.testing.assert_allclose(ghi[k, j], want, rtol=1e-13, atol=1e-16)


def _outgoing_face_values(coef, wall):
    """Face value of each population at the wall face for the quadratic
    state: q(face) - q''/24, face at y = -1/2 (lower) or NY - 1/2 (upper)."""
    yf = -0.5 if wall == 0 else NY - 0.5
    c = coef[wall]
    return _q(c, yf) - 2.0 * c[..., 2] / 24.0     # [25][NX]


@pytest.mark.parametrize("walls", [
    dict(tw_lo=1.0, tw_hi=1.0, uw_lo=0.0, uw_hi=0.0),
    dict(tw_lo=0.8, tw_hi=1.3, uw_lo=0.05, uw_hi=-0.1),
])
def test_wall_density_matches_eq_nw_on_a_non_uniform_state(walls):
    """Eq. nw: n_w = -(outgoing flux through the wall face) / (flux of the
    wall Maxwellian per unit density), the flux being p_y times the face
    value of each population travelling towards the wall; the emitted
    populations then hold n_w g_kx(u_w, T_w) g_ky(0, T_w) in all three ghost
    layers."""
    f, coef = _quadratic_state(2)
    glo, ghi, nlo, nhi = _ghosts(_params(**walls), f)
    for wall, nw_got, G in ((0, nlo, glo), (1, nhi, ghi)):
        tw = walls["tw_lo"] if wall == 0 else walls["tw_hi"]
        uw = walls["uw_lo"] if wall == 0 else walls["uw_hi"]
        face = _outgoing_face_values(coef, wall)
        towards = [ky for ky in range(5) if (RX[ky] < 0 if wall == 0 else RX[ky] > 0)]
        emitted = [ky for ky in range(5) if (RX[ky] > 0 if wall == 0 else RX[ky] < 0)]
        flux = sum(RX[ky] * face[5 * ky + kx] for ky in towards for kx in range(5))
        if tw == 1.0 and uw == 0.0:
            gx = WX.copy()           # g_k(0, 1) = w_k (Eq. g_alpha: only l = 0 survives)
            gy = WX.copy()
        else:
            gx = np.array([oracle.g(k, uw, tw) for k in range(5)])
            gy = np.array([oracle.g(k, 0.0, tw) for k in range(5)])
        den = sum(gx[kx] * gy[ky] * RX[ky] for ky in emitted for kx in range(5))
        want = -flux / den
        np.testing.assert_allclose(nw_got, want, rtol=1e-12)
        # the same order as the density next to the wall (a sanity scale)
        assert np.all((nw_got > 0.5 * 1.2) & (nw_got < 2.0 * 1.2))
        for ky in emitted:
            for kx in range(5):
                k = 5 * ky + kx
                for j in range(3):
                    np.testing.assert_allclose(G[k, j], want * gx[kx] * gy[ky], rtol=1e-12)


def test_specular_plane_ghosts_mirror_the_interior():
    """Sec. 3.4.1 at the low end of y: ghost row -1 - j of population
    (kx, ky) is row j of (kx, 4 - ky)."""
    f, _ = _quadratic_state(3)
    glo, _, nlo, _ = _ghosts(_params(bc_y=2), f)
    for k in range(25):
        km = 5 * (4 - k // 5) + k % 5
        for j in range(3):
            np.testing.assert_array_equal(glo[k, j], f[km, j])
    np.testing.assert_array_equal(nlo, 0.0)
