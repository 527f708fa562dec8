"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the method: it only builds parameter dicts
and initial macroscopic fields (density, velocity, temperature) from closed
forms and a SplitMix64 stream.  Both the oracle and the GPU library receive the
same arrays and turn them into f = f^eq themselves.

Workloads (lattice units: ds = 1/N, m = k_B = 1):
  shear32     32x32 periodic shear wave, a = 9/49, b = 2/21 (T_c = 4/7), T = 1,
              n = 1, u_y = 1e-3 sin(2 pi x), tau = 0.01, dt = 5e-4, ds = 1/32.
  wave2048    2048x2048 periodic, superposed shear (u_y amplitude 1e-3) and
              longitudinal (n amplitude 1e-3) waves along x, wavelength 64
              cells (ds = 1/64), tau = 0.005, dt = 5e-4, T = 1.
  wave64      the 64x64 crop of wave2048 (one wavelength; the 2048 run is this
              one tiled 32x32 times).
  spinodal    periodic spinodal decomposition at T = 0.9 T_c, n = 3.5 (1 +
              0.01 (2U - 1)), u = 0, ds = 1/320, dt = 2e-4, tau = 0.005.
  channel     periodic in x, diffuse walls at y = -ds/2 and (ny - 1/2) ds with
              wall temperature T_w, fluid initially at T_c with n = 3.5 (1 +
              0.005 (2U - 1)) (the cooled-plates quench of Sec. 7).
  channels    256 channels with seeded sizes and wall temperatures.
U is uniform on [0, 1): the top 53 bits of successive SplitMix64 outputs,
drawn in row-major order (y outer, x inner).  Cell centres are
x_i = (i + 1/2) ds, 0-based.
"""
from dataclasses import dataclass, field

import numpy as np

VDW_A = 9.0 / 49.0
VDW_B = 2.0 / 21.0
T_CRIT = 4.0 / 7.0     # critical temperature 8a/(27b) of the EOS above
N_CRIT = 3.5           # critical density 1/(3b)

_M64 = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> np.ndarray:
    """``count`` successive SplitMix64 outputs (Steele, Lea, Flood 2014)."""
    out = np.empty(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _M64)
        # vectorised: state_i = seed + (i+1) * golden
        inc = np.uint64(0x9E3779B97F4A7C15)
        z = state + inc * np.arange(1, count + 1, dtype=np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    out[:] = z
    return out


def uniform(seed: int, count: int) -> np.ndarray:
    """Uniform doubles on [0, 1) from the top 53 bits of SplitMix64."""
    z = splitmix64(seed, count)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class Case:
    name: str
    params: dict
    n: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    steps: int
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def fields(self):
        return self.n, self.ux, self.uy, self.T


def _params(nx, ny, ds, dt, tau, a=VDW_A, b=VDW_B, sigma=1e-4, bc_y=0,
            tw=1.0, uw=0.0, precision=0, rho_ref=1.0, bc_x=0):
    return dict(nx=int(nx), ny=int(ny), ds=float(ds), dt=float(dt), tau=float(tau),
                a=float(a), b=float(b), sigma=float(sigma), bc_x=int(bc_x), bc_y=int(bc_y),
                tw_lo=float(tw), tw_hi=float(tw), uw_lo=float(uw), uw_hi=float(uw),
                precision=int(precision), rho_ref=float(rho_ref))


def _xc(nx, ds):
    return (np.arange(nx) + 0.5) * ds


def shear32(nx=32, ny=32, steps=100, **kw):
    ds = 1.0 / nx
    x = _xc(nx, ds)
    n = np.ones((ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.broadcast_to(1e-3 * np.sin(2 * np.pi * x), (ny, nx)).copy()
    T = np.ones((ny, nx))
    p = _params(nx, ny, ds, 5e-4, 0.01, **kw)
    return Case("shear32", p, n, ux, uy, T, steps)


def wave(nx=2048, ny=2048, cells_per_wavelength=64, steps=1000, **kw):
    ds = 1.0 / cells_per_wavelength
    x = _xc(nx, ds)
    n = np.broadcast_to(1.0 + 1e-3 * np.cos(2 * np.pi * x), (ny, nx)).copy()
    ux = np.zeros((ny, nx))
    uy = np.broadcast_to(1e-3 * np.sin(2 * np.pi * x), (ny, nx)).copy()
    T = np.ones((ny, nx))
    p = _params(nx, ny, ds, 5e-4, 0.005, **kw)
    return Case(f"wave{nx}x{ny}", p, n, ux, uy, T, steps)


def wave2048(**kw):
    """The 64 x 64 wave tiled 32 x 32 times: the inputs are exactly periodic
    (evaluating sin / cos at x up to 32 would not round identically)."""
    return tile(wave(64, 64, **kw), 32, 32)


def wave64(**kw):
    return wave(64, 64, **kw)


def spinodal(nx=4096, ny=4096, seed=3, steps=5000, ds=1.0 / 320, dt=2e-4, tau=0.005,
             temperature=0.9 * T_CRIT, noise=0.01, **kw):
    U = uniform(seed, nx * ny).reshape(ny, nx)
    n = N_CRIT * (1.0 + noise * (2.0 * U - 1.0))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    T = np.full((ny, nx), float(temperature))
    p = _params(nx, ny, ds, dt, tau, **kw)
    return Case(f"spinodal{nx}x{ny}", p, n, ux, uy, T, steps)


def channel(nx=64, ny=128, seed=4, steps=2000, tw=0.8 * T_CRIT, ds=1.0 / 320, dt=2e-4,
            tau=0.005, noise=0.005, t0=T_CRIT, **kw):
    U = uniform(seed, nx * ny).reshape(ny, nx)
    n = N_CRIT * (1.0 + noise * (2.0 * U - 1.0))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    T = np.full((ny, nx), float(t0))
    p = _params(nx, ny, ds, dt, tau, bc_y=1, tw=tw, **kw)
    return Case(f"channel{nx}x{ny}", p, n, ux, uy, T, steps)


def channels(count=256, seed=4, nx_range=(64, 512), ny_range=(128, 1024),
             tw_range=(0.7, 0.95), steps=2000, precision=1, **kw):
    """``count`` walled channels.  One SplitMix64 stream (seed) is consumed in
    the order: per channel nx, ny, T_w; then the noise of every channel, channel
    by channel, row-major."""
    head = uniform(seed, 3 * count).reshape(count, 3)
    lo_x, hi_x = nx_range
    lo_y, hi_y = ny_range
    sizes = []
    for c in range(count):
        nx = lo_x + int(head[c, 0] * (hi_x - lo_x + 1))
        ny = lo_y + int(head[c, 1] * (hi_y - lo_y + 1))
        tw = (tw_range[0] + (tw_range[1] - tw_range[0]) * head[c, 2]) * T_CRIT
        sizes.append((nx, ny, tw))
    total = sum(nx * ny for nx, ny, _ in sizes)
    noise = uniform(seed, 3 * count + total)[3 * count:]
    cases = []
    off = 0
    for c, (nx, ny, tw) in enumerate(sizes):
        U = noise[off:off + nx * ny].reshape(ny, nx)
        off += nx * ny
        n = N_CRIT * (1.0 + 0.005 * (2.0 * U - 1.0))
        z = np.zeros((ny, nx))
        p = _params(nx, ny, 1.0 / 320, 2e-4, 0.005, bc_y=1, tw=tw, precision=precision,
                    rho_ref=N_CRIT, **kw)
        cases.append(Case(f"channel[{c}]{nx}x{ny}", p, n, z, z.copy(),
                          np.full((ny, nx), T_CRIT), steps))
    return cases


def tile(case: Case, rx: int, ry: int) -> Case:
    """The same workload repeated rx times along x and ry times along y."""
    p = dict(case.params)
    p["nx"] = case.params["nx"] * rx
    p["ny"] = case.params["ny"] * ry
    t = lambda a: np.tile(a, (ry, rx))
    return Case(case.name + f"x{rx}x{ry}", p, t(case.n), t(case.ux), t(case.uy), t(case.T),
                case.steps)


def random_f_perturbation(seed: int, shape, amplitude: float) -> np.ndarray:
    """Seeded multiplicative noise (1 + amplitude (2U - 1)) for raw f tests."""
    U = uniform(seed, int(np.prod(shape))).reshape(shape)
    return 1.0 + amplitude * (2.0 * U - 1.0)


# ---------------------------------------------------------- learned closure --
# Fine spinodal samples at T = (0.75 + 0.2 U) T_c, their 4x-coarser
# counterparts (same physical domain and time: ds and dt four times larger),
# random network parameters and random coarse moment fields.

CLOSURE_FACTOR = 4
CLOSURE_PARAM_SHAPES = ((32, 4, 3, 3), (32,), (32, 32, 3, 3), (32,), (4, 32, 3, 3), (4,))


def closure_sample(nx=2048, ny=None, seed=5000, ds=1.0 / 320, dt=2e-4, tau=0.005, noise=0.01):
    """Fine spinodal sample: the first draw of the seed's stream sets T, the
    next nx * ny ones the density noise n = 3.5 (1 + noise (2U - 1)); u = 0."""
    ny = nx if ny is None else ny
    U = uniform(seed, 1 + nx * ny)
    temperature = (0.75 + 0.2 * U[0]) * T_CRIT
    n = N_CRIT * (1.0 + noise * (2.0 * U[1:].reshape(ny, nx) - 1.0))
    z = np.zeros((ny, nx))
    p = _params(nx, ny, ds, dt, tau)
    return Case(f"closure{nx}x{ny}s{seed}", p, n, z, z.copy(), np.full((ny, nx), temperature), 0)


def coarse_params(fine_params, factor=CLOSURE_FACTOR, precision=1):
    """Parameters of the factor-times coarser lattice over the same domain."""
    p = dict(fine_params)
    p["nx"] = fine_params["nx"] // factor
    p["ny"] = fine_params["ny"] // factor
    p["ds"] = fine_params["ds"] * factor
    p["dt"] = fine_params["dt"] * factor
    p["precision"] = precision
    p["rho_ref"] = N_CRIT
    return p


def closure_params(seed=7, last_scale=0.1) -> np.ndarray:
    """Random float32 parameter vector: weights uniform in +-sqrt(6 / fan_in)
    (fan_in = 9 C_in), the last layer's scaled by last_scale, biases zero."""
    out = []
    draws = uniform(seed, sum(int(np.prod(s)) for s in CLOSURE_PARAM_SHAPES))
    o = 0
    for i, shape in enumerate(CLOSURE_PARAM_SHAPES):
        size = int(np.prod(shape))
        if len(shape) == 4:
            bound = np.sqrt(6.0 / (9 * shape[1])) * (last_scale if i == 4 else 1.0)
            out.append(bound * (2.0 * draws[o:o + size] - 1.0))
        else:
            out.append(np.zeros(size))
        o += size
    return np.concatenate(out).astype(np.float32)


def closure_moments(nx, ny, seed=11, amplitude=0.01) -> np.ndarray:
    """Random admissible moment planes (4, ny, nx) near the spinodal state:
    n = 3.5 (1 + a (2U - 1)), u = a (2U - 1), T = 0.85 T_c (1 + a (2U - 1))."""
    U = 2.0 * uniform(seed, 4 * nx * ny).reshape(4, ny, nx) - 1.0
    return np.stack([N_CRIT * (1.0 + amplitude * U[0]), amplitude * U[1], amplitude * U[2],
                     0.85 * T_CRIT * (1.0 + amplitude * U[3])])


# ------------------------------------------------ half channels (specular) --

def half_channel(nx=8, ny=40, seed=9, tw=0.8 * T_CRIT, ds=1.0 / 320, dt=2e-4, tau=0.005, noise=0.01,
                 temperature=None, **kw):
    """Noisy vdW fluid between a specular symmetry plane (low y end) and a
    diffuse wall at T_w (high y end)."""
    U = uniform(seed, nx * ny).reshape(ny, nx)
    n = N_CRIT * (1.0 + noise * (2.0 * U - 1.0))
    z = np.zeros((ny, nx))
    T = np.full((ny, nx), float(tw if temperature is None else temperature))
    p = _params(nx, ny, ds, dt, tau, bc_y=2, tw=tw, **kw)
    return Case(f"half{nx}x{ny}", p, n, z, z.copy(), T, 0)


def box(nx=8, ny=12, seed=13, tw=0.8 * T_CRIT, bc_y=2, ds=1.0 / 320, dt=2e-4, tau=0.005, noise=0.01,
        speed=0.01, temperature=None, **kw):
    """Noisy moving vdW fluid in a box with specular planes at both ends of x
    and, in y, the half channel's specular plane + diffuse wall (bc_y = 2),
    diffuse walls (1) or periodic ends (0)."""
    U = uniform(seed, 3 * nx * ny).reshape(3, ny, nx)
    n = N_CRIT * (1.0 + noise * (2.0 * U[0] - 1.0))
    ux = speed * (2.0 * U[1] - 1.0)
    uy = speed * (2.0 * U[2] - 1.0)
    T = np.full((ny, nx), float(tw if temperature is None else temperature))
    p = _params(nx, ny, ds, dt, tau, bc_y=bc_y, tw=tw, bc_x=3, **kw)
    return Case(f"box{nx}x{ny}y{bc_y}", p, n, ux, uy, T, 0)


def laplace_bubble(R0, n_gas, n_liquid, sigma=5e-5, tw=0.8, N=160, ds=1.0 / 320, dt=2e-4, tau=5e-3,
                   a=9.0 / 8.0, b=1.0 / 3.0):
    """The Laplace test (Sec. 6): a gas bubble of radius R0 centred on the
    corner x = y = 0 of an N x N box (specular planes at x = 0, x = N ds and
    y = 0, a diffuse wall at T_w at y = N ds; the paper's wall is at x = 0.5
    and its top boundary specular, the axes are exchanged here), fluid at rest
    at T_w, the tanh profile of Eq. tanh in R = sqrt(x^2 + y^2) between the
    given gas and liquid densities, width Eq. xiwagner."""
    xi = np.sqrt(8.0 * sigma / (9.0 * (1.0 - tw)))
    c = (np.arange(N) + 0.5) * ds
    R = np.hypot(c[None, :], c[:, None])
    n = n_gas + 0.5 * (n_liquid - n_gas) * (1.0 + np.tanh((R - R0) / xi))
    z = np.zeros((N, N))
    p = _params(N, N, ds, dt, tau, a=a, b=b, sigma=sigma, bc_y=2, tw=tw, bc_x=3)
    return Case(f"laplace{R0:g}", p, n, z, z.copy(), np.full((N, N), float(tw)), 0,
                extra={"R0": float(R0), "xi": float(xi)})


def sound_wave(N, V=0.0, n0=1.0, a=0.0, b=0.0, sigma=0.0, T0=0.8, tau=5e-4, dt=2e-4, du0=1e-3):
    """A longitudinal wave seen from a moving frame (Sec. 6.2): L = 1
    periodic in x with N nodes (one node across y), n = n0, T = T0,
    u_x = V + du0 sin(2 pi x_i), u_y = 0, x_i = (i + 1/2)/N - 1/2."""
    x = (np.arange(N) + 0.5) / N - 0.5
    n = np.full((1, N), float(n0))
    ux = (V + du0 * np.sin(2.0 * np.pi * x))[None, :]
    uy = np.zeros((1, N))
    T = np.full((1, N), float(T0))
    p = _params(N, 1, 1.0 / N, dt, tau, a=a, b=b, sigma=sigma)
    return Case(f"sound{N}_V{V:g}", p, n, ux, uy, T, 0, extra={"V": float(V), "du0": float(du0), "x": x})


def moving_bubble(V, n_gas, n_liquid, R0=0.25, sigma=1e-4, tw=0.8, N=160, ds=1.0 / 320, dt=2e-4, tau=5e-3,
                  a=9.0 / 8.0, b=1.0 / 3.0):
    """The moving-bubble test (Sec. 6.3): a gas bubble of radius R0 centred
    on the specular plane at x = 0 (here y = 0), carried by a uniform
    background velocity V parallel to the plane and to a diffuse wall at T_w
    moving with V at y = N ds; periodic along the flow with length 2 N ds
    (node centres x_i = (i + 1/2) ds - N ds).  Fluid at T_w, the tanh profile
    of Eq. tanh in R with width Eq. xiwagner."""
    xi = np.sqrt(8.0 * sigma / (9.0 * (1.0 - tw)))
    x = (np.arange(2 * N) + 0.5) * ds - N * ds
    y = (np.arange(N) + 0.5) * ds
    R = np.hypot(x[None, :], y[:, None])
    n = n_gas + 0.5 * (n_liquid - n_gas) * (1.0 + np.tanh((R - R0) / xi))
    p = _params(2 * N, N, ds, dt, tau, a=a, b=b, sigma=sigma, bc_y=2, tw=tw, uw=V)
    z = np.zeros((N, 2 * N))
    return Case(f"moving_bubble_V{V:g}", p, n, np.full((N, 2 * N), float(V)), z, np.full((N, 2 * N), float(tw)),
                0, extra={"V": float(V), "R0": float(R0), "xi": float(xi), "x": x, "y": y})


def planar_interface(tw, n_gas, n_liquid, cells=160, ds=1.0 / 320, dt=2e-4, tau=0.005, sigma=1e-4,
                     a=9.0 / 8.0, b=1.0 / 3.0, x0=0.25):
    """The planar-interface test (Sec. 5) on the half channel: one column of
    `cells` nodes from the channel centre (specular plane) to the wall at
    x = cells ds = 0.5, fluid at rest at T = T_w with the tanh profile of
    Eq. tanh between the given gas and liquid densities, width Eq. xiwagner
    (kappa = sigma), interface at x0 (the paper's walls are across x; here
    across y)."""
    xi = np.sqrt(8.0 * sigma / (9.0 * (1.0 - tw)))
    y = (np.arange(cells) + 0.5) * ds
    n = n_gas + 0.5 * (n_liquid - n_gas) * (1.0 + np.tanh((y - x0) / xi))
    z = np.zeros((cells, 1))
    p = _params(1, cells, ds, dt, tau, a=a, b=b, sigma=sigma, bc_y=2, tw=tw)
    return Case(f"planar{tw:g}", p, n[:, None], z, z.copy(), np.full((cells, 1), float(tw)), 0)


def quench(N=320, seed=17, tw=0.8, noise=0.01, dt=2e-4, tau=0.005, sigma=1e-4, a=9.0 / 8.0, b=1.0 / 3.0):
    """Phase separation between suddenly cooled plates (Sec. 7): a vdW fluid
    (a = 9/8, b = 1/3, T_c = n_c = 1) at rest at T = 1 with n = 1 + 0.01 (2U - 1)
    between diffuse walls at T_w, 2N nodes across the walls and N along them,
    ds = 1/N.  The paper's walls are across x; here across y (nx = N periodic,
    ny = 2N)."""
    U = uniform(seed, 2 * N * N).reshape(2 * N, N)
    n = 1.0 + noise * (2.0 * U - 1.0)
    z = np.zeros((2 * N, N))
    p = _params(N, 2 * N, 1.0 / N, dt, tau, a=a, b=b, sigma=sigma, bc_y=1, tw=tw)
    return Case(f"quench{N}", p, n, z, z.copy(), np.ones((2 * N, N)), 0)


def shear_wave(N, V=0.0, n0=1.0, a=0.0, b=0.0, sigma=0.0, T0=0.8, tau=5e-4, dt=2e-4, u0=1e-3):
    """Damping of a shear wave seen from a moving frame (Sec. 6.1): L = 1
    periodic in x with N nodes (one node across y), n = n0, T = T0, u_x = V,
    u_y = u0 sin(2 pi x_i) at the cell centres x_i = (i + 1/2)/N - 1/2
    (0-based i).  a = b = sigma = 0 is the ideal gas; the vdW vapour and
    liquid take their coexistence densities at T0 as n0."""
    x = (np.arange(N) + 0.5) / N - 0.5
    n = np.full((1, N), float(n0))
    ux = np.full((1, N), float(V))
    uy = (u0 * np.sin(2.0 * np.pi * x))[None, :]
    T = np.full((1, N), float(T0))
    p = _params(N, 1, 1.0 / N, dt, tau, a=a, b=b, sigma=sigma)
    return Case(f"shear{N}_V{V:g}", p, n, ux, uy, T, 0, extra={"V": float(V), "u0": float(u0), "x": x})
