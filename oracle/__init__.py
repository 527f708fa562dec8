"""Plain FP64 CPU oracle of the D2Q25 thermal Boltzmann stage update.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It never imports the GPU package,
and the GPU package never imports it.  The arithmetic lives in the C library
``olb_oracle.c``; this module only marshals numpy arrays through ctypes.

Parameters are plain dicts with the keys of ``oolb_params``: nx, ny, ds, dt,
tau, a, b, sigma, bc_x, bc_y, tw_lo, tw_hi, uw_lo, uw_hi (precision and
rho_ref are accepted and ignored).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

OK, E_ARG, E_CFL, E_DOMAIN, E_NONFINITE, E_WORKSPACE, E_DEVICE, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("ds", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("sigma", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("tw_lo", ctypes.c_double), ("tw_hi", ctypes.c_double),
                ("uw_lo", ctypes.c_double), ("uw_hi", ctypes.c_double),
                ("precision", ctypes.c_int32), ("rho_ref", ctypes.c_double)]


_DEFAULTS = dict(bc_x=0, bc_y=0, tw_lo=1.0, tw_hi=1.0, uw_lo=0.0, uw_hi=0.0,
                 precision=0, rho_ref=1.0, sigma=0.0)


def _params(d):
    full = dict(_DEFAULTS)
    full.update(d)
    return _Params(**{k: full[k] for k, _ in _Params._fields_})


_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def lib():
    """Load the oracle library, compiling it first if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oolb_init.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        L.oolb_free.argtypes = [ctypes.c_void_p]
        L.oolb_free.restype = None
        for name in ("oolb_set_fields", "oolb_moments"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.oolb_set_f.argtypes = [ctypes.c_void_p, _dp]
        L.oolb_get_f.argtypes = [ctypes.c_void_p, _dp]
        L.oolb_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.oolb_rhs.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oolb_wall_density.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oolb_wall_ghosts.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oolb_last_error.argtypes = [ctypes.c_void_p]
        L.oolb_last_error.restype = ctypes.c_char_p
        L.oolb_set_threads.argtypes = [ctypes.c_int]
        L.oolb_set_threads.restype = None
        L.oolb_get_threads.restype = ctypes.c_int
        L.oolb_quadrature.argtypes = [_dp, _dp]
        L.oolb_quadrature.restype = None
        L.oolb_hermite.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oolb_hermite.restype = ctypes.c_double
        L.oolb_g.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.oolb_g.restype = ctypes.c_double
        L.oolb_feq.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.oolb_feq.restype = None
        L.oolb_dpf.argtypes = [_dp, _dp, _dp]
        L.oolb_dpf.restype = None
        L.oolb_weno_recon.argtypes = [_dp, _dp]
        L.oolb_weno_recon.restype = ctypes.c_double
        for name in ("oolb_grad", "oolb_glap"):
            getattr(L, name).argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, _dp]
            getattr(L, name).restype = None
        L.oolb_stencil_tables.argtypes = [_dp, _dp]
        L.oolb_stencil_tables.restype = None
        L.oolb_pw.argtypes = [ctypes.c_double] * 4
        L.oolb_pw.restype = ctypes.c_double
        _LIB = L
    return _LIB


def set_threads(n):
    lib().oolb_set_threads(int(n))


def get_threads():
    return int(lib().oolb_get_threads())


# ---------------------------------------------------------------- pieces ----

def quadrature():
    R = np.zeros(5)
    W = np.zeros(5)
    lib().oolb_quadrature(_ptr(R), _ptr(W))
    return R, W


def hermite(l, p):
    return lib().oolb_hermite(int(l), float(p))


def g(k, u, T):
    return lib().oolb_g(int(k), float(u), float(T))


def feq(n, ux, uy, T):
    out = np.zeros(25)
    lib().oolb_feq(float(n), float(ux), float(uy), float(T), _ptr(out))
    return out


def dpf(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    dx = np.zeros(25)
    dy = np.zeros(25)
    lib().oolb_dpf(_ptr(f), _ptr(dx), _ptr(dy))
    return dx, dy


def weno_recon(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.zeros(3)
    r = lib().oolb_weno_recon(_ptr(v), _ptr(w))
    return r, w


def grad(gfield, ds, x, y):
    gfield = np.ascontiguousarray(gfield, dtype=np.float64)
    ny, nx = gfield.shape
    out = np.zeros(2)
    lib().oolb_grad(_ptr(gfield), nx, ny, float(ds), int(x), int(y), _ptr(out))
    return out


def glap(gfield, ds, x, y):
    gfield = np.ascontiguousarray(gfield, dtype=np.float64)
    ny, nx = gfield.shape
    out = np.zeros(2)
    lib().oolb_glap(_ptr(gfield), nx, ny, float(ds), int(x), int(y), _ptr(out))
    return out


def stencil_tables():
    gw = np.zeros(16)
    D = np.zeros(49)
    lib().oolb_stencil_tables(_ptr(gw), _ptr(D))
    return gw.reshape(4, 4), D.reshape(7, 7)


def pw(n, T, a, b):
    return lib().oolb_pw(float(n), float(T), float(a), float(b))


# --------------------------------------------------------------- context ----

class Oracle:
    """One lattice instance advanced by the oracle (host memory)."""

    def __init__(self, params):
        self.params = dict(_DEFAULTS)
        self.params.update(params)
        self.nx = int(self.params["nx"])
        self.ny = int(self.params["ny"])
        self._p = _params(self.params)
        h = ctypes.c_void_p()
        rc = lib().oolb_init(ctypes.byref(self._p), ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().oolb_free(self._h)
            self._h = None

    __del__ = close

    def _check(self, rc):
        if rc != OK:
            raise OracleError(rc, lib().oolb_last_error(self._h).decode())

    def _field(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (self.ny, self.nx):
            raise ValueError(f"field shape {a.shape} != {(self.ny, self.nx)}")
        return a

    def set_fields(self, n, ux, uy, T):
        n, ux, uy, T = (self._field(a) for a in (n, ux, uy, T))
        self._check(lib().oolb_set_fields(self._h, _ptr(n), _ptr(ux), _ptr(uy), _ptr(T)))

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(25, self.ny, self.nx)
        self._check(lib().oolb_set_f(self._h, _ptr(f)))

    def get_f(self):
        f = np.zeros((25, self.ny, self.nx))
        self._check(lib().oolb_get_f(self._h, _ptr(f)))
        return f

    def step(self, nsteps=1):
        self._check(lib().oolb_step(self._h, int(nsteps)))

    def moments(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(4)]
        self._check(lib().oolb_moments(self._h, *(_ptr(a) for a in out)))
        return tuple(out)

    def rhs(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(25, self.ny, self.nx)
        L = np.zeros_like(f)
        self._check(lib().oolb_rhs(self._h, _ptr(f), _ptr(L)))
        return L

    def wall_ghosts(self):
        """Ghost rows of the last ghost fill, two arrays [25][3][nx]: layer j
        is row -1 - j (lower wall) and row ny + j (upper wall)."""
        lo = np.zeros((25, 3, self.nx))
        hi = np.zeros((25, 3, self.nx))
        self._check(lib().oolb_wall_ghosts(self._h, _ptr(lo), _ptr(hi)))
        return lo, hi

    def wall_density(self):
        lo = np.zeros(self.nx)
        hi = np.zeros(self.nx)
        self._check(lib().oolb_wall_density(self._h, _ptr(lo), _ptr(hi)))
        return lo, hi
