"""ctypes binding of the gfx950 D2Q25 library (``libolb.so``, include/olb.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch supplies the device workspace (a uint8 CUDA tensor) and the stream.
The functions keep the C names; ``Lattice`` bundles them for one context.
There is no CPU fallback: without the built library or a GPU every call
raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libolb.so")

OLB_OK, OLB_E_ARG, OLB_E_CFL, OLB_E_DOMAIN, OLB_E_NONFINITE = 0, -1, -2, -3, -4
OLB_E_WORKSPACE, OLB_E_DEVICE, OLB_E_STATE = -5, -6, -7
OLB_BC_PERIODIC, OLB_BC_DIFFUSE, OLB_BC_SPECULAR_DIFFUSE, OLB_BC_SPECULAR = 0, 1, 2, 3
OLB_FP64, OLB_FP32_MIXED = 0, 1


class OlbError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"olb error {code}: {msg}")
        self.code = code


class olb_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("ds", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("sigma", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("tw_lo", ctypes.c_double), ("tw_hi", ctypes.c_double),
                ("uw_lo", ctypes.c_double), ("uw_hi", ctypes.c_double),
                ("precision", ctypes.c_int32), ("rho_ref", ctypes.c_double)]


_DEFAULTS = dict(bc_x=0, bc_y=0, tw_lo=1.0, tw_hi=1.0, uw_lo=0.0, uw_hi=0.0,
                 precision=0, rho_ref=1.0, sigma=0.0)


def make_params(d):
    full = dict(_DEFAULTS)
    full.update(d)
    return olb_params(**{k: full[k] for k, _ in olb_params._fields_})


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p
_LIB = None

# C name -> (argtypes, restype)
_SIGS = {
    "olb_workspace_bytes": ([ctypes.POINTER(olb_params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "olb_init": ([ctypes.POINTER(olb_params), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "olb_set_fields": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "olb_step": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_sync": ([_vp], ctypes.c_int),
    "olb_moments": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "olb_moments_device": ([_vp, _vp], ctypes.c_int),
    "olb_get_f": ([_vp, _dp], ctypes.c_int),
    "olb_set_f": ([_vp, _dp], ctypes.c_int),
    "olb_wall_density": ([_vp, _dp, _dp], ctypes.c_int),
    "olb_set_tile": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_set_base_temperature": ([_vp, ctypes.c_double], ctypes.c_int),
    "olb_set_tile_order": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_batch_set_tile_order": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_launch_counts": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "olb_last_error": ([_vp], ctypes.c_char_p),
    "olb_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "olb_free": ([_vp], None),
    "olb_batch_workspace_bytes": ([ctypes.POINTER(olb_params), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "olb_batch_init": ([ctypes.POINTER(olb_params), ctypes.c_int32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "olb_batch_set_fields": ([_vp, ctypes.c_int32, _dp, _dp, _dp, _dp], ctypes.c_int),
    "olb_batch_set_f": ([_vp, ctypes.c_int32, _dp], ctypes.c_int),
    "olb_batch_get_f": ([_vp, ctypes.c_int32, _dp], ctypes.c_int),
    "olb_batch_step": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_batch_sync": ([_vp], ctypes.c_int),
    "olb_batch_moments": ([_vp, ctypes.c_int32, _dp, _dp, _dp, _dp], ctypes.c_int),
    "olb_batch_wall_density": ([_vp, ctypes.c_int32, _dp, _dp], ctypes.c_int),
    "olb_batch_use_graph": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_batch_set_tile": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_batch_set_base_temperature": ([_vp, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "olb_batch_autotune": ([_vp, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "olb_batch_tiles": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "olb_batch_launch_config": ([_vp] + [ctypes.POINTER(ctypes.c_int32)] * 3, ctypes.c_int),
    "olb_batch_last_error": ([_vp], ctypes.c_char_p),
    "olb_batch_free": ([_vp], None),
    "olb_set_fields_device": ([_vp, _vp], ctypes.c_int),
    "olb_batch_set_fields_device": ([_vp, ctypes.c_int32, _vp], ctypes.c_int),
    "olb_batch_moments_device": ([_vp, ctypes.c_int32, _vp], ctypes.c_int),
    "olb_closure_workspace_bytes": ([ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "olb_closure_init": ([ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "olb_closure_set_norm": ([_vp, _dp, _dp, _dp], ctypes.c_int),
    "olb_closure_set_params": ([_vp, _fp], ctypes.c_int),
    "olb_closure_get_params": ([_vp, _fp], ctypes.c_int),
    "olb_closure_forward": ([_vp, _vp, _vp], ctypes.c_int),
    "olb_closure_forward_layers": ([_vp, _vp, _vp], ctypes.c_int),
    "olb_closure_gradients": ([_vp, _vp, _vp, _fp, _fp], ctypes.c_int),
    "olb_closure_train_step": ([_vp, _vp, _vp, ctypes.c_float, _fp], ctypes.c_int),
    "olb_closure_apply": ([_vp, _vp, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "olb_closure_set_conserve": ([_vp, ctypes.c_int32], ctypes.c_int),
    "olb_closure_nudge": ([_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "olb_closure_forward_noalloc": ([ctypes.c_int32, ctypes.c_int32, _vp, _dp, _dp, _dp, ctypes.c_int32, _vp, _vp,
                                     _vp], ctypes.c_int),
    "olb_closure_last_error": ([_vp], ctypes.c_char_p),
    "olb_closure_free": ([_vp], None),
    "olb_restrict": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp], ctypes.c_int),
}


def lib():
    """Load libolb.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _check(rc, h=None, batch=False):
    if rc != OLB_OK:
        if h:
            get = {False: lib().olb_last_error, True: lib().olb_batch_last_error,
                   "closure": lib().olb_closure_last_error}[batch]
            msg = get(h).decode()
        else:
            msg = ""
        raise OlbError(rc, msg or lib().olb_strerror(rc).decode())


# ------------------------------------------------------------ C-named calls --

def olb_workspace_bytes(params):
    p = make_params(params) if isinstance(params, dict) else params
    n = ctypes.c_size_t()
    _check(lib().olb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return int(n.value)


def olb_init(params, workspace_ptr, nbytes, stream_ptr):
    p = make_params(params) if isinstance(params, dict) else params
    h = _vp()
    _check(lib().olb_init(ctypes.byref(p), _vp(workspace_ptr), nbytes, _vp(stream_ptr), ctypes.byref(h)))
    return h


def olb_set_fields(h, n, ux, uy, T):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (n, ux, uy, T)]
    _check(lib().olb_set_fields(h, *(_ptr(a) for a in arrs)), h)


def olb_set_fields_device(h, dev_ptr):
    _check(lib().olb_set_fields_device(h, _vp(dev_ptr)), h)


def olb_step(h, nsteps):
    _check(lib().olb_step(h, int(nsteps)), h)


def olb_sync(h):
    _check(lib().olb_sync(h), h)


def olb_moments(h, shape):
    out = [np.empty(shape) for _ in range(4)]
    _check(lib().olb_moments(h, *(_ptr(a) for a in out)), h)
    return tuple(out)


def olb_moments_device(h, dev_ptr):
    _check(lib().olb_moments_device(h, _vp(dev_ptr)), h)


def olb_get_f(h, shape):
    f = np.empty((25,) + tuple(shape))
    _check(lib().olb_get_f(h, _ptr(f)), h)
    return f


def olb_set_f(h, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(lib().olb_set_f(h, _ptr(f)), h)


def olb_wall_density(h, nx):
    lo, hi = np.empty(nx), np.empty(nx)
    _check(lib().olb_wall_density(h, _ptr(lo), _ptr(hi)), h)
    return lo, hi


def olb_set_tile(h, by):
    _check(lib().olb_set_tile(h, int(by)), h)


def olb_set_base_temperature(h, T):
    _check(lib().olb_set_base_temperature(h, float(T)), h)


def olb_set_tile_order(h, strip):
    _check(lib().olb_set_tile_order(h, int(strip)), h)


def olb_launch_counts(h):
    s, w = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().olb_launch_counts(h, ctypes.byref(s), ctypes.byref(w)), h)
    return s.value, w.value


def olb_free(h):
    lib().olb_free(h)


# ------------------------------------------------------------- convenience --

def _need_device_f64(t, count):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == count):
        raise ValueError(f"expected a contiguous float64 CUDA tensor of {count} values, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")

class Lattice:
    """One context on ``device`` with a torch-owned workspace and stream."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the D2Q25 library has no CPU path")
        self.params = dict(_DEFAULTS)
        self.params.update(params)
        self.nx, self.ny = int(self.params["nx"]), int(self.params["ny"])
        self.device = torch.device(device)
        nbytes = olb_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = olb_init(self.params, aligned, nbytes, self.stream.cuda_stream)
        self.nbytes = nbytes

    def close(self):
        if getattr(self, "h", None):
            olb_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.ny, self.nx)

    def set_fields(self, n, ux, uy, T):
        olb_set_fields(self.h, n, ux, uy, T)

    def step(self, nsteps=1):
        olb_step(self.h, nsteps)

    def sync(self):
        olb_sync(self.h)

    def moments(self):
        return olb_moments(self.h, self.shape)

    def moments_device(self, out):
        """Moments into a contiguous float64 CUDA tensor of 4 * ny * nx values."""
        _need_device_f64(out, 4 * self.nx * self.ny)
        olb_moments_device(self.h, out.data_ptr())

    def set_fields_device(self, fields):
        """f <- f^eq of a contiguous float64 CUDA tensor [4][ny][nx]."""
        _need_device_f64(fields, 4 * self.nx * self.ny)
        olb_set_fields_device(self.h, fields.data_ptr())

    def get_f(self):
        return olb_get_f(self.h, self.shape)

    def set_f(self, f):
        olb_set_f(self.h, f)

    def wall_density(self):
        return olb_wall_density(self.h, self.nx)

    def set_tile(self, by):
        olb_set_tile(self.h, by)

    def set_base_temperature(self, T):
        """FP32 departure base at rest and temperature T (default 1)."""
        olb_set_base_temperature(self.h, T)

    def set_tile_order(self, strip):
        olb_set_tile_order(self.h, strip)

    def launch_counts(self):
        return olb_launch_counts(self.h)


# ------------------------------------------------------------------ batches --

def _param_array(params_list):
    arr = (olb_params * len(params_list))()
    for i, p in enumerate(params_list):
        arr[i] = make_params(p) if isinstance(p, dict) else p
    return arr


def olb_batch_workspace_bytes(params_list):
    arr = _param_array(params_list)
    n = ctypes.c_size_t()
    _check(lib().olb_batch_workspace_bytes(arr, len(params_list), ctypes.byref(n)))
    return int(n.value)


def olb_batch_init(params_list, workspace_ptr, nbytes, stream_ptr):
    arr = _param_array(params_list)
    h = _vp()
    _check(lib().olb_batch_init(arr, len(params_list), _vp(workspace_ptr), nbytes, _vp(stream_ptr),
                                ctypes.byref(h)))
    return h


def olb_batch_set_fields(h, i, n, ux, uy, T):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (n, ux, uy, T)]
    _check(lib().olb_batch_set_fields(h, int(i), *(_ptr(a) for a in arrs)), h, True)


def olb_batch_set_fields_device(h, i, dev_ptr):
    _check(lib().olb_batch_set_fields_device(h, int(i), _vp(dev_ptr)), h, True)


def olb_batch_moments_device(h, i, dev_ptr):
    _check(lib().olb_batch_moments_device(h, int(i), _vp(dev_ptr)), h, True)


def olb_batch_set_f(h, i, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(lib().olb_batch_set_f(h, int(i), _ptr(f)), h, True)


def olb_batch_get_f(h, i, shape):
    f = np.empty((25,) + tuple(shape))
    _check(lib().olb_batch_get_f(h, int(i), _ptr(f)), h, True)
    return f


def olb_batch_step(h, nsteps):
    _check(lib().olb_batch_step(h, int(nsteps)), h, True)


def olb_batch_sync(h):
    _check(lib().olb_batch_sync(h), h, True)


def olb_batch_moments(h, i, shape):
    out = [np.empty(shape) for _ in range(4)]
    _check(lib().olb_batch_moments(h, int(i), *(_ptr(a) for a in out)), h, True)
    return tuple(out)


def olb_batch_wall_density(h, i, nx):
    lo, hi = np.empty(nx), np.empty(nx)
    _check(lib().olb_batch_wall_density(h, int(i), _ptr(lo), _ptr(hi)), h, True)
    return lo, hi


def olb_batch_use_graph(h, steps_per_graph):
    _check(lib().olb_batch_use_graph(h, int(steps_per_graph)), h, True)


def olb_batch_set_tile(h, by):
    _check(lib().olb_batch_set_tile(h, int(by)), h, True)


def olb_batch_set_base_temperature(h, i, T):
    _check(lib().olb_batch_set_base_temperature(h, int(i), float(T)), h, True)


def olb_batch_set_tile_order(h, strip):
    _check(lib().olb_batch_set_tile_order(h, int(strip)), h, True)


def olb_batch_autotune(h, trial_steps, cache_path=None):
    chosen = ctypes.c_int32()
    path = cache_path.encode() if cache_path else None
    _check(lib().olb_batch_autotune(h, int(trial_steps), path, ctypes.byref(chosen)), h, True)
    return chosen.value


def olb_batch_launch_config(h):
    by, strip, graph = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().olb_batch_launch_config(h, ctypes.byref(by), ctypes.byref(strip), ctypes.byref(graph)), h, True)
    return by.value, strip.value, graph.value


def olb_batch_tiles(h):
    t, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().olb_batch_tiles(h, ctypes.byref(t), ctypes.byref(b)), h, True)
    return t.value, b.value


def olb_batch_free(h):
    lib().olb_batch_free(h)


class Batch:
    """Many instances on ``device``, stepped in lockstep by single launches.
    Uses its own (default-priority) stream so that HIP graphs can be captured."""

    def __init__(self, params_list, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the D2Q25 library has no CPU path")
        self.params = []
        for p in params_list:
            full = dict(_DEFAULTS)
            full.update(p)
            self.params.append(full)
        self.device = torch.device(device)
        nbytes = olb_batch_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.h = olb_batch_init(self.params, aligned, nbytes, self.stream.cuda_stream)
        self.nbytes = nbytes

    def __len__(self):
        return len(self.params)

    def shape(self, i):
        return (int(self.params[i]["ny"]), int(self.params[i]["nx"]))

    def close(self):
        if getattr(self, "h", None):
            olb_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, i, n, ux, uy, T):
        olb_batch_set_fields(self.h, i, n, ux, uy, T)

    def set_f(self, i, f):
        olb_batch_set_f(self.h, i, f)

    def get_f(self, i):
        return olb_batch_get_f(self.h, i, self.shape(i))

    def step(self, nsteps=1):
        olb_batch_step(self.h, nsteps)

    def sync(self):
        olb_batch_sync(self.h)

    def moments(self, i):
        return olb_batch_moments(self.h, i, self.shape(i))

    def moments_device(self, i, out):
        ny, nx = self.shape(i)
        _need_device_f64(out, 4 * nx * ny)
        olb_batch_moments_device(self.h, i, out.data_ptr())

    def set_fields_device(self, i, fields):
        ny, nx = self.shape(i)
        _need_device_f64(fields, 4 * nx * ny)
        olb_batch_set_fields_device(self.h, i, fields.data_ptr())

    def wall_density(self, i):
        return olb_batch_wall_density(self.h, i, self.shape(i)[1])

    def use_graph(self, steps_per_graph):
        olb_batch_use_graph(self.h, steps_per_graph)

    def set_tile(self, by):
        olb_batch_set_tile(self.h, by)

    def set_base_temperature(self, i, T):
        """FP32 departure base of instance i at rest and temperature T."""
        olb_batch_set_base_temperature(self.h, i, T)

    def set_tile_order(self, strip):
        olb_batch_set_tile_order(self.h, strip)

    def autotune(self, trial_steps=3, cache_path=None):
        return olb_batch_autotune(self.h, trial_steps, cache_path)

    def tiles(self):
        return olb_batch_tiles(self.h)

    def launch_config(self):
        """(tile height, strip width, RK-3 steps per graph)."""
        return olb_batch_launch_config(self.h)


# ------------------------------------------------------------------ closure --

NPARAM = 11588
# offsets of the blocks of the flat parameter vector
PARAM_BLOCKS = (("W1", (32, 4, 3, 3)), ("b1", (32,)), ("W2", (32, 32, 3, 3)), ("b2", (32,)),
                ("W3", (4, 32, 3, 3)), ("b3", (4,)))


def olb_closure_workspace_bytes(nx, ny):
    n = ctypes.c_size_t()
    _check(lib().olb_closure_workspace_bytes(int(nx), int(ny), ctypes.byref(n)))
    return int(n.value)


def olb_closure_init(nx, ny, workspace_ptr, nbytes, stream_ptr):
    h = _vp()
    _check(lib().olb_closure_init(int(nx), int(ny), _vp(workspace_ptr), nbytes, _vp(stream_ptr),
                                  ctypes.byref(h)))
    return h


def _f32(a, count):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != count:
        raise ValueError(f"expected {count} values, got {a.size}")
    return a


def olb_closure_set_norm(h, in_mean, in_scale, out_scale):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (in_mean, in_scale, out_scale)]
    for a in arrs:
        if a.size != 4:
            raise ValueError("normalisation vectors have 4 entries")
    _check(lib().olb_closure_set_norm(h, *(_ptr(a) for a in arrs)), h, "closure")


def olb_closure_set_params(h, params):
    p = _f32(params, NPARAM)
    _check(lib().olb_closure_set_params(h, p.ctypes.data_as(_fp)), h, "closure")


def olb_closure_get_params(h):
    p = np.empty(NPARAM, dtype=np.float32)
    _check(lib().olb_closure_get_params(h, p.ctypes.data_as(_fp)), h, "closure")
    return p


def olb_closure_forward(h, dev_moments, dev_delta):
    _check(lib().olb_closure_forward(h, _vp(dev_moments), _vp(dev_delta)), h, "closure")


def olb_closure_forward_layers(h, dev_moments, dev_delta):
    _check(lib().olb_closure_forward_layers(h, _vp(dev_moments), _vp(dev_delta)), h, "closure")


def olb_closure_gradients(h, dev_moments, dev_reference):
    g = np.empty(NPARAM, dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    _check(lib().olb_closure_gradients(h, _vp(dev_moments), _vp(dev_reference), g.ctypes.data_as(_fp),
                                       loss.ctypes.data_as(_fp)), h, "closure")
    return g, float(loss[0])


def olb_closure_train_step(h, dev_moments, dev_reference, lr, want_loss=True):
    loss = np.zeros(1, dtype=np.float32)
    ptr = loss.ctypes.data_as(_fp) if want_loss else None
    _check(lib().olb_closure_train_step(h, _vp(dev_moments), _vp(dev_reference), ctypes.c_float(lr), ptr),
           h, "closure")
    return float(loss[0]) if want_loss else None


def olb_closure_apply(h, ctx):
    skipped = ctypes.c_int32()
    _check(lib().olb_closure_apply(h, ctx, ctypes.byref(skipped)), h, "closure")
    return skipped.value


def olb_closure_nudge(h, ctx, dev_target, dev_moments=None):
    skipped = ctypes.c_int32()
    _check(lib().olb_closure_nudge(h, ctx, _vp(dev_target), _vp(dev_moments) if dev_moments else None,
                                   ctypes.byref(skipped)), h, "closure")
    return skipped.value


def olb_closure_forward_noalloc(nx, ny, dev_params, in_mean, in_scale, out_scale, mask, dev_moments, dev_delta,
                                stream_ptr):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (in_mean, in_scale, out_scale)]
    for a in arrs:
        if a.size != 4:
            raise ValueError("normalisation vectors have 4 entries")
    _check(lib().olb_closure_forward_noalloc(int(nx), int(ny), _vp(dev_params), *(_ptr(a) for a in arrs), int(mask),
                                             _vp(dev_moments), _vp(dev_delta), _vp(stream_ptr)))


def olb_closure_set_conserve(h, mask):
    _check(lib().olb_closure_set_conserve(h, int(mask)), h, "closure")


def olb_closure_free(h):
    lib().olb_closure_free(h)


def olb_restrict(dev_fine, fnx, fny, factor, dev_coarse, stream_ptr):
    _check(lib().olb_restrict(_vp(dev_fine), int(fnx), int(fny), int(factor), _vp(dev_coarse),
                              _vp(stream_ptr)))


def restrict(fine, fnx, fny, factor, out=None, stream=None):
    """Conservative restriction of a float64 CUDA tensor [4][fny][fnx]."""
    import torch
    _need_device_f64(fine, 4 * fnx * fny)
    cnx, cny = fnx // factor, fny // factor
    if out is None:
        out = torch.empty(4 * cnx * cny, dtype=torch.float64, device=fine.device)
    _need_device_f64(out, 4 * cnx * cny)
    stream = stream if stream is not None else torch.cuda.current_stream(fine.device)
    olb_restrict(fine.data_ptr(), fnx, fny, factor, out.data_ptr(), stream.cuda_stream)
    return out


class Closure:
    """The learned coarse-lattice closure on ``device`` (workspace and stream
    from torch)."""

    def __init__(self, nx, ny, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the closure kernels have no CPU path")
        self.nx, self.ny = int(nx), int(ny)
        self.device = torch.device(device)
        nbytes = olb_closure_workspace_bytes(self.nx, self.ny)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = olb_closure_init(self.nx, self.ny, aligned, nbytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            olb_closure_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _planes(self, t):
        _need_device_f64(t, 4 * self.nx * self.ny)
        return t.data_ptr()

    def set_norm(self, in_mean, in_scale, out_scale):
        olb_closure_set_norm(self.h, in_mean, in_scale, out_scale)

    def set_params(self, params):
        olb_closure_set_params(self.h, params)

    def set_conserve(self, mask):
        """Bit c (0 n, 1 u_x, 2 u_y, 3 T): make that correction mean-free."""
        olb_closure_set_conserve(self.h, mask)

    def get_params(self):
        return olb_closure_get_params(self.h)

    def forward(self, moments, delta):
        olb_closure_forward(self.h, self._planes(moments), self._planes(delta))

    def forward_layers(self, moments, delta):
        olb_closure_forward_layers(self.h, self._planes(moments), self._planes(delta))

    def gradients(self, moments, reference):
        return olb_closure_gradients(self.h, self._planes(moments), self._planes(reference))

    def train_step(self, moments, reference, lr, want_loss=True):
        return olb_closure_train_step(self.h, self._planes(moments), self._planes(reference), lr, want_loss)

    def apply(self, lattice):
        return olb_closure_apply(self.h, lattice.h)

    def nudge(self, lattice, target, moments_out=None):
        """Set the lattice's moments to ``target`` keeping its non-equilibrium
        part; its previous moments go to ``moments_out`` if given."""
        out = self._planes(moments_out) if moments_out is not None else None
        return olb_closure_nudge(self.h, lattice.h, self._planes(target), out)
