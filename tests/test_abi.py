"""The C-ABI library loads and exports every symbol its header declares, and
its host-side argument validation (no device work) behaves as documented."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "olb.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(olb_[a-z_]+)\s*\(", text)))


def _lib():
    from paper_1702_01690_amd import olb
    if not os.path.exists(olb.LIB_PATH):
        pytest.fail("libolb.so is not built (run __graft_entry__.build())")
    return olb, olb.lib()


def test_library_exports_every_declared_symbol():
    olb, L = _lib()
    names = _declared()
    assert "olb_step" in names and "olb_init" in names
    for n in names:
        assert hasattr(L, n), n
    # and the binding wraps each one under the same name
    for n in names:
        if n in ("olb_last_error", "olb_strerror", "olb_batch_last_error", "olb_closure_last_error"):
            continue
        assert hasattr(olb, n), n


def _params(**kw):
    p = dict(nx=32, ny=32, ds=1 / 32, dt=5e-4, tau=0.01, a=9 / 49, b=2 / 21, sigma=1e-4)
    p.update(kw)
    return p


def test_workspace_size_and_validation_codes():
    olb, L = _lib()
    nb = olb.olb_workspace_bytes(_params())
    # three FP64 distribution arrays with ghost rows + carries + wall + flag
    assert nb >= 3 * 25 * 38 * 32 * 8 + 2 * 2 * 32 * 32 * 8
    nb32 = olb.olb_workspace_bytes(_params(precision=1, rho_ref=1.0))
    assert nb32 < nb
    cases = [(dict(dt=0.02), olb.OLB_E_CFL), (dict(tau=0.0), olb.OLB_E_DOMAIN),
             (dict(bc_x=1), olb.OLB_E_ARG), (dict(bc_x=2), olb.OLB_E_ARG), (dict(bc_x=3, nx=2), olb.OLB_E_ARG),
             (dict(bc_y=1, ny=2), olb.OLB_E_ARG),
             (dict(nx=0), olb.OLB_E_ARG), (dict(precision=1, rho_ref=0.0), olb.OLB_E_ARG),
             (dict(bc_y=1, tw_lo=0.0), olb.OLB_E_DOMAIN), (dict(sigma=-1.0), olb.OLB_E_ARG),
             # 32-bit byte offsets within a plane: 16384 x 16384 (with its 6 ghost rows) is one
             # plane too many for FP64 values, and the carried FP64 fields bound FP32 storage alike
             (dict(nx=16384, ny=16384), olb.OLB_E_ARG), (dict(nx=16384, ny=16384, precision=1, rho_ref=1.0), olb.OLB_E_ARG)]
    for kw, code in cases:
        with pytest.raises(olb.OlbError) as e:
            olb.olb_workspace_bytes(_params(**kw))
        assert e.value.code == code, kw
    # the largest accepted FP64 lattice of that width: (ny + 6) * 16384 * 8 < 2^31
    assert olb.olb_workspace_bytes(_params(nx=16384, ny=16384 - 7)) > 0


def test_init_rejects_small_or_misaligned_workspace_without_touching_device():
    olb, L = _lib()
    p = olb.make_params(_params())
    h = ctypes.c_void_p()
    nb = olb.olb_workspace_bytes(_params())
    rc = L.olb_init(ctypes.byref(p), ctypes.c_void_p(4096), nb - 1, None, ctypes.byref(h))
    assert rc == olb.OLB_E_WORKSPACE
    rc = L.olb_init(ctypes.byref(p), ctypes.c_void_p(4096 + 8), nb, None, ctypes.byref(h))
    assert rc == olb.OLB_E_WORKSPACE
    assert L.olb_strerror(olb.OLB_E_CFL).decode().startswith("CFL")


def test_closure_validation_without_device_work():
    olb, L = _lib()
    nb = olb.olb_closure_workspace_bytes(64, 48)
    # activations (bf16 and FP32 pre-activations), moments, parameters and Adam state
    assert nb >= 64 * 48 * (32 * 2 * 2 + 32 * 4 * 2) + 4 * olb.NPARAM * 4
    for nx, ny in ((0, 4), (4, -1)):
        with pytest.raises(olb.OlbError) as e:
            olb.olb_closure_workspace_bytes(nx, ny)
        assert e.value.code == olb.OLB_E_ARG
    with pytest.raises(olb.OlbError) as e:
        olb.olb_closure_init(8, 8, 0, 1 << 20, 0)
    assert e.value.code == olb.OLB_E_WORKSPACE
    with pytest.raises(olb.OlbError) as e:
        olb.olb_closure_init(8, 8, 256 * 1000 + 8, 1 << 20, 0)      # misaligned
    assert e.value.code == olb.OLB_E_WORKSPACE
    with pytest.raises(olb.OlbError) as e:
        olb.olb_closure_init(8, 8, 256 * 1000, 16, 0)               # too small
    assert e.value.code == olb.OLB_E_WORKSPACE
    for fnx, fny, r in ((10, 8, 4), (8, 8, 0), (2, 8, 4)):
        with pytest.raises(olb.OlbError) as e:
            olb.olb_restrict(1 << 20, fnx, fny, r, 1 << 21, 0)
        assert e.value.code == olb.OLB_E_ARG
    assert L.olb_closure_last_error(None) == b"null closure"


def test_noalloc_closure_forward_rejects_null_pointers_on_the_host():
    """The allocation-free inference call validates its arguments before it
    touches a device."""
    import numpy as np
    olb, L = _lib()
    one = np.ones(4)
    with pytest.raises(olb.OlbError) as e:
        olb.olb_closure_forward_noalloc(8, 8, None, one, one, one, 0, None, None, None)
    assert e.value.code == olb.OLB_E_ARG
