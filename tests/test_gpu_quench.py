"""Phase separation between suddenly cooled plates (Sec. 7): a 320 x 640
lattice (walls across y) at the paper's parameters, against what the paper
reports: liquid deposits on the cold walls first (at the coexistence liquid
density), the fluid in the centre stays warmer than the walls while it cools,
and the temperature maxima sit at the liquid-vapour interfaces, not at the
walls.  Diffuse walls conserve mass.  A 32 x 64 crop of the same physics is
checked against the oracle."""
import numpy as np
import pytest

import olb_inputs as I
import oracle
from _metrics import moment_errors
from paper_1702_01690_amd import phase

pytestmark = pytest.mark.gpu


def _olb():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1702_01690_amd import olb
    return olb


def test_quench_physics_matches_oracle():
    olb = _olb()
    c = I.quench(N=32, seed=5)
    lat = olb.Lattice(c.params)
    lat.set_fields(*c.fields)
    lat.step(20)
    o = oracle.Oracle(c.params)
    o.set_fields(*c.fields)
    o.step(20)
    err = moment_errors(lat.moments(), o.moments())
    print(f"[quench] 32x64, 20 steps: {err}", flush=True)
    assert max(err.values()) < 1e-11


def test_quench_early_stage():
    olb = _olb()
    c = I.quench()
    tw, dt = c.params["tw_lo"], c.params["dt"]
    lat = olb.Lattice(c.params)
    lat.set_fields(*c.fields)
    m0 = c.n.sum()
    _, n_liq = phase.maxwell_coexistence(tw)
    centre_prev = None
    done = 0
    for t in (2.5, 5.0):
        k = int(round(t / dt)) - done
        lat.step(k)
        done += k
        n, ux, uy, T = lat.moments()
        ny = n.shape[0]
        pn, pT = n.mean(axis=1), T.mean(axis=1)
        film = 0.5 * (pn[:5].mean() + pn[-5:].mean())
        centre = pT[ny // 2 - 5: ny // 2 + 5].mean()
        hot = np.argmax(pT[: ny // 2]), ny - 1 - np.argmax(pT[ny // 2:][::-1])
        print(f"[quench] t={t}: mass {(n.sum() - m0) / m0:+.2e}, wall film n {film:.4f} (Maxwell {n_liq:.4f}), "
              f"centre T {centre:.4f}, hottest rows {hot}", flush=True)
        assert abs(n.sum() - m0) < 1e-11 * m0
        assert abs(film / n_liq - 1.0) < 0.02
        assert tw < centre < 1.0
        assert min(hot[0], ny - 1 - hot[1]) > 10          # inside the fluid, at the film's edge
        if centre_prev is not None:
            assert centre < centre_prev
        centre_prev = centre
