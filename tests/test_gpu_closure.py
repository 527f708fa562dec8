"""Learned closure kernels against the FP64 closure oracle (oracle/cnn.py).

* restriction: FP64 both sides, summation order aside;
* forward pass and gradients: the oracle mirrors the kernels' bf16 rounding
  of weights, activations and back-propagated gradients, so the two differ
  only by FP32-versus-FP64 accumulation and the rare bf16 rounding it flips;
  against the pure-FP64 network the bar is the bf16 precision (2^-9 relative
  per rounding, a few roundings deep);
* one Adam step against the oracle's Adam on the kernel's own gradient;
* the correction with a constant network output (zero weights, biases b3)
  against the oracle's correction of the same f, including skipped nodes,
  and the restart of the solver from the corrected state;
* end to end: a network trained on solver-generated pairs by these kernels
  reduces the coarse lattice's error against the fine one on a held-out
  sample.
"""
import numpy as np
import pytest

import olb_inputs as I
import oracle
from oracle import cnn

pytestmark = pytest.mark.gpu


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1702_01690_amd import olb
    return torch, olb


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device="cuda:0")


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _setup(nx, ny, seed=3, bias=True):
    params = I.closure_params(seed=seed, last_scale=1.0)
    if bias:
        d = cnn.unpack(params.astype(np.float64))
        r = I.uniform(seed + 100, 68) - 0.5
        d["b1"][:], d["b2"][:], d["b3"][:] = 0.1 * r[:32], 0.1 * r[32:64], 0.1 * r[64:68]
        params = cnn.pack(d).astype(np.float32)
    m = I.closure_moments(nx, ny, seed=seed + 1)
    ref = m + 0.01 * (I.closure_moments(nx, ny, seed=seed + 2) - m)
    norm = (m.mean(axis=(1, 2)), m.std(axis=(1, 2)), np.abs(ref - m).std(axis=(1, 2)))
    return params, m, ref, norm


@pytest.mark.parametrize("shape", [(64, 48), (36, 20), (4, 4)])
def test_restriction_matches_oracle(shape):
    torch, olb = _env()
    fnx, fny = shape
    f = I.closure_moments(fnx, fny, seed=71, amplitude=0.05)
    out = olb.restrict(_dev(torch, f), fnx, fny, 4)
    got = out.cpu().numpy().reshape(4, fny // 4, fnx // 4)
    want = cnn.restrict(f, 4)
    print(f"[closure] restrict {shape}: max rel {np.max(np.abs(got - want) / np.abs(want)):.2e}", flush=True)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-16)


def test_restriction_rejects_bad_sizes():
    torch, olb = _env()
    f = _dev(torch, np.ones(4 * 10 * 8))
    with pytest.raises(olb.OlbError):
        olb.olb_restrict(f.data_ptr(), 10, 8, 4, f.data_ptr(), 0)


@pytest.mark.parametrize("shape,mask", [((37, 23), 0), ((64, 32), 0), ((5, 3), 0), ((37, 23), 7),
                                        ((20, 12), 15)])
def test_forward_matches_oracle(shape, mask):
    torch, olb = _env()
    nx, ny = shape
    params, m, _, norm = _setup(nx, ny)
    c = olb.Closure(nx, ny)
    c.set_norm(*norm)
    c.set_params(params)
    c.set_conserve(mask)
    delta = torch.empty(4 * nx * ny, dtype=torch.float64, device="cuda:0")
    c.forward(_dev(torch, m), delta)
    torch.cuda.synchronize()
    got = delta.cpu().numpy().reshape(4, ny, nx)
    mirrored = cnn.correction(params, m, norm, bf16_mirror=True, conserve_mask=mask)
    exact = cnn.correction(params, m, norm, bf16_mirror=False, conserve_mask=mask)
    for ch in range(4):
        if (mask >> ch) & 1:
            assert abs(got[ch].mean()) <= 1e-12 * np.abs(got[ch]).max()
    e_m, e_x = _rel_l2(got, mirrored), _rel_l2(got, exact)
    scale = np.abs(mirrored).max()
    e_max = np.abs(got - mirrored).max() / scale
    print(f"[closure] forward {shape} mask {mask}: rel-L2 vs bf16-mirrored {e_m:.2e} (max {e_max:.2e}), "
          f"vs FP64 {e_x:.2e}", flush=True)
    assert e_m < 1e-3 and e_max < 1e-2
    assert e_x < 3e-2


@pytest.mark.parametrize("shape", [(37, 23), (64, 48), (16, 16), (5, 3), (130, 17), (300, 260), (512, 512)])
def test_fused_inference_equals_layer_by_layer_forward(shape):
    """The fused kernel (ragged edge tiles, lattices smaller than its halo,
    and lattices with more tiles than workgroups, where a workgroup takes
    several tiles in turn) against the training path's per-layer kernels."""
    torch, olb = _env()
    nx, ny = shape
    params, m, _, norm = _setup(nx, ny, seed=17)
    c = olb.Closure(nx, ny)
    c.set_norm(*norm)
    c.set_params(params)
    dm = _dev(torch, m)
    fused, layers = torch.empty_like(dm), torch.empty_like(dm)
    c.set_conserve(0)
    c.forward(dm, fused)
    c.forward_layers(dm, layers)
    torch.cuda.synchronize()
    assert torch.equal(fused, layers)
    c.set_conserve(7)
    c.forward(dm, fused)
    c.forward_layers(dm, layers)
    torch.cuda.synchronize()
    f, l = fused.cpu().numpy(), layers.cpu().numpy()
    assert np.abs(f - l).max() <= 1e-12 * np.abs(l).max()


@pytest.mark.parametrize("shape", [(37, 23), (64, 64)])
def test_gradients_match_oracle(shape):
    torch, olb = _env()
    nx, ny = shape
    params, m, ref, norm = _setup(nx, ny, seed=5)
    c = olb.Closure(nx, ny)
    c.set_norm(*norm)
    c.set_params(params)
    g, loss = c.gradients(_dev(torch, m), _dev(torch, ref))
    L_m, g_m = cnn.loss_and_gradient(params, m, ref, norm, bf16_mirror=True)
    L_x, g_x = cnn.loss_and_gradient(params, m, ref, norm, bf16_mirror=False)
    print(f"[closure] loss gpu {loss:.6e} mirrored {L_m:.6e} fp64 {L_x:.6e}", flush=True)
    assert abs(loss - L_m) <= 1e-4 * L_m
    o = 0
    for name, shape_b in cnn.BLOCKS:
        k = int(np.prod(shape_b))
        em = _rel_l2(g[o:o + k], g_m[o:o + k])
        ex = _rel_l2(g[o:o + k], g_x[o:o + k])
        print(f"[closure] grad {name}: rel-L2 vs mirrored {em:.2e}, vs FP64 {ex:.2e}", flush=True)
        assert em < 5e-3, name
        assert ex < 5e-2, name
        o += k
    cos = float(g @ g_m / (np.linalg.norm(g) * np.linalg.norm(g_m)))
    assert cos > 0.99999


@pytest.mark.parametrize("shape", [(37, 23), (300, 260)])
def test_sums_over_nodes_are_reproducible(shape):
    """Gradients, loss and the projected corrections are sums over nodes
    formed from per-workgroup partial sums in a fixed order: two evaluations
    on the same inputs give the same bits, and so do two training runs."""
    torch, olb = _env()
    nx, ny = shape
    params, m, ref, norm = _setup(nx, ny, seed=11)
    dm, dr = _dev(torch, m), _dev(torch, ref)
    c = olb.Closure(nx, ny)
    c.set_norm(*norm)
    c.set_params(params)
    g1, l1 = c.gradients(dm, dr)
    g2, l2 = c.gradients(dm, dr)
    assert np.array_equal(g1, g2) and l1 == l2
    c.set_conserve(7)
    for fwd in (c.forward, c.forward_layers):
        a, b = torch.empty_like(dm), torch.empty_like(dm)
        fwd(dm, a)
        fwd(dm, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    runs = []
    for _ in range(2):
        c.set_params(params)                   # also resets the Adam state
        for _ in range(3):
            c.train_step(dm, dr, 1e-3)
        runs.append(c.get_params())
    assert np.array_equal(runs[0], runs[1])


def test_train_step_is_adam_on_the_kernel_gradient():
    torch, olb = _env()
    nx, ny = 40, 24
    params, m, ref, norm = _setup(nx, ny, seed=9)
    c = olb.Closure(nx, ny)
    c.set_norm(*norm)
    c.set_params(params)
    dm, dr = _dev(torch, m), _dev(torch, ref)
    g, _ = c.gradients(dm, dr)
    lr = 1e-3
    c.train_step(dm, dr, lr)
    got = c.get_params().astype(np.float64)
    want, _, _ = cnn.adam(params.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr)
    # the kernel's Adam step is FP32: its first step, lr g / (|g| + eps), is
    # lr sign(g) to FP32 rounding unless |g| ~ eps
    err = np.abs(got - want)
    print(f"[closure] adam max |diff| {err.max():.2e} (lr {lr})", flush=True)
    assert np.quantile(err, 0.999) < 1e-6 * lr + 1e-7 and err.max() < lr


def _coarse_lattice(olb, precision, seed=5002):
    fine = I.closure_sample(64, 48, seed=seed)
    cp = I.coarse_params(fine.params, precision=precision)
    lat = olb.Lattice(cp)
    m = I.closure_moments(cp["nx"], cp["ny"], seed=seed + 1)
    lat.set_fields(*m)
    lat.step(3)
    return cp, lat


@pytest.mark.parametrize("precision", [0, 1])
def test_constant_correction_matches_oracle_and_restarts(precision):
    torch, olb = _env()
    cp, lat = _coarse_lattice(olb, precision)
    nx, ny = cp["nx"], cp["ny"]
    f0 = lat.get_f()
    m0 = np.stack(lat.moments())
    params = np.zeros(cnn.NPARAM, dtype=np.float32)
    b3 = np.array([1e-3, 2e-4, -3e-4, 5e-4], dtype=np.float32)
    params[-4:] = b3
    c = olb.Closure(nx, ny)
    c.set_norm(np.zeros(4), np.ones(4), np.ones(4))
    c.set_params(params)
    c.set_conserve(0)           # a uniform correction of every moment
    skipped = c.apply(lat)
    assert skipped == 0
    dm = np.broadcast_to(b3.astype(np.float64)[:, None, None], m0.shape)
    want, mask = cnn.apply_correction(f0, m0, dm, cp["b"], oracle.feq)
    assert not mask.any()
    got = lat.get_f()
    tol = 1e-13 if precision == 0 else 2e-6
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"[closure] apply precision {precision}: max rel f error {err:.2e}", flush=True)
    assert err < tol
    m1 = np.stack(lat.moments())
    np.testing.assert_allclose(m1[0], m0[0] + dm[0], rtol=10 * tol)
    # the solver restarts from the corrected f with a refreshed carried state
    if precision == 0:
        o = oracle.Oracle(cp)
        o.set_f(want)
        o.step(4)
        lat.step(4)
        ref = np.stack(o.moments())
        got_m = np.stack(lat.moments())
        err = np.abs(got_m - ref).max(axis=(1, 2)) / np.abs(ref).max(axis=(1, 2))
        print(f"[closure] restart after apply: {err}", flush=True)
        assert err[0] < 1e-11 and err[3] < 1e-11


def test_correction_skips_inadmissible_nodes():
    torch, olb = _env()
    cp, lat = _coarse_lattice(olb, 0)
    nx, ny = cp["nx"], cp["ny"]
    f0 = lat.get_f()
    m0 = np.stack(lat.moments())
    # dn = 1/b - 3.5 pushes every node with n >= 3.5 out of (0, 1/b)
    dn = np.float32(1.0 / cp["b"] - I.N_CRIT)
    params = np.zeros(cnn.NPARAM, dtype=np.float32)
    params[-4] = dn
    c = olb.Closure(nx, ny)
    c.set_norm(np.zeros(4), np.ones(4), np.ones(4))
    c.set_params(params)
    c.set_conserve(0)
    skipped = c.apply(lat)
    dm = np.zeros_like(m0)
    dm[0] = float(dn)
    want, mask = cnn.apply_correction(f0, m0, dm, cp["b"], oracle.feq)
    print(f"[closure] skipped {skipped} of {nx * ny} (oracle {int(mask.sum())})", flush=True)
    assert 0 < skipped < nx * ny and skipped == int(mask.sum())
    got = lat.get_f()
    np.testing.assert_array_equal(got[:, mask], f0[:, mask])
    assert np.abs(got - want).max() / np.abs(want).max() < 1e-13


def test_conservative_apply_keeps_total_mass():
    torch, olb = _env()
    cp, lat = _coarse_lattice(olb, 0)
    nx, ny = cp["nx"], cp["ny"]
    m0 = np.stack(lat.moments())
    params, _, _, _ = _setup(nx, ny, seed=13)
    c = olb.Closure(nx, ny)
    c.set_norm(m0.mean(axis=(1, 2)), m0.std(axis=(1, 2)), np.array([1e-3, 1e-4, 1e-4, 1e-4]))
    c.set_params(params)        # default projection: n, u_x, u_y mean-free
    assert c.apply(lat) == 0
    m1 = np.stack(lat.moments())
    print(f"[closure] mass before {m0[0].sum():.15e} after {m1[0].sum():.15e}; "
          f"max |dn| {np.abs(m1[0] - m0[0]).max():.2e}", flush=True)
    assert np.abs(m1[0] - m0[0]).max() > 1e-5          # the correction did something
    assert abs(m1[0].sum() - m0[0].sum()) <= 1e-13 * m0[0].sum()


def test_closure_state_errors():
    torch, olb = _env()
    c = olb.Closure(8, 8)
    z = torch.zeros(4 * 64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(olb.OlbError) as e:
        c.forward(z, z.clone())
    assert e.value.code == olb.OLB_E_STATE
    bad = np.zeros(cnn.NPARAM, dtype=np.float32)
    bad[7] = np.nan
    with pytest.raises(olb.OlbError) as e:
        c.set_params(bad)
    assert e.value.code == olb.OLB_E_ARG
    with pytest.raises(olb.OlbError):
        c.set_norm(np.zeros(4), np.zeros(4), np.ones(4))


def test_set_fields_device_matches_host_and_checks_domain():
    torch, olb = _env()
    case = I.spinodal(40, 24, seed=8)
    a, b = olb.Lattice(case.params), olb.Lattice(case.params)
    a.set_fields(*case.fields)
    b.set_fields_device(_dev(torch, np.stack(case.fields)))
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    a.step(2)
    b.step(2)
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    bad = np.stack(case.fields).copy()
    bad[3, 5, 7] = -1.0
    with pytest.raises(olb.OlbError) as e:
        b.set_fields_device(_dev(torch, bad))
    assert e.value.code == olb.OLB_E_DOMAIN
    np.testing.assert_array_equal(a.get_f(), b.get_f())   # previous state kept


def test_trained_closure_gains_over_the_plain_coarse_run():
    """Trains the network on the GPU from 12 fine/coarse trajectories and
    evaluates it on a held-out sample against the restricted fine run:
    after training on nudged pairs, per window through the solver; after one
    round of data aggregation over its own runs, along a free corrected run
    (better in the first windows, bounded later)."""
    torch, olb = _env()
    from paper_1702_01690_amd import closure as C
    nf, windows = 128, 10
    refs, cps = [], []
    for seed in range(5000, 5012):
        s = I.closure_sample(nf, seed=seed)
        cps.append(I.coarse_params(s.params))
        refs.append(C.fine_references(s.params, s.fields, cps[-1], windows))
    net = olb.Closure(nf // 4, nf // 4)
    X = torch.cat([C.nudged_inputs(r, cp, net) for r, cp in zip(refs, cps)])
    R = torch.cat([r[1:] for r in refs])
    net.set_norm(*C.normalisation(X, R))
    net.set_params(I.closure_params(seed=7))
    h = C.train(net, X, R, epochs=30, lr=3e-3, final_lr=3e-4, seed=1)
    print(f"[closure] {X.shape[0]} nudged pairs; loss {h[0]:.3e} -> {h[-1]:.3e}", flush=True)
    assert h[-1] < 0.6 * h[0]

    held = I.closure_sample(nf, seed=6000)
    cp = I.coarse_params(held.params)
    href = C.fine_references(held.params, held.fields, cp, windows)
    plain, fixed = C.window_errors(href, cp, net)
    rp, rf = np.mean([r for _, r in plain]), np.mean([r for _, r in fixed])
    mp, mf = np.mean([m for m, _ in plain]), np.mean([m for m, _ in fixed])
    print(f"[closure] per-window density error, mean over windows: rms {rp:.3e} -> {rf:.3e}, "
          f"max {mp:.3e} -> {mf:.3e}", flush=True)
    assert rf < 0.85 * rp and mf < mp

    X = torch.cat([X] + [C.rollout_inputs(r, cp_, net) for r, cp_ in zip(refs, cps)])
    R = torch.cat([R, R])
    h = C.train(net, X, R, epochs=15, lr=1e-3, final_lr=1e-4, seed=2)
    print(f"[closure] aggregation: {X.shape[0]} pairs, loss {h[0]:.3e} -> {h[-1]:.3e}", flush=True)
    roll_p, _ = C.rollout_errors(href, cp, None)
    roll_f, skipped = C.rollout_errors(href, cp, net)
    print("[closure] free run (max/rms per window) plain:   " + " ".join(f"{a:.2e}/{b:.1e}" for a, b in roll_p),
          flush=True)
    print("[closure] free run (max/rms per window) closure: " + " ".join(f"{a:.2e}/{b:.1e}" for a, b in roll_f),
          flush=True)
    assert skipped == 0
    # first free window: 15 % on the rms; the maximum (one node out of 16k)
    # must improve too (0.73-0.86 measured across kernel builds)
    assert roll_f[0][1] < 0.85 * roll_p[0][1] and roll_f[0][0] < roll_p[0][0]
    # stability, not accuracy: without data aggregation the corrected free
    # run grows x10 within 25 windows; with it, it stays near the plain run
    # (the long horizon is set by modes no coarse state predicts, and moves
    # with FP32 rounding: 1.0-1.32x measured across kernel builds)
    assert max(b for _, b in roll_f) < 1.5 * max(b for _, b in roll_p)
