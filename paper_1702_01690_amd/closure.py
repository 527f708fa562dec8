"""Training and use of the learned coarse-lattice closure.

A coarse lattice (``factor`` times coarser in space and time, FP32 departure
storage) is corrected every ``window`` coarse steps by a small convolutional
network that maps its moments to a moment correction (include/olb.h,
olb_closure_*).  Everything it learns from comes from the solver itself:

  fine run (FP64) --restrict--> reference moments R_0 .. R_W, one per window
  coarse run from R_0, nudged onto R_j at the end of every window (a perfect
      closure: the non-equilibrium part of f is kept) --> inputs X_j
  pair (X_j, R_j): the network learns R_j - X_j

and then, to teach it the states it meets in use (data aggregation), pairs
along coarse runs corrected by the network itself, labelled with the same
fine references.

Python only sequences library calls: the solver, the restriction, the
network's forward and backward passes, Adam and the correction all run in
the library's HIP kernels; torch supplies device memory.
"""
import time

import numpy as np

from . import olb


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the closure has no CPU path")
    return torch


def _check_sizes(fine_params, coarse_params, factor):
    fnx, fny = int(fine_params["nx"]), int(fine_params["ny"])
    cnx, cny = int(coarse_params["nx"]), int(coarse_params["ny"])
    if (cnx * factor, cny * factor) != (fnx, fny):
        raise ValueError("coarse lattice must be the fine one divided by factor")
    return fnx, fny, cnx, cny


def fine_references(fine_params, fields, coarse_params, windows=8, window=10, factor=4, device="cuda:0"):
    """Restricted fine moments at the start and the end of each window:
    float64 CUDA tensor [windows + 1][4 * cny * cnx] (n, u_x, u_y, T planes).
    The fine lattice takes ``factor`` steps per coarse step."""
    torch = _torch()
    fnx, fny, cnx, cny = _check_sizes(fine_params, coarse_params, factor)
    fine = olb.Lattice(fine_params, device=device)
    fine.set_fields(*fields)
    fm = torch.empty(4 * fnx * fny, dtype=torch.float64, device=device)
    refs = torch.empty(windows + 1, 4 * cnx * cny, dtype=torch.float64, device=device)
    for j in range(windows + 1):
        fine.moments_device(fm)
        olb.restrict(fm, fnx, fny, factor, out=refs[j], stream=fine.stream)
        if j < windows:
            fine.step(window * factor)
    fine.sync()
    fine.close()
    return refs


def nudged_inputs(refs, coarse_params, nudger, window=10, device="cuda:0"):
    """Inputs X_1 .. X_W of one continuous coarse run held on the references:
    it starts from f^eq(R_0); at the end of window j its moments are X_j and
    it is then nudged onto R_j.  ``nudger``: any Closure of the coarse size."""
    torch = _torch()
    windows = refs.shape[0] - 1
    coarse = olb.Lattice(coarse_params, device=device)
    coarse.set_fields_device(refs[0])
    X = torch.empty(windows, refs.shape[1], dtype=torch.float64, device=device)
    for j in range(windows):
        coarse.step(window)
        skipped = nudger.nudge(coarse, refs[j + 1], X[j])
        if skipped:
            raise RuntimeError(f"nudge skipped {skipped} nodes")
    coarse.sync()
    coarse.close()
    return X


def rollout_inputs(refs, coarse_params, net, window=10, device="cuda:0"):
    """Inputs X_1 .. X_W of a coarse run from f^eq(R_0) corrected by ``net``
    at the end of every window (moments taken before the correction)."""
    torch = _torch()
    windows = refs.shape[0] - 1
    coarse = olb.Lattice(coarse_params, device=device)
    coarse.set_fields_device(refs[0])
    X = torch.empty(windows, refs.shape[1], dtype=torch.float64, device=device)
    for j in range(windows):
        coarse.step(window)
        coarse.moments_device(X[j])
        net.apply(coarse)
    coarse.sync()
    coarse.close()
    return X


def normalisation(X, R, sample=64):
    """Per-channel input mean and scale and output scale from up to
    ``sample`` pairs spread over the set (host statistics of the data)."""
    k = min(sample, X.shape[0])
    idx = np.linspace(0, X.shape[0] - 1, k).astype(int)
    x = X[idx].cpu().numpy().reshape(k, 4, -1)
    d = (R[idx] - X[idx]).cpu().numpy().reshape(k, 4, -1)
    in_mean = x.mean(axis=(0, 2))
    in_scale = np.maximum(x.std(axis=(0, 2)), 1e-12 + 1e-9 * np.abs(in_mean))
    out_scale = np.maximum(d.std(axis=(0, 2)), 1e-15)
    return in_mean, in_scale, out_scale


def train(net, X, R, epochs=20, lr=1e-3, final_lr=None, seed=0, log=None):
    """Adam over the pairs in a seeded order, one pair per step; the learning
    rate decays geometrically from lr to final_lr.  Returns the mean loss of
    each epoch."""
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    final_lr = lr if final_lr is None else final_lr
    history = []
    total = epochs * n
    step = 0
    for e in range(epochs):
        losses = []
        for i in rng.permutation(n):
            rate = lr * (final_lr / lr) ** (step / max(total - 1, 1))
            losses.append(net.train_step(X[i], R[i], rate, want_loss=True))
            step += 1
        history.append(float(np.mean(losses)))
        if log:
            log(f"epoch {e}: loss {history[-1]:.4e}")
    return history


def train_closure(samples, coarse_params_of, net, windows=8, window=10, factor=4, epochs=30,
                  rounds=2, round_epochs=15, lr=3e-3, round_lr=1e-3, init_params=None, seed=0,
                  log=None, device="cuda:0"):
    """The whole recipe.  ``samples``: (fine_params, fields) pairs;
    ``coarse_params_of(fine_params)`` gives the coarse lattice's parameters.
    Nudged pairs first, then ``rounds`` rounds of data aggregation over the
    network's own runs.  Sets the normalisation and the parameters of
    ``net`` (init_params: float32 vector).  Returns the loss histories, the
    pair count and the normalisation."""
    torch = _torch()
    cps = [coarse_params_of(fp) for fp, _ in samples]
    refs = [fine_references(fp, fl, cp, windows, window, factor, device)
            for (fp, fl), cp in zip(samples, cps)]
    X = torch.cat([nudged_inputs(r, cp, net, window, device) for r, cp in zip(refs, cps)])
    R = torch.cat([r[1:] for r in refs])
    norm = normalisation(X, R)
    net.set_norm(*norm)
    if init_params is not None:
        net.set_params(init_params)
    hist = [train(net, X, R, epochs, lr, lr / 10, seed, log)]
    if log:
        log(f"nudged pairs: {X.shape[0]}, loss {hist[0][0]:.3e} -> {hist[0][-1]:.3e}")
    for k in range(rounds):
        Xn = torch.cat([rollout_inputs(r, cp, net, window, device) for r, cp in zip(refs, cps)])
        X = torch.cat([X, Xn])
        R = torch.cat([R, torch.cat([r[1:] for r in refs])])
        hist.append(train(net, X, R, round_epochs, round_lr, round_lr / 10, seed + 1 + k))
        if log:
            log(f"aggregation round {k + 1}: {X.shape[0]} pairs, loss {hist[-1][0]:.3e} -> {hist[-1][-1]:.3e}")
    return dict(history=hist, pairs=int(X.shape[0]), norm=norm)


def _err(m, ref):
    dn = (m[0] - ref[0]) / ref[0]
    return float(np.abs(dn).max()), float(np.sqrt(np.mean(dn * dn)))


def window_errors(refs, coarse_params, net, window=10, device="cuda:0"):
    """The closure's own job, one window at a time, through the solver: a
    coarse run held on the references (nudged at every window end) gives the
    moments X_j after each window; the density error of X_j (no closure) and
    of X_j + network(X_j) (what apply produces) against R_j.  Returns lists
    of (max relative, rms relative) per window for both."""
    torch = _torch()
    windows = refs.shape[0] - 1
    P4 = refs.shape[1]
    cnx, cny = int(coarse_params["nx"]), int(coarse_params["ny"])
    coarse = olb.Lattice(coarse_params, device=device)
    coarse.set_fields_device(refs[0])
    X = torch.empty(P4, dtype=torch.float64, device=device)
    delta = torch.empty(P4, dtype=torch.float64, device=device)
    plain, fixed = [], []
    for j in range(windows):
        coarse.step(window)
        coarse.moments_device(X)
        coarse.sync()
        net.forward(X, delta)
        x = X.cpu().numpy().reshape(4, cny, cnx)
        d = delta.cpu().numpy().reshape(4, cny, cnx)
        r = refs[j + 1].cpu().numpy().reshape(4, cny, cnx)
        plain.append(_err(x, r))
        fixed.append(_err(x + d, r))
        net.nudge(coarse, refs[j + 1])
    coarse.close()
    return plain, fixed


def rollout_errors(refs, coarse_params, net=None, window=10, device="cuda:0"):
    """Density errors (max relative, rms relative) against R_j at the end of
    each window of a free coarse run from f^eq(R_0), corrected by ``net``
    after every window when given; also the nodes the corrections skipped."""
    windows = refs.shape[0] - 1
    cnx, cny = int(coarse_params["nx"]), int(coarse_params["ny"])
    coarse = olb.Lattice(coarse_params, device=device)
    coarse.set_fields_device(refs[0])
    out, skipped = [], 0
    for j in range(windows):
        coarse.step(window)
        if net is not None:
            skipped += net.apply(coarse)
        m = np.stack(coarse.moments())
        out.append(_err(m, refs[j + 1].cpu().numpy().reshape(4, cny, cnx)))
    coarse.close()
    return out, skipped


def timing(fine_params, fields, coarse_params, net=None, steps=200, window=10, factor=4, device="cuda:0"):
    """Wall-clock seconds of ``steps`` coarse steps (the closure applied every
    ``window`` steps when net is given) and of the same physical time on the
    fine lattice (factor times as many steps).  State resident before each
    timed region."""
    torch = _torch()
    fnx, fny, cnx, cny = _check_sizes(fine_params, coarse_params, factor)
    fine = olb.Lattice(fine_params, device=device)
    fine.set_fields(*fields)
    fine.step(2)
    fine.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fine.step(steps * factor)
    fine.sync()
    t_fine = time.perf_counter() - t0
    fm = torch.empty(4 * fnx * fny, dtype=torch.float64, device=device)
    r0 = torch.empty(4 * cnx * cny, dtype=torch.float64, device=device)
    fine.moments_device(fm)
    olb.restrict(fm, fnx, fny, factor, out=r0, stream=fine.stream)
    fine.sync()
    fine.close()
    coarse = olb.Lattice(coarse_params, device=device)
    coarse.set_fields_device(r0)
    coarse.step(2)
    coarse.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(window, steps - done)
        coarse.step(k)
        done += k
        if net is not None and k == window:
            net.apply(coarse)
    coarse.sync()
    t_coarse = time.perf_counter() - t0
    coarse.close()
    return t_fine, t_coarse
