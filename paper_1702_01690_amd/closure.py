"""Training and use of the learned coarse-lattice closure.

A coarse lattice (factor times coarser in space and time, FP32 departure
storage) is corrected every ``every`` coarse steps by a small convolutional
network that maps its moments to a moment correction (include/olb.h,
olb_closure_*).  Training pairs come from the solver itself:

  fine run (FP64) --restrict--> reference moments R_j at t_j = j * window
  coarse run of ``window`` steps from R_j (f = f^eq)  -->  moments X_j+1
  pair: input X_j+1, reference R_j+1 (the network learns R - X)

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


def trajectory_pairs(fine_params, fields, coarse_params, windows=8, window_steps=10, factor=4,
                     device="cuda:0"):
    """Pairs (X, R) of one fine trajectory: float64 CUDA tensors
    [windows][4 * cny * cnx] of coarse-run moments and restricted fine
    moments ``window_steps`` coarse steps after each restart."""
    torch = _torch()
    fnx, fny = int(fine_params["nx"]), int(fine_params["ny"])
    cnx, cny = int(coarse_params["nx"]), int(coarse_params["ny"])
    if (cnx * factor, cny * factor) != (fnx, fny):
        raise ValueError("coarse lattice must be the fine one divided by factor")
    fine = olb.Lattice(fine_params, device=device)
    fine.set_fields(*fields)
    fm = torch.empty(4 * fnx * fny, dtype=torch.float64, device=device)
    refs = torch.empty(windows + 1, 4 * cnx * cny, dtype=torch.float64, device=device)
    for j in range(windows + 1):
        fine.moments_device(fm)
        olb.restrict(fm, fnx, fny, factor, out=refs[j], stream=fine.stream)
        if j < windows:
            fine.step(window_steps * factor)
    fine.sync()
    fine.close()
    coarse = olb.Batch([coarse_params] * windows, device=device)
    for j in range(windows):
        coarse.set_fields_device(j, refs[j])
    coarse.step(window_steps)
    X = torch.empty(windows, 4 * cnx * cny, dtype=torch.float64, device=device)
    for j in range(windows):
        coarse.moments_device(j, X[j])
    coarse.sync()
    coarse.close()
    return X, refs[1:].clone()


def normalisation(X, R, sample=64):
    """Per-channel input mean and scale and output scale from up to
    ``sample`` pairs (host statistics of the training data)."""
    k = min(sample, X.shape[0])
    x = X[:k].cpu().numpy().reshape(k, 4, -1)
    d = (R[:k] - X[:k]).cpu().numpy().reshape(k, 4, -1)
    in_mean = x.mean(axis=(0, 2))
    in_scale = np.maximum(x.std(axis=(0, 2)), 1e-12 + 1e-9 * np.abs(in_mean))
    out_scale = np.maximum(d.std(axis=(0, 2)), 1e-15)
    return in_mean, in_scale, out_scale


def train(closure, X, R, epochs=20, lr=1e-3, final_lr=None, seed=0, log=None):
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
            losses.append(closure.train_step(X[i], R[i], rate, want_loss=True))
            step += 1
        history.append(float(np.mean(losses)))
        if log:
            log(f"epoch {e}: loss {history[-1]:.4e}")
    return history


def _rel(a, ref):
    return float(np.max(np.abs(a - ref) / np.abs(ref)))


def evaluate(fine_params, fields, coarse_params, closure=None, horizon=80, every=10, factor=4,
             device="cuda:0"):
    """Run the fine lattice (FP64) and the coarse one (from the restricted
    initial state) for ``horizon`` coarse steps, the coarse one corrected
    every ``every`` steps when a closure is given.  Returns the coarse run's
    max pointwise relative errors of n and T and the max |u| error against
    the restricted fine moments, the nodes the correction skipped, and the
    wall-clock times of both runs."""
    torch = _torch()
    fnx, fny = int(fine_params["nx"]), int(fine_params["ny"])
    cnx, cny = int(coarse_params["nx"]), int(coarse_params["ny"])
    fine = olb.Lattice(fine_params, device=device)
    fine.set_fields(*fields)
    fm = torch.empty(4 * fnx * fny, dtype=torch.float64, device=device)
    r0 = torch.empty(4 * cnx * cny, dtype=torch.float64, device=device)
    fine.moments_device(fm)
    olb.restrict(fm, fnx, fny, factor, out=r0, stream=fine.stream)
    fine.sync()
    coarse = olb.Lattice(coarse_params, device=device)
    coarse.set_fields_device(r0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fine.step(horizon * factor)
    fine.sync()
    t_fine = time.perf_counter() - t0

    skipped = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < horizon:
        k = min(every, horizon - done)
        coarse.step(k)
        done += k
        if closure is not None and k == every:
            skipped += closure.apply(coarse)
    coarse.sync()
    t_coarse = time.perf_counter() - t0

    fine.moments_device(fm)
    ref = torch.empty_like(r0)
    olb.restrict(fm, fnx, fny, factor, out=ref, stream=fine.stream)
    fine.sync()
    rn, rux, ruy, rT = ref.cpu().numpy().reshape(4, cny, cnx)
    n, ux, uy, T = coarse.moments()
    du = np.sqrt((ux - rux) ** 2 + (uy - ruy) ** 2).max()
    out = dict(n=_rel(n, rn), T=_rel(T, rT), u_abs=float(du), skipped=int(skipped),
               fine_s=t_fine, coarse_s=t_coarse,
               ref_n_range=float(rn.max() - rn.min()))
    fine.close()
    coarse.close()
    return out
