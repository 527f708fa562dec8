"""Galilean invariance of shear-wave damping (Sec. 6.1 of the paper) and of
longitudinal waves (Sec. 6.2).

A shear wave u_y = u0 sin(k x) (k = 2 pi, L = 1, periodic in x) decays as
u0 exp(-nu_an t) with nu_an = k^2 eta_0 / rho_0 = k^2 tau T0 (Eq. shear_sol,
eta_0 = tau n0 T0, unit mass).  Seen from a frame moving with -V, the same
wave rides on a uniform u_x = V and its profile is u~(t) sin[k (x - V t)]
(Eq. shear_sol_V).  The solver runs every (medium, N_x, V) case as one
instance of a batch; the amplitude is projected out of u_y every ``every``
steps (the discrete Eq. shear_ut) and analysed on the host:

  * eta_app / eta_0 = nu_app / nu_an, nu_app the least-squares fit of
    u0 exp(-nu t) to the sampled amplitudes (u0 held at its initial value);
  * the L2 norm of u~_s / u~_lin(t_s) - 1 by the trapezoid rule
    (Eq. shear_L2);
  * convergence orders: the slope of log|err| against log dx over
    N_x = 20 .. 60 (Tab. shear_ux), and the slope of log of the departure
    from V = 0 against log V over 0 < V <= 0.5 (Tab. shear_nx).

Python only sequences library calls and reads the moments back; the
stepping runs in the library's HIP kernels.
"""
import time

import numpy as np

from . import olb

K = 2.0 * np.pi


def amplitude(uy, x, V, t):
    """Discrete Eq. shear_ut: (2 / N) sum_i u_y,i sin[k (x_i - V t)]."""
    uy = np.asarray(uy, dtype=np.float64).reshape(-1)
    return 2.0 / uy.size * float(np.sum(uy * np.sin(K * (x - V * t))))


def sweep(cases, samples=200, every=1000, graph=10, device="cuda:0", log=None, component="uy"):
    """Run the wave ``cases`` (olb_inputs.shear_wave / sound_wave) as one batch
    for samples * every steps; the amplitude is projected from u_y (shear
    waves) or from u_x - V (component "ux", longitudinal waves).  Returns
    (times [samples + 1], amplitudes [len(cases)][samples + 1], seconds spent
    stepping on the GPU)."""
    if component not in ("uy", "ux"):
        raise ValueError("component is 'uy' or 'ux'")
    plane = 2 if component == "uy" else 1
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the shear-wave sweep has no CPU path")
    dt = float(cases[0].params["dt"])
    if any(float(c.params["dt"]) != dt for c in cases):
        raise ValueError("all cases of a sweep share one time step")
    batch = olb.Batch([c.params for c in cases], device=device)
    if graph:
        batch.use_graph(graph)
    for i, c in enumerate(cases):
        batch.set_fields(i, *c.fields)
    sizes = [4 * c.params["nx"] * c.params["ny"] for c in cases]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    buf = torch.empty(int(offs[-1]), dtype=torch.float64, device=device)
    times = np.arange(samples + 1) * every * dt
    amps = np.empty((len(cases), samples + 1))
    def wave(u, c):
        return u if component == "uy" else u - c.extra["V"]

    for i, c in enumerate(cases):
        amps[i, 0] = amplitude(wave(c.uy if component == "uy" else c.ux, c), c.extra["x"], c.extra["V"], 0.0)
    secs = 0.0
    t0 = time.perf_counter()
    for s in range(1, samples + 1):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(batch.stream)
        batch.step(every)
        ev1.record(batch.stream)
        for i in range(len(cases)):
            batch.moments_device(i, buf[offs[i]:offs[i + 1]])
        batch.sync()
        secs += ev0.elapsed_time(ev1) / 1e3
        host = buf.cpu().numpy()
        for i, c in enumerate(cases):
            n = c.params["nx"] * c.params["ny"]
            u = host[offs[i] + plane * n: offs[i] + (plane + 1) * n]
            amps[i, s] = amplitude(wave(u, c), c.extra["x"], c.extra["V"], times[s])
        if log and s % max(samples // 10, 1) == 0:
            log(f"sample {s}/{samples} ({time.perf_counter() - t0:.1f} s)")
    batch.close()
    return times, amps, secs


def decay_rate(amps, times, u0):
    """nu minimising sum_s (u~_s - u0 exp(-nu t_s))^2: Newton's method on the
    stationarity condition, from the rate of the last sample."""
    a = np.asarray(amps, dtype=np.float64)
    t = np.asarray(times, dtype=np.float64)
    nu = -np.log(max(a[-1] / u0, 1e-300)) / t[-1] if a[-1] > 0 else 1.0 / t[-1]
    for _ in range(100):
        e = u0 * np.exp(-nu * t)
        r = a - e
        g = np.sum(r * t * e)                      # (1/2) d/dnu of the squared residual
        h = np.sum((t * e) ** 2 - r * t * t * e)   # its derivative
        step = g / h
        nu -= step
        if abs(step) <= 1e-16 * abs(nu):
            break
    return float(nu)


def viscosity_ratio(amps, times, u0, tau, T0):
    """eta_app / eta_0 = nu_app / nu_an."""
    return decay_rate(amps, times, u0) / (K * K * tau * T0)


def l2_norm(amps, times, u0, tau, T0):
    """Eq. shear_L2: trapezoid rule over the S + 1 samples, weights 1/2 at
    both ends, normalised by S."""
    a = np.asarray(amps, dtype=np.float64)
    lin = u0 * np.exp(-K * K * tau * T0 * np.asarray(times))
    w = np.ones(a.size)
    w[0] = w[-1] = 0.5
    return float(np.sqrt(np.sum(w * (a / lin - 1.0) ** 2) / (a.size - 1)))


def order(h, err):
    """Exponent gamma of the least-squares fit of err = c h^gamma in log-log."""
    return float(np.polyfit(np.log(np.asarray(h, dtype=np.float64)),
                            np.log(np.abs(np.asarray(err, dtype=np.float64))), 1)[0])


def orders(results, media, sizes, dx_speeds=(0.0, 0.5, 1.0, 2.0), v_speeds=(0.1, 0.2, 0.3, 0.4, 0.5)):
    """Both tables from ``results[(medium, N, V)] = (eta_ratio, L2)``.

    dx: {medium: {V: (eta order, L2 order)}} over ``sizes`` (Tab. shear_ux);
    V:  {medium: {N: (eta order, L2 order)}} over ``v_speeds`` against V = 0
    (Tab. shear_nx)."""
    dx, vv = {}, {}
    for m in media:
        dx[m] = {}
        for V in dx_speeds:
            h = [1.0 / N for N in sizes]
            dx[m][V] = (order(h, [results[(m, N, V)][0] - 1.0 for N in sizes]),
                        order(h, [results[(m, N, V)][1] for N in sizes]))
        vv[m] = {}
        for N in sizes:
            e0, l0 = results[(m, N, 0.0)]
            vv[m][N] = (order(v_speeds, [results[(m, N, V)][0] - e0 for V in v_speeds]),
                        order(v_speeds, [results[(m, N, V)][1] - l0 for V in v_speeds]))
    return dx, vv


def sound_linear(n0, T0, tau, k=K, a=0.0, b=0.0, sigma=0.0):
    """Linearised longitudinal wave of this model (Eqs. sound_cs, long_coeff,
    long_usol): P_eta = p^w (Eq. vdw), P_kappa = p^i = n T, eta = tau n T,
    kappa_T = 2 tau n T (m = 1).  Returns (c_s, nu_a, nu_t, S) with S the
    sine coefficient of Eq. long_usol for a wave started with delta n =
    delta T = 0."""
    dPdn = T0 / (1.0 - b * n0) ** 2 - 2.0 * a * n0
    dPdT = n0 / (1.0 - b * n0)
    cs2 = dPdn + (n0 * T0) / (n0 * n0) * dPdT + n0 * k * k * sigma
    cs = float(np.sqrt(cs2))
    eta, kap = tau * n0 * T0, 2.0 * tau * n0 * T0
    nu_t = k * k * kap / (n0 * cs2) * (dPdn + n0 * k * k * sigma)
    nu_a = k * k * (eta + kap) / (2.0 * n0) - 0.5 * nu_t
    S = ((k * k * kap - n0 * nu_a) ** 2 - n0 * n0 * nu_a * nu_t) / (n0 * k * cs * (k * k * kap - n0 * (nu_a - nu_t)))
    return cs, float(nu_a), float(nu_t), float(S)


def sound_fit(amps, times, du0, nu0, c0, S0=None, k=K):
    """Least-squares fit of Eq. long_usol_2, du0 e^{-nu t} [cos(c k t) +
    S sin(c k t)], to sampled amplitudes: (nu, c, S); with S0 None the sine
    term is dropped (the ideal-gas fit of two parameters)."""
    from scipy.optimize import curve_fit
    t = np.asarray(times, dtype=np.float64)
    a = np.asarray(amps, dtype=np.float64)
    if S0 is None:
        f = lambda tt, nu, c: du0 * np.exp(-nu * tt) * np.cos(c * k * tt)
        (nu, c), _ = curve_fit(f, t, a, p0=[nu0, c0], xtol=1e-15, ftol=1e-15)
        return float(nu), float(c), 0.0
    f = lambda tt, nu, c, S: du0 * np.exp(-nu * tt) * (np.cos(c * k * tt) + S * np.sin(c * k * tt))
    (nu, c, S), _ = curve_fit(f, t, a, p0=[nu0, c0, S0], xtol=1e-15, ftol=1e-15)
    return float(nu), float(c), float(S)
