"""Steady planar interfaces and the solver's liquid-vapour coexistence curve
(Sec. 5 of the paper: half channel between a specular symmetry plane and a
diffuse wall at T_w).

Python only sequences library calls (a batch of half channels stepped in HIP
graphs); the densities are read back at the end of each chunk.
"""
import numpy as np

from . import olb


def relax(batch, chunk=10000, rtol=1e-8, max_steps=600000, log=None):
    """Step every instance of ``batch`` until the largest density change over
    one chunk, relative to the density, is below ``rtol`` (or ``max_steps``).
    Returns (steps taken, last relative change)."""
    prev = [batch.moments(i)[0].copy() for i in range(len(batch))]
    steps, change = 0, np.inf
    while steps < max_steps:
        batch.step(chunk)
        steps += chunk
        change = 0.0
        for i in range(len(batch)):
            n = batch.moments(i)[0]
            change = max(change, float(np.max(np.abs(n - prev[i]) / n)))
            prev[i] = n.copy()
        if log:
            log(f"{steps} steps: relative density change per chunk {change:.3e}")
        if change < rtol:
            break
    return steps, change


def coexistence(n):
    """Gas and liquid densities of a steady half-channel profile, taken where
    the paper takes them: the node at the channel centre (next to the
    symmetry plane) and the node next to the wall."""
    n = np.asarray(n).reshape(-1)
    return float(n[0]), float(n[-1])


def spurious(moments, tw):
    """Largest speed and largest temperature excess T - T_w of a profile."""
    n, ux, uy, T = (np.asarray(a) for a in moments)
    return float(np.max(np.hypot(ux, uy))), float(np.max(T - tw))
