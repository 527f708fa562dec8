"""Parity metrics shared by the GPU tests.

n and T: pointwise max |a - b| / |b|.  Velocity: normwise, the largest error
of the vector u over the lattice divided by the largest |u_ref| (a component
that vanishes by symmetry cannot blow up the ratio).
"""
import numpy as np


def rel_scalar(a, ref):
    return float(np.max(np.abs(a - ref) / np.abs(ref)))


def rel_vector(ax, ay, rx, ry):
    err = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2)
    scale = np.sqrt(rx ** 2 + ry ** 2).max()
    return float(err.max() / scale) if scale > 0 else float(err.max())


def moment_errors(gpu, ref):
    n, ux, uy, T = gpu
    rn, rux, ruy, rT = ref
    return {"n": rel_scalar(n, rn), "u": rel_vector(ux, uy, rux, ruy), "T": rel_scalar(T, rT)}
