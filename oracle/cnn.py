"""Plain FP64 CPU reference of the learned coarse-lattice closure.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` alone.  It shares no code
with the GPU package.

The closure is an extension beyond the paper (whose method has no learned
part), so every function below is the textbook definition of its operation,
written out with numpy in float64:

* periodic 3x3 cross-correlation (the convolution layers), ReLU, the mean
  squared error on normalised corrections;
* back-propagation by the chain rule, one layer at a time;
* Adam (Kingma and Ba, 2015) with bias correction;
* conservative restriction: block averages of the density n, the momentum
  density n u and the energy density n (|u|^2 + 2 T) (unit mass, D = 2, as
  in the moments of Sec. 2.2), then u and T recovered from them;
* the correction of a coarse distribution, f + f^eq(m + dm) - f^eq(m), with
  the Hermite equilibrium of Eqs. feq and g_alpha taken from the FP64 solver
  oracle.

``bf16=True`` mirrors the GPU kernels' precision choices: weights,
activations and back-propagated gradients that enter the matrix cores are
rounded to bfloat16 (8 significant bits, round to nearest, ties to even);
sums stay float64 here.  With ``bf16=False`` the network is pure float64,
which the finite-difference pins use.

Parameter vector layout (float, 11588 values):
[W1 (32,4,3,3) | b1 (32) | W2 (32,32,3,3) | b2 (32) | W3 (4,32,3,3) | b3 (4)],
W[o][c][ky][kx] weighting input (x + kx - 1, y + ky - 1).
"""
import numpy as np

BLOCKS = (("W1", (32, 4, 3, 3)), ("b1", (32,)), ("W2", (32, 32, 3, 3)), ("b2", (32,)),
          ("W3", (4, 32, 3, 3)), ("b3", (4,)))
NPARAM = sum(int(np.prod(s)) for _, s in BLOCKS)


def unpack(params):
    """Flat parameter vector -> dict of float64 arrays."""
    p = np.asarray(params, dtype=np.float64).ravel()
    if p.size != NPARAM:
        raise ValueError(f"expected {NPARAM} parameters, got {p.size}")
    out, o = {}, 0
    for name, shape in BLOCKS:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in BLOCKS])


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: half to even


def conv3x3(x, W, b):
    """out[o, y, x] = b[o] + sum_{c, ky, kx} W[o, c, ky, kx] in[c, y+ky-1, x+kx-1]
    with periodic wrap.  x: (C, H, W)."""
    out = np.broadcast_to(b[:, None, None], (W.shape[0],) + x.shape[1:]).astype(np.float64).copy()
    for ky in range(3):
        for kx in range(3):
            # shifted[c, y, x] = x[c, y + ky - 1, x + kx - 1]
            shifted = np.roll(x, shift=(1 - ky, 1 - kx), axis=(1, 2))
            out += np.einsum("oc,chw->ohw", W[:, :, ky, kx], shifted)
    return out


def conv3x3_backward(x, W, g, need_dx=True):
    """Gradients of sum(g * conv3x3(x, W, b)) with respect to W, b and x."""
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            shifted = np.roll(x, shift=(1 - ky, 1 - kx), axis=(1, 2))
            dW[:, :, ky, kx] = np.einsum("ohw,chw->oc", g, shifted)
    db = g.sum(axis=(1, 2))
    dx = None
    if need_dx:
        dx = np.zeros_like(x)
        for ky in range(3):
            for kx in range(3):
                # in[c, q] feeds out[o, q - (ky - 1, kx - 1)]
                back = np.roll(g, shift=(ky - 1, kx - 1), axis=(1, 2))
                dx += np.einsum("oc,ohw->chw", W[:, :, ky, kx], back)
    return dW, db, dx


def _r(x, on):
    return bf16(x) if on else x


def forward(params, m, norm, bf16_mirror=False):
    """Network on moment planes m (4, H, W).  norm = (in_mean, in_scale,
    out_scale), 4 values each.  Returns the intermediates and the
    normalised output z3 (4, H, W)."""
    P = unpack(params)
    in_mean, in_scale, _ = (np.asarray(v, dtype=np.float64) for v in norm)
    W = {k: (_r(P[k], bf16_mirror) if k.startswith("W") else P[k]) for k in P}
    x0 = _r((m - in_mean[:, None, None]) / in_scale[:, None, None], bf16_mirror)
    z1 = conv3x3(x0, W["W1"], W["b1"])
    a1 = _r(np.maximum(z1, 0.0), bf16_mirror)
    z2 = conv3x3(a1, W["W2"], W["b2"])
    a2 = _r(np.maximum(z2, 0.0), bf16_mirror)
    z3 = conv3x3(a2, W["W3"], W["b3"])
    return dict(W=W, x0=x0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3)


def correction(params, m, norm, bf16_mirror=False, conserve_mask=0):
    """Moment correction dm (4, H, W) = network output times out_scale; the
    channels c with bit c of conserve_mask set have their lattice mean
    removed (a conservative correction: zero net change of the total)."""
    out_scale = np.asarray(norm[2], dtype=np.float64)
    z3 = forward(params, m, norm, bf16_mirror)["z3"]
    for c in range(4):
        if (conserve_mask >> c) & 1:
            z3[c] = z3[c] - z3[c].mean()
    return z3 * out_scale[:, None, None]


def loss_and_gradient(params, m, ref, norm, bf16_mirror=False):
    """L = mean over nodes and channels of (z3 - (ref - m) / out_scale)^2 and
    dL/dparams (flat, float64)."""
    out_scale = np.asarray(norm[2], dtype=np.float64)
    s = forward(params, m, norm, bf16_mirror)
    t = (ref - m) / out_scale[:, None, None]
    d = s["z3"] - t
    L = float(np.mean(d * d))
    g3 = _r(2.0 * d / d.size, bf16_mirror)
    W = s["W"]
    dW3, db3, da2 = conv3x3_backward(s["a2"], W["W3"], g3)
    g2 = _r(da2 * (s["z2"] > 0.0), bf16_mirror)
    dW2, db2, da1 = conv3x3_backward(s["a1"], W["W2"], g2)
    g1 = _r(da1 * (s["z1"] > 0.0), bf16_mirror)
    dW1, db1, _ = conv3x3_backward(s["x0"], W["W1"], g1, need_dx=False)
    grad = pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))
    return L, grad


def adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1).  Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def restrict(fields, r):
    """Conservative r x r restriction of moment planes (4, H, W) = (n, u_x,
    u_y, T); H and W multiples of r."""
    n, ux, uy, T = (np.asarray(a, dtype=np.float64) for a in fields)
    H, W = n.shape
    if H % r or W % r:
        raise ValueError("lattice not divisible by the restriction factor")

    def block_mean(a):
        return a.reshape(H // r, r, W // r, r).mean(axis=(1, 3))

    N = block_mean(n)
    Jx = block_mean(n * ux)
    Jy = block_mean(n * uy)
    E = block_mean(n * (ux * ux + uy * uy + 2.0 * T))
    cux, cuy = Jx / N, Jy / N
    cT = 0.5 * (E / N - cux * cux - cuy * cuy)
    return np.stack([N, cux, cuy, cT])


def admissible(m, b):
    n, ux, uy, T = m
    ok = np.isfinite(n) & np.isfinite(ux) & np.isfinite(uy) & np.isfinite(T) & (n > 0.0) & (T > 0.0)
    if b > 0.0:
        ok &= n * b < 1.0
    return ok


def apply_correction(f, m, dm, b, feq):
    """f (25, H, W) + f^eq(m + dm) - f^eq(m) at admissible nodes of m + dm;
    feq(n, ux, uy, T) -> 25 values (the solver oracle's equilibrium).
    Returns the corrected f and the mask of skipped nodes."""
    f = np.array(f, dtype=np.float64)
    new = m + dm
    ok = admissible(new, b)
    H, W = ok.shape
    for y in range(H):
        for x in range(W):
            if ok[y, x]:
                f[:, y, x] += feq(*new[:, y, x]) - feq(*m[:, y, x])
    return f, ~ok
