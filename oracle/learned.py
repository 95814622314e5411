"""Oracle (test infrastructure): the learned initial guess's network in FP64.

Plain numpy, channel-first arrays (C, n, n, n) on the periodic n^3 grid
(z slowest, matching the canonical point order of diag(n, n, n) patterns).
Only tests/ and the benchmark's baseline leg use this module.

The network (the growth step "learned initial guess" of the method's
statement): four levels n, n/2, n/4, n/8 with channels ch = (32, 64, 96, 128);
two periodic 3x3x3 convolutions with ReLU per encoder level, 2x2x2 average
pooling between levels; the decoder upsamples by nearest neighbour, applies a
convolution with ReLU, adds the encoder activation of that level (additive
skip), then a second convolution with ReLU; a last convolution (no
activation) gives 36 channels = fluctuation strain (11,22,33,23,13,12) of the
six Mandel unit loads.  Inputs: phase indicator, mu/mu0 - 1, lambda/lambda0 - 1.
Loss: C0-energy norm of the strain error over mu0, averaged over loads and
points.  Optimiser: Adam (Kingma and Ba) with bias correction.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# ---------------------------------------------------------------- layers
def conv3d(x, w, b=None):
    """Periodic cross-correlation: y[o, p] = sum_{i, t} w[o, i, t] x[i, p + t] (+ b[o]).

    x: (Ci, n, n, n); w: (Co, Ci, 27) with tap t = 9 (dz+1) + 3 (dy+1) + (dx+1).
    """
    co = w.shape[0]
    y = np.zeros((co,) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))   # xs[p] = x[p + t]
        y += np.einsum("oi,izyx->ozyx", w[:, :, t], xs)
    if b is not None:
        y += b[:, None, None, None]
    return y


def conv3d_adjoint(dy, w):
    """dx[i, p] = sum_{o, t} w[o, i, t] dy[o, p - t]  (adjoint of conv3d in x)."""
    ci = w.shape[1]
    dx = np.zeros((ci,) + dy.shape[1:])
    for t, (dz, ddy, ddx) in enumerate(TAPS):
        g = np.einsum("oi,ozyx->izyx", w[:, :, t], dy)
        dx += np.roll(g, shift=(dz, ddy, ddx), axis=(1, 2, 3))   # value at p comes from p - t
    return dx


def conv3d_wgrad(x, dy):
    """dw[o, i, t] = sum_p dy[o, p] x[i, p + t]  (gradient of <dy, conv3d(x, w)> in w)."""
    out = np.zeros((dy.shape[0], x.shape[0], 27))
    for t, (dz, ddy, ddx) in enumerate(TAPS):
        xs = np.roll(x, shift=(-dz, -ddy, -ddx), axis=(1, 2, 3))
        out[:, :, t] = np.einsum("ozyx,izyx->oi", dy, xs)
    return out


def avgpool2(x):
    c, n = x.shape[0], x.shape[1]
    return x.reshape(c, n // 2, 2, n // 2, 2, n // 2, 2).mean(axis=(2, 4, 6))


def avgpool2_adjoint(y):
    return np.repeat(np.repeat(np.repeat(y, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def upsample2_adjoint(y):
    c, n = y.shape[0], y.shape[1]
    return y.reshape(c, n // 2, 2, n // 2, 2, n // 2, 2).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


# ---------------------------------------------------------------- network
CH = (32, 64, 96, 128)


def layer_shapes(ch=CH, n_in=3, n_out=36):
    """(cout, cin) of the 15 convolutions in evaluation order."""
    c0, c1, c2, c3 = ch
    return [(c0, n_in), (c0, c0), (c1, c0), (c1, c1), (c2, c1), (c2, c2), (c3, c2), (c3, c3),
            (c2, c3), (c2, c2), (c1, c2), (c1, c1), (c0, c1), (c0, c0), (n_out, c0)]


def net_input(phase, lame, lam0, mu0, n):
    """Three input channels on the grid from phase ids (canonical order) and the phase table."""
    phase = np.asarray(phase).reshape(n, n, n)
    lame = np.asarray(lame, dtype=np.float64).reshape(-1, 2)
    lam, mu = lame[phase, 0], lame[phase, 1]
    return np.stack([(phase != 0).astype(np.float64), mu / mu0 - 1.0, (lam / lam0 - 1.0) if lam0 != 0 else 0.0 * lam])


def _keep(a):
    return a


def forward(params, x, store=None):
    """Network output (36, n, n, n) and the cache for backward.

    ``store`` (optional) rounds every tensor the network keeps between layers
    (input, activations, skip sums, pooled maps) to a storage format, e.g.
    BF16; the output layer stays unrounded.  Without it everything is FP64."""
    q = store or _keep
    c = {}

    def conv(k, inp, act=True):
        w, b = params[k]
        z = conv3d(inp, w, b)
        return q(relu(z)) if act else z

    c["x0"] = q(x)
    c["e0a"] = conv(0, c["x0"])
    c["e0"] = conv(1, c["e0a"])
    c["p1"] = q(avgpool2(c["e0"]))
    c["e1a"] = conv(2, c["p1"])
    c["e1"] = conv(3, c["e1a"])
    c["p2"] = q(avgpool2(c["e1"]))
    c["e2a"] = conv(4, c["p2"])
    c["e2"] = conv(5, c["e2a"])
    c["p3"] = q(avgpool2(c["e2"]))
    c["e3a"] = conv(6, c["p3"])
    c["e3"] = conv(7, c["e3a"])
    c["u2"] = upsample2(c["e3"])
    c["d2a"] = conv(8, c["u2"])
    c["s2"] = q(c["d2a"] + c["e2"])
    c["d2"] = conv(9, c["s2"])
    c["u1"] = upsample2(c["d2"])
    c["d1a"] = conv(10, c["u1"])
    c["s1"] = q(c["d1a"] + c["e1"])
    c["d1"] = conv(11, c["s1"])
    c["u0"] = upsample2(c["d1"])
    c["d0a"] = conv(12, c["u0"])
    c["s0"] = q(c["d0a"] + c["e0"])
    c["d0"] = conv(13, c["s0"])
    out = conv(14, c["d0"], act=False)
    return out, c


def backward(params, c, dout, store=None):
    """Gradients [(dw, db)] of the 15 convolutions for output gradient dout.

    ``store`` rounds the gradients kept between layers (the output gradient,
    each layer's input gradient, the pooling/upsampling adjoints with their
    skip sums) as ``forward``'s does; weight and bias gradients stay exact."""
    q = store or _keep
    grads = [None] * 15

    def conv_back(k, inp, dz):
        w, _ = params[k]
        grads[k] = (conv3d_wgrad(inp, dz), dz.sum(axis=(1, 2, 3)))
        return q(conv3d_adjoint(dz, w))

    def rb(da, a):   # through ReLU, given its output a
        return da * (a > 0)

    g = conv_back(14, c["d0"], q(dout))
    ds0 = conv_back(13, c["s0"], rb(g, c["d0"]))
    g = conv_back(12, c["u0"], rb(ds0, c["d0a"]))
    g = q(upsample2_adjoint(g))
    ds1 = conv_back(11, c["s1"], rb(g, c["d1"]))
    g = conv_back(10, c["u1"], rb(ds1, c["d1a"]))
    g = q(upsample2_adjoint(g))
    ds2 = conv_back(9, c["s2"], rb(g, c["d2"]))
    g = conv_back(8, c["u2"], rb(ds2, c["d2a"]))
    g = q(upsample2_adjoint(g))
    g = conv_back(7, c["e3a"], rb(g, c["e3"]))
    g = conv_back(6, c["p3"], rb(g, c["e3a"]))
    g = q(avgpool2_adjoint(g) + ds2)
    g = conv_back(5, c["e2a"], rb(g, c["e2"]))
    g = conv_back(4, c["p2"], rb(g, c["e2a"]))
    g = q(avgpool2_adjoint(g) + ds1)
    g = conv_back(3, c["e1a"], rb(g, c["e1"]))
    g = conv_back(2, c["p1"], rb(g, c["e1a"]))
    g = q(avgpool2_adjoint(g) + ds0)
    g = conv_back(1, c["e0a"], rb(g, c["e0"]))
    conv_back(0, c["x0"], rb(g, c["e0a"]))
    return grads


# ---------------------------------------------------------------- loss, optimiser
def energy_loss(pred, label, lam0, mu0, batch=1):
    """Mean over loads and points of e : C0 : e / mu0 with e = pred - label.

    pred, label: (36, n, n, n) = 6 loads x components (11,22,33,23,13,12).
    C0 isotropic: e : C0 : e = lambda0 (tr e)^2 + 2 mu0 (sum of e_ij^2 over
    all nine entries).  Returns (loss, d loss / d pred); batch divides both.
    """
    e = (pred - label).reshape(6, 6, -1)
    P = e.shape[2]
    tr = e[:, 0] + e[:, 1] + e[:, 2]
    r = lam0 / mu0
    sq = e[:, 0] ** 2 + e[:, 1] ** 2 + e[:, 2] ** 2 + 2.0 * (e[:, 3] ** 2 + e[:, 4] ** 2 + e[:, 5] ** 2)
    scale = 1.0 / (6.0 * P * batch)
    loss = scale * float(np.sum(r * tr ** 2 + 2.0 * sq))
    g = np.empty_like(e)
    for c in range(3):
        g[:, c] = scale * (2.0 * r * tr + 4.0 * e[:, c])
    for c in range(3, 6):
        g[:, c] = scale * 8.0 * e[:, c]
    return loss, g.reshape(pred.shape)


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step number t >= 1; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def label_from_strain(strain, n):
    """(6 loads, 6 comps, n^3) fluctuation -> (36, n, n, n) network target."""
    return np.asarray(strain, dtype=np.float64).reshape(36, n, n, n)
