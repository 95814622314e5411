"""Pins of the learned-guess oracle (CPU, FP64): each layer against an
independent definition, the whole network against finite differences."""
import numpy as np
import pytest

from oracle import learned as NN
from tests import net_layout


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_equals_fft_circular_correlation():
    """y[o] = sum_i corr(x[i], w[o, i]) computed with the 3-D FFT (correlation theorem)."""
    n, ci, co = 6, 3, 4
    x = rnd((ci, n, n, n), 1)
    w = rnd((co, ci, 27), 2)
    y = NN.conv3d(x, w)
    ref = np.zeros_like(y)
    for o in range(co):
        for i in range(ci):
            k = np.zeros((n, n, n))
            for t, (dz, dy, dx) in enumerate(NN.TAPS):
                k[dz % n, dy % n, dx % n] += w[o, i, t]
            # sum_t k[t] x[p + t] = IFFT(FFT(x) conj(FFT(k)))
            ref[o] += np.real(np.fft.ifftn(np.fft.fftn(x[i]) * np.conj(np.fft.fftn(k))))
    assert np.allclose(y, ref, atol=1e-10)


def test_conv_bias_and_single_tap():
    """A centre-tap identity kernel plus bias returns x + b."""
    x = rnd((2, 4, 4, 4), 3)
    w = np.zeros((2, 2, 27))
    w[0, 0, 13] = w[1, 1, 13] = 1.0
    y = NN.conv3d(x, w, np.array([0.5, -1.0]))
    assert np.allclose(y[0], x[0] + 0.5) and np.allclose(y[1], x[1] - 1.0)
    # tap (dz, dy, dx) = (0, 0, +1) reads the next x
    w2 = np.zeros((1, 1, 27))
    w2[0, 0, 14] = 1.0
    assert np.allclose(NN.conv3d(x[:1], w2)[0], np.roll(x[0], -1, axis=2))


def test_conv_adjoints():
    """<conv(x), y> = <x, adjoint(y)> and <conv(x; dw), y> = <dw, wgrad(x, y)>."""
    n, ci, co = 4, 3, 5
    x, y = rnd((ci, n, n, n), 4), rnd((co, n, n, n), 5)
    w, dw = rnd((co, ci, 27), 6), rnd((co, ci, 27), 7)
    lhs = np.sum(NN.conv3d(x, w) * y)
    assert np.isclose(lhs, np.sum(x * NN.conv3d_adjoint(y, w)), rtol=1e-12)
    assert np.isclose(np.sum(NN.conv3d(x, dw) * y), np.sum(dw * NN.conv3d_wgrad(x, y)), rtol=1e-12)


def test_pool_upsample_pairs():
    x, y = rnd((2, 8, 8, 8), 8), rnd((2, 4, 4, 4), 9)
    assert np.isclose(np.sum(NN.avgpool2(x) * y), np.sum(x * NN.avgpool2_adjoint(y)), rtol=1e-12)
    assert np.isclose(np.sum(NN.upsample2(y) * x), np.sum(y * NN.upsample2_adjoint(x)), rtol=1e-12)
    assert np.allclose(NN.avgpool2(NN.upsample2(y)), y)
    assert np.isclose(NN.avgpool2(np.ones((1, 4, 4, 4))).mean(), 1.0)


def test_energy_loss_closed_form_and_gradient():
    """Uniform error e on every load: loss = (lambda0 tr^2 + 2 mu0 e:e) / mu0."""
    n, lam0, mu0 = 2, 1.7, 0.6
    e = np.array([0.1, -0.2, 0.05, 0.03, -0.04, 0.02])   # 11,22,33,23,13,12
    pred = np.tile(e[None, :, None], (6, 1, n ** 3)).reshape(36, n, n, n)
    L, g = NN.energy_loss(pred, np.zeros_like(pred), lam0, mu0)
    E = np.array([[e[0], e[5], e[4]], [e[5], e[1], e[3]], [e[4], e[3], e[2]]])
    assert np.isclose(L, (lam0 * np.trace(E) ** 2 + 2 * mu0 * np.sum(E * E)) / mu0, rtol=1e-14)
    lab = rnd((36, n, n, n), 10)
    pr = rnd((36, n, n, n), 11)
    L0, g = NN.energy_loss(pr, lab, lam0, mu0)
    d = rnd(pr.shape, 12)
    h = 1e-6
    fd = (NN.energy_loss(pr + h * d, lab, lam0, mu0)[0] - NN.energy_loss(pr - h * d, lab, lam0, mu0)[0]) / (2 * h)
    assert np.isclose(fd, np.sum(g * d), rtol=1e-7)


def small_params(seed, ch, scale=0.3):
    r = np.random.default_rng(seed)
    out = []
    for co, ci in NN.layer_shapes(ch):
        out.append((r.standard_normal((co, ci, 27)) * scale / np.sqrt(27 * ci), r.standard_normal(co) * 0.05))
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_network_gradient_matches_finite_differences(seed):
    """Whole encoder-decoder (tiny channels) on 8^3: backward vs central differences."""
    ch, n = (4, 5, 6, 7), 8
    params = small_params(seed, ch)
    r = np.random.default_rng(100 + seed)
    x = r.standard_normal((3, n, n, n))
    lab = r.standard_normal((36, n, n, n)) * 0.1
    lam0, mu0 = 1.3, 0.8

    def loss_of(p):
        out, _ = NN.forward(p, x)
        return NN.energy_loss(out, lab, lam0, mu0)[0]

    out, cache = NN.forward(params, x)
    _, dout = NN.energy_loss(out, lab, lam0, mu0)
    grads = NN.backward(params, cache, dout)
    h = 1e-6
    for k in (0, 5, 8, 14):
        dw = r.standard_normal(params[k][0].shape)
        db = r.standard_normal(params[k][1].shape)
        pp = list(params)
        pm = list(params)
        pp[k] = (params[k][0] + h * dw, params[k][1] + h * db)
        pm[k] = (params[k][0] - h * dw, params[k][1] - h * db)
        fd = (loss_of(pp) - loss_of(pm)) / (2 * h)
        an = np.sum(grads[k][0] * dw) + np.sum(grads[k][1] * db)
        assert np.isclose(fd, an, rtol=1e-5, atol=1e-12), (k, fd, an)


def test_flat_layout_roundtrip():
    params = small_params(3, NN.CH, 1.0)
    flat = net_layout.flatten(params)
    back = net_layout.unflatten(flat)
    assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(params, back))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g from zero moments, the bias-corrected step is lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    w = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    for t in range(1, 6):
        w_new, m, v = NN.adam(w, g, m, v, t, lr)
        assert np.allclose(w - w_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
        w = w_new
