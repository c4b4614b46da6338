"""Pins of the FP64 network reference (oracle/convnet.py): the valid complex convolution
against scipy's correlation, and the analytic Wirtinger gradients against central finite
differences of the loss."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import convnet


def _setup(C=3, B=2, H=6, W=9, seed=0):
    rng = np.random.default_rng(seed)
    params = convnet.unflat(rng.standard_normal(
        sum(2 * co * ci * 25 + 2 * co for ci, co in zip([1, C, C, C], [C, C, C, 1]))) * 0.3, C)
    x = rng.standard_normal((B, 1, H + 16, W + 16)) + 1j * rng.standard_normal((B, 1, H + 16, W + 16))
    tgt = rng.standard_normal((B, 1, H, W)) + 1j * rng.standard_normal((B, 1, H, W))
    row0 = np.array([0, 5])[:B]
    return params, x, tgt, row0


def test_conv_valid_matches_scipy_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 2, 11, 13)) + 1j * rng.standard_normal((1, 2, 11, 13))
    w = rng.standard_normal((3, 2, 5, 5)) + 1j * rng.standard_normal((3, 2, 5, 5))
    b = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    y = convnet.conv_valid(x, w, b)
    for co in range(3):
        want = b[co] + sum(correlate(x[0, ci], np.conj(w[co, ci]), mode="valid") for ci in range(2))
        assert np.max(np.abs(y[0, co] - want)) < 1e-12


def test_flat_round_trip():
    params, *_ = _setup()
    v = convnet.flat(params)
    back = convnet.unflat(v, 3)
    for (w0, b0), (w1, b1) in zip(params, back):
        assert np.array_equal(w0, w1) and np.array_equal(b0, b1)


@pytest.mark.parametrize("layer", [0, 1, 3])
def test_gradients_match_finite_differences(layer):
    params, x, tgt, row0 = _setup()
    out, acts = convnet.forward(params, x)
    grads = convnet.backward(params, acts, out, tgt, row0)
    rng = np.random.default_rng(layer)
    w, b = params[layer]
    h = 1e-6
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in w.shape)
        for part, unit in ((0, 1.0), (1, 1j)):
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[layer][0][idx] += h * unit
            wm[layer][0][idx] -= h * unit
            fd = (convnet.loss(convnet.forward(wp, x)[0], tgt, row0) -
                  convnet.loss(convnet.forward(wm, x)[0], tgt, row0)) / (2 * h)
            g = grads[layer][0][idx]
            an = g.real if part == 0 else g.imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (layer, idx, part, fd, an)
    # bias gradient
    co = 0
    for unit, part in ((1.0, 0), (1j, 1)):
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[layer][1][co] += h * unit
        bm[layer][1][co] -= h * unit
        fd = (convnet.loss(convnet.forward(bp, x)[0], tgt, row0) - convnet.loss(convnet.forward(bm, x)[0], tgt, row0)) / (2 * h)
        g = grads[layer][1][co]
        assert abs(fd - (g.real if part == 0 else g.imag)) <= 1e-6 * max(1.0, abs(g)) + 1e-9
