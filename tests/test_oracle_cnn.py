"""Pins of the FP64 reference network (oracle/cnn.py): the forward pass
against scipy's 2-D correlation, the backward pass against central finite
differences of the loss, and planted mistakes that those pins must catch."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((B, 256, 8))
    x[:, :, :5] = rng.normal(size=(B, 256, 5))
    t = rng.normal(size=(B, 256, 16))
    return x, t


def _scipy_forward(params, x):
    """Each layer as sums of scipy 2-D correlations (zero padding, 'same')."""
    a = x.reshape(-1, 16, 16, 8)
    for Wt, b, relu in cnn.unpack(params):
        B, cin, cout = a.shape[0], Wt.shape[2], Wt.shape[0]
        z = np.zeros((B, 16, 16, cout))
        for n in range(B):
            for co in range(cout):
                acc = np.full((16, 16), b[co])
                for ci in range(cin):
                    acc += correlate2d(a[n, :, :, ci], Wt[co, :, ci].reshape(3, 3), mode="same")
                z[n, :, :, co] = acc
        a = np.maximum(z, 0.0) if relu else z
    return a.reshape(a.shape[0], 256, -1)


def test_layout_matches_documented_sizes():
    lay, n = cnn.layout()
    assert [l[2] for l in lay] == [80, 288, 288, 288]
    assert n == 32 * 80 + 32 + 2 * (32 * 288 + 32) + 16 * 288 + 16


def test_forward_matches_scipy_correlation():
    p = cnn.he_params(1)
    x, _ = _inputs(2, 2)
    np.testing.assert_allclose(cnn.forward(p, x), _scipy_forward(p, x), rtol=1e-12, atol=1e-12)


def test_single_tap_is_a_shift():
    """A network whose only non-zero weight is one tap of identity channels
    shifts the input: a closed form independent of the loop structure."""
    lay, n = cnn.layout()
    p = np.zeros(n)
    for li, (wo, cout, kp, cin, bo, relu) in enumerate(lay):
        W = np.zeros((cout, kp))
        for c in range(min(cin, cout)):
            tap = 5 if li == 0 else 4        # layer 1: neighbour (dy, dx) = (0, +1)
            W[c, tap * cin + c] = 1.0
        p[wo:wo + cout * kp] = W.ravel()
    x = np.zeros((1, 256, 8))
    x[0, :, 0] = np.abs(np.random.default_rng(3).normal(size=256))
    y = cnn.forward(p, x)[0, :, 0].reshape(16, 16)
    img = x[0, :, 0].reshape(16, 16)
    expect = np.zeros((16, 16))
    expect[:, :-1] = img[:, 1:]
    np.testing.assert_array_equal(y, expect)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    p = cnn.he_params(10 + seed)
    x, t = _inputs(2, 20 + seed)
    L, g = cnn.loss_grad(p, x, t)
    assert L == pytest.approx(cnn.loss(p, x, t), rel=1e-14)
    lay, n = cnn.layout()
    rng = np.random.default_rng(seed)
    idx = []
    for wo, cout, kp, cin, bo, _ in lay:
        real = [wo + co * kp + k for co in range(cout) for k in range(9 * cin)]
        idx += list(rng.choice(real, 12, replace=False)) + list(bo + rng.choice(cout, 3, replace=False))
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cnn.loss(pp, x, t) - cnn.loss(pm, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_padding_entries_get_zero_gradient():
    p = cnn.he_params(5)
    x, t = _inputs(1, 6)
    _, g = cnn.loss_grad(p, x, t)
    wo, cout, kp, cin, bo, _ = cnn.layout()[0][0]
    W = g[wo:wo + cout * kp].reshape(cout, kp)
    assert np.all(W[:, 72:] == 0.0)                          # tap 10 of layer 1
    assert np.all(W[:, :72].reshape(cout, 9, 8)[:, :, 5:] == 0.0)   # zero input channels


def test_planted_mistakes_fail_the_pins(monkeypatch):
    p = cnn.he_params(7)
    x, t = _inputs(1, 8)
    ref = _scipy_forward(p, x)
    # transposed taps (row and column offsets swapped)
    orig = cnn._shift
    monkeypatch.setattr(cnn, "_shift", lambda a, dy, dx: orig(a, dx, dy))
    assert not np.allclose(cnn.forward(p, x), ref, rtol=1e-6)
    monkeypatch.setattr(cnn, "_shift", orig)
    # backward without the ReLU mask: forward() hands the backward
    # pre-activations that all look positive
    L, g = cnn.loss_grad(p, x, t)
    forward_orig = cnn.forward

    def unmasked(params, xx, keep=False):
        y, acts, pres = forward_orig(params, xx, keep=True)
        return y, acts, [np.abs(z) + 1.0 for z in pres]

    monkeypatch.setattr(cnn, "forward", unmasked)
    _, g_bad = cnn.loss_grad(p, x, t)
    monkeypatch.setattr(cnn, "forward", forward_orig)
    i = cnn.layout()[0][0][0] + 4 * 8     # a centre-tap weight of layer 1
    h = 1e-6
    pp, pm = p.copy(), p.copy()
    pp[i] += h
    pm[i] -= h
    fd = (cnn.loss(pp, x, t) - cnn.loss(pm, x, t)) / (2 * h)
    assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 1e-12
    assert abs(fd - g_bad[i]) > 1e-3 * abs(fd)
