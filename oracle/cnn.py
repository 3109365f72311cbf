"""FP64 CPU reference of the convolutional surrogate of the basis functions.

Test infrastructure only (imported by tests/ and nothing else).

The network is not part of the paper's method: it is a learned
approximation of the local basis functions of section 3 (the solutions of
the local Robin problems of eq. (mrc1) for each interface function), whose
output the solver checks with the residual of those local problems before
using it.  This module defines what the network computes, in float64 and
with plain numpy loops over the nine taps of each 3x3 convolution:

* input  x : [B, 256, 8] on the 16 x 16 cells of a subdomain, channels last
  (cell l = 16*row + column); channel 0 is (ln kappa - mean ln kappa) / 4,
  channels 1..4 mark the cells next to the W, E, S, N sides that lie on the
  skeleton, channels 5..7 are zero;
* layers : 3x3 convolutions with zero padding, 8 -> 32 -> 32 -> 32 -> 16
  channels, ReLU after the first three, none after the last;
* output : [B, 256, 16], one channel per interface basis function;
* loss   : mean over all B*256*16 outputs of the squared difference to the
  targets.

Parameter vector (float32 in the library, read here as float64): for each
layer, the weights W[co, tap, ci] with tap = 3*(dy+1) + (dx+1) for the
neighbour at row offset dy and column offset dx, stored [Cout][taps][Cin],
the K extent (taps x Cin) rounded up to a multiple of 16 (layer 1: 10 taps
of 8 channels), then the Cout biases.

parity pinned by: scipy's 2-D correlation for the forward pass, central
finite differences of the loss for the backward pass (tests/test_oracle_cnn.py).
"""
from __future__ import annotations

import numpy as np

H = W_ = 16
CHANNELS = [(8, 32, True), (32, 32, True), (32, 32, True), (32, 16, False)]


def _kpad(cin):
    return -(-9 * cin // 16) * 16


def layout():
    """[(w_offset, cout, kpad, cin, b_offset, relu)] per layer, and the total."""
    out, o = [], 0
    for cin, cout, relu in CHANNELS:
        kp = _kpad(cin)
        out.append((o, cout, kp, cin, o + cout * kp, relu))
        o += cout * kp + cout
    return out, o


def n_params():
    return layout()[1]


def unpack(params):
    """Per layer (W [Cout, 9, Cin] float64, b [Cout] float64, relu)."""
    p = np.asarray(params, dtype=np.float64)
    lay, n = layout()
    assert p.size == n
    out = []
    for wo, cout, kp, cin, bo, relu in lay:
        Wfull = p[wo:wo + cout * kp].reshape(cout, kp)
        Wt = Wfull[:, :9 * cin].reshape(cout, 9, cin)
        out.append((Wt, p[bo:bo + cout], relu))
    return out


def _shift(x, dy, dx):
    """y[b, r, c, :] = x[b, r + dy, c + dx, :], zero outside the 16 x 16 patch."""
    y = np.zeros_like(x)
    r0, r1 = max(0, -dy), min(H, H - dy)
    c0, c1 = max(0, -dx), min(W_, W_ - dx)
    y[:, r0:r1, c0:c1, :] = x[:, r0 + dy:r1 + dy, c0 + dx:c1 + dx, :]
    return y


def _conv(x, Wt, b):
    """out[b, r, c, co] = b[co] + sum_{tap, ci} Wt[co, tap, ci] x[b, r+dy, c+dx, ci]."""
    B = x.shape[0]
    out = np.broadcast_to(b, (B, H, W_, Wt.shape[0])).copy()
    for tap in range(9):
        dy, dx = tap // 3 - 1, tap % 3 - 1
        out += _shift(x, dy, dx) @ Wt[:, tap, :].T
    return out


def forward(params, x, keep=False):
    """Network output [B, 256, 16] for inputs x [B, 256, 8]; with keep=True
    also the list of layer inputs and pre-activations (for backward)."""
    a = np.asarray(x, dtype=np.float64).reshape(-1, H, W_, 8)
    acts, pres = [], []
    for Wt, b, relu in unpack(params):
        acts.append(a)
        z = _conv(a, Wt, b)
        pres.append(z)
        a = np.maximum(z, 0.0) if relu else z
    y = a.reshape(a.shape[0], H * W_, -1)
    return (y, acts, pres) if keep else y


def loss(params, x, target):
    y = forward(params, x)
    d = y - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d))


def loss_grad(params, x, target):
    """(loss, gradient of the loss with respect to the parameter vector)."""
    y, acts, pres = forward(params, x, keep=True)
    t = np.asarray(target, dtype=np.float64).reshape(y.shape)
    d = y - t
    L = float(np.mean(d * d))
    g = (2.0 / d.size) * d.reshape(pres[-1].shape)       # dL/d(output)
    lay, n = layout()
    grad = np.zeros(n)
    layers = unpack(params)
    for li in range(len(layers) - 1, -1, -1):
        Wt, b, relu = layers[li]
        wo, cout, kp, cin, bo, _ = lay[li]
        if relu:
            g = g * (pres[li] > 0.0)                        # through the ReLU
        a = acts[li]
        gW = np.zeros((cout, kp))
        for tap in range(9):
            dy, dx = tap // 3 - 1, tap % 3 - 1
            xs = _shift(a, dy, dx)
            gW[:, tap * cin:(tap + 1) * cin] = np.einsum("brco,brci->oi", g, xs)
        grad[wo:wo + cout * kp] = gW.ravel()
        grad[bo:bo + cout] = g.sum(axis=(0, 1, 2))
        if li > 0:
            # input gradient: the transpose of the correlation
            ga = np.zeros_like(a)
            for tap in range(9):
                dy, dx = tap // 3 - 1, tap % 3 - 1
                ga += _shift(g @ Wt[:, tap, :], -dy, -dx)
            g = ga
    return L, grad


def he_params(seed):
    """Random parameters of the documented layout (He-normal weights on the
    real channels, small random biases), for tests."""
    rng = np.random.default_rng(seed)
    lay, n = layout()
    p = np.zeros(n)
    real_cin = [5, 32, 32, 32]
    for (wo, cout, kp, cin, bo, _), rc in zip(lay, real_cin):
        Wt = np.zeros((cout, 9, cin))
        Wt[:, :, :rc] = rng.normal(0.0, np.sqrt(2.0 / (9 * rc)), size=(cout, 9, rc))
        Wfull = np.zeros((cout, kp))
        Wfull[:, :9 * cin] = Wt.reshape(cout, 9 * cin)
        p[wo:wo + cout * kp] = Wfull.ravel()
        p[bo:bo + cout] = rng.normal(0.0, 0.1, size=cout)
    return p
