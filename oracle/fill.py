"""FP64 CPU reference of the learned stale fill (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU leg of ``bench.py``
may import this module; the product library never loads it and shares no code
with it.

The fill is a small convolutional network that predicts the brightness of
stale pixels from the readout of the reconstruction.  It is not part of the
paper's method: it reads a readout and never writes into the reconstruction
state.  Definitions followed here:

* Input per pixel, channels in this order: brightness L, stale mask (1 for a
  stale pixel, else 0), log(1 + age) with age = newest index - last index.
* Four 3x3 layers with zero padding, channels 3 -> 16 -> 16 -> 16 -> 1, ReLU
  after each of the first three.  Cross-correlation (no kernel flip):
  y[o, i, j] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] x[c, i + dy - 1, j + dx - 1]
  with x = 0 outside the image.
* Prediction = L + the last layer's output: the network learns a correction
  of the brightness the reconstruction shows (its Gaussian fill at stale
  pixels), so zero last-layer parameters give back L exactly.
* Loss: the mean of (prediction - target)^2 over the stale pixels of the batch.
* Optimiser: Adam (Kingma and Ba, 2015, Algorithm 1) with bias correction.

Parameters travel as one flat float vector, layer by layer: w_l in
[Cout][Cin][3][3] order, then b_l.  Everything here is FP64; the network runs
on arrays of shape [N, C, H, W].
"""
from __future__ import annotations

import numpy as np

CHANNELS = (3, 16, 16, 16, 1)
N_LAYERS = len(CHANNELS) - 1


def layer_shapes():
    """[(w shape, b shape)] per layer."""
    return [((CHANNELS[l + 1], CHANNELS[l], 3, 3), (CHANNELS[l + 1],)) for l in range(N_LAYERS)]


N_PARAMS = sum(int(np.prod(ws)) + int(np.prod(bs)) for ws, bs in layer_shapes())


def unflatten(flat):
    """Flat parameter vector -> [(w, b)] (FP64 copies)."""
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.shape == (N_PARAMS,)
    out, k = [], 0
    for ws, bs in layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((flat[k:k + nw].reshape(ws).copy(), flat[k + nw:k + nw + nb].copy()))
        k += nw + nb
    return out


def flatten(params):
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def conv3x3(x, w, b):
    """Zero-padded 3x3 cross-correlation, x [N, Cin, H, W] -> [N, Cout, H, W]:
    one matrix product over channels per tap, summed over the 9 taps."""
    n, cin, h, wd = x.shape
    xp = np.zeros((n, cin, h + 2, wd + 2))
    xp[:, :, 1:h + 1, 1:wd + 1] = x
    y = np.broadcast_to(b.reshape(1, -1, 1, 1), (n, w.shape[0], h, wd)).copy()
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("nchw,oc->nohw", xp[:, :, dy:dy + h, dx:dx + wd], w[:, :, dy, dx])
    return y


def conv3x3_backward(x, w, gy):
    """Gradients of sum(gy * conv3x3(x, w, b)) with respect to x, w and b."""
    n, cin, h, wd = x.shape
    xp = np.zeros((n, cin, h + 2, wd + 2))
    xp[:, :, 1:h + 1, 1:wd + 1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("nohw,nchw->oc", gy, xp[:, :, dy:dy + h, dx:dx + wd])
            gxp[:, :, dy:dy + h, dx:dx + wd] += np.einsum("nohw,oc->nchw", gy, w[:, :, dy, dx])
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:h + 1, 1:wd + 1], gw, gb


def forward(params, x):
    """Prediction [N, H, W] (input channel 0 plus the network's output) and
    the per-layer inputs / pre-activations."""
    cache = []
    a = x
    for l, (w, b) in enumerate(params):
        z = conv3x3(a, w, b)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if l < N_LAYERS - 1 else z
    return x[:, 0] + a[:, 0], cache


def backward(params, cache, gpred):
    """Gradients of the loss with respect to every layer's (w, b), given
    gpred = dloss/dprediction [N, H, W]."""
    grads = [None] * N_LAYERS
    g = gpred[:, None]
    for l in range(N_LAYERS - 1, -1, -1):
        a_in, z = cache[l]
        if l < N_LAYERS - 1:
            g = g * (z > 0)                      # through the ReLU of layer l
        gx, gw, gb = conv3x3_backward(a_in, params[l][0], g)
        grads[l] = (gw, gb)
        g = gx
    return grads


def masked_mse(pred, target, mask):
    """Mean of (pred - target)^2 over mask != 0, and its gradient in pred."""
    m = (mask != 0).astype(np.float64)
    cnt = m.sum()
    if cnt == 0:
        return 0.0, np.zeros_like(pred, dtype=np.float64)
    d = (pred - target) * m
    return float((d * d).sum() / cnt), 2.0 * d / cnt


def loss_and_grad(flat, x, target, mask):
    params = unflatten(flat)
    pred, cache = forward(params, x)
    loss, gpred = masked_mse(pred, target, mask)
    return loss, flatten(backward(params, cache, gpred))


def make_input(L, stale, log_age):
    """Network input [N, 3, H, W] from readout planes [N, H, W]."""
    return np.stack([np.asarray(L, np.float64), (np.asarray(stale) != 0).astype(np.float64),
                     np.asarray(log_age, np.float64)], axis=1)


class Adam:
    """Adam with bias correction; state per parameter."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
