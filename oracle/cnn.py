"""CPU (float64) oracle for the bracket-proposal CNN (test infrastructure only).

The learned proposal is not part of the paper: it is a small network that
predicts, for every 8x8 cell of an image, a value bracket [lo, hi] that should
contain the medians of the cell's pixels.  The exact filter then only ranks
the pixels whose values fall inside a tile's bracket and falls back to the
plain filter where the bracket misses.  This module is the plain definition
of that network and of its gradients, against which the GPU kernels are
checked:

* conv3x3(x, w, b): 'same' correlation with zero padding,
    y[i, j, o] = b[o] + sum_{dy, dx, c} w[o, dy + 1, dx + 1, c] x[i + dy, j + dx, c]
  with activations laid out (H, W, C) and weights (Cout, 3, 3, Cin).
* network: conv -> ReLU, three times, then a conv to two outputs (lo, hi).
* pinball (quantile) loss: rho_tau(u) = u (tau - [u < 0]), u = target - pred,
  averaged over cells; tau_lo = 0.02 for lo, tau_hi = 0.98 for hi.
* backward passes by the chain rule, written out per layer.
* Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015,
  Algorithm 1): exponential moving averages of the gradient and of its
  square, each divided by its bias correction 1 - beta^t, and the step
  -lr * mhat / (sqrt(vhat) + eps).
"""

from __future__ import annotations

import numpy as np

TAU_LO = 0.02
TAU_HI = 0.98
CELL = 8


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    H, W, C = x.shape
    O = w.shape[0]
    assert w.shape == (O, 3, 3, C)
    xp = np.zeros((H + 2, W + 2, C), dtype=np.float64)
    xp[1:-1, 1:-1] = x
    y = np.broadcast_to(b.astype(np.float64), (H, W, O)).copy()
    for ky in range(3):
        for kx in range(3):
            patch = xp[ky:ky + H, kx:kx + W, :]             # x[i + ky - 1, j + kx - 1, :]
            y += patch @ w[:, ky, kx, :].T.astype(np.float64)
    return y


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients of sum(dy * conv3x3(x, w, b)) with respect to x, w and b."""
    H, W, C = x.shape
    O = w.shape[0]
    xp = np.zeros((H + 2, W + 2, C), dtype=np.float64)
    xp[1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros((O, 3, 3, C), dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            patch = xp[ky:ky + H, kx:kx + W, :]
            dw[:, ky, kx, :] = np.einsum("ijo,ijc->oc", dy, patch)
            dxp[ky:ky + H, kx:kx + W, :] += dy @ w[:, ky, kx, :].astype(np.float64)
    db = dy.sum(axis=(0, 1))
    return dxp[1:-1, 1:-1], dw, db


def relu(x):
    return np.maximum(x, 0.0)


def forward(x, params):
    """params: list of 4 (w, b).  Returns (output, cache of layer inputs/pre-activations)."""
    cache = []
    h = x
    for li, (w, b) in enumerate(params):
        pre = conv3x3(h, w, b)
        cache.append((h, pre))
        h = relu(pre) if li < len(params) - 1 else pre
    return h, cache


def pinball(pred, target, tau):
    u = target - pred
    return u * (tau - (u < 0))


def loss_and_grad(out, t_lo, t_hi):
    """Mean pinball loss over cells for out[..., 0] = lo, out[..., 1] = hi."""
    n = t_lo.size
    L = (pinball(out[..., 0], t_lo, TAU_LO).sum() + pinball(out[..., 1], t_hi, TAU_HI).sum()) / n
    g = np.zeros_like(out, dtype=np.float64)
    u0 = t_lo - out[..., 0]
    u1 = t_hi - out[..., 1]
    g[..., 0] = -(TAU_LO - (u0 < 0)) / n
    g[..., 1] = -(TAU_HI - (u1 < 0)) / n
    return L, g


def backward(params, cache, dout):
    grads = [None] * len(params)
    d = dout
    for li in range(len(params) - 1, -1, -1):
        h_in, pre = cache[li]
        if li < len(params) - 1:
            d = d * (pre > 0)
        dx, dw, db = conv3x3_backward(h_in, params[li][0], d)
        grads[li] = (dw, db)
        d = dx
    return grads


def adam_step(p, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step number `step` (1-based) in float64; returns the
    new (p, m, v).  m and v start at zero before step 1."""
    p, m, v, g = (np.asarray(a, dtype=np.float64) for a in (p, m, v, g))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def cell_features(img: np.ndarray, radius: int, maxval: float) -> np.ndarray:
    """Network input per 8x8 cell: mean of the cell's values / maxval, and the
    radius plane radius / 64.  Cells beyond the image edge average what they
    cover."""
    H, W = img.shape
    h, w = -(-H // CELL), -(-W // CELL)
    f = np.zeros((h, w, 2), dtype=np.float64)
    for i in range(h):
        for j in range(w):
            f[i, j, 0] = img[i * CELL:(i + 1) * CELL, j * CELL:(j + 1) * CELL].astype(np.float64).mean() / maxval
    f[..., 1] = radius / 64.0
    return f


def cell_targets(median: np.ndarray, maxval: float):
    """Per cell: (min, max) of the exact median image over the cell, / maxval."""
    H, W = median.shape
    h, w = -(-H // CELL), -(-W // CELL)
    lo = np.zeros((h, w))
    hi = np.zeros((h, w))
    for i in range(h):
        for j in range(w):
            blk = median[i * CELL:(i + 1) * CELL, j * CELL:(j + 1) * CELL].astype(np.float64)
            lo[i, j] = blk.min() / maxval
            hi[i, j] = blk.max() / maxval
    return lo, hi


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
