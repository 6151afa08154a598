"""Pins for the CNN oracle: its convolution against scipy's correlate, its
gradients against central finite differences of its own forward pass (an
independent check of every backward formula), and the pinball loss against
its definition at hand-picked points."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def rand_params(rng, cin=2, width=4, cout=2):
    shapes = [(width, 3, 3, cin), (width, 3, 3, width), (width, 3, 3, width), (cout, 3, 3, width)]
    return [(rng.normal(0, 0.5, s), rng.normal(0, 0.1, s[0])) for s in shapes]


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(7, 9, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(ndimage.correlate(x[:, :, c], w[o, :, :, c], mode="constant", cval=0.0)
                         for c in range(3))
        assert np.allclose(y[:, :, o], ref, rtol=1e-12, atol=1e-12)


def test_conv_identity_kernel_and_padding():
    x = np.arange(20, dtype=np.float64).reshape(4, 5, 1)
    w = np.zeros((1, 3, 3, 1))
    w[0, 1, 2, 0] = 1.0            # picks x[i, j + 1]
    y = cnn.conv3x3(x, w, np.zeros(1))
    assert np.array_equal(y[:, :-1, 0], x[:, 1:, 0])
    assert np.all(y[:, -1, 0] == 0)   # zero padding beyond the right edge


def test_pinball_definition():
    assert cnn.pinball(np.array(1.0), np.array(3.0), 0.25) == pytest.approx(0.5)
    assert cnn.pinball(np.array(3.0), np.array(1.0), 0.25) == pytest.approx(1.5)


@pytest.mark.parametrize("seed", [1, 2])
def test_network_gradients_by_finite_differences(seed):
    rng = np.random.default_rng(seed)
    params = rand_params(rng)
    x = rng.normal(size=(5, 6, 2))
    t_lo = rng.normal(size=(5, 6))
    t_hi = t_lo + 0.5

    def total_loss(ps):
        out, _ = cnn.forward(x, ps)
        return cnn.loss_and_grad(out, t_lo, t_hi)[0]

    out, cache = cnn.forward(x, params)
    _, dout = cnn.loss_and_grad(out, t_lo, t_hi)
    grads = cnn.backward(params, cache, dout)
    eps = 1e-6
    for li in range(4):
        for which in (0, 1):
            arr = params[li][which]
            idxs = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
            for idx in idxs:
                old = arr[idx]
                arr[idx] = old + eps
                lp = total_loss(params)
                arr[idx] = old - eps
                lm = total_loss(params)
                arr[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = grads[li][which][idx]
                assert abs(fd - an) <= 1e-5 + 1e-4 * abs(fd), (li, which, idx, fd, an)


def test_input_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4, 4, 3))
    w = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    dy = rng.normal(size=(4, 4, 2))
    dx, _, _ = cnn.conv3x3_backward(x, w, dy)
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 2, 1), (3, 3, 2), (2, 0, 1)]:
        xp = x.copy(); xp[idx] += eps
        xm = x.copy(); xm[idx] -= eps
        fd = ((cnn.conv3x3(xp, w, b) * dy).sum() - (cnn.conv3x3(xm, w, b) * dy).sum()) / (2 * eps)
        assert fd == pytest.approx(dx[idx], rel=1e-6, abs=1e-8)


def test_cell_features_and_targets():
    img = np.arange(16 * 24, dtype=np.uint16).reshape(16, 24)
    f = cnn.cell_features(img, 32, 65535.0)
    assert f.shape == (2, 3, 2)
    assert f[0, 0, 0] == pytest.approx(img[:8, :8].mean() / 65535.0)
    assert np.all(f[..., 1] == 0.5)
    lo, hi = cnn.cell_targets(img, 65535.0)
    assert lo[1, 2] == pytest.approx(img[8:16, 16:24].min() / 65535.0)
    assert hi[1, 2] == pytest.approx(img[8:16, 16:24].max() / 65535.0)


def test_bf16_round():
    assert cnn.bf16_round(np.array([1.0, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9])).tolist() == \
        [1.0, 1.0, 1.0 + 2 ** -7]


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g from zero moments, m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected moments are exactly g and
    g^2 and every step moves p by -lr * g / (|g| + eps), whatever b1 and b2
    are.  Tiny gradients (|g| ~ eps) separate eps outside the root from
    eps inside it."""
    g = np.array([1.0, -2.5, 3e-4, -1e-8, 2e-8, 0.0])
    lr, eps = 1e-3, 1e-8
    for b1, b2 in ((0.9, 0.999), (0.5, 0.75)):
        p = np.array([0.3, -1.0, 2.0, 5.0, -5.0, 7.0])
        m = np.zeros_like(g)
        v = np.zeros_like(g)
        p0 = p.copy()
        for t in range(1, 8):
            p, m, v = cnn.adam_step(p, m, v, g, lr, t, b1=b1, b2=b2, eps=eps)
            assert np.allclose(m, (1 - b1 ** t) * g, rtol=1e-12, atol=0)
            assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12, atol=0)
            exp = p0 - t * lr * g / (np.abs(g) + eps)
            assert np.allclose(p, exp, rtol=1e-12, atol=1e-17)
    # |g| = eps: the step is half of lr (eps added under the root would give about 1e-4 lr)
    p, _, _ = cnn.adam_step(np.zeros(1), np.zeros(1), np.zeros(1), np.array([1e-8]), 1.0, 1)
    assert p[0] == pytest.approx(-0.5, rel=1e-12)


def test_adam_two_gradients_weighted_average():
    """Two steps with gradients g1 then g2: the bias-corrected moments are the
    normalised weighted averages (b1 g1 + g2) / (1 + b1) and
    (b2 g1^2 + g2^2) / (1 + b2) (sum of a geometric series of weights)."""
    b1, b2, lr, eps = 0.9, 0.999, 0.1, 1e-8
    g1, g2 = np.array([1.0, -2.0, 0.5]), np.array([3.0, 1.0, -0.5])
    p, m, v = cnn.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g1, lr, 1)
    p1 = p.copy()
    p, m, v = cnn.adam_step(p, m, v, g2, lr, 2)
    mhat = (b1 * g1 + g2) / (1 + b1)
    vhat = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    assert np.allclose(p - p1, -lr * mhat / (np.sqrt(vhat) + eps), rtol=1e-12, atol=0)


def test_adam_zero_gradient_keeps_parameters():
    p = np.array([1.0, -2.0])
    out, m, v = cnn.adam_step(p, np.zeros(2), np.zeros(2), np.zeros(2), 0.5, 1)
    assert np.array_equal(out, p) and np.all(m == 0) and np.all(v == 0)
