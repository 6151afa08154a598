"""Per-element error bounds between the bracket CNN's GPU chain and the
float64 oracle (a test helper, not a test module).

The GPU keeps weights, cell features, hidden activations and backward
gradients as bfloat16 and accumulates in float32.  The expected values are
the oracle's float64 chain (`oracle.cnn`) rounded to bfloat16 at the same
points.  The bound on each element follows that arithmetic:

* float32 sums: a product of two bf16 values is exact in float32.  A sum of
  K terms (a bias included) accumulated in float32 is within gamma(K) *
  sum|terms| of the exact sum.  The worst case over all orders is K * u
  (u = 2^-24); with rounding errors taken as independent and of mean zero
  it is lambda * sqrt(K) * u except with probability below
  2 K exp(-lambda^2 / 2) (Higham and Mary, "A New Approach to Probabilistic
  Rounding Error Analysis", SIAM J. Sci. Comput. 2019, Theorem 2.4).
  lambda = 8 here: below 1e-11 per sum of up to a few thousand terms.
* bf16 stores: rounding (to float32, then to bf16 nearest-even) is monotone.
  If the GPU's float32 value lies within e of the exact value x, its stored
  bf16 value lies between round(x - e) and round(x + e), so its distance to
  the oracle's round(x) is at most the larger distance to those two.  Away
  from a rounding midpoint both ends round to round(x): the stored values
  are then identical and the bound is 0, so an error confined to a few cells
  or channels (a wrong mask, a wrong tap) exceeds it.
* the pinball gradient depends on the sign of target - output only; where
  the output's bound does not decide the sign, either value is allowed.
* a ReLU mask taken from a stored activation is uncertain only where the
  activation's own interval holds both 0 and a positive value.
"""

from __future__ import annotations

import numpy as np

from oracle import cnn as OC

U = 2.0 ** -24
EPS64 = 1e-15      # slack for the oracle's own float64 rounding, relative to magnitudes


def gamma(k: int) -> float:
    return 8.0 * np.sqrt(k) * U


def bf16_interval(x, e, relu=False):
    """(round(x), bound on |round(y) - round(x)| for |y - x| <= e)."""
    f = (lambda a: OC.bf16_round(np.maximum(a, 0.0))) if relu else OC.bf16_round
    c = f(x)
    return c, np.maximum(np.abs(f(x + e) - c), np.abs(f(x - e) - c))


def pad32(a):
    out = np.zeros(a.shape[:2] + (32,))
    out[..., :a.shape[2]] = a
    return out


def forward(img, radius, maxval, Ws, bs):
    """Oracle forward chain with bounds.  Ws[l]: bf16-valued weights
    (cout, 3, 3, 32); bs[l]: float32-valued biases.  Returns a dict with the
    layer inputs h[l] (bf16 values) and bounds eh[l], the pre-activations
    pre[l] with bounds epre[l]; pre[3] is the output."""
    f = OC.cell_features(img, radius, maxval)
    # GPU: exact integer sum, one division by the pixel count, one product
    # by float32(1 / maxval): within 3u relative (4u taken); radius / 64 is exact
    ef = 4 * U * np.abs(f)
    ef[..., 1] = 0.0
    h, eh = bf16_interval(f, ef)
    h, eh = pad32(h), pad32(eh)
    H, EH, PRE, EPRE = [], [], [], []
    for l in range(4):
        W, b = Ws[l], bs[l]
        pre = OC.conv3x3(h, W, b)
        mag = OC.conv3x3(np.abs(h) + eh, np.abs(W), np.abs(b))
        e = OC.conv3x3(eh, np.abs(W), np.zeros_like(b)) + (gamma(9 * 32 + 1) + EPS64) * mag
        H.append(h)
        EH.append(eh)
        PRE.append(pre)
        EPRE.append(e)
        if l < 3:
            h, eh = bf16_interval(pre, e, relu=True)
    return {"h": H, "eh": EH, "pre": PRE, "epre": EPRE}


def pinball_grad(out, eout, median, maxval):
    """Gradient of the summed pinball loss with respect to (lo, hi) as the
    GPU stores it (bf16, 16 channels, 2..15 zero), with bounds."""
    t_lo, t_hi = OC.cell_targets(median, maxval)
    n = t_lo.size
    _, g = OC.loss_and_grad(out[..., :2], t_lo, t_hi)
    d = np.zeros(out.shape[:2] + (16,))
    ed = np.zeros_like(d)
    d[..., :2] = OC.bf16_round(g * n)
    for c, (t, tau) in enumerate(((t_lo, OC.TAU_LO), (t_hi, OC.TAU_HI))):
        # targets on the GPU: float32(v) * float32(1 / maxval), within 2u relative
        et = 3 * U * np.abs(t)
        unsure = np.abs(t - out[..., c]) <= eout[..., c] + et
        below = (t - out[..., c]) < 0
        alt = OC.bf16_round(-(tau - (~below).astype(np.float64)))   # the other sign's value
        ed[..., c] = np.where(unsure, np.abs(alt - d[..., c]), 0.0)
    return d, ed


def backward(fw, Ws, d, ed):
    """Weight and bias gradients of every layer with bounds, backward from
    the output gradient d (bound ed).  Returns lists dw, edw, db, edb indexed
    by layer."""
    ncell = d.shape[0] * d.shape[1]
    DW, EDW, DB, EDB = [None] * 4, [None] * 4, [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        W = Ws[l]
        cout = W.shape[0]
        h, eh = fw["h"][l], fw["eh"][l]
        zw = np.zeros_like(W)
        _, dw, db = OC.conv3x3_backward(h, zw, d)
        _, mdw, mdb = OC.conv3x3_backward(np.abs(h) + eh, zw, np.abs(d) + ed)
        _, t1, _ = OC.conv3x3_backward(np.abs(h), zw, ed)
        _, t2, _ = OC.conv3x3_backward(eh, zw, np.abs(d) + ed)
        # split-K partials over cell blocks, then a sum of the partials
        g = gamma(2 * ncell) + EPS64
        DW[l], EDW[l] = dw, t1 + t2 + g * mdw
        DB[l], EDB[l] = db, ed.sum(axis=(0, 1)) + g * mdb
        if l == 0:
            break
        zx = np.zeros_like(h)
        dx, _, _ = OC.conv3x3_backward(zx, W, d)
        mdx, _, _ = OC.conv3x3_backward(zx, np.abs(W), np.abs(d) + ed)
        edx0, _, _ = OC.conv3x3_backward(zx, np.abs(W), ed)
        edx = edx0 + (gamma(9 * cout) + EPS64) * mdx
        # mask: the stored activation h[l] = bf16(relu(pre[l-1])) > 0
        pre, epre = fw["pre"][l - 1], fw["epre"][l - 1]
        a_lo = OC.bf16_round(np.maximum(pre - epre, 0.0))
        a_hi = OC.bf16_round(np.maximum(pre + epre, 0.0))
        on, off = a_lo > 0, a_hi <= 0
        mask = h > 0
        dm, _ = bf16_interval(dx, edx)
        nd = dm * mask
        c_lo, c_hi = OC.bf16_round(dx - edx), OC.bf16_round(dx + edx)
        e_val = np.maximum(np.abs(c_lo - nd), np.abs(c_hi - nd))   # GPU value if its mask is on
        e_unsure = np.maximum(e_val, np.abs(nd))                    # ... or 0 if it is off
        d = nd
        ed = np.where(on, e_val, np.where(off, 0.0, e_unsure))
    return DW, EDW, DB, EDB


def chain_case(img, radius, seed, flip=0.2):
    """A network and a training target for the end-to-end gradient check.

    Weights are non-negative (so forward sums do not cancel, which keeps the
    bounds tight) and each hidden channel's bias is minus a quantile (30-70 %)
    of its pre-bias sums over the image, so every layer's ReLU masks are
    partly on and partly off.  The output layer puts lo in [0.1, 0.4] and
    hi in [0.55, 0.85].  The target median image puts each cell's min and max
    0.05 above the oracle's (lo, hi) output, or below it in a fraction
    `flip` of the cells, so both branches of the pinball gradient occur and
    no output is near its target.  Returns (Ws, bs, median)."""
    rng = np.random.default_rng(seed)
    f = OC.cell_features(img, radius, 65535.0)
    h = pad32(OC.bf16_round(f))
    Ws, bs = [], []
    for l in range(4):
        cout = 32 if l < 3 else 16
        cin = 2 if l == 0 else 32
        w = np.zeros((cout, 3, 3, 32))
        w[:, :, :, :cin] = np.abs(rng.normal(0, np.sqrt(2.0 / (9 * cin)), (cout, 3, 3, cin)))
        if l == 3:
            w[2:] = 0
        s = OC.conv3x3(h, OC.bf16_round(w), np.zeros(cout))
        b = np.zeros(cout)
        if l < 3:
            q = rng.uniform(0.3, 0.7, cout)
            b = -np.array([np.quantile(s[..., o], q[o]) for o in range(cout)])
        else:
            w[:2] *= 0.3 / np.max(s[..., :2], axis=(0, 1))[:, None, None, None]
            b[:2] = (0.1, 0.55)
        w = OC.bf16_round(w)
        b = b.astype(np.float32).astype(np.float64)
        Ws.append(w)
        bs.append(b)
        pre = OC.conv3x3(h, w, b)
        h = OC.bf16_round(np.maximum(pre, 0)) if l < 3 else pre
    out = h[..., :2]
    sgn = lambda: np.where(rng.random(out.shape[:2]) < flip, -1.0, 1.0)
    t_lo = out[..., 0] + 0.05 * sgn()
    t_hi = out[..., 1] + 0.05 * sgn()
    assert t_lo.min() > 0 and t_hi.max() < 1 and np.all(t_lo < t_hi), "targets out of range"
    med = np.zeros(img.shape, dtype=np.uint16)
    for i in range(out.shape[0]):
        for j in range(out.shape[1]):
            lo = int(round(t_lo[i, j] * 65535))
            hi = int(round(t_hi[i, j] * 65535))
            blk = med[8 * i:8 * i + 8, 8 * j:8 * j + 8]
            blk[...] = (lo + hi) // 2
            blk[0, 0] = lo
            blk[-1, -1] = hi
    return Ws, bs, med


def magnitudes(fw, Ws, d):
    """The same backward pass on absolute values: per-layer weight-gradient
    magnitudes (what one cell's term is measured against)."""
    out = [None] * 4
    dcur = np.abs(d)
    for l in range(3, -1, -1):
        _, mdw, _ = OC.conv3x3_backward(np.abs(fw["h"][l]), np.zeros_like(Ws[l]), dcur)
        out[l] = mdw
        if l > 0:
            dx, _, _ = OC.conv3x3_backward(np.zeros_like(fw["h"][l]), np.abs(Ws[l]), dcur)
            dcur = dx * (fw["h"][l] > 0)
    return out
