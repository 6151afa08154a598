"""GPU parity of the bracket-CNN kernels against the float64 CPU oracle.

Inputs are rounded to bfloat16 on the host and the oracle sees the same
rounded values, so the only differences are the float32 accumulation order
on MFMA (and bf16 rounding of bf16 outputs).  Tolerances below follow from
that: a sum of K products of bf16 values in f32 has relative error about
K * 2^-24 of the sum of magnitudes; a bf16 output adds 2^-9 relative.
"""

import numpy as np
import pytest

from oracle import cnn as OC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    import paper_2505_22938_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    m.lib()
    return m


def to_bf16_dev(a):
    """float64 array -> (device bf16 tensor, the bf16-rounded float64 values)."""
    r = OC.bf16_round(a)
    t = torch.from_numpy(np.ascontiguousarray(r.astype(np.float32))).to(torch.bfloat16).cuda()
    return t, r


def from_bf16(t):
    return t.float().cpu().numpy().astype(np.float64)


def close(got, exp, scale, rel):
    err = np.abs(got - exp)
    assert np.all(err <= rel * scale + 1e-30), (float(err.max()), float(scale.max()))


def test_mfma_operand_layout(mf):
    rng = np.random.default_rng(0)
    A, Ar = to_bf16_dev(rng.normal(size=(16, 32)))
    B, Br = to_bf16_dev(rng.normal(size=(32, 16)))
    D = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    mf.cnn.mfma_probe(A, B, D)
    torch.cuda.synchronize()
    exp = Ar @ Br
    mag = np.abs(Ar) @ np.abs(Br)
    close(D.cpu().numpy().astype(np.float64), exp, mag, 32 * 2.0 ** -23)


def make_layer(rng, cout, cin_real=32):
    w = rng.normal(0, 0.2, size=(cout, 3, 3, 32))
    w[:, :, :, cin_real:] = 0
    b = rng.normal(0, 0.1, size=cout)
    return w, b


@pytest.mark.parametrize("H,W", [(5, 37), (16, 64), (1, 16), (3, 3)])
def test_conv_forward_modes(mf, H, W):
    rng = np.random.default_rng(H * 100 + W)
    x, xr = to_bf16_dev(rng.normal(size=(H, W, 32)))
    w, b = make_layer(rng, 32)
    wd, wr = to_bf16_dev(w)
    bd = torch.from_numpy(b.astype(np.float32)).cuda()
    exp = OC.conv3x3(xr, wr, b.astype(np.float32).astype(np.float64))
    mag = OC.conv3x3(np.abs(xr), np.abs(wr), np.abs(b))
    y1 = torch.empty((H, W, 32), dtype=torch.float32, device="cuda")
    mf.cnn.conv_forward(x, H, W, wd, bd, 32, 1, y1)
    y0 = torch.empty((H, W, 32), dtype=torch.bfloat16, device="cuda")
    mf.cnn.conv_forward(x, H, W, wd, bd, 32, 0, y0)
    torch.cuda.synchronize()
    close(y1.cpu().numpy().astype(np.float64), exp, mag, 300 * 2.0 ** -24)
    close(from_bf16(y0), np.maximum(exp, 0), mag, 2.0 ** -8)
    # output layer: 16 channels, f32
    w4, b4 = make_layer(rng, 16)
    w4d, w4r = to_bf16_dev(w4)
    b4d = torch.from_numpy(b4.astype(np.float32)).cuda()
    y4 = torch.empty((H, W, 16), dtype=torch.float32, device="cuda")
    mf.cnn.conv_forward(x, H, W, w4d, b4d, 16, 1, y4)
    torch.cuda.synchronize()
    exp4 = OC.conv3x3(xr, w4r, b4.astype(np.float32).astype(np.float64))
    mag4 = OC.conv3x3(np.abs(xr), np.abs(w4r), np.abs(b4))
    close(y4.cpu().numpy().astype(np.float64), exp4, mag4, 300 * 2.0 ** -24)


@pytest.mark.parametrize("cout", [32, 16])
def test_conv_backward_data(mf, cout):
    rng = np.random.default_rng(7 + cout)
    H, W = 6, 40
    w, _ = make_layer(rng, cout)
    wd, wr = to_bf16_dev(w)
    dy = np.zeros((H, W, 32))
    dy[:, :, :cout] = rng.normal(size=(H, W, cout))
    dyd, dyr = to_bf16_dev(dy)
    act = rng.normal(size=(H, W, 32))            # previous layer output (mask > 0)
    actd, actr = to_bf16_dev(np.maximum(act, 0))
    wf = torch.empty((32, 9, 32), dtype=torch.bfloat16, device="cuda")
    mf.cnn.flip_weights(wd, cout, wf)
    dx = torch.empty((H, W, 32), dtype=torch.float32, device="cuda")
    mf.cnn.conv_forward(dyd, H, W, wf, None, 32, 1, dx)
    dxm = torch.empty((H, W, 32), dtype=torch.bfloat16, device="cuda")
    mf.cnn.conv_forward(dyd, H, W, wf, None, 32, 2, dxm, mask=actd)
    torch.cuda.synchronize()
    exp, _, _ = OC.conv3x3_backward(np.zeros((H, W, 32)), wr, dyr[:, :, :cout])
    mag, _, _ = OC.conv3x3_backward(np.zeros((H, W, 32)), np.abs(wr), np.abs(dyr[:, :, :cout]))
    close(dx.cpu().numpy().astype(np.float64), exp, mag, 300 * 2.0 ** -24)
    close(from_bf16(dxm), exp * (actr > 0), mag, 2.0 ** -8)


@pytest.mark.parametrize("cout", [32, 16])
@pytest.mark.parametrize("H,W,spb", [(7, 70, 3), (16, 64, 8), (2, 20, 1)])
def test_conv_weight_gradient(mf, cout, H, W, spb):
    rng = np.random.default_rng(H + W + cout)
    x, xr = to_bf16_dev(rng.normal(size=(H, W, 32)))
    dy = np.zeros((H, W, 32))
    dy[:, :, :cout] = rng.normal(size=(H, W, cout))
    dyd, dyr = to_bf16_dev(dy)
    ws = torch.empty(mf.cnn.wgrad_workspace(H, W, cout, spb), dtype=torch.float32, device="cuda")
    dw = torch.empty((cout, 9, 32), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    mf.cnn.conv_wgrad(x, dyd, H, W, cout, ws, dw, db, segs_per_block=spb)
    torch.cuda.synchronize()
    _, edw, edb = OC.conv3x3_backward(xr, np.zeros((cout, 3, 3, 32)), dyr[:, :, :cout])
    _, mdw, mdb = OC.conv3x3_backward(np.abs(xr), np.zeros((cout, 3, 3, 32)),
                                      np.abs(dyr[:, :, :cout]))
    close(dw.cpu().numpy().reshape(cout, 3, 3, 32).astype(np.float64), edw, mdw,
          H * W * 2.0 ** -22)
    close(db.cpu().numpy().astype(np.float64), edb, mdb, H * W * 2.0 ** -22)


def test_pinball_loss_and_gradient(mf):
    rng = np.random.default_rng(3)
    n = 1000
    out = rng.normal(size=(n, 16)).astype(np.float32)
    tgt = rng.normal(size=(n, 2)).astype(np.float32)
    outd = torch.from_numpy(out).cuda()
    tgtd = torch.from_numpy(tgt).cuda()
    dout = torch.empty((n, 32), dtype=torch.bfloat16, device="cuda")
    part = torch.empty((n + 255) // 256, dtype=torch.float32, device="cuda")
    mf.cnn.pinball(outd, 16, tgtd, n, OC.TAU_LO, OC.TAU_HI, dout, part)
    torch.cuda.synchronize()
    L, g = OC.loss_and_grad(out[:, :2].astype(np.float64), tgt[:, 0].astype(np.float64),
                            tgt[:, 1].astype(np.float64))
    assert float(part.sum()) == pytest.approx(L * n, rel=1e-5)
    got = from_bf16(dout)
    assert np.allclose(got[:, :2], OC.bf16_round(g * n), rtol=0, atol=1e-12)
    assert np.all(got[:, 2:] == 0)


def test_features_and_targets(mf):
    import workloads
    img = workloads.natural_u16(100, 75, seed=1)
    feat = torch.empty((10, 13, 32), dtype=torch.bfloat16, device="cuda")
    d = torch.from_numpy(img).cuda()
    mf.cnn.features(d, 32, feat)
    tgt = torch.empty((10 * 13, 2), dtype=torch.float32, device="cuda")
    mf.cnn.targets(d, tgt)
    torch.cuda.synchronize()
    ef = OC.cell_features(img, 32, 65535.0)
    got = from_bf16(feat)
    assert np.allclose(got[..., :2], OC.bf16_round(ef), rtol=2.0 ** -8, atol=0)
    assert np.all(got[..., 2:] == 0)
    lo, hi = OC.cell_targets(img, 65535.0)
    t = tgt.cpu().numpy().reshape(10, 13, 2).astype(np.float64)
    assert np.allclose(t[..., 0], lo, rtol=1e-6) and np.allclose(t[..., 1], hi, rtol=1e-6)


def test_adam_step(mf):
    """Two Adam steps with different gradients against the float64 oracle
    (oracle.cnn.adam_step).  Tolerance from the kernel's float32 arithmetic:
    each step's update lr * mhat / (sqrt(vhat) + eps) is formed in a dozen
    float32 operations (relative error within 16u of its magnitude, u =
    2^-24, counting the moments' sums term by term), and the parameter is
    rounded once per step (u |p|); errors of step 1 carry into step 2.  The
    oracle takes the float32 values of lr, beta1, beta2 and eps that the
    kernel computes with.  The bf16 copy is the kernel's own float32
    parameter rounded to nearest even."""
    rng = np.random.default_rng(9)
    n = 777
    p = rng.normal(size=n).astype(np.float32)
    gs = [rng.normal(size=n).astype(np.float32) for _ in range(2)]
    gs[1][::7] = -gs[0][::7]          # opposite signs: the first moment cancels there
    pd = torch.from_numpy(p.copy()).cuda()
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    pb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    lr, u = 1e-2, 2.0 ** -24
    f32 = lambda x: float(np.float32(x))
    pp, mm, vv = p.astype(np.float64), np.zeros(n), np.zeros(n)
    mmag, vmag = np.zeros(n), np.zeros(n)
    tol = np.zeros(n)
    for step, g in ((1, gs[0]), (2, gs[1])):
        mf.cnn.adam(pd, m, v, torch.from_numpy(g).cuda(), lr, step, pb)
        pp, mm, vv = OC.adam_step(pp, mm, vv, g, f32(lr), step, b1=f32(0.9), b2=f32(0.999),
                                  eps=f32(1e-8))
        mmag = 0.9 * mmag + 0.1 * np.abs(g)
        vmag = 0.999 * vmag + 0.001 * g.astype(np.float64) ** 2
        upd = (mmag / (1 - 0.9 ** step)) / (np.sqrt(vv / (1 - 0.999 ** step)) + 1e-8)
        tol += 16 * u * lr * upd + 2 * u * np.abs(pp)
    torch.cuda.synchronize()
    got = pd.cpu().numpy().astype(np.float64)
    err = np.abs(got - pp)
    assert np.all(err <= tol), float(np.max(err / tol))
    assert np.array_equal(from_bf16(pb), OC.bf16_round(got))


@pytest.mark.parametrize("dtype,w,h,radius", [("u16", 37, 53, 16), ("u8", 300, 129, 4),
                                               ("u16", 1, 1, 32), ("u16", 200, 200, 64),
                                               ("u8", 512, 384, 0), ("u16", 1000, 17, 8)])
def test_fused_network_equals_layers(mf, dtype, w, h, radius):
    """The one-launch network (features + four layers in LDS) against the
    layer-by-layer kernels on the same bf16 weights: equal bit for bit, on
    grids that are not multiples of the 16-cell block and on the 1-cell
    grid (every layer's zero padding matters there)."""
    import workloads
    rng = np.random.default_rng(w * 7 + h)
    img = torch.from_numpy(workloads.uniform(w, h, dtype, w + h)).cuda()
    layers = [make_layer(rng, 32, cin_real=2), make_layer(rng, 32), make_layer(rng, 32),
              make_layer(rng, 16)]
    wd = [to_bf16_dev(wl)[0] for wl, _ in layers]
    bd = [torch.from_numpy(b.astype(np.float32)).cuda() for _, b in layers]
    H, W = (h + 7) // 8, (w + 7) // 8
    act = [torch.empty((H, W, 32), dtype=torch.bfloat16, device="cuda") for _ in range(4)]
    mf.cnn.features(img, radius, act[0])
    for l in range(3):
        mf.cnn.conv_forward(act[l], H, W, wd[l], bd[l], 32, 0, act[l + 1])
    ref = torch.empty((H, W, 16), dtype=torch.float32, device="cuda")
    mf.cnn.conv_forward(act[3], H, W, wd[3], bd[3], 16, 1, ref)
    got = torch.full((H, W, 16), float("nan"), dtype=torch.float32, device="cuda")
    mf.cnn.net_forward(img, radius, wd, bd, got)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
