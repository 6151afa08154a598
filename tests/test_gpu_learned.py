"""GPU tests of the learned-bracket path: exactness at any fallback rate,
forced fallback with wrong brackets, the exact set of recomputed tiles for
injected brackets, the network forward pass against the float64 oracle, and
a short training run."""

import numpy as np
import pytest

import workloads
from oracle import cnn as OC
from oracle import footprints as OF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    import paper_2505_22938_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    m.lib()
    return m


@pytest.fixture(scope="module")
def net(mf):
    n = mf.LearnedNet(seed=1)
    yield n
    n.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def tile_info(mf, w, h, dtype_code, fp):
    tx, ty = mf.LearnedNet.tile_grid(w, h, dtype_code, fp)
    tw, th = mf.LearnedNet.tile_shape(w, h, dtype_code, fp)
    assert tx == -(-w // tw) and ty == -(-h // th)
    return tx, ty, tw, th


def brackets_dev(br):
    return torch.from_numpy(np.ascontiguousarray(br.astype(np.int64).astype(np.uint32)
                                                 .view(np.int32))).cuda()


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_forced_fallback_wrong_brackets(mf, net, oracle_mod, dtype):
    img = workloads.natural_u16(300, 200, seed=2)
    if dtype == "u8":
        img = (img >> 8).astype(np.uint8)
    code = mf.MF_U8 if dtype == "u8" else mf.MF_U16
    fp = mf.Footprint.disc(8)
    tx, ty, tw, th = tile_info(mf, 300, 200, code, fp)
    br = np.zeros((ty * tx, 2))
    br[:, 1] = 0          # bracket [0, 0]: wrong for every tile of this image
    out, fb = net.filter_bracketed(dev(img), fp, brackets_dev(br))
    torch.cuda.synchronize()
    exp = oracle_mod.filter(img, OF.disc(8), "clamp")
    assert np.array_equal(out.cpu().numpy(), exp)
    assert fb == int((exp != 0).sum())   # every pixel whose median is not 0


@pytest.mark.parametrize("shape", ["ellipse", "disc3"])
def test_full_bracket_fallback_by_capacity(mf, net, oracle_mod, shape):
    """A full-range bracket holds every box pixel: tiles run bracketed (no
    fallback) when the box fits the bracketed layout's capacity, and go to
    the plain pass whole otherwise; the output is exact either way."""
    img = workloads.natural_u16(257, 131, seed=3)
    if shape == "ellipse":
        fp, ofp = mf.Footprint.ellipse(9, 4, 20), OF.ellipse(9, 4, 20)
    else:
        fp, ofp = mf.Footprint.disc(3), OF.disc(3)
    tx, ty, tw, th = tile_info(mf, 257, 131, mf.MF_U16, fp)
    cap = mf.LearnedNet.tile_grid(257, 131, mf.MF_U16, fp, with_capacity=True)[2]
    box = (tw + fp.dx_max - fp.dx_min) * (th + fp.dy_max - fp.dy_min)
    br = np.zeros((ty * tx, 2))
    br[:, 1] = 65535
    out, fb = net.filter_bracketed(dev(img), fp, brackets_dev(br), boundary="mirror")
    torch.cuda.synchronize()
    assert fb == (0 if box <= cap else 257 * 131), (box, cap, fb)
    assert np.array_equal(out.cpu().numpy(), oracle_mod.filter(img, ofp, "mirror"))


def box_counts(img, r, tx, ty, tw, th, br):
    """Per tile: box pixels (clamp boundary) inside the tile's bracket."""
    pad = np.pad(img, ((r, r + th), (r, r + tw)), mode="edge")
    out = np.zeros(tx * ty, dtype=np.int64)
    for t in range(tx * ty):
        x0, y0 = (t % tx) * tw, (t // tx) * th
        box = pad[y0:y0 + th + 2 * r, x0:x0 + tw + 2 * r]
        out[t] = int(((box >= br[t, 0]) & (box <= br[t, 1])).sum())
    return out


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_injected_brackets_fail_exactly_where_medians_escape(mf, net, oracle_mod, seed):
    """Random per-tile brackets, some containing every median of their tile
    and some not.  The fallback count is exact: every pixel whose median is
    outside its tile's bracket, plus every pixel of a tile with more
    in-bracket box pixels than the bracketed layout holds.  Radii 40 and 64
    use uniform noise (concentrated medians) and the large-box layout."""
    rng = np.random.default_rng(seed)
    W, H = 320, 260
    r = [4, 12, 20, 40, 64][seed]
    img = (workloads.natural_u16(W, H, seed=10 + seed) if r <= 20
           else workloads.uniform(W, H, "u16", 10 + seed))
    fp = mf.Footprint.disc(r)
    exp = oracle_mod.filter(img, OF.disc(r), "clamp")
    tx, ty, tw, th = tile_info(mf, W, H, mf.MF_U16, fp)
    cap = mf.LearnedNet.tile_grid(W, H, mf.MF_U16, fp, with_capacity=True)[2]
    br = np.zeros((ty * tx, 2), dtype=np.int64)
    for t in range(tx * ty):
        x0, y0 = (t % tx) * tw, (t // tx) * th
        med = exp[y0:y0 + th, x0:x0 + tw]
        lo, hi = int(med.min()), int(med.max())
        mode = rng.integers(0, 4)
        if mode == 0:          # exact range: no miss
            br[t] = (lo, hi)
        elif mode == 1:        # generous: no miss
            br[t] = (max(0, lo - 500), min(65535, hi + 500))
        elif mode == 2:        # too high at the bottom: some medians escape
            br[t] = (min(lo + 1, hi), hi) if hi > lo else (lo + 1, hi + 1)
        else:                  # too low at the top
            br[t] = (lo, max(hi - 1, lo)) if hi > lo else (lo - 1, hi - 1)
    br = np.clip(br, 0, 65535)
    ts = box_counts(img, r, tx, ty, tw, th, br)
    expect = 0
    for t in range(tx * ty):
        x0, y0 = (t % tx) * tw, (t // tx) * th
        med = exp[y0:y0 + th, x0:x0 + tw]
        if ts[t] > cap:
            expect += med.size
        else:
            expect += int(((med < br[t, 0]) | (med > br[t, 1])).sum())
    out, fb = net.filter_bracketed(dev(img), fp, brackets_dev(br))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), exp)
    assert fb == expect


@pytest.mark.parametrize("dtype,r", [("u16", 64), ("u8", 64), ("u16", 100)])
def test_large_box_bracket_overflow_and_narrow(mf, net, oracle_mod, dtype, r):
    """Large boxes: a full-range bracket holds more pixels than the bracketed
    layout can rank, so every tile goes to the plain pass (global-scratch
    plan); a bracket of exactly each tile's median range ranks few pixels
    and needs no fallback.  Both exact."""
    W, H = 300, 211
    img = workloads.uniform(W, H, dtype, 21)   # medians concentrate: narrow exact brackets
    code = mf.MF_U8 if dtype == "u8" else mf.MF_U16
    maxv = 255 if dtype == "u8" else 65535
    fp = mf.Footprint.disc(r)
    exp = oracle_mod.filter(img, OF.disc(r), "mirror")
    tx, ty, tw, th = tile_info(mf, W, H, code, fp)
    full = np.zeros((tx * ty, 2))
    full[:, 1] = maxv
    out, fb = net.filter_bracketed(dev(img), fp, brackets_dev(full), boundary="mirror")
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), exp)
    assert fb == W * H
    exact = np.zeros((tx * ty, 2), dtype=np.int64)
    for t in range(tx * ty):
        x0, y0 = (t % tx) * tw, (t // tx) * th
        med = exp[y0:y0 + th, x0:x0 + tw]
        exact[t] = (int(med.min()), int(med.max()))
    mf.work_counters(1)
    out, fb = net.filter_bracketed(dev(img), fp, brackets_dev(exact), boundary="mirror")
    torch.cuda.synchronize()
    ranked = mf.work_counters(-1)[7]
    mf.work_counters(0)
    assert np.array_equal(out.cpu().numpy(), exp)
    assert fb == 0
    assert ranked < tx * ty * (tw + 2 * r) * (th + 2 * r)


def _flat_params(Ws, bs):
    """Network parameters in the library's flat layout (per layer: weights
    [cout][9][32], then the biases)."""
    offW, offB = _layer_slices()
    p = np.zeros(offB[3] + 16, dtype=np.float64)
    for l in range(4):
        p[offW[l]:offW[l] + Ws[l].size] = Ws[l].reshape(-1)
        p[offB[l]:offB[l] + bs[l].size] = bs[l]
    return p.astype(np.float32)


def _check_within(got, exp, bound, what):
    err = np.abs(got - exp)
    bad = err > bound
    assert not bad.any(), (what, int(bad.sum()), float(err[bad].max()), float(bound[bad].min()))


@pytest.mark.parametrize("case", ["chain", "random"])
def test_network_forward_matches_oracle(mf, case):
    """The network's (lo, hi) output per cell against the float64 oracle
    chain, element by element, within the per-element bound of
    tests/cnn_bounds.py (bf16 stores at the kernels' points, float32
    accumulation).  'chain': the end-to-end test network (non-negative
    weights, ReLUs half on); 'random': the library's random initialisation
    with a random output layer (sign changes everywhere)."""
    from tests import cnn_bounds as CB
    img = workloads.natural_u16(130, 70, seed=5)
    n = mf.LearnedNet(seed=7)
    if case == "chain":
        Ws, bs, _ = CB.chain_case(img, 16, seed=7)
        n.set_params(_flat_params(Ws, bs))
    else:
        params = n.get_params().astype(np.float64)
        offW, offB = _layer_slices()
        rng = np.random.default_rng(0)
        params[offW[3]:offW[3] + 2 * 9 * 32] = rng.normal(0, 0.05, 2 * 9 * 32)
        n.set_params(params.astype(np.float32))
        p32 = params.astype(np.float32).astype(np.float64)
        Ws = [OC.bf16_round(p32[offW[l]:offW[l] + (32 if l < 3 else 16) * 9 * 32]
                            .reshape(-1, 3, 3, 32)) for l in range(4)]
        bs = [p32[offB[l]:offB[l] + (32 if l < 3 else 16)] for l in range(4)]
    out = n.forward(dev(img), 16)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)[..., :2]
    fw = CB.forward(img, 16, 65535.0, Ws, bs)
    _check_within(got, fw["pre"][3][..., :2], fw["epre"][3][..., :2], "out")
    n.close()


def test_training_decreases_loss_and_filter_stays_exact(mf, oracle_mod):
    n = mf.LearnedNet(seed=3)
    fp = mf.Footprint.disc(8)
    imgs = [dev(workloads.natural_u16(256, 256, seed=100 + i)) for i in range(4)]
    meds = [mf.median_filter(im, fp, "clamp") for im in imgs]
    torch.cuda.synchronize()
    losses = []
    for step in range(60):
        i = step % 4
        losses.append(n.train_step(imgs[i], meds[i], 8, 3e-3))
    assert np.mean(losses[-8:]) < 0.7 * np.mean(losses[:8]), losses[:4] + losses[-4:]
    test = workloads.natural_u16(256, 256, seed=999)
    n.set_margin(0.02)
    out, fb = n.filter(dev(test), fp)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle_mod.filter(test, OF.disc(8), "clamp"))
    assert 0 <= fb <= 256 * 256
    n.close()


def _layer_slices():
    W = 32 * 9 * 32
    offW = [0, W + 32, 2 * (W + 32), 3 * (W + 32)]
    offB = [W, 2 * W + 32, 3 * W + 64, 3 * (W + 32) + 16 * 9 * 32]
    return offW, offB


def test_train_step_gradient_matches_oracle(mf):
    """One training step's parameter gradient, every element of every layer,
    against the float64 oracle's forward and backward chain with bf16
    rounding where the kernels store bf16, within the per-element bound of
    tests/cnn_bounds.py.  The network and target (tests/cnn_bounds.py:
    chain_case) put both pinball branches and both ReLU states in every layer
    and keep the bound below one cell's share of each gradient entry's
    magnitude for nearly all entries (checked on the CPU by
    tests/test_cnn_bounds.py, which also shows that one cell's flipped
    mask, or a shifted tap, exceeds it)."""
    from tests import cnn_bounds as CB
    offW, offB = _layer_slices()
    img = workloads.natural_u16(96, 72, seed=8)
    Ws, bs, med = CB.chain_case(img, 8, seed=5)
    n = mf.LearnedNet(seed=5)
    n.set_params(_flat_params(Ws, bs))
    d_img = dev(img)
    loss = n.train_step(d_img, dev(med), 8, 1e-7)
    torch.cuda.synchronize()
    g = n.get_grads().astype(np.float64)

    fw = CB.forward(img, 8, 65535.0, Ws, bs)
    d, ed = CB.pinball_grad(fw["pre"][3], fw["epre"][3], med, 65535.0)
    assert np.all(ed == 0), "an output is too close to its target"
    t_lo, t_hi = OC.cell_targets(med, 65535.0)
    L, _ = OC.loss_and_grad(fw["pre"][3][..., :2], t_lo, t_hi)
    assert loss == pytest.approx(L, rel=1e-4)
    DW, EDW, DB, EDB = CB.backward(fw, Ws, d, ed)
    for l in range(4):
        cout = 32 if l < 3 else 16
        gw = g[offW[l]:offW[l] + cout * 9 * 32].reshape(cout, 3, 3, 32)
        gb = g[offB[l]:offB[l] + cout]
        _check_within(gw, DW[l], EDW[l], ("W", l))
        _check_within(gb, DB[l], EDB[l], ("b", l))
    n.close()


def test_trained_network_gain_over_plain(mf, oracle_mod):
    """What the trained network buys: on i.i.d. uniform uint16 noise (the
    learned-proposal workload) the committed network's brackets rank a small
    fraction of the box pixels that the method without it (the plain filter)
    ranks, with the output still exact and few pixels recomputed."""
    import os
    path = os.path.join(os.path.dirname(mf.__file__), "weights", "bracket_net.npz")
    net = mf.LearnedNet.load(path)
    img_np = workloads.uniform(512, 384, "u16", 42)
    img = dev(img_np)
    ranked = {}
    for r in (16, 32):
        fp = mf.Footprint.disc(r)
        exp = oracle_mod.filter(img_np, OF.disc(r), "clamp")
        mf.work_counters(1)
        out, fb = net.filter(img, fp)
        torch.cuda.synchronize()
        learned = mf.work_counters(-1)[7]
        mf.work_counters(0)
        assert np.array_equal(out.cpu().numpy(), exp)
        mf.work_counters(1)
        out2 = mf.median_filter(img, fp, "clamp")
        torch.cuda.synchronize()
        plain = mf.work_counters(-1)[7]
        mf.work_counters(0)
        assert np.array_equal(out2.cpu().numpy(), exp)
        ranked[r] = learned / plain
        assert fb <= 0.1 * 512 * 384, (r, fb)
    assert max(ranked.values()) < 0.5, ranked
    net.close()


@pytest.mark.parametrize("kind", ["uniform", "natural"])
def test_learned_full_size_sampled(mf, oracle_mod, kind):
    """2048x2048 uint16 (the learned-proposal workload) at radii 16, 32, 64
    with the committed network: every pixel equals the plain filter's and
    2000 seeded pixels equal the oracle's."""
    import os
    net = mf.LearnedNet.load(os.path.join(os.path.dirname(mf.__file__), "weights",
                                          "bracket_net.npz"))
    img_np = (workloads.uniform_u16(2048, 2048, seed=4) if kind == "uniform"
              else workloads.natural_u16(2048, 2048, seed=4))
    img = dev(img_np)
    for r in (16, 32, 64):
        fp = mf.Footprint.disc(r)
        out, fb = net.filter(img, fp)
        ref = mf.median_filter(img, fp, "clamp")
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy()), r
        rng = np.random.default_rng(r)
        xs, ys = rng.integers(0, 2048, 2000), rng.integers(0, 2048, 2000)
        exp = oracle_mod.filter_points(img_np, OF.disc(r), xs, ys, "clamp")
        assert np.array_equal(got[ys, xs], exp), r
        assert 0 <= fb <= 2048 * 2048
    net.close()


def test_trained_network_gain_over_untrained_and_full_bracket(mf, oracle_mod):
    """What training buys, against the method without the trained network:
    on i.i.d. uniform uint16 (the learned-proposal workload) the committed
    network recomputes a small fraction of the pixels, while the same
    network untrained (full-range output, every bracket dropped) and a
    constant full-range bracket per tile send every pixel to the plain pass;
    all three are exact."""
    import os
    S = 512
    img_np = workloads.uniform(S, S, "u16", 77)
    img = dev(img_np)
    fp = mf.Footprint.disc(32)
    exp = oracle_mod.filter(img_np, OF.disc(32), "clamp")
    trained = mf.LearnedNet.load(os.path.join(os.path.dirname(mf.__file__), "weights",
                                              "bracket_net.npz"))
    untrained = mf.LearnedNet(seed=4)
    untrained.set_margin(trained.margin)
    out_t, fb_t = trained.filter(img, fp)
    out_u, fb_u = untrained.filter(img, fp)
    tx, ty = mf.LearnedNet.tile_grid(S, S, mf.MF_U16, fp)
    full = torch.tensor([0, 65535], dtype=torch.int32, device="cuda").repeat(tx * ty)
    out_f, fb_f = trained.filter_bracketed(img, fp, full)
    torch.cuda.synchronize()
    for o in (out_t, out_u, out_f):
        assert np.array_equal(o.cpu().numpy(), exp)
    assert fb_u == S * S and fb_f == S * S, (fb_u, fb_f)
    assert fb_t <= 0.05 * S * S, fb_t
    trained.close()
    untrained.close()


def test_failed_tiles_recomputed_on_the_plain_plan(mf, net, oracle_mod):
    """Failed bracketed tiles are recomputed on the plain filter's own tile
    plan when its tiles split them evenly (here 64x64 plain tiles under
    64x128 bracketed tiles): every other bracketed tile gets an empty
    bracket (it fails), the rest a full-range one; the output equals the
    plain filter's bit for bit and the fallback count is the failed tiles'
    pixels."""
    W = H = 2048
    img_np = workloads.natural_u16(W, H, seed=9)
    img = dev(img_np)
    fp = mf.Footprint.disc(16)
    tw, th = mf.LearnedNet.tile_shape(W, H, mf.MF_U16, fp)
    plain = mf.query_plan(W, H, mf.MF_U16, fp)
    assert plain["tile_w"] == tw and th % plain["tile_h"] == 0 and th > plain["tile_h"], (
        (tw, th), plain)
    tx, ty = mf.LearnedNet.tile_grid(W, H, mf.MF_U16, fp)
    br = np.zeros((tx * ty, 2))
    br[:, 1] = 65535
    fail = (np.arange(tx * ty) % 2) == 1
    br[fail, 0] = 1          # lo > hi: no bracket, the tile fails
    br[fail, 1] = 0
    out, fb = net.filter_bracketed(img, fp, brackets_dev(br))
    ref = mf.median_filter(img, fp, "clamp")
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    cap = mf.LearnedNet.tile_grid(W, H, mf.MF_U16, fp, with_capacity=True)[2]
    box = (tw + fp.dx_max - fp.dx_min) * (th + fp.dy_max - fp.dy_min)
    expect = int(fail.sum()) * tw * th if box <= cap else W * H
    assert fb == expect, (fb, expect, box, cap)
    rng = np.random.default_rng(5)
    xs, ys = rng.integers(0, W, 1000), rng.integers(0, H, 1000)
    assert np.array_equal(out.cpu().numpy()[ys, xs],
                          oracle_mod.filter_points(img_np, OF.disc(16), xs, ys, "clamp"))
