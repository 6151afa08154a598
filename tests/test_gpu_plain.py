"""GPU parity of the plain filter against the CPU oracle, bit for bit.

Small cases compare every pixel.  Full-size workloads compare a seeded
sample of pixels that the oracle computes one by one, in the same launch
configuration the benchmark uses.
"""

import numpy as np
import pytest

import workloads
from oracle import footprints as OF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    import paper_2505_22938_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    m.lib()
    return m


def to_dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(mf, img, fp, boundary, **kw):
    out = mf.median_filter(to_dev(img), fp, boundary, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def assert_same(got, exp, what=""):
    if not np.array_equal(bits(got), bits(exp)):
        bad = np.argwhere(got.view(np.uint8 if got.dtype == np.uint8 else
                                   (np.uint16 if got.dtype == np.uint16 else np.uint32)) !=
                          exp.view(np.uint8 if exp.dtype == np.uint8 else
                                   (np.uint16 if exp.dtype == np.uint16 else np.uint32)))
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at {bad[:5].tolist()}")


FOOTPRINTS = {
    "disc1": (lambda m: m.Footprint.disc(1), lambda: OF.disc(1)),
    "disc3": (lambda m: m.Footprint.disc(3), lambda: OF.disc(3)),
    "disc8": (lambda m: m.Footprint.disc(8), lambda: OF.disc(8)),
    "paper_disc2": (lambda m: m.Footprint.disc_limit(6), lambda: OF.disc_limit(6)),
    "ellipse": (lambda m: m.Footprint.ellipse(9, 3, 30), lambda: OF.ellipse(9, 3, 30)),
    "hexagon": (lambda m: m.Footprint.regular_polygon(6, 7), lambda: OF.regular_polygon(6, 7)),
    "triangle": (lambda m: m.Footprint.polygon([(0, -5), (6, 4), (-4, 3)]),
                 lambda: OF.polygon([(0, -5), (6, 4), (-4, 3)])),
}


def make_img(dtype, w, h, seed):
    if dtype == "f32":
        return workloads.special_floats(w, h, seed)
    if dtype == "u16":
        return workloads.natural_u16(w, h, seed)
    return workloads.uniform(w, h, dtype, seed)


def test_plain_u8_256_disc4(mf, oracle_mod):
    img = workloads.plain_u8(256, 256, 0)
    fp = mf.Footprint.disc(4)
    assert fp.taps == 49
    assert_same(run(mf, img, fp, "clamp"), oracle_mod.filter(img, OF.disc(4), "clamp"), "c1")


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
@pytest.mark.parametrize("fpname", list(FOOTPRINTS))
def test_plain_matrix(mf, oracle_mod, dtype, boundary, fpname):
    mk, mko = FOOTPRINTS[fpname]
    img = make_img(dtype, 150, 77, 3)          # ragged in both directions
    got = run(mf, img, mk(mf), boundary)
    assert_same(got, oracle_mod.filter(img, mko(), boundary), f"{dtype}/{boundary}/{fpname}")


@pytest.mark.parametrize("w,h", [(1, 1), (1, 37), (41, 1), (2, 2), (3, 5), (64, 64), (65, 63)])
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
def test_plain_degenerate_sizes(mf, oracle_mod, w, h, boundary):
    img = workloads.uniform(w, h, "u16", w * 100 + h)
    for r in (0, 1, 5, 12):
        got = run(mf, img, mf.Footprint.disc(r), boundary)
        assert_same(got, oracle_mod.filter(img, OF.disc(r), boundary), f"{w}x{h} r={r}")


def test_plain_padded_stride(mf, oracle_mod):
    base = workloads.uniform(100, 50, "u8", 5)
    dev = torch.zeros((50, 128), dtype=torch.uint8, device="cuda")
    dev[:, :100] = to_dev(base)
    view = dev[:, :100]
    out = mf.median_filter(view, mf.Footprint.disc(3), "mirror")
    torch.cuda.synchronize()
    assert out.stride() == view.stride()
    assert_same(out.cpu().numpy(), oracle_mod.filter(base, OF.disc(3), "mirror"), "stride")


def test_plain_constant_and_binary(mf, oracle_mod):
    c = np.full((70, 90), 1234, dtype=np.uint16)
    assert_same(run(mf, c, mf.Footprint.disc(6), "clamp"), c, "constant")
    b = workloads.binary(90, 70, 1, hi=255)
    fp = OF.disc(5)
    assert_same(run(mf, b, mf.Footprint.disc(5), "clamp"), oracle_mod.filter(b, fp, "clamp"),
                "binary")


def test_plain_rank_parameter(mf, oracle_mod):
    img = workloads.uniform(80, 60, "u16", 9)
    fp = OF.disc(4)
    for k in (0, 10, 48):
        got = run(mf, img, mf.Footprint.disc(4), "clamp", rank=k)
        assert_same(got, oracle_mod.filter(img, fp, "clamp", rank=k), f"rank {k}")


def test_plain_adversarial(mf, oracle_mod):
    img = workloads.adversarial_u16(256, 256, border=40)
    got = run(mf, img, mf.Footprint.disc(16), "clamp")
    assert_same(got, oracle_mod.filter(img, OF.disc(16), "clamp"), "adversarial")


@pytest.mark.parametrize("r", [16, 32, 40, 48])
def test_plain_large_radius_u16(mf, oracle_mod, r):
    img = workloads.natural_u16(300, 200, seed=1)
    got = run(mf, img, mf.Footprint.disc(r), "clamp")
    assert_same(got, oracle_mod.filter(img, OF.disc(r), "clamp"), f"r={r}")


def sample_points(w, h, n, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, w, n)
    ys = rng.integers(0, h, n)
    # always include the corners and edges
    xs = np.concatenate([xs, [0, w - 1, 0, w - 1, w // 2, 0]])
    ys = np.concatenate([ys, [0, 0, h - 1, h - 1, 0, h // 2]])
    return xs, ys


@pytest.mark.parametrize("r", [56, 64, 80, 100])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_plain_global_scratch_radius(mf, oracle_mod, r, dtype):
    # boxes too large for LDS: sort, omnigram and reverse map in global scratch
    img = make_img(dtype, 150, 130, 7)
    got = run(mf, img, mf.Footprint.disc(r), "mirror")
    assert_same(got, oracle_mod.filter(img, OF.disc(r), "mirror"), f"{dtype} r={r}")


@pytest.mark.parametrize("case", ["one_high_half", "three_octaves_signed"])
def test_global_scratch_f32_order_of_high_halves(mf, oracle_mod, case):
    """Float keys in global scratch are ranked by a counting pass over their
    low 16 bits and then stable passes over the high 16 bits.  Inputs whose
    pixels share few high halves but differ in the low ones make every
    median depend on both orders: one high half for all pixels (values in
    [1, 1 + 2^-7)), and three octaves of both signs with low bits drawn at
    random (so equal high halves are common and their low halves decide)."""
    rng = np.random.default_rng(5)
    w, h = 210, 170
    if case == "one_high_half":
        img = (1.0 + rng.random((h, w)) * (2.0 ** -7)).astype(np.float32)
    else:
        hi = rng.choice(np.array([0x3F80, 0x4000, 0x4080, 0xBF80, 0xC000], np.uint32), (h, w))
        img = ((hi << 16) | rng.integers(0, 1 << 16, (h, w), dtype=np.uint32)).view(np.float32)
    fp = mf.Footprint.disc(64)
    p = mf.query_plan(w, h, mf.MF_F32, fp)
    assert p["box_w"] * p["box_h"] * 8 > 160 * 1024, p   # a global-scratch plan
    for boundary in ("clamp", "mirror"):
        assert_same(run(mf, img, fp, boundary), oracle_mod.filter(img, OF.disc(64), boundary),
                    f"{case} {boundary}")


@pytest.mark.parametrize("name", ["disc48", "ellipse", "hexagon"])
def test_lognormal_f32_footprints(mf, oracle_mod, name):
    # float32 planes with +-1e6 outliers under the mirror boundary
    mk = {"disc48": (lambda: mf.Footprint.disc(48), lambda: OF.disc(48)),
          "ellipse": (lambda: mf.Footprint.ellipse(60, 20, 30), lambda: OF.ellipse(60, 20, 30)),
          "hexagon": (lambda: mf.Footprint.regular_polygon(6, 40), lambda: OF.regular_polygon(6, 40))}
    a, b = mk[name]
    img = workloads.lognormal_f32(320, 180, planes=1, seed=2)[0]
    got = run(mf, img, a(), "mirror")
    assert_same(got, oracle_mod.filter(img, b(), "mirror"), name)


@pytest.mark.parametrize("r", [8, 32, 100])
def test_natural_u16_4096_sampled(mf, oracle_mod, r):
    img = workloads.natural_u16(4096, 4096, seed=1)
    got = run(mf, img, mf.Footprint.disc(r), "clamp")
    xs, ys = sample_points(4096, 4096, 4000, 17)
    exp = oracle_mod.filter_points(img, OF.disc(r), xs, ys, "clamp")
    assert_same(got[ys, xs], exp, f"4096 r={r}")


def test_natural_u16_4096_disc8_every_pixel(mf, oracle_mod):
    """The 4096^2 natural-like image at radius 8, every output pixel against
    the oracle (radius 32, the headline, is checked in full by the
    benchmark's CPU leg)."""
    img = workloads.natural_u16(4096, 4096, seed=1)
    got = run(mf, img, mf.Footprint.disc(8), "clamp")
    assert_same(got, oracle_mod.filter(img, OF.disc(8), "clamp"), "4096 r=8, all pixels")


@pytest.mark.parametrize("dtype,fpname,tile", [
    ("u16", "disc8", (40, 24)),      # width not dividing 64, last band shorter
    ("u8", "ellipse", (48, 20)),
    ("f32", "hexagon", (24, 40)),    # two bands per wave, 16 lanes idle
    ("u16", "triangle", (64, 20)),
    ("u16", "disc3", (7, 9)),
])
def test_plain_general_tile_shapes(mf, oracle_mod, dtype, fpname, tile):
    """Tile shapes outside the power-of-two grid (forced through the tile
    override), on ragged images with both boundaries."""
    mk, ofp = FOOTPRINTS[fpname]
    img = make_img(dtype, 203, 117, 31)
    mf.set_tile_override(*tile)
    try:
        for boundary in ("clamp", "mirror"):
            assert_same(run(mf, img, mk(mf), boundary), oracle_mod.filter(img, ofp(), boundary),
                        f"{dtype} {fpname} {tile} {boundary}")
    finally:
        mf.set_tile_override(0, 0)


@pytest.mark.parametrize("tile", [(54, 56), (40, 36)])
def test_plain_large_radius_odd_tiles(mf, oracle_mod, tile):
    """Radius 100 on global-scratch plans with odd tile shapes (the default
    54x56 and a smaller one)."""
    img = workloads.natural_u16(300, 260, 32)
    mf.set_tile_override(*tile)
    try:
        assert_same(run(mf, img, mf.Footprint.disc(100), "clamp"),
                    oracle_mod.filter(img, OF.disc(100), "clamp"), f"r100 {tile}")
    finally:
        mf.set_tile_override(0, 0)


@pytest.mark.parametrize("name", ["disc48", "ellipse", "hexagon"])
def test_lognormal_f32_full_size_sampled(mf, oracle_mod, name):
    """3840x2160 float32 log-normal plane with +-1e6 outliers, mirror
    boundary, at full size in the default launch configuration; 3000
    seeded output pixels against the oracle."""
    mk = {"disc48": (lambda: mf.Footprint.disc(48), lambda: OF.disc(48)),
          "ellipse": (lambda: mf.Footprint.ellipse(60, 20, 30), lambda: OF.ellipse(60, 20, 30)),
          "hexagon": (lambda: mf.Footprint.regular_polygon(6, 40), lambda: OF.regular_polygon(6, 40))}
    a, b = mk[name]
    img = workloads.lognormal_f32(3840, 2160, planes=1, seed=2)[0]
    got = run(mf, img, a(), "mirror")
    rng = np.random.default_rng(7)
    xs = rng.integers(0, 3840, 3000)
    ys = rng.integers(0, 2160, 3000)
    exp = oracle_mod.filter_points(img, b(), xs, ys, "mirror")
    assert np.array_equal(got[ys, xs].view(np.uint32), exp.view(np.uint32))


def test_lognormal_f32_three_planes_all_windows(mf, oracle_mod):
    """The whole float32 workload: three 3840x2160 log-normal planes with
    +-1e6 outliers (one seeded stack), each plane filtered on its own under
    the mirror boundary with the disc r=48, ellipse 60x20 at 30 degrees and
    hexagon R=40 windows; 1000 seeded output pixels per plane and window
    against the oracle."""
    stack = workloads.lognormal_f32(3840, 2160, planes=3, seed=2)
    wins = [(mf.Footprint.disc(48), OF.disc(48)),
            (mf.Footprint.ellipse(60, 20, 30), OF.ellipse(60, 20, 30)),
            (mf.Footprint.regular_polygon(6, 40), OF.regular_polygon(6, 40))]
    for p in range(3):
        img = stack[p]
        rng = np.random.default_rng(100 + p)
        xs = rng.integers(0, 3840, 1000)
        ys = rng.integers(0, 2160, 1000)
        for q, (fa, fb) in enumerate(wins):
            got = run(mf, img, fa, "mirror")
            exp = oracle_mod.filter_points(img, fb, xs, ys, "mirror")
            assert np.array_equal(got[ys, xs].view(np.uint32), exp.view(np.uint32)), (p, q)


@pytest.mark.parametrize("dt,r,w,h", [("u8", 123, 41, 29), ("f32", 118, 37, 23), ("u16", 110, 70, 45)])
def test_plain_largest_windows(mf, oracle_mod, dt, r, w, h):
    """Windows up to the largest the 8-bit box coordinates allow (width 247,
    radius 123: 8x8 output tiles under a 254x254 box in global scratch)."""
    img = workloads.uniform(w, h, dt, r) if dt != "f32" else workloads.special_floats(w, h, r)
    got = run(mf, img, mf.Footprint.disc(r), "mirror")
    assert_same(got, oracle_mod.filter(img, OF.disc(r), "mirror"), f"{dt} r={r}")


def test_autotune_records_shape_and_cache_round_trip(mf, oracle_mod, tmp_path):
    """The autotuner times the candidate shapes on the caller's image, records
    the fastest for (dtype, footprint); later calls and plan queries use it,
    outputs stay exact, and the table survives a JSON save / load."""
    import json
    img = workloads.natural_u16(300, 210, seed=8)
    fp, ofp = mf.Footprint.ellipse(7.5, 4, 10), OF.ellipse(7.5, 4, 10)   # used by no other test
    d = to_dev(img)
    tw, th, ms = mf.autotune(d, fp, "mirror", reps=2)
    assert 1 <= tw <= 64 and th >= 1 and ms > 0
    p = mf.query_plan(300, 210, mf.MF_U16, fp)
    assert (p["tile_w"], p["tile_h"]) == (tw, th)
    got = mf.median_filter(d, fp, "mirror")
    torch.cuda.synchronize()
    assert_same(got.cpu().numpy(), oracle_mod.filter(img, ofp, "mirror"), "tuned shape")
    path = str(tmp_path / "tune.json")
    mf.tune_cache_save(path)
    entries = json.load(open(path))
    mine = [e for e in entries if (e["tile_w"], e["tile_h"]) == (tw, th)]
    assert mine and all(set(e) == {"key", "tile_w", "tile_h", "ms"} for e in entries)
    mf.tune_cache_load(path)
    assert (mf.query_plan(300, 210, mf.MF_U16, fp)["tile_w"],
            mf.query_plan(300, 210, mf.MF_U16, fp)["tile_h"]) == (tw, th)


def test_global_scratch_on_two_streams(mf, oracle_mod):
    """Global-scratch tiles are claimed at run time through counters kept
    with each stream's scratch: calls queued on two streams without
    synchronising in between, and a graph of such a call replayed on its
    stream, all stay exact."""
    a = workloads.natural_u16(230, 170, seed=41)
    b = workloads.uniform(190, 210, "u16", 42)
    fp = mf.Footprint.disc(64)
    exp_a = oracle_mod.filter(a, OF.disc(64), "clamp")
    exp_b = oracle_mod.filter(b, OF.disc(64), "mirror")
    da, db = to_dev(a), to_dev(b)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs_a = [torch.empty_like(da) for _ in range(3)]
    outs_b = [torch.empty_like(db) for _ in range(3)]
    for i in range(3):
        with torch.cuda.stream(s1):
            mf.median_filter(da, fp, "clamp", out=outs_a[i])
        with torch.cuda.stream(s2):
            mf.median_filter(db, fp, "mirror", out=outs_b[i])
    torch.cuda.synchronize()
    for i in range(3):
        assert_same(outs_a[i].cpu().numpy(), exp_a, f"stream 1 call {i}")
        assert_same(outs_b[i].cpu().numpy(), exp_b, f"stream 2 call {i}")
    g = torch.cuda.CUDAGraph()
    out_g = torch.empty_like(da)
    with torch.cuda.graph(g, stream=s1):
        mf.median_filter(da, fp, "clamp", out=out_g)
    for rep in range(3):
        out_g.zero_()
        g.replay()
        with torch.cuda.stream(s2):
            mf.median_filter(db, fp, "mirror", out=outs_b[0])
        torch.cuda.synchronize()
        assert_same(out_g.cpu().numpy(), exp_a, f"replay {rep}")
        assert_same(outs_b[0].cpu().numpy(), exp_b, f"stream 2 beside replay {rep}")


def test_graph_capture_after_warm_call_and_release(mf, oracle_mod):
    """A plain call is captured into a graph once one uncaptured call on the
    same stream has uploaded its footprint and sized its scratch (radius 100:
    global-scratch tiles).  Replays, with eager work in between, match the
    eager outputs and the oracle.  A footprint never used on the device
    cannot be captured (MF_ERR_UNSUPPORTED, nothing enqueued).  After
    mf_release_scratch the next call allocates again and is still exact."""
    img = workloads.natural_u16(400, 300, seed=31)
    d_img = to_dev(img)
    fps = [mf.Footprint.disc(100), mf.Footprint.disc(8)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager = [mf.median_filter(d_img, fp, "clamp") for fp in fps]
    s.synchronize()
    outs = [torch.empty_like(d_img) for _ in fps]
    fresh = mf.Footprint.disc(5)
    status = None
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for fp, o in zip(fps, outs):
            mf.median_filter(d_img, fp, "clamp", out=o)
        try:
            mf.median_filter(d_img, fresh, "clamp")
        except mf.MedianFilterError as e:
            status = e.status
    assert status == -3
    for rep in range(3):
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep
        # eager work between replays
        mf.median_filter(d_img, mf.Footprint.disc(3), "mirror")
        torch.cuda.synchronize()
    exp = oracle_mod.filter(img, OF.disc(100), "clamp")
    assert_same(outs[0].cpu().numpy(), exp, "captured r=100")
    del g
    torch.cuda.synchronize()
    mf.release_scratch()
    got = run(mf, img, mf.Footprint.disc(100), "clamp")
    assert_same(got, exp, "after release")
