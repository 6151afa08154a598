"""GPU parity of several windows from one ordinal transform per tile (the
paper's multi-parameter filtering over radii and shapes) against the CPU
oracle and the single-window filter, bit for bit.  Each case runs with every
window in one pass (fused) and with the library's grouping by box size
(auto), which splits windows of very different sizes into passes."""

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


@pytest.fixture(params=["fused", "auto"])
def fusion(request, mf):
    mf.set_window_fusion(request.param == "fused")
    yield request.param
    mf.set_window_fusion(False)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                          np.ascontiguousarray(b).view(np.uint8))


def image(dt, w, h, seed):
    if dt == "f32":
        return workloads.special_floats(w, h, seed)
    return workloads.uniform(w, h, dt, seed)


@pytest.mark.parametrize("dt", ["u8", "u16", "f32"])
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
def test_radii_one_pass(mf, oracle_mod, fusion, dt, boundary):
    """Medians over discs of radius 3, 8 and 17 from one call, on an image
    spanning several tiles with ragged edges: each plane equals the oracle
    and the single-window filter."""
    radii = (3, 8, 17)
    w, h = 150, 97
    img = image(dt, w, h, 41)
    d = dev(img)
    outs = mf.window_filter(d, [mf.Footprint.disc(r) for r in radii], boundary)
    torch.cuda.synchronize()
    for r, o in zip(radii, outs):
        got = o.cpu().numpy()
        assert same(got, oracle_mod.filter(img, OF.disc(r), boundary)), (dt, r)
        single = mf.median_filter(d, mf.Footprint.disc(r), boundary)
        torch.cuda.synchronize()
        assert same(got, single.cpu().numpy()), (dt, r)


@pytest.mark.parametrize("dt", ["u16", "f32"])
def test_mixed_shapes_ranks_and_maps(mf, oracle_mod, fusion, dt):
    """A disc, an ellipse, a hexagon and off-centre shapes, at medians,
    constant ranks and a per-pixel rank map (span membership for all)."""
    w, h = 121, 83
    img = image(dt, w, h, 42)
    d = dev(img)
    tri = [(-4.0, -3.0), (6.0, -1.0), (0.0, 5.0)]
    wins = [
        (mf.Footprint.disc(5), OF.disc(5), -1),
        (mf.Footprint.ellipse(9, 3, 30), OF.ellipse(9, 3, 30), 7),
        (mf.Footprint.regular_polygon(6, 7), OF.regular_polygon(6, 7), None),
        (mf.Footprint.polygon(tri), OF.polygon(tri), 0),
        (mf.Footprint.disc(11), OF.disc(11), "map"),
    ]
    spec = []
    maps = {}
    for q, (fp, ofp, rk) in enumerate(wins):
        if rk is None:
            spec.append(fp)
        elif rk == "map":
            maps[q] = workloads.random_ranks(w, h, len(ofp), 9)
            spec.append((fp, dev(maps[q])))
        else:
            spec.append((fp, rk))
    outs = mf.window_filter(d, spec, "mirror")
    torch.cuda.synchronize()
    for q, ((fp, ofp, rk), o) in enumerate(zip(wins, outs)):
        if rk == "map":
            exp = oracle_mod.filter(img, ofp, "mirror", rank_map=maps[q])
        elif rk is None or rk < 0:
            exp = oracle_mod.filter(img, ofp, "mirror")
        else:
            exp = oracle_mod.filter(img, ofp, "mirror", rank=rk)
        assert same(o.cpu().numpy(), exp), (dt, q)


def test_rank_map_clamped_to_its_own_window(mf, oracle_mod, fusion):
    """A rank-map plane on a small window beside a larger one: its entries
    beyond its own N are clamped to its own maximum, not the larger
    window's."""
    w, h = 77, 53
    img = image("u16", w, h, 47)
    small = OF.disc(4)
    rm = workloads.random_ranks(w, h, len(small), 13)
    outs = mf.window_filter(dev(img), [mf.Footprint.disc(12), (mf.Footprint.disc(4), dev(rm))],
                            "clamp")
    torch.cuda.synchronize()
    assert same(outs[0].cpu().numpy(), oracle_mod.filter(img, OF.disc(12), "clamp"))
    assert same(outs[1].cpu().numpy(), oracle_mod.filter(img, small, "clamp", rank_map=rm))


@pytest.mark.parametrize("dt,radii", [("u16", (64, 8)), ("u8", (1, 60)), ("f32", (40, 2, 20))])
def test_large_boxes(mf, oracle_mod, fusion, dt, radii):
    """Boxes taken by the global-scratch and largest register plans, with a
    small window beside the large one."""
    w, h = 140, 75
    img = image(dt, w, h, 43)
    outs = mf.window_filter(dev(img), [mf.Footprint.disc(r) for r in radii], "clamp")
    torch.cuda.synchronize()
    for r, o in zip(radii, outs):
        assert same(o.cpu().numpy(), oracle_mod.filter(img, OF.disc(r), "clamp")), (dt, r)


@pytest.mark.parametrize("tile", [(24, 40), (7, 33)])
def test_odd_tile_shapes(mf, oracle_mod, fusion, tile):
    w, h = 101, 67
    img = image("u16", w, h, 44)
    mf.set_tile_override(*tile)
    try:
        outs = mf.window_filter(dev(img), [mf.Footprint.disc(6), mf.Footprint.disc(2)], "clamp")
        torch.cuda.synchronize()
    finally:
        mf.set_tile_override(0, 0)
    for r, o in zip((6, 2), outs):
        assert same(o.cpu().numpy(), oracle_mod.filter(img, OF.disc(r), "clamp")), (tile, r)


def test_off_centre_windows_beyond_one_box(mf, oracle_mod, fusion):
    """Two 201-pixel-wide bars on opposite sides of the centre: each fits a
    box, their common rectangle (401 wide) does not, so each gets its own
    pass even when one pass is requested."""
    right = [(0.0, -3.0), (200.0, -3.0), (200.0, 3.0), (0.0, 3.0)]
    left = [(-200.0, -3.0), (0.0, -3.0), (0.0, 3.0), (-200.0, 3.0)]
    w, h = 90, 23
    img = image("u8", w, h, 46)
    outs = mf.window_filter(dev(img), [mf.Footprint.polygon(right), mf.Footprint.polygon(left)],
                            "mirror")
    torch.cuda.synchronize()
    for verts, o in zip((right, left), outs):
        assert same(o.cpu().numpy(), oracle_mod.filter(img, OF.polygon(verts), "mirror"))


def test_errors_and_empty(mf, fusion):
    d = dev(image("u8", 40, 30, 45))
    fp = mf.Footprint.disc(2)
    with pytest.raises(ValueError):
        mf.window_filter(d, [fp] * 9)
    with pytest.raises(mf.MedianFilterError):
        mf.window_filter(d, [(fp, 13)])                   # rank >= N
    o = torch.empty_like(d)
    with pytest.raises(mf.MedianFilterError):
        mf.window_filter(d, [fp, mf.Footprint.disc(3)], outs=[o, o])
    empty = torch.empty((0, 5), dtype=torch.uint8, device="cuda")
    mf.window_filter(empty, [fp, mf.Footprint.disc(9)])


@pytest.mark.parametrize("radii,fused", [((24, 32, 40), False), ((8, 16, 32), True)])
def test_radii_full_size(mf, oracle_mod, radii, fused):
    """4096x4096 uint16 natural-like image (the headline workload), three
    disc radii in one call: every pixel equals the single-window median
    filter and 1000 seeded pixels per plane equal the oracle.  Radii 24/32/40
    share one pass under the default grouping; 8/16/32 are forced into one."""
    S = 4096
    img = workloads.natural_u16(S, S, seed=1)
    d = dev(img)
    mf.set_window_fusion(fused)
    try:
        outs = mf.window_filter(d, [mf.Footprint.disc(r) for r in radii], "clamp")
        torch.cuda.synchronize()
    finally:
        mf.set_window_fusion(False)
    rng = np.random.default_rng(23)
    for r, o in zip(radii, outs):
        got = o.cpu().numpy()
        single = mf.median_filter(d, mf.Footprint.disc(r), "clamp").cpu().numpy()
        assert np.array_equal(got, single), r
        xs, ys = rng.integers(0, S, 1000), rng.integers(0, S, 1000)
        assert np.array_equal(got[ys, xs], oracle_mod.filter_points(img, OF.disc(r), xs, ys,
                                                                    "clamp")), r


def test_lognormal_f32_three_shapes_full_size(mf, oracle_mod):
    """The float workload: one 3840x2160 log-normal plane with +-1e6
    outliers, disc r=48, ellipse 60x20 at 30 degrees and hexagon R=40 in one
    call (mirror), which the default grouping runs as one pass: every pixel
    equals the single-window filter bit for bit, and 400 seeded pixels per
    plane equal the oracle."""
    img = np.ascontiguousarray(workloads.lognormal_f32(3840, 2160, planes=1, seed=2)[0])
    d = dev(img)
    wins = [(mf.Footprint.disc(48), OF.disc(48)),
            (mf.Footprint.ellipse(60, 20, 30), OF.ellipse(60, 20, 30)),
            (mf.Footprint.regular_polygon(6, 40), OF.regular_polygon(6, 40))]
    outs = mf.window_filter(d, [w[0] for w in wins], "mirror")
    torch.cuda.synchronize()
    rng = np.random.default_rng(29)
    h, w = img.shape
    for (fp, ofp), o in zip(wins, outs):
        got = o.cpu().numpy()
        single = mf.median_filter(d, fp, "mirror").cpu().numpy()
        assert same(got, single)
        xs, ys = rng.integers(0, w, 400), rng.integers(0, h, 400)
        assert same(got[ys, xs], oracle_mod.filter_points(img, ofp, xs, ys, "mirror"))
