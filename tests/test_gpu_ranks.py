"""GPU parity of the general rank outputs against the CPU oracle, bit for bit:
per-pixel rank maps (the percentile varying across the image) and several
rank planes from one ordinal transform per tile."""

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                          np.ascontiguousarray(b).view(np.uint8))


def image(dt, w, h, seed):
    if dt == "f32":
        return workloads.special_floats(w, h, seed)
    return workloads.uniform(w, h, dt, seed)


FPS = {
    "disc5": (lambda m: m.Footprint.disc(5), lambda: OF.disc(5)),
    "disc24": (lambda m: m.Footprint.disc(24), lambda: OF.disc(24)),
    "ellipse": (lambda m: m.Footprint.ellipse(9, 3, 30), lambda: OF.ellipse(9, 3, 30)),
    "hexagon": (lambda m: m.Footprint.regular_polygon(6, 7), lambda: OF.regular_polygon(6, 7)),
}


@pytest.mark.parametrize("dt", ["u8", "u16", "f32"])
@pytest.mark.parametrize("fpname", list(FPS))
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
def test_rank_map_matches_oracle(mf, oracle_mod, dt, fpname, boundary):
    """Random ranks (some outside [0, N)) and a 0..100 % percentile ramp on
    images spanning several tiles with ragged right and bottom edges."""
    fp, ofp = FPS[fpname][0](mf), FPS[fpname][1]()
    n = len(ofp)
    w, h = 150, 97
    img = image(dt, w, h, 3)
    d = dev(img)
    for rm in (workloads.random_ranks(w, h, n, 7), workloads.percentile_ramp(w, h, n)):
        got = mf.rank_map_filter(d, fp, dev(rm), boundary)
        torch.cuda.synchronize()
        exp = oracle_mod.filter(img, ofp, boundary, rank_map=rm)
        assert same(got.cpu().numpy(), exp), (dt, fpname, boundary)


@pytest.mark.parametrize("dt,r", [("u16", 60), ("f32", 40), ("u8", 64)])
def test_rank_map_large_windows(mf, oracle_mod, dt, r):
    """Windows whose boxes take the global-scratch or largest register plans."""
    fp, ofp = mf.Footprint.disc(r), OF.disc(r)
    w, h = 140, 75
    img = image(dt, w, h, 11)
    rm = workloads.random_ranks(w, h, len(ofp), 12)
    got = mf.rank_map_filter(dev(img), fp, dev(rm), "mirror")
    torch.cuda.synchronize()
    assert same(got.cpu().numpy(), oracle_mod.filter(img, ofp, "mirror", rank_map=rm))


@pytest.mark.parametrize("tile", [(24, 40), (7, 33), (64, 16)])
def test_rank_map_odd_tile_shapes(mf, oracle_mod, tile):
    fp, ofp = mf.Footprint.disc(6), OF.disc(6)
    w, h = 101, 67
    img = image("u16", w, h, 5)
    rm = workloads.random_ranks(w, h, len(ofp), 6)
    mf.set_tile_override(*tile)
    try:
        got = mf.rank_map_filter(dev(img), fp, dev(rm), "clamp")
        torch.cuda.synchronize()
    finally:
        mf.set_tile_override(0, 0)
    assert same(got.cpu().numpy(), oracle_mod.filter(img, ofp, "clamp", rank_map=rm)), tile


def test_several_ranks_one_pass(mf, oracle_mod):
    """25th / 50th / 75th percentile planes and a rank-map plane from one
    call equal the oracle and the single-rank plain filter."""
    fp, ofp = mf.Footprint.disc(9), OF.disc(9)
    n = len(ofp)
    w, h = 133, 88
    img = image("u16", w, h, 21)
    d = dev(img)
    ks = [(n - 1) // 4, (n - 1) // 2, 3 * (n - 1) // 4]
    rm = workloads.percentile_ramp(w, h, n)
    outs = mf.rank_filter(d, fp, ks + [dev(rm)], "mirror")
    torch.cuda.synchronize()
    for k, o in zip(ks, outs):
        got = o.cpu().numpy()
        assert same(got, oracle_mod.filter(img, ofp, "mirror", rank=k)), k
        single = mf.median_filter(d, fp, "mirror", rank=k)
        torch.cuda.synchronize()
        assert same(got, single.cpu().numpy()), k
    assert same(outs[3].cpu().numpy(), oracle_mod.filter(img, ofp, "mirror", rank_map=rm))


def test_eight_planes_and_argument_errors(mf, oracle_mod):
    fp, ofp = mf.Footprint.ellipse(6, 3, 20), OF.ellipse(6, 3, 20)
    n = len(ofp)
    w, h = 70, 45
    img = image("f32", w, h, 31)
    d = dev(img)
    ranks = [0, 1, n // 3, (n - 1) // 2, n - 2, n - 1,
             dev(workloads.random_ranks(w, h, n, 1)), dev(workloads.random_ranks(w, h, n, 2))]
    outs = mf.rank_filter(d, fp, ranks, "clamp")
    torch.cuda.synchronize()
    for q, (rk, o) in enumerate(zip(ranks, outs)):
        if isinstance(rk, int):
            exp = oracle_mod.filter(img, ofp, "clamp", rank=rk)
        else:
            exp = oracle_mod.filter(img, ofp, "clamp", rank_map=rk.cpu().numpy())
        assert same(o.cpu().numpy(), exp), q
    with pytest.raises(ValueError):
        mf.rank_filter(d, fp, [0] * 9)
    with pytest.raises(mf.MedianFilterError):
        mf.rank_filter(d, fp, [n])                       # constant rank out of range
    o = torch.empty_like(d)
    with pytest.raises(mf.MedianFilterError):
        mf.rank_filter(d, fp, [0, 1], outs=[o, o])       # two planes into one buffer
    rm = torch.zeros((h, w), dtype=torch.int32, device="cuda")
    with pytest.raises(mf.MedianFilterError):             # rank map overlapping an output
        mf.rank_filter(d, fp, [rm], outs=[rm.view(torch.float32)])
    empty = torch.empty((0, 5), dtype=torch.uint8, device="cuda")
    mf.rank_filter(empty, fp, [0, 1])                     # nothing to do


def test_rank_map_full_size_sampled(mf, oracle_mod):
    """4096x4096 uint16 natural-like image, disc r=32, percentile ramp 0..100 %
    across the width (the paper's varying-percentile example): 3000 seeded
    pixels equal the oracle's, and every column whose rank is the median's
    equals the median filter, bit for bit."""
    S = 4096
    img = workloads.natural_u16(S, S, seed=1)
    fp, ofp = mf.Footprint.disc(32), OF.disc(32)
    n = len(ofp)
    rm = workloads.percentile_ramp(S, S, n)
    d = dev(img)
    got = mf.rank_map_filter(d, fp, dev(rm), "clamp").cpu().numpy()
    med = mf.median_filter(d, fp, "clamp").cpu().numpy()
    torch.cuda.synchronize()
    cols = np.nonzero(rm[0] == (n - 1) // 2)[0]
    assert len(cols) > 0 and np.array_equal(got[:, cols], med[:, cols])
    rng = np.random.default_rng(17)
    xs, ys = rng.integers(0, S, 3000), rng.integers(0, S, 3000)
    exp = oracle_mod.filter_points(img, ofp, xs, ys, "clamp", ranks=rm[ys, xs])
    assert np.array_equal(got[ys, xs], exp)
