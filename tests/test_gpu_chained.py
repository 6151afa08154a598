"""GPU parity of chained tiles (median_filter_chained): tiles of a column
re-rank only their new rows and merge them with the kept part of the box
above, and start their first band from forwarded last-row solutions.  The
output must equal median_filter's (and so the oracle's) bit for bit for
every dtype, window shape, boundary, ragged image size and chain length,
including inputs with many ties (where forwarding is only exact if the kept
part keeps its order)."""

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
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


def image(kind, w, h, seed):
    if kind == "u8":
        return workloads.uniform(w, h, "u8", seed)
    if kind == "u8smooth":   # few distinct values: long runs of ties
        return (workloads.natural_u16(w, h, seed) >> 12).astype(np.uint8)
    if kind == "u16":
        return workloads.natural_u16(w, h, seed)
    return workloads.lognormal_f32(w, h, planes=1, seed=seed)[0]


FPS = {
    "disc3": lambda m: m.Footprint.disc(3),
    "disc8": lambda m: m.Footprint.disc(8),
    "disc20": lambda m: m.Footprint.disc(20),
    "ellipse": lambda m: m.Footprint.ellipse(9, 4, 30),
    "hexagon": lambda m: m.Footprint.regular_polygon(6, 7),
}


@pytest.mark.parametrize("kind", ["u8", "u8smooth", "u16", "f32"])
@pytest.mark.parametrize("fpn", sorted(FPS))
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
def test_chained_equals_plain(mf, kind, fpn, boundary):
    img = dev(image(kind, 333, 517, 5))
    fp = FPS[fpn](mf)
    ref = mf.median_filter(img, fp, boundary)
    for chain in (1, 2, 3, 100):
        got = mf.median_filter_chained(img, fp, chain, boundary)
        torch.cuda.synchronize()
        assert same(got.cpu().numpy(), ref.cpu().numpy()), f"chain {chain}"


def test_chained_matches_oracle_small(mf, oracle_mod):
    for kind, r, b in [("u8smooth", 5, "clamp"), ("u16", 9, "mirror"), ("f32", 4, "mirror")]:
        host = image(kind, 70, 301, 9)
        got = mf.median_filter_chained(dev(host), mf.Footprint.disc(r), 4, b)
        torch.cuda.synchronize()
        exp = oracle_mod.filter(host, OF.disc(r), b)
        assert same(got.cpu().numpy(), exp), (kind, r, b)


def test_chained_headline_size(mf):
    """4096^2 uint16 natural-like, disc r=32 (the headline workload), chains
    of 8 tiles: every pixel equals the plain filter's."""
    img = dev(workloads.natural_u16(4096, 4096, 1))
    fp = mf.Footprint.disc(32)
    ref = mf.median_filter(img, fp, "clamp")
    got = mf.median_filter_chained(img, fp, 8, "clamp")
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_chained_limits(mf):
    img = dev(image("u16", 300, 300, 1))
    with pytest.raises(mf.MedianFilterError) as e:
        mf.median_filter_chained(img, mf.Footprint.disc(100), 4)   # global-scratch box
    assert e.value.status == -3
    with pytest.raises(mf.MedianFilterError) as e:
        mf.median_filter_chained(img, mf.Footprint.disc(3), 0)
    assert e.value.status == -1
    empty = torch.empty((0, 5), dtype=torch.uint16, device="cuda")
    mf.median_filter_chained(empty, mf.Footprint.disc(3), 2)
