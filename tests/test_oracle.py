"""Pins for the CPU oracle, against facts that do not come from the oracle itself.

Each test names what fixes the expected value: the paper, a closed form, a
library routine that reduces to the same definition, brute force, or an
invariant of rank-order filtering.
"""

import math
import os

import numpy as np
import pytest

import workloads
from oracle import footprints as F

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- footprints

def gauss_circle_count(r: int) -> int:
    """Lattice points with x^2+y^2 <= r^2 by Gauss's closed form
    N(r) = 1 + 4r + 4 * sum_{i=1..r} floor(sqrt(r^2 - i^2))."""
    return 1 + 4 * r + 4 * sum(math.isqrt(r * r - i * i) for i in range(1, r + 1))


# Leading values of the Gauss circle problem sequence N(r), r = 0..12.
GAUSS_SEQUENCE = [1, 5, 13, 29, 49, 81, 113, 149, 197, 253, 317, 377, 441]


@pytest.mark.parametrize("r", list(range(0, 13)) + [16, 32, 48, 64, 100])
def test_disc_counts_match_gauss_closed_form(r):
    n = len(F.disc(r))
    assert n == gauss_circle_count(r)
    if r < len(GAUSS_SEQUENCE):
        assert n == GAUSS_SEQUENCE[r]


def test_disc_r4_has_49_taps():
    # the 256x256 uint8 plain workload: disc r=4, dx^2+dy^2 <= 16, 49 taps
    assert len(F.disc(4)) == 49


def test_paper_radius2_window_is_21_taps():
    # Paper, Huang-sliding figure: the radius-2 circular window has 21 taps,
    # the 5x5 square without its four corners; on the lattice this is the
    # disc with limit r(r+1).
    fp = F.disc_limit(2 * 3)
    assert len(fp) == 21
    s = {tuple(p) for p in fp}
    sq = {(x, y) for x in range(-2, 3) for y in range(-2, 3)}
    assert sq - s == {(-2, -2), (-2, 2), (2, -2), (2, 2)}


def test_paper_radius48_tile_census():
    # Paper, GPU tile-geometry figure: at radius 48 a 64x64 output tile needs
    # a rounded-rectangle input tile of 23584 pixels, of which 16192 can be a
    # median.  Both follow from the r(r+1) disc: union of windows over the
    # tile, and T - N + 1.
    fp = F.disc_limit(48 * 49)
    n = len(fp)
    cover = np.zeros((64 + 96 + 1, 64 + 96 + 1), dtype=bool)
    for dx, dy in fp:
        cover[48 + dy:48 + dy + 64, 48 + dx:48 + dx + 64] = True
    T = int(cover.sum())
    assert T == 23584
    assert T - n + 1 == 16192


def _row_interval_count_ellipse(a, b, th_deg):
    # Independent count: per row dy, solve the quadratic in dx for the
    # ellipse boundary and count integers in the closed interval.
    t = math.radians(th_deg)
    c, s = math.cos(t), math.sin(t)
    # (dx c + dy s)^2 / a^2 + (-dx s + dy c)^2 / b^2 <= 1
    A = c * c / a ** 2 + s * s / b ** 2
    total = 0
    R = int(math.ceil(max(a, b))) + 1
    for dy in range(-R, R + 1):
        B = 2 * dy * (c * s / a ** 2 - s * c / b ** 2)
        Cc = dy * dy * (s * s / a ** 2 + c * c / b ** 2) - 1
        disc = B * B - 4 * A * Cc
        if disc < 0:
            continue
        lo = (-B - math.sqrt(disc)) / (2 * A)
        hi = (-B + math.sqrt(disc)) / (2 * A)
        total += max(0, math.floor(hi + 1e-9) - math.ceil(lo - 1e-9) + 1)
    return total


def test_ellipse_60x20_rot30():
    fp = F.ellipse(60, 20, 30)
    assert len(fp) == _row_interval_count_ellipse(60, 20, 30) == 3771
    # major axis along (cos30, sin30): down-right on screen (dy grows downward)
    s = {tuple(p) for p in fp}
    assert (51, 29) in s and (-51, -29) in s and (51, -29) not in s
    assert abs(len(fp) - math.pi * 60 * 20) < 0.01 * math.pi * 60 * 20


def test_regular_hexagon_r40():
    fp = F.regular_polygon(6, 40.0)
    # independent count: flat top/bottom hexagon with a vertex on +x;
    # row dy (|dy| <= 40 sin60) spans |dx| <= 40 - |dy| / tan(60 deg).
    h = 40 * math.sin(math.radians(60))
    total = 0
    for dy in range(-41, 42):
        if abs(dy) > h + 1e-9:
            continue
        half = 40 - abs(dy) / math.tan(math.radians(60))
        total += 2 * math.floor(half + 1e-9) + 1
    assert len(fp) == total == 4145
    s = {tuple(p) for p in fp}
    assert (40, 0) in s and (-40, 0) in s          # vertices lie on the lattice: inclusive
    assert (0, 34) in s and (0, 35) not in s


@pytest.mark.parametrize("fp", [F.disc(0), F.disc(5), F.disc_limit(30), F.ellipse(9, 3, 30),
                                F.ellipse(7.5, 7.5, 0), F.regular_polygon(6, 8),
                                F.regular_polygon(5, 7, 10), F.polygon([(0, -4), (5, 3), (-3, 2)])])
def test_footprints_row_and_column_convex(fp):
    s = {tuple(p) for p in fp}
    for axis in (0, 1):
        lines = {}
        for p in s:
            lines.setdefault(p[1 - axis], []).append(p[axis])
        for vals in lines.values():
            vals = sorted(vals)
            assert vals == list(range(vals[0], vals[-1] + 1))


def test_polygon_winding_invariant_and_square():
    sq_ccw = [(-3, -3), (3, -3), (3, 3), (-3, 3)]
    a = {tuple(p) for p in F.polygon(sq_ccw)}
    b = {tuple(p) for p in F.polygon(sq_ccw[::-1])}
    assert a == b == {(x, y) for x in range(-3, 4) for y in range(-3, 4)}


def test_median_rank_convention():
    # Paper: for a 7x7 window the median is the 25th of 49 values.
    assert F.median_rank(49) + 1 == 25


# ---------------------------------------------------------------- boundary

@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_remap_matches_numpy_pad(oracle_mod, n):
    pad = 3 * n + 5
    base = np.arange(n)
    for boundary, mode in (("clamp", "edge"), ("mirror", "reflect")):
        if boundary == "mirror" and n == 1:
            exp = np.zeros(n + 2 * pad, dtype=int)   # reflect-101 of one pixel: itself
        else:
            exp = np.pad(base, pad, mode=mode)
        got = [oracle_mod.remap(x, n, boundary) for x in range(-pad, n + pad)]
        assert list(exp) == got, (boundary, n)


# ---------------------------------------------------------------- float order

def _bits(x):
    return int(np.array(x, dtype=np.float32).view(np.uint32))


def test_total_order_hand_cases(oracle_mod):
    seq = [-np.inf, -1e30, -1.0, -1e-40, -1e-45, -0.0, 0.0, 1e-45, 1e-40, 1.0, 1e30, np.inf]
    b = [_bits(v) for v in seq]
    for i in range(len(b)):
        for j in range(len(b)):
            assert oracle_mod.total_order_less(b[i], b[j]) == (i < j)
    # NaNs: negative NaN below -inf, positive NaN above +inf
    assert oracle_mod.total_order_less(0xFFC00000, _bits(-np.inf))
    assert oracle_mod.total_order_less(_bits(np.inf), 0x7FC00000)


def test_total_order_matches_numpy_sort(oracle_mod):
    rng = np.random.default_rng(7)
    v = (rng.standard_normal(400) * 10.0 ** rng.integers(-30, 30, 400)).astype(np.float32)
    v = v[v != 0]
    order = np.sort(v)
    b = order.view(np.uint32)
    for i in range(len(b) - 1):
        if order[i] < order[i + 1]:
            assert oracle_mod.total_order_less(int(b[i]), int(b[i + 1]))
            assert not oracle_mod.total_order_less(int(b[i + 1]), int(b[i]))


# ---------------------------------------------------------------- ordinal transform

def test_fig4_ordinal_transform_example(oracle_mod):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "fig4_ordinal.txt"))
            if l.strip() and not l.startswith("#")]
    vals = np.array([int(r[0]) for r in rows], dtype=np.uint16)
    ords = [int(r[1]) for r in rows]
    perm = np.random.default_rng(0).permutation(len(vals))
    C, omega, ordinal = oracle_mod.ordinal_transform(vals[perm])
    assert list(C) == list(vals)                      # reverse map = sorted cardinals
    assert sorted(ordinal) == ords                    # a permutation of 0..n-1
    assert all(C[ordinal[i]] == vals[perm][i] for i in range(len(vals)))
    # duplicates get consecutive ordinals, in index order (stable)
    i29 = [i for i in range(len(perm)) if vals[perm][i] == 29]
    assert sorted(ordinal[i29]) == [3, 4] and ordinal[min(i29)] == 3
    # I(Omega[v]) = v  (Eq. 4)
    assert all(ordinal[omega[v]] == v for v in range(len(vals)))


# ---------------------------------------------------------------- whole filter

SMALL_FPS = {
    "disc0": F.disc(0),
    "disc1": F.disc(1),
    "disc3": F.disc(3),
    "disc_rr1_2": F.disc_limit(6),
    "ellipse": F.ellipse(5, 2, 30),
    "hexagon": F.regular_polygon(6, 4),
    "triangle": F.polygon([(0, -3), (3, 2), (-3, 2)]),
}


def _img(dtype, w, h, seed):
    if dtype == "f32":
        return workloads.special_floats(w, h, seed)
    return workloads.uniform(w, h, dtype, seed)


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
@pytest.mark.parametrize("fpname", list(SMALL_FPS))
def test_oracle_equals_full_sort(oracle_mod, dtype, boundary, fpname):
    fp = SMALL_FPS[fpname]
    for (w, h, seed) in [(13, 9, 1), (1, 7, 2), (6, 1, 3), (2, 2, 4)]:
        img = _img(dtype, w, h, seed)
        got = oracle_mod.filter(img, fp, boundary)
        exp = oracle_mod.tiny_filter(img, fp, boundary)
        assert np.array_equal(got.view(np.uint8), exp.view(np.uint8)), (w, h)


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("boundary,mode", [("clamp", "nearest"), ("mirror", "mirror")])
def test_oracle_equals_scipy(oracle_mod, dtype, boundary, mode):
    from scipy import ndimage
    fp = F.ellipse(6, 2.5, 30)          # asymmetric in x/y: catches swapped axes
    assert len(fp) % 2 == 1
    R = int(np.abs(fp).max())
    mask = np.zeros((2 * R + 1, 2 * R + 1), dtype=bool)
    mask[fp[:, 1] + R, fp[:, 0] + R] = True
    img = workloads.uniform(37, 23, dtype, 11)
    if dtype == "f32":
        img = (img * 2 - 1).astype(np.float32)
        img[img == 0] = 0.5
    got = oracle_mod.filter(img, fp, boundary)
    exp = ndimage.median_filter(img, footprint=mask, mode=mode)
    assert np.array_equal(got, exp)


def test_radius0_identity(oracle_mod):
    for dt in ("u8", "u16", "f32"):
        img = _img(dt, 20, 11, 5)
        for b in ("clamp", "mirror"):
            assert np.array_equal(oracle_mod.filter(img, F.disc(0), b).view(np.uint8),
                                  img.view(np.uint8))


def test_constant_image_fixed_point(oracle_mod):
    for dt, v in (("u8", 77), ("u16", 40000), ("f32", -3.25)):
        img = np.full((9, 14), v, dtype=workloads.NUMPY_DTYPE[dt])
        assert np.array_equal(oracle_mod.filter(img, F.disc(4), "mirror"), img)


def test_monotone_remap_commutes(oracle_mod):
    img = workloads.uniform(31, 17, "u8", 3)
    lut = np.round(255 * (np.arange(256) / 255.0) ** 2.2).astype(np.uint8)   # gamma, non-decreasing
    fp = F.ellipse(4, 2, 60)
    a = oracle_mod.filter(lut[img], fp, "clamp")
    b = lut[oracle_mod.filter(img, fp, "clamp")]
    assert np.array_equal(a, b)
    f = workloads.uniform(31, 17, "f32", 4)
    g = np.exp(3 * f).astype(np.float32)             # increasing on f32
    assert np.array_equal(oracle_mod.filter(g, fp, "mirror"),
                          np.exp(3 * oracle_mod.filter(f, fp, "mirror")).astype(np.float32))


def test_binary_image_majority_vote(oracle_mod):
    img = workloads.binary(29, 21, 9, hi=255)
    fp = F.disc(3)
    n = len(fp)
    k = (n - 1) // 2
    out = oracle_mod.filter(img, fp, "clamp")
    ones = oracle_mod.filter((img > 0).astype(np.uint8), fp, "clamp", rank=0)  # sanity of rank arg
    assert ones.shape == img.shape
    # count of 255s in each window, by direct summation
    H, W = img.shape
    cnt = np.zeros_like(img, dtype=int)
    for dx, dy in fp:
        ys = np.clip(np.arange(H) + dy, 0, H - 1)
        xs = np.clip(np.arange(W) + dx, 0, W - 1)
        cnt += (img[ys][:, xs] > 0)
    assert np.array_equal(out == 255, cnt >= n - k)


def test_order_reversal(oracle_mod):
    fp = F.disc(3)
    u = workloads.uniform(25, 19, "u16", 8)
    assert np.array_equal(oracle_mod.filter(65535 - u, fp, "mirror"),
                          65535 - oracle_mod.filter(u, fp, "mirror"))
    f = workloads.special_floats(25, 19, 8)
    a = oracle_mod.filter(-f, fp, "clamp")
    b = -oracle_mod.filter(f, fp, "clamp")
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))   # bitwise, incl. signed zeros


def test_flip_and_transpose_equivariance(oracle_mod):
    fp = F.disc(4)
    img = workloads.uniform(23, 18, "u8", 12)
    base = oracle_mod.filter(img, fp, "mirror")
    assert np.array_equal(oracle_mod.filter(img[:, ::-1].copy(), fp, "mirror"), base[:, ::-1])
    assert np.array_equal(oracle_mod.filter(img[::-1].copy(), fp, "mirror"), base[::-1])
    assert np.array_equal(oracle_mod.filter(img.T.copy(), fp, "mirror"), base.T)


def test_certificate_and_interior_translation(oracle_mod):
    fp = F.regular_polygon(6, 5)
    n = len(fp)
    k = (n - 1) // 2
    img = workloads.uniform(40, 30, "u16", 13)
    out = oracle_mod.filter(img, fp, "clamp")
    for y in range(0, 30, 3):
        for x in range(0, 40, 3):
            win = np.array([img[min(max(y + dy, 0), 29), min(max(x + dx, 0), 39)] for dx, dy in fp])
            v = out[y, x]
            assert v in win
            assert (win < v).sum() <= k < (win <= v).sum()
    # interior translation: shifting the image shifts the interior output
    sh = np.roll(img, (2, 3), axis=(0, 1))
    o2 = oracle_mod.filter(sh, fp, "clamp")
    assert np.array_equal(o2[10:22, 10:30], np.roll(out, (2, 3), axis=(0, 1))[10:22, 10:30])


def test_filter_points_matches_full(oracle_mod):
    img = workloads.natural_u16(96, 80, seed=1)
    fp = F.disc(8)
    full = oracle_mod.filter(img, fp, "clamp")
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 96, 200)
    ys = rng.integers(0, 80, 200)
    assert np.array_equal(oracle_mod.filter_points(img, fp, xs, ys, "clamp"), full[ys, xs])


# ------------------------------------------------------------ rank maps
# A rank per output pixel (the percentile may vary across the image, paper
# Conclusion and the varying-percentile figure); entries outside [0, N) are
# clamped, i.e. select the window minimum or maximum.

def _maps(n, w, h, seed):
    return [workloads.random_ranks(w, h, n, seed), workloads.percentile_ramp(w, h, n)]


def test_percentile_ramp_ends_and_monotone():
    rm = workloads.percentile_ramp(11, 3, 49)
    assert rm[:, 0].tolist() == [0, 0, 0] and rm[:, -1].tolist() == [48, 48, 48]
    assert (np.diff(rm[0]) >= 0).all()
    assert rm[0, 5] == 24                 # q = 1/2 -> the median rank (N - 1) / 2
    assert workloads.percentile_ramp(1, 2, 7).tolist() == [[0], [0]]


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("boundary", ["clamp", "mirror"])
@pytest.mark.parametrize("fpname", ["disc1", "disc3", "ellipse", "triangle"])
def test_rank_map_equals_full_sort(oracle_mod, dtype, boundary, fpname):
    fp = SMALL_FPS[fpname]
    n = len(fp)
    for (w, h, seed) in [(13, 9, 1), (1, 7, 2), (6, 1, 3)]:
        img = _img(dtype, w, h, seed)
        for rm in _maps(n, w, h, seed):
            got = oracle_mod.filter(img, fp, boundary, rank_map=rm)
            exp = oracle_mod.tiny_filter(img, fp, boundary, rank_map=rm)
            assert np.array_equal(got.view(np.uint8), exp.view(np.uint8)), (w, h)


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("boundary,mode", [("clamp", "nearest"), ("mirror", "mirror")])
def test_rank_map_extremes_are_min_and_max_filters(oracle_mod, dtype, boundary, mode):
    from scipy import ndimage
    fp = F.ellipse(6, 2.5, 30)
    n = len(fp)
    R = int(np.abs(fp).max())
    mask = np.zeros((2 * R + 1, 2 * R + 1), dtype=bool)
    mask[fp[:, 1] + R, fp[:, 0] + R] = True
    img = workloads.uniform(37, 23, dtype, 11)
    if dtype == "f32":
        img = (img * 2 - 1).astype(np.float32)
        img[img == 0] = 0.5
    rng = np.random.default_rng(0)
    low = -rng.integers(0, 5, size=img.shape).astype(np.int32)          # 0 or below
    high = (n - 1 + rng.integers(0, 5, size=img.shape)).astype(np.int32)  # N - 1 or above
    assert np.array_equal(oracle_mod.filter(img, fp, boundary, rank_map=low),
                          ndimage.minimum_filter(img, footprint=mask, mode=mode))
    assert np.array_equal(oracle_mod.filter(img, fp, boundary, rank_map=high),
                          ndimage.maximum_filter(img, footprint=mask, mode=mode))


def test_rank_map_certificate(oracle_mod):
    fp = F.regular_polygon(6, 5)
    n = len(fp)
    img = workloads.uniform(40, 30, "u16", 14)
    rm = workloads.random_ranks(40, 30, n, 5)
    out = oracle_mod.filter(img, fp, "mirror", rank_map=rm)
    for y in range(0, 30, 2):
        for x in range(0, 40, 3):
            win = np.array([img[oracle_mod.remap(y + dy, 30, "mirror"),
                                oracle_mod.remap(x + dx, 40, "mirror")] for dx, dy in fp])
            k = min(max(int(rm[y, x]), 0), n - 1)
            v = out[y, x]
            assert (win < v).sum() <= k < (win <= v).sum(), (x, y, k)


def test_rank_map_constant_equals_rank(oracle_mod):
    fp = F.disc(3)
    n = len(fp)
    img = workloads.uniform(21, 17, "f32", 6)
    for k in (0, 7, (n - 1) // 2, n - 1):
        rm = np.full(img.shape, k, dtype=np.int32)
        a = oracle_mod.filter(img, fp, "clamp", rank_map=rm)
        b = oracle_mod.filter(img, fp, "clamp", rank=k)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), k


def test_filter_points_ranks_match_rank_map(oracle_mod):
    img = workloads.natural_u16(64, 48, seed=2)
    fp = F.disc(5)
    rm = workloads.random_ranks(64, 48, len(fp), 9)
    full = oracle_mod.filter(img, fp, "mirror", rank_map=rm)
    rng = np.random.default_rng(1)
    xs, ys = rng.integers(0, 64, 150), rng.integers(0, 48, 150)
    got = oracle_mod.filter_points(img, fp, xs, ys, "mirror", ranks=rm[ys, xs])
    assert np.array_equal(got, full[ys, xs])
