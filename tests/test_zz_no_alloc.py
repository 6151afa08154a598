"""GPU test of the allocation-free median filter against the ordinary one.

median_filter_noalloc runs the same kernels as median_filter with its span
table and sort scratch in the library's fixed per-GPU array.  Its output must
equal median_filter's bit for bit, on two calls in a row whose second input
is smaller (the array keeps the first call's contents), for windows in LDS
tiles and for windows large enough to need the global-scratch sort, and it
must leave the device's free memory unchanged.
"""

import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    import paper_2505_22938_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    m.lib()
    return m


def _call(fn, img, fp, boundary, out):
    L = ctypes.c_void_p
    es = img.element_size()
    h, w = img.shape
    code = {torch.uint8: 0, torch.uint16: 1, torch.float32: 2}[img.dtype]
    stream = L(torch.cuda.current_stream().cuda_stream)
    rc = fn(L(img.data_ptr()), w, h, img.stride(0) * es, code, fp.handle,
            {"clamp": 0, "mirror": 1}[boundary], L(out.data_ptr()), stream)
    assert rc == 0, f"status {rc}"


def _both(mf, img_np, fp, boundary):
    img = torch.from_numpy(np.ascontiguousarray(img_np)).cuda()
    ref = torch.empty_like(img)
    got = torch.full_like(img, 7)
    _call(mf.lib().median_filter, img, fp, boundary, ref)
    _call(mf.lib().median_filter_noalloc, img, fp, boundary, got)
    torch.cuda.synchronize()
    a = ref.cpu().numpy().view(np.uint8)
    b = got.cpu().numpy().view(np.uint8)
    assert np.array_equal(a, b), f"{int((a != b).sum())} bytes differ"


def _img(kind, w, h, seed):
    if kind == "u8":
        return workloads.uniform(w, h, "u8", seed)
    if kind == "u16":
        return workloads.natural_u16(w, h, seed)
    return workloads.lognormal_f32(w, h, planes=1, seed=seed)[0]


CASES = [
    # (dtype, footprint maker, boundary, first size, second size)
    ("u8", lambda m: m.Footprint.disc(4), "clamp", (517, 389), (131, 77)),
    ("u16", lambda m: m.Footprint.disc(32), "mirror", (1100, 700), (300, 211)),
    ("u16", lambda m: m.Footprint.disc(64), "clamp", (1500, 1200), (400, 333)),
    ("u16", lambda m: m.Footprint.disc(100), "clamp", (1200, 900), (500, 401)),
    ("f32", lambda m: m.Footprint.ellipse(60, 20, 30), "mirror", (1000, 640), (257, 190)),
    ("f32", lambda m: m.Footprint.disc(48), "mirror", (900, 700), (200, 300)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_median_filter_twice(mf, case):
    kind, make, boundary, s1, s2 = CASES[case]
    fp = make(mf)
    print(f"noalloc case {case}: {kind} taps={fp.taps} {boundary} {s1} then {s2}", flush=True)
    _both(mf, _img(kind, *s1, seed=10 + case), fp, boundary)
    _both(mf, _img(kind, *s2, seed=20 + case), fp, boundary)


def test_noalloc_cases_include_global_scratch_plans(mf):
    """Radius 100 cannot sort in LDS (its box alone needs more than 160 KiB
    at 4 bytes per pixel), so the cases above exercise the fixed array's
    sort-slot region as well as its span table."""
    p = mf.query_plan(1200, 900, mf.MF_U16, mf.Footprint.disc(100))
    assert p["box_w"] * p["box_h"] * 4 > 160 * 1024


def test_noalloc_allocates_no_device_memory(mf):
    """After one call has set the array up, calls with footprints the library
    has never seen (whose ordinary path would upload a span table and, for
    the large window, allocate sort scratch) leave free memory unchanged."""
    img = torch.from_numpy(workloads.natural_u16(640, 480, 5)).cuda()
    out = torch.empty_like(img)
    _call(mf.lib().median_filter_noalloc, img, mf.Footprint.disc(3), "clamp", out)
    _call(mf.lib().median_filter_noalloc, img, mf.Footprint.disc(70), "clamp", out)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for fp in (mf.Footprint.disc(5), mf.Footprint.disc(71), mf.Footprint.ellipse(40, 13, 10)):
        _call(mf.lib().median_filter_noalloc, img, fp, "clamp", out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, f"free device memory changed by {free0 - free1} bytes"
