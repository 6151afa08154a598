"""Python binding of libmedianfilter (exact isotropic median filtering on gfx950).

Argument marshalling only: every step of the filter runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  If the compiled
library is missing the import of this module still succeeds, but every call
raises ``RuntimeError`` -- there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmedianfilter.so")

MF_U8, MF_U16, MF_F32 = 0, 1, 2
MF_CLAMP, MF_MIRROR = 0, 1
STATUS = {0: "MF_OK", -1: "MF_ERR_INVALID_ARG", -2: "MF_ERR_ALIAS", -3: "MF_ERR_UNSUPPORTED",
          -4: "MF_ERR_NOMEM", -5: "MF_ERR_HIP"}
BOUNDARY = {"clamp": MF_CLAMP, "mirror": MF_MIRROR}

_lib = None


class MedianFilterError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)}")
        self.status = status


def lib():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2505_22938_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, LL, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong,
                       ctypes.c_size_t)
    PP = ctypes.POINTER(ctypes.c_void_p)
    IP = ctypes.POINTER(ctypes.c_int)
    sig = {
        "mf_status_string": ([I], ctypes.c_char_p),
        "mf_footprint_disc": ([I, PP], I),
        "mf_footprint_disc_limit": ([LL, PP], I),
        "mf_footprint_ellipse": ([D, D, D, PP], I),
        "mf_footprint_polygon": ([P, I, PP], I),
        "mf_footprint_regular_polygon": ([I, D, D, PP], I),
        "mf_footprint_info": ([P, IP, IP, IP, IP, IP, IP], I),
        "mf_footprint_row_spans": ([P, IP, IP], I),
        "mf_footprint_destroy": ([P], None),
        "median_filter": ([P, I, I, SZ, I, P, I, P, P], I),
        "median_filter_rank": ([P, I, I, SZ, I, P, I, I, P, P], I),
        "mf_set_tile_override": ([I, I], I),
        "mf_query_plan": ([I, I, I, P, IP, IP, IP, IP, IP], I),
        "mf_work_counters": ([I, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(fn: str, rc: int):
    if rc != 0:
        raise MedianFilterError(fn, rc)


class Footprint:
    """A filter window: an immutable set of integer offsets (dx right, dy down)."""

    def __init__(self, handle: ctypes.c_void_p, desc: str):
        self._h = handle
        self.desc = desc
        taps, rank, x0, x1, y0, y1 = (ctypes.c_int() for _ in range(6))
        _check("mf_footprint_info", lib().mf_footprint_info(self._h, ctypes.byref(taps),
                                                            ctypes.byref(rank), ctypes.byref(x0),
                                                            ctypes.byref(x1), ctypes.byref(y0),
                                                            ctypes.byref(y1)))
        self.taps, self.rank = taps.value, rank.value
        self.dx_min, self.dx_max, self.dy_min, self.dy_max = x0.value, x1.value, y0.value, y1.value

    @classmethod
    def _make(cls, fn: str, desc: str, *args):
        h = ctypes.c_void_p()
        _check(fn, getattr(lib(), fn)(*args, ctypes.byref(h)))
        return cls(h, desc)

    @classmethod
    def disc(cls, r: int):
        return cls._make("mf_footprint_disc", f"disc(r={r})", int(r))

    @classmethod
    def disc_limit(cls, limit: int):
        return cls._make("mf_footprint_disc_limit", f"disc_limit({limit})", int(limit))

    @classmethod
    def ellipse(cls, a: float, b: float, theta_deg: float):
        return cls._make("mf_footprint_ellipse", f"ellipse({a},{b},{theta_deg})", float(a),
                         float(b), float(theta_deg))

    @classmethod
    def polygon(cls, vertices):
        flat = [float(c) for v in vertices for c in v]
        arr = (ctypes.c_double * len(flat))(*flat)
        return cls._make("mf_footprint_polygon", f"polygon({len(vertices)})",
                         ctypes.cast(arr, ctypes.c_void_p), len(vertices))

    @classmethod
    def regular_polygon(cls, n_sides: int, circumradius: float, rot_deg: float = 0.0):
        return cls._make("mf_footprint_regular_polygon",
                         f"regular_polygon({n_sides},{circumradius},{rot_deg})", int(n_sides),
                         float(circumradius), float(rot_deg))

    def row_spans(self):
        n = self.dy_max - self.dy_min + 1
        lo = (ctypes.c_int * n)()
        hi = (ctypes.c_int * n)()
        _check("mf_footprint_row_spans", lib().mf_footprint_row_spans(self._h, lo, hi))
        return list(lo), list(hi)

    def offsets(self):
        """All (dx, dy) of the window, row by row (host-side, for tests)."""
        lo, hi = self.row_spans()
        return [(dx, self.dy_min + i) for i in range(len(lo)) for dx in range(lo[i], hi[i] + 1)]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.mf_footprint_destroy(h)
            self._h = None

    def __repr__(self):
        return f"Footprint({self.desc}, taps={self.taps})"


def _dtype_code(t):
    import torch
    if t.dtype == torch.uint8:
        return MF_U8, 1
    if t.dtype == torch.uint16:
        return MF_U16, 2
    if t.dtype == torch.float32:
        return MF_F32, 4
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _plane_args(img):
    if img.dim() != 2:
        raise ValueError("expected a 2-D plane (h, w)")
    if not img.is_cuda:
        raise ValueError("image must be a device tensor")
    code, es = _dtype_code(img)
    h, w = img.shape
    if img.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    stride_bytes = img.stride(0) * es if h > 1 else w * es
    return code, es, w, h, stride_bytes


def median_filter(img, fp: Footprint, boundary: str = "clamp", out=None, rank: int | None = None,
                  stream=None):
    """Filter a (h, w) device tensor (uint8, uint16 or float32); returns `out`.

    `out`, if given, must have the same shape, dtype and row stride as `img`.
    `rank` (zero-based, default the median (N-1)/2) selects a percentile.
    """
    import torch
    code, es, w, h, stride_bytes = _plane_args(img)
    if out is None:
        out = torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
    elif out.shape != img.shape or out.dtype != img.dtype or out.stride() != img.stride():
        raise ValueError("out must match img in shape, dtype and strides")
    L = lib()
    if rank is None:
        rc = L.median_filter(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                             fp.handle, BOUNDARY[boundary], ctypes.c_void_p(out.data_ptr()),
                             _stream_ptr(stream))
        _check("median_filter", rc)
    else:
        rc = L.median_filter_rank(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                                  fp.handle, BOUNDARY[boundary], int(rank),
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        _check("median_filter_rank", rc)
    return out


def set_tile_override(tile_w: int = 0, tile_h: int = 0):
    _check("mf_set_tile_override", lib().mf_set_tile_override(int(tile_w), int(tile_h)))


def work_counters(enable: int):
    """enable=1: start (and zero) the device work counters; 0: stop; -1: read
    them -> [blocks scanned, seeds, clk sort, clk rows, clk sweeps, waves, 0, 0]."""
    buf = (ctypes.c_ulonglong * 8)()
    _check("mf_work_counters", lib().mf_work_counters(int(enable),
                                                      ctypes.cast(buf, ctypes.c_void_p)))
    return list(buf) if enable < 0 else None


def query_plan(w: int, h: int, dtype: int, fp: Footprint):
    vals = [ctypes.c_int() for _ in range(5)]
    _check("mf_query_plan", lib().mf_query_plan(w, h, dtype, fp.handle,
                                                *[ctypes.byref(v) for v in vals]))
    return dict(zip(("tile_w", "tile_h", "box_w", "box_h", "lds_bytes"), (v.value for v in vals)))
