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
          -4: "MF_ERR_NOMEM", -5: "MF_ERR_HIP", -6: "MF_ERR_SCRATCH_LIMIT"}
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
        "median_filter_noalloc": ([P, I, I, SZ, I, P, I, P, P], I),
        "median_filter_chained": ([P, I, I, SZ, I, P, I, I, P, P], I),
        "median_filter_ranks": ([P, I, I, SZ, I, P, I, P, I, P], I),
        "median_filter_rank_map": ([P, I, I, SZ, I, P, I, P, SZ, P, P], I),
        "median_filter_windows": ([P, I, I, SZ, I, I, P, I, P], I),
        "mf_set_window_fusion": ([I], I),
        "mf_set_tile_override": ([I, I], I),
        "mf_release_scratch": ([], I),
        "mf_query_plan": ([I, I, I, P, IP, IP, IP, IP, IP], I),
        "mf_work_counters": ([I, P], I),
        "mf_autotune": ([P, I, I, SZ, I, P, I, P, P, I, IP, IP,
                         ctypes.POINTER(ctypes.c_float)], I),
        "mf_tune_cache_load": ([ctypes.c_char_p], I),
        "mf_plan_create": ([P, I, ctypes.c_char_p, PP], I),
        "mf_plan_launch": ([P, P], I),
        "mf_plan_capture": ([P, P], I),
        "mf_plan_replay": ([P, P], I),
        "mf_plan_info": ([P, IP, IP, IP, ctypes.POINTER(ctypes.c_longlong)], I),
        "mf_plan_groups": ([P, IP, IP], I),
        "mf_plan_destroy": ([P], None),
        "median_filter_batched": ([P, I, P], I),
        "mf_plan_autotune": ([P, I, P, I, ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_float), IP], I),
        "mf_mfma_probe": ([P, P, P, P], I),
        "mf_cnn_conv_forward": ([P, I, I, P, P, I, I, P, P, P], I),
        "mf_cnn_flip_weights": ([P, I, P, P], I),
        "mf_cnn_wgrad_workspace": ([I, I, I, I], ctypes.c_longlong),
        "mf_cnn_conv_wgrad": ([P, P, I, I, I, I, P, P, P, P], I),
        "mf_cnn_pinball": ([P, I, P, I, ctypes.c_float, ctypes.c_float, P, P, P], I),
        "mf_cnn_features": ([P, I, I, SZ, I, I, P, P], I),
        "mf_cnn_net_forward": ([P, I, I, SZ, I, I, P, P, P, P], I),
        "mf_cnn_targets": ([P, I, I, SZ, I, P, P], I),
        "mf_cnn_adam": ([P, P, P, P, I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                         ctypes.c_float, I, P, P], I),
        "mf_learned_create": ([ctypes.c_ulonglong, PP], I),
        "mf_learned_destroy": ([P], None),
        "mf_learned_param_count": ([], I),
        "mf_learned_get_params": ([P, P], I),
        "mf_learned_set_params": ([P, P], I),
        "mf_learned_get_grads": ([P, P], I),
        "mf_learned_set_margin": ([P, ctypes.c_float], I),
        "mf_learned_forward": ([P, P, I, I, SZ, I, I, P, P], I),
        "mf_learned_train_step": ([P, P, P, I, I, SZ, I, I, ctypes.c_float,
                                   ctypes.POINTER(ctypes.c_float), P], I),
        "mf_learned_tile_grid": ([I, I, I, P, IP, IP, IP, IP, IP], I),
        "median_filter_bracketed": ([P, I, I, SZ, I, P, I, P, P, P,
                                     ctypes.POINTER(ctypes.c_ulonglong), P], I),
        "median_filter_learned": ([P, I, I, SZ, I, P, I, P, P,
                                   ctypes.POINTER(ctypes.c_ulonglong), P], I),
        "mf_tune_cache_save": ([ctypes.c_char_p], I),
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


def median_filter_chained(img, fp: Footprint, chain: int, boundary: str = "clamp", out=None,
                          stream=None):
    """median_filter with chained tiles: `chain` tiles of a tile column per
    workgroup, top to bottom, each re-ranking the box part it shares with
    the tile above and starting from its forwarded last-row solutions."""
    import torch
    code, es, w, h, stride_bytes = _plane_args(img)
    if out is None:
        out = torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
    elif out.shape != img.shape or out.dtype != img.dtype or out.stride() != img.stride():
        raise ValueError("out must match img in shape, dtype and strides")
    rc = lib().median_filter_chained(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                                     fp.handle, BOUNDARY[boundary], int(chain),
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _check("median_filter_chained", rc)
    return out


def median_filter_noalloc(img, fp: Footprint, out, boundary: str = "clamp", stream=None):
    """median_filter without any device allocation: `out` (same shape, dtype
    and strides as `img`) must be given; span table and sort scratch come
    from the library's fixed per-GPU array (calls that overlap on one GPU
    race on it)."""
    code, es, w, h, stride_bytes = _plane_args(img)
    if out.shape != img.shape or out.dtype != img.dtype or out.stride() != img.stride():
        raise ValueError("out must match img in shape, dtype and strides")
    rc = lib().median_filter_noalloc(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                                     fp.handle, BOUNDARY[boundary],
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _check("median_filter_noalloc", rc)
    return out


MAX_RANK_OUTPUTS = 8


class _RankOutput(ctypes.Structure):
    _fields_ = [("out", ctypes.c_void_p), ("rank", ctypes.c_int), ("rank_map", ctypes.c_void_p),
                ("rank_map_stride_bytes", ctypes.c_size_t)]


def rank_filter(img, fp: Footprint, ranks, boundary: str = "clamp", outs=None, stream=None):
    """Several rank planes of `img` from one ordinal transform per tile.

    `ranks` lists one entry per output plane: an int (a constant zero-based
    rank in [0, N)) or a (h, w) int32 device tensor of per-pixel ranks
    (clamped to [0, N - 1]).  Returns the list of output tensors (`outs`, if
    given, must match `img` in shape, dtype and strides)."""
    import torch
    code, es, w, h, stride_bytes = _plane_args(img)
    ranks = list(ranks)
    if not 1 <= len(ranks) <= MAX_RANK_OUTPUTS:
        raise ValueError(f"1..{MAX_RANK_OUTPUTS} rank planes per call")
    if outs is None:
        outs = [torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
                for _ in ranks]
    if len(outs) != len(ranks):
        raise ValueError("one output per rank entry")
    arr = (_RankOutput * len(ranks))()
    for q, (rk, o) in enumerate(zip(ranks, outs)):
        if o.shape != img.shape or o.dtype != img.dtype or o.stride() != img.stride():
            raise ValueError("outputs must match img in shape, dtype and strides")
        if isinstance(rk, int):
            arr[q] = _RankOutput(o.data_ptr(), int(rk), None, 0)
        else:
            if rk.dtype != torch.int32 or tuple(rk.shape) != (h, w) or not rk.is_cuda:
                raise ValueError("a rank map is an int32 (h, w) device tensor")
            if rk.stride(1) != 1:
                raise ValueError("rank map rows must be contiguous")
            arr[q] = _RankOutput(o.data_ptr(), 0, rk.data_ptr(),
                                 rk.stride(0) * 4 if h > 1 else w * 4)
    rc = lib().median_filter_ranks(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                                   fp.handle, BOUNDARY[boundary], ctypes.cast(arr, ctypes.c_void_p),
                                   len(ranks), _stream_ptr(stream))
    _check("median_filter_ranks", rc)
    return outs


def rank_map_filter(img, fp: Footprint, rank_map, boundary: str = "clamp", out=None,
                    stream=None):
    """One plane whose rank varies per pixel (int32 (h, w) device tensor,
    clamped to [0, N - 1]); returns `out`."""
    import torch
    code, es, w, h, stride_bytes = _plane_args(img)
    if out is None:
        out = torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
    elif out.shape != img.shape or out.dtype != img.dtype or out.stride() != img.stride():
        raise ValueError("out must match img in shape, dtype and strides")
    if rank_map.dtype != torch.int32 or tuple(rank_map.shape) != (h, w) or not rank_map.is_cuda:
        raise ValueError("a rank map is an int32 (h, w) device tensor")
    if rank_map.stride(1) != 1:
        raise ValueError("rank map rows must be contiguous")
    rc = lib().median_filter_rank_map(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                                      fp.handle, BOUNDARY[boundary],
                                      ctypes.c_void_p(rank_map.data_ptr()),
                                      rank_map.stride(0) * 4 if h > 1 else w * 4,
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _check("median_filter_rank_map", rc)
    return out


class _WindowOutput(ctypes.Structure):
    _fields_ = [("out", ctypes.c_void_p), ("footprint", ctypes.c_void_p), ("rank", ctypes.c_int),
                ("rank_map", ctypes.c_void_p), ("rank_map_stride_bytes", ctypes.c_size_t)]


def window_filter(img, windows, boundary: str = "clamp", outs=None, stream=None):
    """Planes of `img` over several windows from one ordinal transform per tile.

    `windows` lists one entry per output plane: a Footprint (its median), or
    a (Footprint, rank) pair where rank is an int (zero-based, < N of that
    footprint; negative: the median) or a (h, w) int32 device tensor of
    per-pixel ranks (clamped to [0, N - 1]).  Returns the list of output
    tensors (`outs`, if given, must match `img` in shape, dtype and strides).
    Each plane equals the single-window filter of the same footprint and rank.
    Windows whose boxes are of similar size share one ordinal transform per
    tile; the others run in passes of their own (set_window_fusion)."""
    import torch
    code, es, w, h, stride_bytes = _plane_args(img)
    windows = [wi if isinstance(wi, tuple) else (wi, -1) for wi in windows]
    if not 1 <= len(windows) <= MAX_RANK_OUTPUTS:
        raise ValueError(f"1..{MAX_RANK_OUTPUTS} planes per call")
    if outs is None:
        outs = [torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
                for _ in windows]
    if len(outs) != len(windows):
        raise ValueError("one output per window")
    arr = (_WindowOutput * len(windows))()
    for q, ((fp, rk), o) in enumerate(zip(windows, outs)):
        if o.shape != img.shape or o.dtype != img.dtype or o.stride() != img.stride():
            raise ValueError("outputs must match img in shape, dtype and strides")
        if isinstance(rk, int):
            arr[q] = _WindowOutput(o.data_ptr(), fp.handle, int(rk), None, 0)
        else:
            if rk.dtype != torch.int32 or tuple(rk.shape) != (h, w) or not rk.is_cuda:
                raise ValueError("a rank map is an int32 (h, w) device tensor")
            if rk.stride(1) != 1:
                raise ValueError("rank map rows must be contiguous")
            arr[q] = _WindowOutput(o.data_ptr(), fp.handle, 0, rk.data_ptr(),
                                   rk.stride(0) * 4 if h > 1 else w * 4)
    rc = lib().median_filter_windows(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes, code,
                                     BOUNDARY[boundary], ctypes.cast(arr, ctypes.c_void_p),
                                     len(windows), _stream_ptr(stream))
    _check("median_filter_windows", rc)
    return outs


def set_window_fusion(all_in_one_pass: bool):
    """window_filter: one pass for all windows (True) or the default grouping
    by box size (False).  Process-wide."""
    lib().mf_set_window_fusion(1 if all_in_one_pass else 0)


def set_tile_override(tile_w: int = 0, tile_h: int = 0):
    _check("mf_set_tile_override", lib().mf_set_tile_override(int(tile_w), int(tile_h)))


def release_scratch():
    """Free the scratch buffers the filters cache per (device, stream); waits
    for the devices to go idle."""
    _check("mf_release_scratch", lib().mf_release_scratch())


def work_counters(enable: int):
    """enable=1: start (and zero) the device work counters; 0: stop; -1: read
    them -> [blocks scanned, seeds, clk sort, clk rows, clk sweeps, waves, lane groups,
    pixels ranked, clk seeds, clk load]."""
    buf = (ctypes.c_ulonglong * 10)()
    _check("mf_work_counters", lib().mf_work_counters(int(enable),
                                                      ctypes.cast(buf, ctypes.c_void_p)))
    return list(buf) if enable < 0 else None


def autotune(img, fp: Footprint, boundary: str = "clamp", out=None, reps: int = 3, stream=None):
    """Time every tile shape for this dtype and footprint on `img`; the
    fastest is used by later calls.  Returns (tile_w, tile_h, ms)."""
    import torch
    code, es, w, h, stride_bytes = _plane_args(img)
    if out is None:
        out = torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
    tw, th, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    _check("mf_autotune", lib().mf_autotune(ctypes.c_void_p(img.data_ptr()), w, h, stride_bytes,
                                            code, fp.handle, BOUNDARY[boundary],
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream),
                                            int(reps), ctypes.byref(tw), ctypes.byref(th),
                                            ctypes.byref(ms)))
    return tw.value, th.value, ms.value


def tune_cache_load(path: str):
    _check("mf_tune_cache_load", lib().mf_tune_cache_load(path.encode()))


def tune_cache_save(path: str):
    _check("mf_tune_cache_save", lib().mf_tune_cache_save(path.encode()))


def query_plan(w: int, h: int, dtype: int, fp: Footprint):
    vals = [ctypes.c_int() for _ in range(5)]
    _check("mf_query_plan", lib().mf_query_plan(w, h, dtype, fp.handle,
                                                *[ctypes.byref(v) for v in vals]))
    return dict(zip(("tile_w", "tile_h", "box_w", "box_h", "lds_bytes"), (v.value for v in vals)))


class _ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("w", ctypes.c_int),
                ("h", ctypes.c_int), ("stride_bytes", ctypes.c_size_t), ("dtype", ctypes.c_int),
                ("fp", ctypes.c_void_p), ("boundary", ctypes.c_int)]


def _descs(items):
    arr = (_ImageDesc * max(1, len(items)))()
    for i, (img, out, fp, boundary) in enumerate(items):
        code, es, w, h, stride_bytes = _plane_args(img)
        if out.shape != img.shape or out.dtype != img.dtype or out.stride() != img.stride():
            raise ValueError("out must match img in shape, dtype and strides")
        arr[i] = _ImageDesc(img.data_ptr(), out.data_ptr(), w, h, stride_bytes, code, fp.handle,
                            BOUNDARY[boundary])
    return arr


class BatchPlan:
    """A persistent batched launch over many (img, out, footprint, boundary)
    entries; keep the tensors and footprints alive as long as the plan."""

    def __init__(self, items, tune_cache: str | None = None):
        self.items = list(items)
        self._arr = _descs(self.items)
        h = ctypes.c_void_p()
        _check("mf_plan_create", lib().mf_plan_create(
            ctypes.cast(self._arr, ctypes.c_void_p), len(self.items),
            tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check("mf_plan_launch", lib().mf_plan_launch(self._h, _stream_ptr(stream)))

    def capture(self, stream):
        _check("mf_plan_capture", lib().mf_plan_capture(self._h, _stream_ptr(stream)))

    def replay(self, stream):
        _check("mf_plan_replay", lib().mf_plan_replay(self._h, _stream_ptr(stream)))

    def info(self):
        t, g, l = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        s = ctypes.c_longlong()
        _check("mf_plan_info", lib().mf_plan_info(self._h, ctypes.byref(t), ctypes.byref(g),
                                                  ctypes.byref(l), ctypes.byref(s)))
        ng, ns = ctypes.c_int(), ctypes.c_int()
        _check("mf_plan_groups", lib().mf_plan_groups(self._h, ctypes.byref(ng), ctypes.byref(ns)))
        return dict(tiles=t.value, grid=g.value, lds_bytes=l.value, scratch_bytes=s.value,
                    groups=ng.value, streams=ns.value)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.mf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def plan_autotune(items, reps: int = 3, stream=None):
    """Batch-aware tuning of the tuned-shape table for this batch (see the
    header): returns (batch ms before, batch ms after, shapes dropped)."""
    arr = _descs(items)
    b, a = ctypes.c_float(), ctypes.c_float()
    d = ctypes.c_int()
    _check("mf_plan_autotune", lib().mf_plan_autotune(ctypes.cast(arr, ctypes.c_void_p), len(items),
                                                       _stream_ptr(stream), int(reps),
                                                       ctypes.byref(b), ctypes.byref(a),
                                                       ctypes.byref(d)))
    return b.value, a.value, d.value


def median_filter_batched(items, stream=None):
    """Filter every (img, out, footprint, boundary) entry in one persistent launch."""
    arr = _descs(list(items))
    _check("median_filter_batched", lib().median_filter_batched(
        ctypes.cast(arr, ctypes.c_void_p), len(items), _stream_ptr(stream)))


# ---------------------------------------------------------------------------
# Bracket-proposal CNN kernels (include/mf_cnn.h)
# ---------------------------------------------------------------------------

def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class cnn:
    """Thin wrappers of the CNN kernels; tensors are device tensors whose
    dtype holds the right bytes (bf16 data may be passed as torch.bfloat16
    or as raw uint16)."""

    @staticmethod
    def mfma_probe(a, b, d, stream=None):
        _check("mf_mfma_probe", lib().mf_mfma_probe(_p(a), _p(b), _p(d), _stream_ptr(stream)))

    @staticmethod
    def conv_forward(x, H, W, w, bias, cout, mode, y, mask=None, stream=None):
        _check("mf_cnn_conv_forward", lib().mf_cnn_conv_forward(
            _p(x), H, W, _p(w), _p(bias), cout, mode, _p(mask), _p(y), _stream_ptr(stream)))

    @staticmethod
    def flip_weights(w, cout, wf, stream=None):
        _check("mf_cnn_flip_weights", lib().mf_cnn_flip_weights(_p(w), cout, _p(wf),
                                                                 _stream_ptr(stream)))

    @staticmethod
    def wgrad_workspace(H, W, cout, segs_per_block=8):
        return int(lib().mf_cnn_wgrad_workspace(H, W, cout, segs_per_block))

    @staticmethod
    def conv_wgrad(x, dy, H, W, cout, workspace, dw, db, segs_per_block=8, stream=None):
        _check("mf_cnn_conv_wgrad", lib().mf_cnn_conv_wgrad(
            _p(x), _p(dy), H, W, cout, segs_per_block, _p(workspace), _p(dw), _p(db),
            _stream_ptr(stream)))

    @staticmethod
    def pinball(out, out_ch, tgt, ncell, tau_lo, tau_hi, dout, part_loss, stream=None):
        _check("mf_cnn_pinball", lib().mf_cnn_pinball(_p(out), out_ch, _p(tgt), ncell, tau_lo,
                                                      tau_hi, _p(dout), _p(part_loss),
                                                      _stream_ptr(stream)))

    @staticmethod
    def features(img, radius, feat, stream=None):
        code, es, w, h, sb = _plane_args(img)
        _check("mf_cnn_features", lib().mf_cnn_features(_p(img), w, h, sb, code, radius,
                                                        _p(feat), _stream_ptr(stream)))

    @staticmethod
    def net_forward(img, radius, weights, biases, out, stream=None):
        """The four-layer network in one launch: weights[l] bf16 and
        biases[l] f32 device tensors (cout 32, 32, 32, 16), out f32
        [ceil(h/8)][ceil(w/8)][16]."""
        code, es, w, h, sb = _plane_args(img)
        wl = (ctypes.c_void_p * 4)(*[_p(t) for t in weights])
        bl = (ctypes.c_void_p * 4)(*[_p(t) for t in biases])
        _check("mf_cnn_net_forward", lib().mf_cnn_net_forward(
            _p(img), w, h, sb, code, int(radius), ctypes.cast(wl, ctypes.c_void_p),
            ctypes.cast(bl, ctypes.c_void_p), _p(out), _stream_ptr(stream)))

    @staticmethod
    def targets(med, tgt, stream=None):
        code, es, w, h, sb = _plane_args(med)
        _check("mf_cnn_targets", lib().mf_cnn_targets(_p(med), w, h, sb, code, _p(tgt),
                                                      _stream_ptr(stream)))

    @staticmethod
    def adam(p, m, v, grad, lr, step, p_bf16=None, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        _check("mf_cnn_adam", lib().mf_cnn_adam(_p(p), _p(m), _p(v), _p(grad), p.numel(), lr, b1,
                                                b2, eps, step, _p(p_bf16), _stream_ptr(stream)))


class LearnedNet:
    """The bracket-proposal network (parameters, Adam state, workspace)."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check("mf_learned_create", lib().mf_learned_create(int(seed), ctypes.byref(h)))
        self._h = h

    @classmethod
    def load(cls, path: str):
        """A network from an .npz written by train_bracket (params, margin)."""
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            params = z["params"]
            margin = float(z["margin"])
        net = cls(seed=0)
        net.set_params(params)
        net.set_margin(margin)
        net.margin = margin
        return net

    @staticmethod
    def param_count():
        return int(lib().mf_learned_param_count())

    def get_params(self):
        import numpy as np
        a = np.empty(self.param_count(), dtype=np.float32)
        _check("mf_learned_get_params", lib().mf_learned_get_params(self._h,
                                                                    a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def get_grads(self):
        import numpy as np
        a = np.empty(self.param_count(), dtype=np.float32)
        _check("mf_learned_get_grads", lib().mf_learned_get_grads(self._h,
                                                                  a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def set_params(self, a):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        assert a.size == self.param_count()
        _check("mf_learned_set_params", lib().mf_learned_set_params(
            self._h, a.ctypes.data_as(ctypes.c_void_p)))

    def set_margin(self, margin: float):
        _check("mf_learned_set_margin", lib().mf_learned_set_margin(self._h, float(margin)))

    def forward(self, img, radius: int, out_cells=None, stream=None):
        import torch
        code, es, w, h, sb = _plane_args(img)
        if out_cells is None:
            out_cells = torch.empty(((h + 7) // 8, (w + 7) // 8, 16), dtype=torch.float32,
                                    device=img.device)
        _check("mf_learned_forward", lib().mf_learned_forward(
            self._h, _p(img), w, h, sb, code, int(radius), _p(out_cells), _stream_ptr(stream)))
        return out_cells

    def train_step(self, img, median, radius: int, lr: float, stream=None):
        code, es, w, h, sb = _plane_args(img)
        loss = ctypes.c_float()
        _check("mf_learned_train_step", lib().mf_learned_train_step(
            self._h, _p(img), _p(median), w, h, sb, code, int(radius), float(lr),
            ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value

    def filter(self, img, fp: Footprint, boundary: str = "clamp", out=None, stream=None,
               count_fallback: bool = True):
        """Exact median via learned brackets; returns (out, fallback_pixels).
        With count_fallback=False the call stays asynchronous and the count
        is None."""
        import torch
        code, es, w, h, sb = _plane_args(img)
        if out is None:
            out = torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
        fb = ctypes.c_ulonglong()
        _check("median_filter_learned", lib().median_filter_learned(
            _p(img), w, h, sb, code, fp.handle, BOUNDARY[boundary], self._h, _p(out),
            ctypes.byref(fb) if count_fallback else None, _stream_ptr(stream)))
        return out, (fb.value if count_fallback else None)

    def filter_bracketed(self, img, fp: Footprint, brackets, boundary: str = "clamp", out=None,
                         stream=None):
        """Exact median with caller-supplied per-tile brackets (device uint32 [tiles][2])."""
        import torch
        code, es, w, h, sb = _plane_args(img)
        if out is None:
            out = torch.empty_strided(img.shape, img.stride(), dtype=img.dtype, device=img.device)
        fb = ctypes.c_ulonglong()
        _check("median_filter_bracketed", lib().median_filter_bracketed(
            _p(img), w, h, sb, code, fp.handle, BOUNDARY[boundary], _p(brackets), self._h,
            _p(out), ctypes.byref(fb), _stream_ptr(stream)))
        return out, fb.value

    @staticmethod
    def tile_grid(w: int, h: int, dtype: int, fp: Footprint, with_capacity: bool = False):
        """(tiles_x, tiles_y) of the bracketed filters; with_capacity also
        returns the most in-bracket box pixels a tile can rank."""
        tx, ty, cap = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check("mf_learned_tile_grid", lib().mf_learned_tile_grid(w, h, dtype, fp.handle,
                                                                  ctypes.byref(tx),
                                                                  ctypes.byref(ty),
                                                                  ctypes.byref(cap), None, None))
        return (tx.value, ty.value, cap.value) if with_capacity else (tx.value, ty.value)

    @staticmethod
    def tile_shape(w: int, h: int, dtype: int, fp: Footprint):
        """(tile_w, tile_h) of the bracketed filters' output tiles."""
        tw, th = ctypes.c_int(), ctypes.c_int()
        _check("mf_learned_tile_grid", lib().mf_learned_tile_grid(w, h, dtype, fp.handle, None,
                                                                  None, None, ctypes.byref(tw),
                                                                  ctypes.byref(th)))
        return tw.value, th.value

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.mf_learned_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
