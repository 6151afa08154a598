"""CPU oracle for exact rank-order filtering (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
use this package.  It shares no code with the GPU library and does not import
it.  Two implementations live here:

* ``filter`` / ``filter_points``: the C++ brute force in
  ``median_oracle.cpp`` (gather the window, take the rank-k element with
  std::nth_element under the dtype's total order), OpenMP over rows.
* ``tiny_filter``: a numpy full sort of every window, for small inputs, used
  to pin the C++ oracle.

Both follow the definition in the paper's "Core concepts" passage: the median
is the element of zero-based rank (N-1)/2 of the window's values.  Any other
rank, constant or given per pixel by a rank map (the Conclusion's percentile
filtering, with the percentile free to vary across the image), is the same
selection at that rank; a map entry outside [0, N) is clamped to it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import footprints  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "median_oracle.cpp")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libmforacle.so")

DTYPE_CODE = {"u8": 0, "u16": 1, "f32": 2}
BOUNDARY_CODE = {"clamp": 0, "mirror": 1}
_NP = {"u8": np.uint8, "u16": np.uint16, "f32": np.float32}

_lib = None


def build(force: bool = True) -> str:
    """Compile the C++ oracle into oracle/_build/libmforacle.so."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L = ctypes.c_longlong
        lib.oracle_filter.argtypes = [P, I, I, L, I, P, P, I, I, I, P, L, I]
        lib.oracle_filter_points.argtypes = [P, I, I, L, I, P, P, I, I, I, P, P, I, P, I]
        lib.oracle_filter_rank_map.argtypes = [P, I, I, L, I, P, P, I, P, L, I, P, L, I]
        lib.oracle_filter_points_ranks.argtypes = [P, I, I, L, I, P, P, I, P, I, P, P, I, P, I]
        lib.oracle_remap.argtypes = [I, I, I]
        lib.oracle_total_order_less.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.oracle_ordinal_transform.argtypes = [P, I, I, P, P, P]
        _lib = lib
    return _lib


def dtype_name(arr: np.ndarray) -> str:
    for k, v in _NP.items():
        if arr.dtype == v:
            return k
    raise TypeError(f"unsupported dtype {arr.dtype}")


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def _offsets(fp):
    fp = np.ascontiguousarray(np.asarray(fp, dtype=np.int32).reshape(-1, 2))
    dx = np.ascontiguousarray(fp[:, 0])
    dy = np.ascontiguousarray(fp[:, 1])
    return dx, dy


def filter(img: np.ndarray, fp, boundary: str = "clamp", rank: int | None = None,
           nthreads: int | None = None, rank_map: np.ndarray | None = None) -> np.ndarray:
    """Rank-order filter a 2-D plane; fp is an (N, 2) array of (dx, dy) offsets.

    rank_map (int32, same shape): a rank per output pixel, entries outside
    [0, N) clamped to it (the window minimum or maximum); overrides `rank`.
    """
    img = np.ascontiguousarray(img)
    if img.ndim != 2:
        raise ValueError("expected a 2-D plane")
    dt = dtype_name(img)
    dx, dy = _offsets(fp)
    n = len(dx)
    k = (n - 1) // 2 if rank is None else int(rank)
    out = np.empty_like(img)
    h, w = img.shape
    if rank_map is not None:
        rm = np.ascontiguousarray(rank_map, dtype=np.int32)
        if rm.shape != img.shape:
            raise ValueError("rank_map must have the image's shape")
        rc = _load().oracle_filter_rank_map(img.ctypes.data, w, h, w, DTYPE_CODE[dt],
                                            dx.ctypes.data, dy.ctypes.data, n, rm.ctypes.data,
                                            w, BOUNDARY_CODE[boundary], out.ctypes.data, w,
                                            nthreads or default_threads())
    else:
        rc = _load().oracle_filter(img.ctypes.data, w, h, w, DTYPE_CODE[dt], dx.ctypes.data,
                                   dy.ctypes.data, n, k, BOUNDARY_CODE[boundary],
                                   out.ctypes.data, w, nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_filter rejected its arguments")
    return out


def filter_points(img: np.ndarray, fp, xs, ys, boundary: str = "clamp",
                  rank: int | None = None, nthreads: int | None = None,
                  ranks=None) -> np.ndarray:
    """Rank-order filter only at the listed pixels; returns a 1-D array.
    ranks: optional rank per listed pixel (clamped to [0, N)), overriding
    `rank`."""
    img = np.ascontiguousarray(img)
    dt = dtype_name(img)
    dx, dy = _offsets(fp)
    n = len(dx)
    k = (n - 1) // 2 if rank is None else int(rank)
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.int32))
    vals = np.empty(len(xs), dtype=img.dtype)
    h, w = img.shape
    if ranks is not None:
        ks = np.ascontiguousarray(np.clip(np.asarray(ranks, dtype=np.int64),
                                          -2**31, 2**31 - 1).astype(np.int32))
        if ks.shape != xs.shape:
            raise ValueError("one rank per listed pixel")
        rc = _load().oracle_filter_points_ranks(img.ctypes.data, w, h, w, DTYPE_CODE[dt],
                                                dx.ctypes.data, dy.ctypes.data, n,
                                                ks.ctypes.data, BOUNDARY_CODE[boundary],
                                                xs.ctypes.data, ys.ctypes.data, len(xs),
                                                vals.ctypes.data, nthreads or default_threads())
    else:
        rc = _load().oracle_filter_points(img.ctypes.data, w, h, w, DTYPE_CODE[dt],
                                          dx.ctypes.data, dy.ctypes.data, n, k,
                                          BOUNDARY_CODE[boundary], xs.ctypes.data,
                                          ys.ctypes.data, len(xs), vals.ctypes.data,
                                          nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_filter_points rejected its arguments")
    return vals


def remap(x: int, n: int, boundary: str) -> int:
    return _load().oracle_remap(int(x), int(n), BOUNDARY_CODE[boundary])


def total_order_less(a_bits: int, b_bits: int) -> bool:
    return bool(_load().oracle_total_order_less(int(a_bits), int(b_bits)))


def ordinal_transform(vals: np.ndarray):
    """Stable ordinal transform of a 1-D array: returns (C, omega, ordinal)."""
    vals = np.ascontiguousarray(vals)
    dt = dtype_name(vals)
    n = vals.size
    C = np.empty(n, dtype=vals.dtype)
    omega = np.empty(n, dtype=np.int32)
    ordinal = np.empty(n, dtype=np.int32)
    rc = _load().oracle_ordinal_transform(vals.ctypes.data, n, DTYPE_CODE[dt], C.ctypes.data,
                                          omega.ctypes.data, ordinal.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_ordinal_transform rejected its arguments")
    return C, omega, ordinal


# ---------------------------------------------------------------------------
# numpy full-sort oracle for small inputs
# ---------------------------------------------------------------------------

def _np_remap(idx: np.ndarray, n: int, boundary: str) -> np.ndarray:
    if boundary == "clamp":
        return np.clip(idx, 0, n - 1)
    if n == 1:
        return np.zeros_like(idx)
    period = 2 * (n - 1)
    m = np.mod(idx, period)
    return np.where(m >= n, period - m, m)


def _sort_keys_f32(vals: np.ndarray) -> np.ndarray:
    """Order key for float32 without NaN: ascending by value, -0 before +0.

    Built with a lexicographic sort (value first, then sign), not with the
    bit-flipping key transform, so it is an independent route to totalOrder.
    """
    flat = vals.reshape(-1)
    order = np.lexsort((~np.signbit(flat), flat.astype(np.float64)))
    ranks = np.empty(flat.size, dtype=np.int64)
    ranks[order] = np.arange(flat.size)
    return ranks.reshape(vals.shape)


def tiny_filter(img: np.ndarray, fp, boundary: str = "clamp",
                rank: int | None = None, rank_map: np.ndarray | None = None) -> np.ndarray:
    """Full np.sort of every window.  Small images only (memory h*w*N).
    rank_map: a rank per pixel, clamped to [0, N)."""
    img = np.asarray(img)
    h, w = img.shape
    fp = np.asarray(fp).reshape(-1, 2)
    n = len(fp)
    k = (n - 1) // 2 if rank is None else int(rank)
    if rank_map is not None:
        k = np.clip(np.asarray(rank_map, dtype=np.int64), 0, n - 1)[:, :, None]
    ys = np.arange(h)[:, None, None] + fp[None, None, :, 1]
    xs = np.arange(w)[None, :, None] + fp[None, None, :, 0]
    ys = _np_remap(ys, h, boundary)
    xs = _np_remap(xs, w, boundary)
    win = img[np.broadcast_to(ys, (h, w, n)), np.broadcast_to(xs, (h, w, n))]
    if img.dtype == np.float32:
        if np.isnan(img).any():
            raise ValueError("tiny_filter does not order NaN")
        keys = _sort_keys_f32(img)
        kwin = keys[np.broadcast_to(ys, (h, w, n)), np.broadcast_to(xs, (h, w, n))]
        order = np.argsort(kwin, axis=2, kind="stable")
        if rank_map is None:
            pos = order[:, :, k]
        else:
            pos = np.take_along_axis(order, k, axis=2)[:, :, 0]
        return np.ascontiguousarray(np.take_along_axis(win, pos[:, :, None], axis=2)[:, :, 0])
    srt = np.sort(win, axis=2)
    if rank_map is None:
        return np.ascontiguousarray(srt[:, :, k])
    return np.ascontiguousarray(np.take_along_axis(srt, k, axis=2)[:, :, 0])
