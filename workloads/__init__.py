"""Seeded synthetic inputs for the median-filter workloads.

This module is shared by the test oracle and the GPU path and therefore holds
no median arithmetic at all: it only draws pixels.  Every generator takes an
explicit seed and uses ``numpy.random.default_rng``.

The paper benchmarks on a 37-megapixel greyscale photograph and illustrates
with photographs (Results section; teaser, rotational-invariance and
percentile figures).  None of those images is available, so these generators
stand in for them with the shapes, value distributions and structure listed
below.

Workloads
---------
``plain_u8_256``      256x256 uint8, i.i.d. uniform 0..255, seed 0.
``natural_u16``       w x h uint16 "natural-like" image: sum of 8 random
                      low-frequency plane waves, min-max scaled to 0..65535,
                      plus Gaussian noise (sigma 800), clipped and rounded,
                      then 5 % salt-and-pepper impulses at 0 / 65535.
                      4096x4096 with seed 1 is the headline workload.
``lognormal_f32``     3 planes of 3840x2160 float32, exp(N(0,1)), with 2 % of
                      pixels replaced by +-1e6 outliers (no NaN), seed 2.
``mixed_batch``       64 images, w,h ~ U{128..2048}, dtype ~ U{u8,u16,f32},
                      disc radius ~ U{1..64}; values uniform over the dtype
                      range (float32: U[0,1)), seed 3.
``uniform_u16``       2048x2048 i.i.d. uniform uint16, seed 4.
``adversarial_u16``   high-frequency 0/65535 checkerboard inside a thick
                      border of mid-grey 32768 (the slow case the paper's
                      limitations section describes).
``percentile_ramp``   int32 rank map for a window of N taps whose percentile
                      runs from 0 % at the left column to 100 % at the right
                      one (the paper's varying-percentile figure): q = x /
                      (w - 1), rank = floor(q * (N - 1) + 1/2).
``random_ranks``      int32 rank map, i.i.d. uniform over -3 .. N + 2 (a few
                      entries outside [0, N) on purpose), seeded.
"""

from __future__ import annotations

import numpy as np

DTYPES = ("u8", "u16", "f32")
NUMPY_DTYPE = {"u8": np.uint8, "u16": np.uint16, "f32": np.float32}


def plain_u8(w: int = 256, h: int = 256, seed: int = 0) -> np.ndarray:
    """i.i.d. uniform uint8 image, shape (h, w)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(h, w), dtype=np.uint8)


def uniform(w: int, h: int, dtype: str, seed: int) -> np.ndarray:
    """i.i.d. uniform image over the dtype's range (float32: U[0,1))."""
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        return rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    if dtype == "u16":
        return rng.integers(0, 65536, size=(h, w), dtype=np.uint16)
    if dtype == "f32":
        return rng.random(size=(h, w), dtype=np.float32)
    raise ValueError(dtype)


def natural_u16(w: int = 4096, h: int = 4096, seed: int = 1,
                n_waves: int = 8, noise_sigma: float = 800.0,
                impulse_frac: float = 0.05) -> np.ndarray:
    """Natural-like uint16 image, shape (h, w).

    Sum of ``n_waves`` plane waves (amplitude U(0.5,1), direction U[0,2pi),
    frequency U(1,8) cycles per image width, phase U[0,2pi)), min-max scaled
    to [0, 65535], plus N(0, sigma^2) noise, clipped and rounded to nearest,
    then a Bernoulli(impulse_frac) mask of pixels set to 0 or 65535 (1/2 each).
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.0, n_waves)
    ang = rng.uniform(0.0, 2 * np.pi, n_waves)
    freq = rng.uniform(1.0, 8.0, n_waves)
    phase = rng.uniform(0.0, 2 * np.pi, n_waves)
    xs = np.arange(w, dtype=np.float64) / w
    ys = (np.arange(h, dtype=np.float64) / w)[:, None]
    img = np.zeros((h, w), dtype=np.float64)
    for a, t, f, p in zip(amp, ang, freq, phase):
        kx = 2 * np.pi * f * np.cos(t)
        ky = 2 * np.pi * f * np.sin(t)
        img += a * np.sin(kx * xs[None, :] + ky * ys + p)
    lo, hi = img.min(), img.max()
    img = (img - lo) * (65535.0 / (hi - lo)) if hi > lo else img * 0.0
    img += rng.normal(0.0, noise_sigma, size=(h, w))
    img = np.rint(np.clip(img, 0.0, 65535.0)).astype(np.uint16)
    hit = rng.random((h, w)) < impulse_frac
    salt = rng.random((h, w)) < 0.5
    img[hit & salt] = 65535
    img[hit & ~salt] = 0
    return img


def lognormal_f32(w: int = 3840, h: int = 2160, planes: int = 3, seed: int = 2,
                  outlier_frac: float = 0.02) -> np.ndarray:
    """Planar float32 stack, shape (planes, h, w): exp(N(0,1)) with +-1e6 outliers."""
    rng = np.random.default_rng(seed)
    img = np.exp(rng.normal(0.0, 1.0, size=(planes, h, w))).astype(np.float32)
    hit = rng.random((planes, h, w)) < outlier_frac
    sign = rng.random((planes, h, w)) < 0.5
    img[hit & sign] = np.float32(1e6)
    img[hit & ~sign] = np.float32(-1e6)
    return img


def mixed_batch_specs(n: int = 64, seed: int = 3, size_lo: int = 128,
                      size_hi: int = 2048, r_lo: int = 1, r_hi: int = 64):
    """Per-image (w, h, dtype, radius, image-seed) for the mixed batch."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        w = int(rng.integers(size_lo, size_hi + 1))
        h = int(rng.integers(size_lo, size_hi + 1))
        dt = DTYPES[int(rng.integers(0, 3))]
        r = int(rng.integers(r_lo, r_hi + 1))
        specs.append(dict(w=w, h=h, dtype=dt, radius=r, seed=seed * 1000 + i))
    return specs


def mixed_batch(n: int = 64, seed: int = 3, **kw):
    """List of (image, spec) for the mixed batch; images are uniform over the dtype range."""
    out = []
    for s in mixed_batch_specs(n, seed, **kw):
        out.append((uniform(s["w"], s["h"], s["dtype"], s["seed"]), s))
    return out


def uniform_u16(w: int = 2048, h: int = 2048, seed: int = 4) -> np.ndarray:
    return uniform(w, h, "u16", seed)


def adversarial_u16(w: int = 1024, h: int = 1024, border: int = 96) -> np.ndarray:
    """0/65535 one-pixel checkerboard inside a ``border``-wide frame of 32768."""
    yy, xx = np.mgrid[0:h, 0:w]
    img = np.where(((xx + yy) & 1) == 0, 0, 65535).astype(np.uint16)
    img[:border, :] = 32768
    img[-border:, :] = 32768
    img[:, :border] = 32768
    img[:, -border:] = 32768
    return img


def binary(w: int, h: int, seed: int, hi: int = 255, p: float = 0.5,
           dtype=np.uint8) -> np.ndarray:
    """Binary noise image with values {0, hi}."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((h, w)) < p, hi, 0).astype(dtype)


def special_floats(w: int, h: int, seed: int) -> np.ndarray:
    """float32 image mixing +-0, +-inf, subnormals and ordinary values (no NaN)."""
    rng = np.random.default_rng(seed)
    pool = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 1e-40, -1e-40,
                     1.0, -1.0, 3.5, -2.25, 1e30, -1e30], dtype=np.float32)
    img = rng.normal(0, 1, size=(h, w)).astype(np.float32)
    pick = rng.random((h, w)) < 0.5
    img[pick] = pool[rng.integers(0, len(pool), size=int(pick.sum()))]
    return img


def percentile_ramp(w: int, h: int, taps: int) -> np.ndarray:
    """Rank map whose percentile grows linearly from 0 (left) to 1 (right);
    the percentile q becomes rank floor(q * (taps - 1) + 1/2)."""
    q = np.arange(w, dtype=np.float64) / max(1, w - 1)
    k = np.floor(q * (taps - 1) + 0.5).astype(np.int32)
    return np.ascontiguousarray(np.broadcast_to(k[None, :], (h, w)))


def random_ranks(w: int, h: int, taps: int, seed: int) -> np.ndarray:
    """Rank map uniform over -3 .. taps + 2 (some entries out of range)."""
    rng = np.random.default_rng(seed)
    return rng.integers(-3, taps + 3, size=(h, w)).astype(np.int32)
