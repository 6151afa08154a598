"""CPU checks of the per-element tolerance used by the CNN chain's GPU parity
tests (tests/cnn_bounds.py): a float32/bf16 emulation of the GPU's
arithmetic, written independently with numpy float32 products in another
summation order, stays within the bounds; the bounds are 0 on most elements
(so they are not vacuous); and mistakes planted in the emulation -- one cell's
ReLU mask flipped, one weight tap moved -- exceed them."""

import numpy as np
import pytest

import workloads
from oracle import cnn as OC
from tests import cnn_bounds as CB

F32 = np.float32


def bf(a):
    return OC.bf16_round(np.asarray(a, dtype=np.float32))


def conv32(x, w, b):
    """float32 'same' 3x3 correlation: per-tap float32 matrix products summed in float32."""
    H, W_, _ = x.shape
    xp = np.zeros((H + 2, W_ + 2, x.shape[2]), dtype=F32)
    xp[1:-1, 1:-1] = x.astype(F32)
    y = np.zeros((H, W_, w.shape[0]), dtype=F32)
    for ky in (2, 0, 1):
        for kx in (1, 2, 0):
            y += xp[ky:ky + H, kx:kx + W_] @ w[:, ky, kx, :].T.astype(F32)
    return y + b.astype(F32)


def dgrad32(d, w):
    H, W_, _ = d.shape
    dxp = np.zeros((H + 2, W_ + 2, w.shape[3]), dtype=F32)
    for ky in range(3):
        for kx in range(3):
            dxp[ky:ky + H, kx:kx + W_] += d.astype(F32) @ w[:, ky, kx, :].astype(F32)
    return dxp[1:-1, 1:-1]


def wgrad32(x, d):
    H, W_, C = x.shape
    xp = np.zeros((H + 2, W_ + 2, C), dtype=F32)
    xp[1:-1, 1:-1] = x.astype(F32)
    dw = np.zeros((d.shape[2], 3, 3, C), dtype=F32)
    for ky in range(3):
        for kx in range(3):
            pa = xp[ky:ky + H, kx:kx + W_].reshape(-1, C)
            dw[:, ky, kx, :] = d.reshape(-1, d.shape[2]).astype(F32).T @ pa
    return dw, d.astype(F32).sum(axis=(0, 1))


def emulate(img, radius, med, Ws, bs, plant=None):
    """The GPU's chain in float32 with bf16 stores.  plant: None, 'mask'
    (one cell's mask flipped in layer 2's backward) or 'tap' (layer 1's
    backward-data weights shifted by one tap)."""
    Hc, Wc = -(-img.shape[0] // 8), -(-img.shape[1] // 8)
    f = np.zeros((Hc, Wc, 32), dtype=F32)
    inv = F32(1.0) / F32(65535.0)
    for i in range(Hc):
        for j in range(Wc):
            blk = img[8 * i:8 * i + 8, 8 * j:8 * j + 8]
            f[i, j, 0] = F32(blk.astype(F32).sum()) / F32(blk.size) * inv
    f[..., 1] = F32(radius / 64.0)
    h = bf(f)
    acts = []
    for l in range(4):
        acts.append(h)
        pre = conv32(h, Ws[l], bs[l])
        h = bf(np.maximum(pre, 0)) if l < 3 else pre
    out = h
    lo, hi = OC.cell_targets(med, 65535.0)
    d = np.zeros((Hc, Wc, 16), dtype=F32)
    for c, (t, tau) in enumerate(((lo, OC.TAU_LO), (hi, OC.TAU_HI))):
        t32 = (med_cells(med, c) * inv).astype(F32)
        u = t32 - out[..., c]
        d[..., c] = bf(-(F32(tau) - (u < 0).astype(F32)))
    dws, dbs = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        dws[l], dbs[l] = wgrad32(acts[l], d)
        if l == 0:
            break
        w = Ws[l]
        if plant == "tap" and l == 1:
            w = np.roll(w, 1, axis=2)
        dx = dgrad32(d, w)
        mask = acts[l] > 0
        if plant == "mask" and l == 2:
            mask = mask.copy()
            mask[1, 2, :] = ~mask[1, 2, :]
        d = bf(dx * mask)
    return out, dws, dbs


def med_cells(med, c):
    Hc, Wc = -(-med.shape[0] // 8), -(-med.shape[1] // 8)
    r = np.zeros((Hc, Wc), dtype=F32)
    for i in range(Hc):
        for j in range(Wc):
            blk = med[8 * i:8 * i + 8, 8 * j:8 * j + 8].astype(F32)
            r[i, j] = blk.min() if c == 0 else blk.max()
    return r


def chain(seed):
    img = workloads.natural_u16(72, 56, seed=seed)
    Ws, bs, med = CB.chain_case(img, 8, seed)
    fw = CB.forward(img, 8, 65535.0, Ws, bs)
    d, ed = CB.pinball_grad(fw["pre"][3], fw["epre"][3], med, 65535.0)
    assert np.all(ed == 0), "an output is too close to its target"
    return img, med, Ws, bs, fw, d, CB.backward(fw, Ws, d, ed)


@pytest.mark.parametrize("seed", [1, 3, 4])
def test_float32_emulation_within_bounds(seed):
    img, med, Ws, bs, fw, d, (DW, EDW, DB, EDB) = chain(seed)
    out, dws, dbs = emulate(img, 8, med, Ws, bs)
    assert np.all(np.abs(out[..., :2] - fw["pre"][3][..., :2]) <= fw["epre"][3][..., :2])
    for l in range(4):
        assert np.all(np.abs(dws[l] - DW[l]) <= EDW[l]), l
        assert np.all(np.abs(dbs[l] - DB[l]) <= EDB[l]), l
    # both pinball branches and both mask states occur
    assert len(np.unique(d[..., 0])) == 2 and len(np.unique(d[..., 1])) == 2
    for l in range(1, 4):
        on = np.mean(fw["h"][l][..., :32] > 0)
        assert 0.2 < on < 0.8, (l, on)
    # the bounds are tight: measured in units of one cell's share of an
    # entry's magnitude (mdw / ncell), the median bound is below 1/2 and
    # nine in ten entries are below 1, so a term missing or wrong in one
    # cell shows
    ncell = d.shape[0] * d.shape[1]
    for l, mdw in enumerate(CB.magnitudes(fw, Ws, d)):
        live = mdw > 0
        r = EDW[l][live] / mdw[live] * ncell
        assert np.median(r) < 0.5 and np.mean(r < 1) > 0.9, (l, np.median(r), np.mean(r < 1))


@pytest.mark.parametrize("plant", ["mask", "tap"])
def test_planted_mistakes_exceed_bounds(plant):
    img, med, Ws, bs, fw, d, (DW, EDW, DB, EDB) = chain(1)
    _, dws, dbs = emulate(img, 8, med, Ws, bs, plant=plant)
    worst = max(float(np.max(np.abs(dws[l] - DW[l]) - EDW[l])) for l in range(4))
    assert worst > 0, plant
