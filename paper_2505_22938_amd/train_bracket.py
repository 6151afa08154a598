"""Train the bracket-proposal network and calibrate its margin.

    python -m paper_2505_22938_amd.train_bracket --out bracket_net.npz
        [--images 512] [--size 512] [--radii 16,32,64] [--epochs 2] [--lr 3e-3]
        [--holdout 16] [--fail-target 0.02] [--seed 4]

Training pairs are method-generated: each image (uint16, alternately the
natural-like generator and i.i.d. uniform values) is filtered exactly by the
library's plain median filter at a radius drawn from --radii, and the
network is trained (library kernels: forward, backward, Adam) to predict, per
8x8 cell, the min and max of the median image over the cell with a pinball
loss.  The margin is then calibrated on held-out images: for every tile the
widening that would make its bracket contain all its medians is measured, and
the margin is set to the (1 - fail_target) quantile of those widenings.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def make_image(i: int, size: int, seed: int):
    import workloads
    s = seed * 100000 + i
    if i % 2 == 0:
        return workloads.natural_u16(size, size, seed=s)
    return workloads.uniform(size, size, "u16", s)


def tile_margins(cells_out: np.ndarray, median: np.ndarray, tw: int, th: int) -> np.ndarray:
    """Per tile: the widening (in full-range units) its cell-union bracket
    needs to contain every median of the tile."""
    h, w = median.shape
    hc, wc = cells_out.shape[:2]
    lo = np.minimum(cells_out[..., 0], cells_out[..., 1])
    hi = np.maximum(cells_out[..., 0], cells_out[..., 1])
    edge = 4   # as the library's bracket kernel: border cells are ignored when possible
    out = []
    for ty in range(0, h, th):
        for tx in range(0, w, tw):
            m = median[ty:ty + th, tx:tx + tw].astype(np.float64) / 65535.0
            r0, r1 = ty // 8, min(hc, (ty + th + 7) // 8)
            c0, c1 = tx // 8, min(wc, (tx + tw + 7) // 8)
            ir0, ir1, ic0, ic1 = max(r0, edge), min(r1, hc - edge), max(c0, edge), min(c1, wc - edge)
            if ir0 < ir1 and ic0 < ic1:
                r0, r1, c0, c1 = ir0, ir1, ic0, ic1
            cl = lo[r0:r1, c0:c1]
            ch = hi[r0:r1, c0:c1]
            need = max(cl.min() - m.min(), m.max() - ch.max(), 0.0)
            out.append(need)
    return np.array(out)


def train(images=512, size=512, radii=(16, 32, 64), epochs=2, lr=3e-3, holdout=16,
          fail_target=0.02, seed=4, log=print):
    import torch

    import paper_2505_22938_amd as mf

    net = mf.LearnedNet(seed=seed)
    fps = {r: mf.Footprint.disc(r) for r in radii}
    rng = np.random.default_rng(seed)
    pairs = []
    t0 = time.time()
    for i in range(images):
        img = torch.from_numpy(make_image(i, size, seed)).cuda()
        r = int(rng.choice(radii))
        med = mf.median_filter(img, fps[r], "clamp")
        pairs.append((img, med, r))
    torch.cuda.synchronize()
    log(f"# {images} training pairs ({size}x{size}) in {time.time() - t0:.1f}s")
    step = 0
    nsteps = epochs * images
    losses = []
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(images)
        for j in order:
            img, med, r = pairs[j]
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / nsteps))   # cosine decay
            losses.append(net.train_step(img, med, r, max(lr_t, lr * 0.02)))
            step += 1
        log(f"# epoch {ep}: mean loss {np.mean(losses[-images:]):.5f}")
    log(f"# {nsteps} steps in {time.time() - t0:.1f}s")
    # margin calibration on held-out images
    need = []
    for i in range(holdout):
        img_np = make_image(images + i, size, seed + 1)
        img = torch.from_numpy(img_np).cuda()
        for r in radii:
            med = mf.median_filter(img, fps[r], "clamp")
            cells = net.forward(img, r)
            torch.cuda.synchronize()
            try:
                mf.LearnedNet.tile_grid(size, size, mf.MF_U16, fps[r])
            except mf.MedianFilterError:
                continue   # no bracketed plan for this footprint
            tw, th = mf.LearnedNet.tile_shape(size, size, mf.MF_U16, fps[r])
            need.append(tile_margins(cells.cpu().numpy(), med.cpu().numpy(), tw, th))
    need = np.concatenate(need) if need else np.zeros(1)
    margin = float(np.quantile(need, 1.0 - fail_target))
    log(f"# margin {margin:.5f} (quantile {1 - fail_target:.3f} of {need.size} held-out tiles)")
    params = net.get_params()
    net.close()
    return params, margin, losses


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--images", type=int, default=512)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--radii", default="16,32,64")
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--holdout", type=int, default=16)
    ap.add_argument("--fail-target", type=float, default=0.02)
    ap.add_argument("--seed", type=int, default=4)
    a = ap.parse_args()
    radii = tuple(int(r) for r in a.radii.split(","))
    params, margin, losses = train(a.images, a.size, radii, a.epochs, a.lr, a.holdout,
                                   a.fail_target, a.seed)
    meta = dict(images=a.images, size=a.size, radii=list(radii), epochs=a.epochs, lr=a.lr,
                seed=a.seed, fail_target=a.fail_target, final_loss=float(np.mean(losses[-64:])))
    np.savez(a.out, params=params, margin=np.float32(margin), meta=json.dumps(meta))
    print(json.dumps(dict(out=a.out, margin=margin, **meta)))


if __name__ == "__main__":
    main()
