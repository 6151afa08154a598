"""Train the bracket-proposal network and calibrate its margin.

    python -m paper_2505_22938_amd.train_bracket --out bracket_net.npz
        [--images 512] [--size 512] [--radii 16,32,64] [--epochs 2] [--lr 3e-3]
        [--holdout 8] [--calibration-size 2048] [--fail-target 0.0005] [--seed 4]

Training pairs are method-generated: each image (uint16, alternately the
natural-like generator and i.i.d. uniform values) is filtered exactly by the
library's plain median filter at a radius drawn from --radii, and the
network is trained (library kernels: forward, backward, Adam) to predict, per
8x8 cell, the min and max of the median image over the cell with a pinball
loss.  The margin is then calibrated on held-out images: for every output
pixel of a tile the filter would rank in the bracketed layout (cell-union
bracket at most 0.3 of the range and holding at most a quarter of the tile's
box), the widening that would make the tile's bracket contain the pixel's
median is measured, and the margin is set to the (1 - fail_target) quantile
of those widenings (fail_target: the fraction of such pixels left to the
per-pixel recompute).

    python -m paper_2505_22938_amd.train_bracket --calibrate-only WEIGHTS --out OUT
        recalibrates the margin of existing weights the same way.
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


def tile_margins(cells_out: np.ndarray, median: np.ndarray, tw: int, th: int,
                 img: np.ndarray | None = None, radius: int = 0) -> np.ndarray:
    """Per output pixel: the widening (in full-range units) its tile's
    cell-union bracket needs to contain the pixel's median.  With the input
    image, the pixels of tiles
    that the filter never ranks in the bracketed layout whatever the margin
    are left out: a cell-union bracket wider than 0.3 of the range (the
    bracket is dropped) or one that already holds more than a quarter of the
    tile's box (clamp boundary, the window extent `radius`; the tile goes to
    the plain pass)."""
    h, w = median.shape
    pad = None
    if img is not None:
        pad = np.pad(img, ((radius, radius + th), (radius, radius + tw)), mode="edge")
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
            if pad is not None:
                blo, bhi = float(cl.min()), float(ch.max())
                if bhi - blo > 0.3:
                    continue
                box = pad[ty:ty + th + 2 * radius, tx:tx + tw + 2 * radius] / 65535.0
                if ((box >= blo) & (box <= bhi)).sum() > box.size / 4:
                    continue
            need = np.maximum(np.maximum(cl.min() - m, m - ch.max()), 0.0)
            out.append(need.ravel())
    return np.concatenate(out) if out else np.zeros(0)


def calibrate(net, images, radii, holdout, size, seed, fail_target, log=print):
    """The bracket margin: on held-out images (the training generator with
    seed + 1, numbered after the `images` training images), the widening
    each pixel's tile bracket needs to hold the pixel's median, at the
    (1 - fail_target) quantile over the pixels of tiles that can be
    bracketed: fail_target is the fraction of those pixels whose median
    escapes and is recomputed on its own."""
    import torch

    import paper_2505_22938_amd as mf

    fps = {r: mf.Footprint.disc(r) for r in radii}
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
            need.append(tile_margins(cells.cpu().numpy(), med.cpu().numpy(), tw, th, img_np, r))
    need = np.concatenate(need) if need else np.zeros(1)
    margin = float(np.quantile(need, 1.0 - fail_target)) if need.size else 0.0
    log(f"# margin {margin:.5f} (quantile {1 - fail_target:.4f} of {need.size} held-out pixels "
        f"of tiles that can be bracketed)")
    return margin


def train(images=512, size=512, radii=(16, 32, 64), epochs=2, lr=3e-3, holdout=8,
          fail_target=0.0005, seed=4, log=print, calibration_size=2048):
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
    margin = calibrate(net, images, radii, holdout, calibration_size, seed, fail_target, log)
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
    ap.add_argument("--holdout", type=int, default=8)
    ap.add_argument("--calibration-size", type=int, default=2048,
                    help="side of the held-out images the margin is calibrated on")
    ap.add_argument("--fail-target", type=float, default=0.0005)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--calibrate-only", metavar="WEIGHTS", default=None,
                    help="keep the parameters of WEIGHTS and only recalibrate the margin")
    a = ap.parse_args()
    radii = tuple(int(r) for r in a.radii.split(","))
    if a.calibrate_only:
        import torch

        import paper_2505_22938_amd as mf
        torch.cuda.init()   # torch's device set-up before the library's first HIP call
        with np.load(a.calibrate_only, allow_pickle=False) as z:
            params = z["params"]
            meta = json.loads(str(z["meta"]))
        net = mf.LearnedNet(seed=0)
        net.set_params(params)
        margin = calibrate(net, meta.get("images", a.images), radii, a.holdout,
                           a.calibration_size, meta.get("seed", a.seed), a.fail_target)
        net.close()
        meta.update(fail_target=a.fail_target, calibration_radii=list(radii),
                    calibration_holdout=a.holdout, calibration_size=a.calibration_size,
                    calibration="pixel quantile over tiles that can be bracketed")
        np.savez(a.out, params=params, margin=np.float32(margin), meta=json.dumps(meta))
        print(json.dumps(dict(out=a.out, margin=margin, **meta)))
        return
    params, margin, losses = train(a.images, a.size, radii, a.epochs, a.lr, a.holdout,
                                   a.fail_target, a.seed, calibration_size=a.calibration_size)
    meta = dict(images=a.images, size=a.size, radii=list(radii), epochs=a.epochs, lr=a.lr,
                seed=a.seed, fail_target=a.fail_target, final_loss=float(np.mean(losses[-64:])))
    np.savez(a.out, params=params, margin=np.float32(margin), meta=json.dumps(meta))
    print(json.dumps(dict(out=a.out, margin=margin, **meta)))


if __name__ == "__main__":
    main()
