"""Benchmark: exact median filter, 4096x4096 uint16 natural-like image, disc r=32, clamp.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--radius R] [--size S]
                    [--no-cpu] [--cpu-seconds T] [--legs plain,batched,learned,ranks,windows,stress]
                    [--weights PATH] [--copy-check]

One step = one call of the plain filter over the whole image (every step of
the hot path: tile load, ordinal transform, sliding and omnigram scans,
reverse map), with the input already resident in device memory.  Prints one
JSON line.  The CPU-baseline leg times the brute-force oracle on a bounded
sample of output pixels on the host cores and counts mismatches of the GPU
output on that sample.

Comparison legs in the same line:
  batched  - 64 mixed images (w, h uniform in 128..2048, u8/u16/f32, disc
             r uniform in 1..64, clamp): one replay of the captured persistent
             launch against 64 sequential plain launches on one stream;
  learned  - 2048x2048 uint16 (i.i.d. uniform, and the natural-like
             generator), disc r = 16, 32, 64: CNN bracket proposal + bracketed
             tiles + exact fallback against the plain filter, with the
             fallback rate;
  ranks    - the headline image: 25/50/75 % percentile planes in one call
             (one ordinal transform per tile) against three single-rank
             calls, and a per-pixel rank map running 0..100 % across the
             width against the median filter;
  windows  - the headline image: medians over discs of radius 24/32/40 and
             8/16/32 in one call each (windows of similar box size share one
             ordinal transform per tile), and one 3840x2160 float32
             log-normal plane with its disc r=48, ellipse and hexagon windows
             (mirror), each against one plain call per window;
  stress   - the slow input of the paper's limitations discussion (1024^2
             0/65535 checkerboard in a mid-grey frame, r=32), reported only.
Each compares every output pixel with the plain filter's and a random sample
with the oracle.  --copy-check adds a 256 MiB device copy (three launches),
whose hardware byte counters calibrate the filter's in a counter run.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T int32 VALU lane-ops/s
VALU_PEAK_OPS = 256 * 64 * 2.4e9

# Sources the plain kernel is built from; with the launch plan (tile, box,
# LDS bytes) they determine the kernel's memory traffic.
PLAIN_SOURCES = ("tile_engine.h", "tile_common.h", "mf_internal.h", "median_plain.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles",
                            "mf_plain_kernel_u16_4096x4096_disc_r32_hbm_bytes.md")


def kernel_sources_hash(plan):
    import hashlib
    h = hashlib.sha256()
    for name in PLAIN_SOURCES:
        with open(os.path.join(ROOT, "paper_2505_22938_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    geo = [plan[k] for k in ("tile_w", "tile_h", "box_w", "box_h", "lds_bytes")]
    h.update(("plan:" + ",".join(str(v) for v in geo)).encode())
    return h.hexdigest()


def measured_traffic(plan):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources or the launch plan changed since the counters were
    taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(l.split(": ", 1) for l in f.read().splitlines() if ": " in l)
        if kv.get("kernel_sources_sha256", "").strip() != kernel_sources_hash(plan):
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def work_model(plan, taps, rows, cols, w, h, passes, blocks, seeds, groups):
    """Algorithmic lane-operations of one filter call:
    sort 3 ops/element/4-bit pass + 1 op/element for the ordinal image,
    2*cols compare-accumulates per vertically slid pixel, 2*rows per
    horizontally slid pixel, 64 membership tests per wave-cooperative scan
    block, 8 per group tested by one lane, and one histogram update per tap
    of each seed window."""
    tw, th = plan["tile_w"], plan["tile_h"]
    T = plan["box_w"] * plan["box_h"]
    tiles = -(-w // tw) * -(-h // th)
    npx = tiles * tw * th                      # computed pixels incl. ragged tiles
    seed_rows = seeds * tw                     # first rows of bands
    sort_ops = tiles * T * (3 * passes + 1)
    slide_ops = (npx - seed_rows) * 2 * cols + (seed_rows - seeds) * 2 * rows
    scan_ops = 64 * blocks + 8 * groups
    seed_ops = seeds * taps
    total = sort_ops + slide_ops + scan_ops + seed_ops
    return dict(total=total, sort=sort_ops, slide=slide_ops, scan=scan_ops, seed=seed_ops,
                blocks_per_px=blocks / npx, groups_per_px=groups / npx, tiles=tiles,
                computed_px=npx)


def _time_events(torch, fn, stream, reps):
    """Per-call device time (ms) of fn() bracketed by events on `stream`."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def _oracle_sample(img_np, ofp, got, n, seed):
    """Mismatches of `got` against the oracle at n random pixels."""
    import oracle
    h, w = img_np.shape
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, w, n)
    ys = rng.integers(0, h, n)
    exp = oracle.filter_points(img_np, ofp, xs, ys, "clamp", nthreads=oracle.default_threads())
    a = got[ys, xs]
    if a.dtype == np.float32:
        return int((a.view(np.uint32) != exp.view(np.uint32)).sum())
    return int((a != exp).sum())


def leg_batched(torch, mf, reps, check_oracle, log, autotune=True):
    """Mixed batch of 64 images: captured persistent launch vs sequential plain launches."""
    import workloads
    from oracle import footprints as OF
    batch = workloads.mixed_batch(64, 3)
    fps, items, plain_out = {}, [], []
    for img_np, sp in batch:
        r = sp["radius"]
        if r not in fps:
            fps[r] = mf.Footprint.disc(r)
        img = torch.from_numpy(img_np).cuda()
        items.append((img, torch.empty_like(img), fps[r], "clamp"))
        plain_out.append(torch.empty_like(img))
    px = sum(int(i[0].numel()) for i in items)
    stream = torch.cuda.current_stream()

    def plain_all():
        for (img, _, fp, b), o in zip(items, plain_out):
            mf.median_filter(img, fp, b, out=o)

    def measure():
        """(plain sequential ms, graph replay ms, plan info, mismatches vs plain)"""
        plain_all()
        torch.cuda.synchronize()
        tp = float(np.median(_time_events(torch, plain_all, stream, reps)))
        plan = mf.BatchPlan(items)
        side = torch.cuda.Stream()
        plan.capture(side)
        plan.replay(side)
        side.synchronize()
        tb = float(np.median(_time_events(torch, lambda: plan.replay(side), side, reps)))
        info = plan.info()
        plan.close()
        mism = sum(int((it[1] != o).sum()) for it, o in zip(items, plain_out))
        return tp, tb, info, mism

    # default tile shapes, then autotuned ones (one tuning run per (dtype,
    # radius) on its first image; plain calls and the batched plan then both
    # use the tuned table)
    res = {"default": measure()}
    tuned, t_tune = 0, 0.0
    if autotune:
        t0 = time.perf_counter()
        seen = set()
        for (img, out, fp, b), (img_np, sp) in zip(items, batch):
            key = (sp["dtype"], sp["radius"])
            if key in seen:
                continue
            seen.add(key)
            mf.autotune(img, fp, b, out=out, reps=2)
            tuned += 1
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
        res["autotuned"] = measure()
    omism, ochk = None, 0
    if check_oracle:
        omism = 0
        for i, ((img_np, sp), it) in enumerate(zip(batch, items)):
            omism += _oracle_sample(img_np, OF.disc(sp["radius"]), it[1].cpu().numpy(), 64, i)
            ochk += 64
    best_plain = min(res, key=lambda k: res[k][0])
    best_batch = min(res, key=lambda k: res[k][1])
    mp, mb = res[best_plain][0], res[best_batch][1]
    log(f"# batched: {px / 1e6:.1f} Mpx; " + "; ".join(
        f"{k}: plain {v[0]:.2f} ms, graph {v[1]:.2f} ms" for k, v in res.items()))
    return {"images": 64, "megapixels": px / 1e6,
            "policies": {k: {"plain_sequential_ms": v[0], "graph_replay_ms": v[1],
                             "speedup": v[0] / v[1], "plan": v[2], "mismatches_vs_plain": v[3]}
                         for k, v in res.items()},
            "plain_sequential_ms": mp, "graph_replay_ms": mb, "speedup_vs_plain": mp / mb,
            "best": {"plain": best_plain, "batched": best_batch},
            "plain_mpx_s": px / 1e3 / mp, "batched_mpx_s": px / 1e3 / mb,
            "mismatches_vs_plain": sum(v[3] for v in res.values()),
            "oracle_mismatches": omism, "oracle_checked_px": ochk,
            "autotune": f"{tuned} (dtype, radius) shapes tuned in {t_tune:.1f} s" if autotune
                        else "off"}


def leg_learned(torch, mf, weights, reps, check_oracle, log):
    """2048x2048 uint16: learned bracket path vs the plain filter."""
    import workloads
    from oracle import footprints as OF
    if not os.path.exists(weights):
        return {"skipped": f"no trained weights at {os.path.relpath(weights, ROOT)}"}
    net = mf.LearnedNet.load(weights)
    stream = torch.cuda.current_stream()
    S = 2048
    rows = []
    for kind in ("uniform", "natural"):
        img_np = (workloads.uniform_u16(S, S, seed=4) if kind == "uniform"
                  else workloads.natural_u16(S, S, seed=4))
        img = torch.from_numpy(img_np).cuda()
        ref = torch.empty_like(img)
        out = torch.empty_like(img)
        for r in (16, 32, 64):
            fp = mf.Footprint.disc(r)
            mf.median_filter(img, fp, "clamp", out=ref)
            tp = _time_events(torch, lambda: mf.median_filter(img, fp, "clamp", out=ref), stream,
                              reps)
            mf.work_counters(1)
            mf.median_filter(img, fp, "clamp", out=ref)
            torch.cuda.synchronize()
            cp = mf.work_counters(-1)
            mf.work_counters(0)
            row = {"image": kind, "radius": r, "plain_ms": float(np.median(tp))}
            try:
                _, fb = net.filter(img, fp, out=out)
            except mf.MedianFilterError as e:
                row["learned"] = f"unsupported: {e}"
                rows.append(row)
                continue
            tl = _time_events(torch, lambda: net.filter(img, fp, out=out, count_fallback=False),
                              stream, reps)
            mf.work_counters(1)
            net.filter(img, fp, out=out)
            torch.cuda.synchronize()
            cl = mf.work_counters(-1)
            mf.work_counters(0)
            row.update(learned_ms=float(np.median(tl)), fallback_rate=fb / (S * S),
                       speedup_vs_plain=row["plain_ms"] / float(np.median(tl)),
                       ranked_px_fraction=cl[7] / max(cp[7], 1),
                       mismatches_vs_plain=int((out != ref).sum()))
            if check_oracle:
                row["oracle_mismatches"] = _oracle_sample(img_np, OF.disc(r), out.cpu().numpy(),
                                                          2000, r)
            log(f"# learned {kind} r={r}: plain {row['plain_ms']:.3f} ms, learned "
                f"{row['learned_ms']:.3f} ms, fallback {row['fallback_rate']:.4f}")
            rows.append(row)
    net.close()
    return {"weights": os.path.relpath(weights, ROOT), "margin": net.margin,
            "size": [S, S], "dtype": "u16", "results": rows}


def leg_ranks(torch, mf, img, img_np, fp, ofp, reps, check_oracle, log):
    """Headline image: 25/50/75 % percentile planes from one ordinal
    transform per tile against three single-rank calls, and a rank map whose
    percentile runs 0..100 % across the width against the median filter."""
    import workloads
    stream = torch.cuda.current_stream()
    n = fp.taps
    ks = [(n - 1) // 4, (n - 1) // 2, 3 * (n - 1) // 4]
    singles = [torch.empty_like(img) for _ in ks]
    multi = [torch.empty_like(img) for _ in ks]

    def run_singles():
        for k, o in zip(ks, singles):
            mf.median_filter(img, fp, "clamp", out=o, rank=k)

    run_singles()
    mf.rank_filter(img, fp, ks, "clamp", outs=multi)
    t_single = float(np.median(_time_events(torch, run_singles, stream, reps)))
    t_multi = float(np.median(_time_events(
        torch, lambda: mf.rank_filter(img, fp, ks, "clamp", outs=multi), stream, reps)))
    mism = sum(int((a != b).sum()) for a, b in zip(singles, multi))
    S_h, S_w = img_np.shape
    rm_np = workloads.percentile_ramp(S_w, S_h, n)
    rm = torch.from_numpy(rm_np).cuda()
    ramp = torch.empty_like(img)
    med = torch.empty_like(img)
    mf.rank_map_filter(img, fp, rm, "clamp", out=ramp)
    mf.median_filter(img, fp, "clamp", out=med)
    t_ramp = float(np.median(_time_events(
        torch, lambda: mf.rank_map_filter(img, fp, rm, "clamp", out=ramp), stream, reps)))
    t_med = float(np.median(_time_events(
        torch, lambda: mf.median_filter(img, fp, "clamp", out=med), stream, reps)))
    cols = np.nonzero(rm_np[0] == (n - 1) // 2)[0]
    ramp_np = ramp.cpu().numpy()
    col_mism = int((ramp_np[:, cols] != med.cpu().numpy()[:, cols]).sum())
    res = {"ranks": ks, "three_single_calls_ms": t_single, "one_three_plane_call_ms": t_multi,
           "speedup": t_single / t_multi, "mismatches_multi_vs_single": mism,
           "percentile_ramp_ms": t_ramp, "median_ms": t_med,
           "ramp_median_columns_mismatches": col_mism}
    if check_oracle:
        import oracle
        rng = np.random.default_rng(99)
        xs, ys = rng.integers(0, S_w, 2000), rng.integers(0, S_h, 2000)
        exp = oracle.filter_points(img_np, ofp, xs, ys, "clamp", ranks=rm_np[ys, xs],
                                   nthreads=oracle.default_threads())
        res["ramp_oracle_mismatches"] = int((ramp_np[ys, xs] != exp).sum())
        res["ramp_oracle_checked_px"] = 2000
    log(f"# ranks: 3 single {t_single:.2f} ms, one 3-plane call {t_multi:.2f} ms; "
        f"ramp {t_ramp:.2f} ms vs median {t_med:.2f} ms")
    return res


def leg_windows(torch, mf, img, img_np, reps, check_oracle, log):
    """Headline image: medians over several disc radii in one call (the
    library's grouping by box size) against one plain call per radius; radii
    24/32/40 share one ordinal transform per tile, 8/16/32 are split into
    passes (forced into one pass too, for comparison)."""
    import workloads
    from oracle import footprints as OF
    discs = lambda radii: ([mf.Footprint.disc(r) for r in radii],   # noqa: E731
                           [OF.disc(r) for r in radii], [f"disc r={r}" for r in radii])
    res = {"similar": _windows_case(torch, mf, img, img_np, reps, check_oracle, log,
                                    *discs((24, 32, 40)), "clamp"),
           "disparate": _windows_case(torch, mf, img, img_np, reps, check_oracle, log,
                                      *discs((8, 16, 32)), "clamp")}
    # the float workload: one 3840x2160 log-normal plane, its three windows
    f32 = np.ascontiguousarray(workloads.lognormal_f32(3840, 2160, planes=1, seed=2)[0])
    res["f32_three_shapes"] = _windows_case(
        torch, mf, torch.from_numpy(f32).cuda(), f32, reps, check_oracle, log,
        [mf.Footprint.disc(48), mf.Footprint.ellipse(60, 20, 30),
         mf.Footprint.regular_polygon(6, 40)],
        [OF.disc(48), OF.ellipse(60, 20, 30), OF.regular_polygon(6, 40)],
        ["disc r=48", "ellipse 60x20 @30", "hexagon R=40"], "mirror")
    return res


def _windows_case(torch, mf, img, img_np, reps, check_oracle, log, fps, ofps, names, boundary):
    """One window_filter call over `fps` against one plain call per window,
    and the same windows forced into one pass."""
    stream = torch.cuda.current_stream()
    singles = [torch.empty_like(img) for _ in fps]
    multi = [torch.empty_like(img) for _ in fps]

    def run_singles():
        for f, o in zip(fps, singles):
            mf.median_filter(img, f, boundary, out=o)

    run_singles()
    mf.window_filter(img, fps, boundary, outs=multi)
    t_single = float(np.median(_time_events(torch, run_singles, stream, reps)))
    t_multi = float(np.median(_time_events(
        torch, lambda: mf.window_filter(img, fps, boundary, outs=multi), stream, reps)))
    bits = (lambda t: t.view(torch.int32)) if img.dtype == torch.float32 else (lambda t: t)
    mism = sum(int((bits(a) != bits(b)).sum()) for a, b in zip(singles, multi))
    mf.set_window_fusion(True)
    try:
        fused = [torch.empty_like(img) for _ in fps]
        t_fused = float(np.median(_time_events(
            torch, lambda: mf.window_filter(img, fps, boundary, outs=fused), stream, reps)))
    finally:
        mf.set_window_fusion(False)
    mism += sum(int((bits(a) != bits(b)).sum()) for a, b in zip(singles, fused))
    res = {"windows": names, "boundary": boundary, "dtype": str(img.dtype).replace("torch.", ""),
           "size": [int(img.shape[1]), int(img.shape[0])],
           "single_calls_ms": t_single, "one_call_ms": t_multi,
           "speedup": t_single / t_multi, "all_in_one_pass_ms": t_fused,
           "mismatches_multi_vs_single": mism}
    if check_oracle:
        import oracle
        h, w = img_np.shape
        rng = np.random.default_rng(200 + len(names))
        bad = 0
        for ofp, o in zip(ofps, multi):
            xs, ys = rng.integers(0, w, 500), rng.integers(0, h, 500)
            exp = oracle.filter_points(img_np, ofp, xs, ys, boundary,
                                       nthreads=oracle.default_threads())
            got = o.cpu().numpy()[ys, xs]
            bad += int((got.view(np.uint8).reshape(500, -1) != exp.view(np.uint8).reshape(500, -1))
                       .any(axis=1).sum())
        res["oracle_mismatches"] = bad
        res["oracle_checked_px"] = 500 * len(names)
    log(f"# windows {names}: {len(names)} plain calls {t_single:.2f} ms, "
        f"one call {t_multi:.2f} ms, all in one pass {t_fused:.2f} ms")
    return res


def leg_stress(torch, mf, reps, check_oracle, log):
    """1024x1024 uint16 0/65535 checkerboard inside a mid-grey frame, disc
    r=32: the input the paper's limitations discussion describes as slow
    (medians jump across the whole value range between neighbours).
    Reported, not a target."""
    import workloads
    from oracle import footprints as OF
    img_np = workloads.adversarial_u16(1024, 1024, border=96)
    img = torch.from_numpy(img_np).cuda()
    out = torch.empty_like(img)
    fp = mf.Footprint.disc(32)
    mf.median_filter(img, fp, "clamp", out=out)
    ts = _time_events(torch, lambda: mf.median_filter(img, fp, "clamp", out=out),
                      torch.cuda.current_stream(), reps)
    mf.work_counters(1)
    mf.median_filter(img, fp, "clamp", out=out)
    torch.cuda.synchronize()
    c = mf.work_counters(-1)
    mf.work_counters(0)
    ms = float(np.median(ts))
    res = {"image": "1024x1024 u16 checkerboard 0/65535 in a 96-px frame of 32768",
           "radius": 32, "ms": ms, "mpx_s": 1024 * 1024 / 1e3 / ms,
           "scan_blocks_per_px": c[0] / (1024 * 1024), "lane_groups_per_px": c[6] / (1024 * 1024)}
    if check_oracle:
        res["oracle_mismatches"] = _oracle_sample(img_np, OF.disc(32), out.cpu().numpy(), 2000, 5)
        res["oracle_checked_px"] = 2000
    log(f"# stress: adversarial 1024^2 r=32 {ms:.3f} ms")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--radius", type=int, default=32)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--legs", default="plain,batched,learned,ranks,windows,stress")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2505_22938_amd", "weights",
                                                      "bracket_net.npz"))
    ap.add_argument("--copy-check", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched leg: default tile shapes instead of autotuned ones")
    args = ap.parse_args()
    legs = set(args.legs.split(","))

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the filter shards by image bands, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2505_22938_amd as mf
    import workloads

    dev = torch.device("cuda:0")
    S, r = args.size, args.radius
    t0 = time.time()
    img_np = workloads.natural_u16(S, S, seed=1)
    img = torch.from_numpy(img_np).to(dev)
    out = torch.empty_like(img)
    fp = mf.Footprint.disc(r)
    plan = mf.query_plan(S, S, mf.MF_U16, fp)
    print(f"# input ready in {time.time() - t0:.1f}s; plan {plan}", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        mf.median_filter(img, fp, "clamp", out=out)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        mf.median_filter(img, fp, "clamp", out=out)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    mpx = S * S / 1e6
    value = mpx * args.steps / wall

    # work counters (separate, untimed call)
    mf.work_counters(1)
    mf.median_filter(img, fp, "clamp", out=out)
    torch.cuda.synchronize()
    cnt = mf.work_counters(-1)
    blocks, seeds, groups = cnt[0], cnt[1], cnt[6]
    nw = max(cnt[5], 1)
    phase_clk = {"sort": cnt[2] / nw, "rows": cnt[3] / nw, "sweep": cnt[4] / nw}
    mf.work_counters(0)
    lo, hi = fp.row_spans()
    rows = len(lo)
    cols = fp.dx_max - fp.dx_min + 1
    wm = work_model(plan, fp.taps, rows, cols, S, S, 4, blocks, seeds, groups)
    kmean = float(np.mean(kern_ms))
    achieved = wm["total"] / (kmean * 1e-3)
    traffic = measured_traffic(plan) if (S, r) == (4096, 32) else None
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Top/s (int32 lane-ops)", "frac": achieved / VALU_PEAK_OPS,
                "traffic": traffic, "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "hbm_gb_s": traffic / (kmean * 1e-3) / 1e9 if traffic else None,
                "hbm_frac_of_8tb_s": traffic / (kmean * 1e-3) / 8e12 if traffic else None,
                "kernel_ms_mean": kmean, "kernel_ms_min": float(np.min(kern_ms)),
                "work_lane_ops": wm, "clocks_per_wave": phase_clk}
    gpu_out = out.cpu().numpy()

    if args.copy_check:
        # a plain device copy of known size, for calibrating byte counters
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if "ranks" in legs:
        from oracle import footprints as OF
        ranks = leg_ranks(torch, mf, img, img_np, fp, OF.disc(r), 5, not args.no_cpu, log)
    else:
        ranks = None
    windows = (leg_windows(torch, mf, img, img_np, 5, not args.no_cpu, log)
               if "windows" in legs else None)
    learned = (leg_learned(torch, mf, args.weights, 5, not args.no_cpu, log)
               if "learned" in legs else None)
    stress = leg_stress(torch, mf, 5, not args.no_cpu, log) if "stress" in legs else None
    # last: the batched leg records autotuned tile shapes, which every later
    # plan in this process would use instead of the default ones
    batched = (leg_batched(torch, mf, 5, not args.no_cpu, log, autotune=not args.no_autotune)
               if "batched" in legs else None)

    cpu = None
    mismatches = None
    if not args.no_cpu:
        import oracle
        from oracle import footprints as OF
        ofp = OF.disc(r)
        cores = oracle.default_threads()
        rng = np.random.default_rng(123)
        n0 = 20000
        xs = rng.integers(0, S, n0)
        ys = rng.integers(0, S, n0)
        c0 = time.perf_counter()
        v0 = oracle.filter_points(img_np, ofp, xs, ys, "clamp", nthreads=cores)
        d0 = time.perf_counter() - c0
        n1 = int(min(S * S, max(n0, n0 * args.cpu_seconds / max(d0, 1e-3))))
        xs1 = rng.integers(0, S, n1)
        ys1 = rng.integers(0, S, n1)
        c1 = time.perf_counter()
        v1 = oracle.filter_points(img_np, ofp, xs1, ys1, "clamp", nthreads=cores)
        d1 = time.perf_counter() - c1
        mismatches = int((gpu_out[ys, xs] != v0).sum() + (gpu_out[ys1, xs1] != v1).sum())
        # one thread on a 512x512 crop of output pixels, for scaling
        C = min(512, S)
        cy, cx = np.mgrid[0:C, 0:C]
        c2 = time.perf_counter()
        x2, y2 = cx.ravel() + (S - C) // 2, cy.ravel() + (S - C) // 2
        v2 = oracle.filter_points(img_np, ofp, x2, y2, "clamp", nthreads=1)
        d2 = time.perf_counter() - c2
        mismatches += int((gpu_out[y2, x2] != v2).sum())
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                             "")
        except OSError:
            pass
        cpu = {"value": n1 / d1 / 1e6, "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
               "cpu_model": model, "one_thread_mpx_s": C * C / d2 / 1e6,
               "one_thread_sample": f"central {C}x{C} crop, {d2:.1f}s",
               "sample": f"{n1} random output pixels of the same {S}x{S} image, disc r={r} "
                         f"({fp.taps} taps), brute force gather + nth_element, {d1:.1f}s",
               "mismatches_vs_gpu": mismatches, "checked_px": n0 + n1 + C * C}

    line = {
        "metric": "Mpixel/s, r=32 disc uint16 4K, learned/batched vs plain GPU, bit-exact",
        "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"plain median filter, {S}x{S} uint16 natural-like (8 plane "
                               f"waves + N(0,800) + 5% impulses, seed 1), disc r={r} "
                               f"({fp.taps} taps), clamp",
                   "tile": [plan["tile_w"], plan["tile_h"]], "box": [plan["box_w"], plan["box_h"]],
                   "lds_bytes": plan["lds_bytes"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "learned": learned,
        "ranks": ranks,
        "windows": windows,
        "stress": stress,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
