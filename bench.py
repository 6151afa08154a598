"""Benchmark: exact median filter, 4096x4096 uint16 natural-like image, disc r=32, clamp.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--radius R] [--size S]
                    [--no-cpu] [--legs plain,batched,learned,ranks,windows,stress]
                    [--weights PATH] [--copy-check]

One step = one call of the plain filter over the whole image (every step of
the hot path: tile load, ordinal transform, sliding and omnigram scans,
reverse map), with the input already resident in device memory.  Prints one
JSON line.  The CPU-baseline leg runs the brute-force oracle over every
output pixel of the same image on the host cores (about 20 s on 16 cores),
timing it and counting mismatches of the GPU output.

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
MIX_FILE = os.path.join(ROOT, "profiles",
                        "mf_plain_kernel_u16_4096x4096_disc_r32_instruction_mix.md")


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


def box_union_px(lo, hi, dy_min, tw, th):
    """Pixels of the union of the windows centred on a tw x th tile (the
    rounded rectangle the method must rank): for each box row, the x range
    covered by the footprint rows that reach it from some tile row."""
    nrows = len(lo)
    total = 0
    for y in range(dy_min, th + dy_min + nrows - 1):     # box row, tile coords
        dys = [y - ty for ty in range(th) if 0 <= y - ty - dy_min < nrows]
        if not dys:
            continue
        xl = min(lo[dy - dy_min] for dy in dys)
        xh = max(hi[dy - dy_min] for dy in dys) + tw - 1
        total += xh - xl + 1
    return total


def band_geometry(plan, w, h):
    """Output pixels, histogram seeds, 16-column seed moves and horizontally
    slid pixels of one plain-filter launch, from the plan: bands of
    ceil(th / (16 * 64 / tw)) rows, each band's first row cut into 16-column
    chunks (the first from a histogram, the others moved from the previous
    chunk's seed window), the rest of each chunk slid horizontally."""
    tw, th = plan["tile_w"], plan["tile_h"]
    segs = 64 // tw
    R = -(-th // (16 * segs))
    npx = seeds = moves = hslid = 0
    for ty0 in range(0, h, th):
        rows_in = min(th, h - ty0)
        bands = -(-rows_in // R)
        for tx0 in range(0, w, tw):
            cols_in = min(tw, w - tx0)
            chunks = -(-cols_in // 16)
            npx += rows_in * cols_in
            seeds += bands
            moves += bands * (chunks - 1)
            hslid += bands * (cols_in - chunks)
    first_row = seeds + moves + hslid
    return dict(px=npx, seeds=seeds, moves=moves, hslid=hslid, vslid=npx - first_row)


def work_model(plan, fp, w, h, key_bits, blocks, groups):
    """Algorithmic lane-operations of one plain-filter launch (the method's own
    work, not the kernel's instruction count):
      sort   A * P * 3 per output pixel: ranking the union of the tile's
             windows (T_union box pixels per tile) with P = key_bits / 8 byte
             passes of about 3 operations per element;
      slides 2 * cols compares per vertically slid pixel, 2 * rows per
             horizontally slid pixel (a 16-column seed move counts as 16
             horizontal slides);
      scans  64 omnigram tests per wave-cooperative block, 8 per lane group
             (both counted by the kernel);
      seeds  N histogram updates per histogram seed."""
    tw, th = plan["tile_w"], plan["tile_h"]
    lo, hi = fp.row_spans()
    rows = len(lo)
    cols = fp.dx_max - fp.dx_min + 1
    tiles = -(-w // tw) * -(-h // th)
    t_union = box_union_px(lo, hi, fp.dy_min, tw, th)
    passes = key_bits // 8
    g = band_geometry(plan, w, h)
    sort_ops = tiles * t_union * passes * 3
    slide_ops = g["vslid"] * 2 * cols + (g["hslid"] + 16 * g["moves"]) * 2 * rows
    scan_ops = 64 * blocks + 8 * groups
    seed_ops = g["seeds"] * fp.taps
    total = sort_ops + slide_ops + scan_ops + seed_ops
    return dict(total=total, sort=sort_ops, slide=slide_ops, scan=scan_ops, seed=seed_ops,
                t_union=t_union, t_box=plan["box_w"] * plan["box_h"], byte_passes=passes,
                amplification=t_union / (tw * th), blocks_per_px=blocks / g["px"],
                groups_per_px=groups / g["px"], tiles=tiles, per_px=total / g["px"], **g)


def issued_lane_ops(plan):
    """VALU lane-instructions per launch (SQ_INSTS_VALU x 64) from the committed
    counter summary, or None when the kernel or plan changed since."""
    try:
        with open(MIX_FILE) as f:
            kv = dict(l.split(": ", 1) for l in f.read().splitlines() if ": " in l)
        if kv.get("kernel_sources_sha256", "").strip() != kernel_sources_hash(plan):
            return None
        return int(kv["valu_lane_ops_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


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


def _oracle_sample(img_np, ofp, got, n, seed, boundary="clamp"):
    """Mismatches of `got` against the oracle at n random pixels."""
    import oracle
    h, w = img_np.shape
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, w, n)
    ys = rng.integers(0, h, n)
    exp = oracle.filter_points(img_np, ofp, xs, ys, boundary, nthreads=oracle.default_threads())
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
        # keep a per-image shape only where it makes the whole batch faster
        bt_before, bt_after, dropped = mf.plan_autotune(items, reps=3)
        t_tune = time.perf_counter() - t0
        res["autotuned"] = measure()
    omism, ochk = None, 0
    if check_oracle:
        omism = 0
        for i, ((img_np, sp), it) in enumerate(zip(batch, items)):
            omism += _oracle_sample(img_np, OF.disc(sp["radius"]), it[1].cpu().numpy(), 64, i)
            ochk += 64
    # the headline compares both forms under one tile-shape policy: the
    # autotuned shapes the batched workload specifies (default shapes when
    # tuning is off), each plain launch given the same shape as its batch entry
    pol = "autotuned" if "autotuned" in res else "default"
    mp, mb = res[pol][0], res[pol][1]
    log(f"# batched: {px / 1e6:.1f} Mpx; " + "; ".join(
        f"{k}: plain {v[0]:.2f} ms, graph {v[1]:.2f} ms" for k, v in res.items()))
    return {"images": 64, "megapixels": px / 1e6,
            "policies": {k: {"plain_sequential_ms": v[0], "graph_replay_ms": v[1],
                             "speedup": v[0] / v[1], "plan": v[2], "mismatches_vs_plain": v[3]}
                         for k, v in res.items()},
            "policy": pol, "plain_sequential_ms": mp, "graph_replay_ms": mb,
            "speedup_vs_plain": mp / mb,
            "plain_mpx_s": px / 1e3 / mp, "batched_mpx_s": px / 1e3 / mb,
            "mismatches_vs_plain": sum(v[3] for v in res.values()),
            "oracle_mismatches": omism, "oracle_checked_px": ochk,
            "autotune": (f"{tuned} (dtype, radius) shapes tuned per image, then {dropped} "
                         f"dropped where the batch ran faster without them (batch "
                         f"{bt_before:.2f} -> {bt_after:.2f} ms); {t_tune:.1f} s")
                        if autotune else "off"}


def leg_learned(torch, mf, weights, reps, check_oracle, log):
    """2048x2048 uint16: learned bracket path vs the plain filter."""
    import workloads
    from oracle import footprints as OF
    if not os.path.exists(weights):
        return {"skipped": f"no trained weights at {os.path.relpath(weights, ROOT)}"}
    net = mf.LearnedNet.load(weights)
    # the method without the trained network: the same network untrained (its
    # output layer starts at the full range, so every bracket is dropped), and
    # a constant full-range bracket for every tile
    untrained = mf.LearnedNet(seed=4)
    untrained.set_margin(net.margin)
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
            # gain over the method without the trained network
            out2 = torch.empty_like(img)
            _, fbu = untrained.filter(img, fp, out=out2)
            tu = _time_events(torch, lambda: untrained.filter(img, fp, out=out2,
                                                              count_fallback=False), stream, reps)
            row["untrained"] = {"ms": float(np.median(tu)), "fallback_rate": fbu / (S * S),
                                "mismatches_vs_plain": int((out2 != ref).sum())}
            tx, ty = mf.LearnedNet.tile_grid(S, S, mf.MF_U16, fp)
            full = torch.tensor([0, 65535], dtype=torch.int32, device="cuda").repeat(tx * ty)
            _, fbf = net.filter_bracketed(img, fp, full, out=out2)
            tf = _time_events(torch, lambda: net.filter_bracketed(img, fp, full, out=out2), stream,
                              reps)
            row["full_range_bracket"] = {"ms": float(np.median(tf)),
                                         "fallback_rate": fbf / (S * S),
                                         "mismatches_vs_plain": int((out2 != ref).sum())}
            log(f"# learned {kind} r={r}: plain {row['plain_ms']:.3f} ms, learned "
                f"{row['learned_ms']:.3f} ms, fallback {row['fallback_rate']:.4f}; untrained "
                f"{row['untrained']['ms']:.3f} ms (fallback {row['untrained']['fallback_rate']:.3f}),"
                f" full-range bracket {row['full_range_bracket']['ms']:.3f} ms")
            rows.append(row)
    net.close()
    untrained.close()
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


def leg_configs(torch, mf, img, img_np, reps, check_oracle, log):
    """The plain filter on the other workloads it is specified on: the
    256x256 uint8 i.i.d. image under a radius-4 disc (checked in full); the
    headline image at radii 8 and 100 (radius 32 is the headline); the
    3-channel 3840x2160 float32 log-normal image, channels filtered
    independently, under each of its three windows (mirror)."""
    import workloads
    from oracle import footprints as OF
    stream = torch.cuda.current_stream()
    res = {}
    u8 = workloads.plain_u8(256, 256, 0)
    d8 = torch.from_numpy(u8).cuda()
    o8 = torch.empty_like(d8)
    fp = mf.Footprint.disc(4)
    mf.median_filter(d8, fp, "clamp", out=o8)
    ms = float(np.median(_time_events(
        torch, lambda: mf.median_filter(d8, fp, "clamp", out=o8), stream, reps)))
    r = {"image": "256x256 uint8 i.i.d. uniform, seed 0", "window": "disc r=4 (49 taps)",
         "boundary": "clamp", "ms": ms, "mpx_s": 256 * 256 / 1e3 / ms}
    if check_oracle:
        import oracle
        exp = oracle.filter(u8, OF.disc(4), "clamp", nthreads=oracle.default_threads())
        r["oracle_mismatches"] = int((o8.cpu().numpy() != exp).sum())
        r["oracle_checked_px"] = 256 * 256
    res["u8_256_disc4"] = r
    log(f"# configs: 256^2 u8 disc 4 {ms:.3f} ms")
    h, w = img_np.shape
    out = torch.empty_like(img)
    for rad in (8, 100):
        fp = mf.Footprint.disc(rad)
        mf.median_filter(img, fp, "clamp", out=out)
        ms = float(np.median(_time_events(
            torch, lambda: mf.median_filter(img, fp, "clamp", out=out), stream, reps)))
        r = {"image": f"{w}x{h} uint16 natural-like (the headline image)",
             "window": f"disc r={rad} ({fp.taps} taps)", "boundary": "clamp", "ms": ms,
             "mpx_s": w * h / 1e3 / ms, "plan": mf.query_plan(w, h, mf.MF_U16, fp)}
        if check_oracle:
            r["oracle_mismatches"] = _oracle_sample(img_np, OF.disc(rad), out.cpu().numpy(),
                                                    1000, 40 + rad)
            r["oracle_checked_px"] = 1000
        res[f"u16_{w}_disc{rad}"] = r
        log(f"# configs: {w}^2 u16 disc {rad} {ms:.3f} ms")
    f32 = workloads.lognormal_f32(3840, 2160, planes=3, seed=2)
    planes = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in f32]
    outs = [torch.empty_like(p) for p in planes]
    for name, fp, ofp in (("disc r=48", mf.Footprint.disc(48), OF.disc(48)),
                          ("ellipse 60x20 @30", mf.Footprint.ellipse(60, 20, 30),
                           OF.ellipse(60, 20, 30)),
                          ("hexagon R=40", mf.Footprint.regular_polygon(6, 40),
                           OF.regular_polygon(6, 40))):
        def run():
            for p, o in zip(planes, outs):
                mf.median_filter(p, fp, "mirror", out=o)

        run()
        ms = float(np.median(_time_events(torch, run, stream, reps)))
        r = {"image": "3840x2160x3 float32 log-normal (mu 0, sigma 1) with 2% +-1e6 outliers, "
                      "seed 2, channels filtered independently",
             "window": f"{name} ({fp.taps} taps)", "boundary": "mirror", "ms_3_channels": ms,
             "mpx_s": 3 * 3840 * 2160 / 1e3 / ms}
        if check_oracle:
            r["oracle_mismatches"] = sum(
                _oracle_sample(f32[c], ofp, outs[c].cpu().numpy(), 300, 60 + c, "mirror")
                for c in range(3))
            r["oracle_checked_px"] = 900
        res[f"f32_3840x2160x3_{name.split()[0]}"] = r
        log(f"# configs: 3840x2160x3 f32 {name} {ms:.3f} ms (3 channels)")
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
    ap.add_argument("--legs", default="plain,configs,batched,learned,ranks,windows,stress")
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
    phase_clk = {"sort": cnt[2] / nw, "rows": cnt[3] / nw, "sweep": cnt[4] / nw,
                 "seeds": cnt[8] / nw, "load": cnt[9] / nw}
    mf.work_counters(0)
    wm = work_model(plan, fp, S, S, 16, blocks, groups)
    if wm["seeds"] != seeds:
        print(f"# note: kernel counted {seeds} histogram seeds, plan geometry {wm['seeds']}",
              file=sys.stderr, flush=True)
    kmean = float(np.mean(kern_ms))
    achieved = wm["total"] / (kmean * 1e-3)
    full = (S, r) == (4096, 32)
    traffic = measured_traffic(plan) if full else None
    issued = issued_lane_ops(plan) if full else None
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Top/s (int32 lane-ops)", "frac": achieved / VALU_PEAK_OPS,
                "traffic": traffic, "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "hbm_gb_s": traffic / (kmean * 1e-3) / 1e9 if traffic else None,
                "hbm_frac_of_8tb_s": traffic / (kmean * 1e-3) / 8e12 if traffic else None,
                "kernel_ms_mean": kmean, "kernel_ms_min": float(np.min(kern_ms)),
                "algorithmic_lane_ops": wm["total"],
                "issued_lane_ops": issued,
                "issued_over_algorithmic": issued / wm["total"] if issued else None,
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
    configs = (leg_configs(torch, mf, img, img_np, 5, not args.no_cpu, log)
               if "configs" in legs else None)
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
        # every output pixel of the headline image, on all host cores
        c1 = time.perf_counter()
        exp = oracle.filter(img_np, ofp, "clamp", nthreads=cores)
        d1 = time.perf_counter() - c1
        n1 = S * S
        mismatches = int((gpu_out != exp).sum())
        del exp
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
               "sample": f"all {n1} output pixels of the same {S}x{S} image, disc r={r} "
                         f"({fp.taps} taps), brute force gather + nth_element, {d1:.1f}s",
               "mismatches_vs_gpu": mismatches, "checked_px": n1 + C * C}

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
        "configs": configs,
        "batched": batched,
        "learned": learned,
        "ranks": ranks,
        "windows": windows,
        "stress": stress,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
