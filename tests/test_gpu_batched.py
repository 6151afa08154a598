"""GPU parity of the batched launch: every image of a mixed batch
equals the plain filter's output and the oracle's, bit for bit, and graph
replays reproduce it."""

import numpy as np
import pytest

import workloads
from oracle import footprints as OF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    import paper_2505_22938_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def small_batch(mf, seed=3, n=12, size_hi=300, r_hi=64):
    specs = workloads.mixed_batch_specs(n=n, seed=seed, size_lo=8, size_hi=size_hi, r_hi=r_hi)
    items, hosts = [], []
    for s in specs:
        img = workloads.uniform(s["w"], s["h"], s["dtype"], s["seed"])
        fp = mf.Footprint.disc(s["radius"])
        boundary = "clamp" if s["seed"] % 2 else "mirror"
        d = dev(img)
        items.append((d, torch.empty_like(d), fp, boundary))
        hosts.append((img, s["radius"], boundary))
    return items, hosts


def check(items, hosts, oracle_mod, what):
    for (d, out, fp, b), (img, r, _) in zip(items, hosts):
        got = out.cpu().numpy()
        exp = oracle_mod.filter(img, OF.disc(r), b)
        assert np.array_equal(got.view(np.uint8), exp.view(np.uint8)), \
            f"{what}: {img.shape} {img.dtype} r={r} {b}"


def test_batched_mixed_matches_oracle(mf, oracle_mod):
    items, hosts = small_batch(mf)
    plan = mf.BatchPlan(items)
    info = plan.info()
    assert info["tiles"] > 0 and info["grid"] > 0
    plan.launch()
    torch.cuda.synchronize()
    check(items, hosts, oracle_mod, "launch")
    plan.close()


def test_batched_equals_plain_and_footprint_mix(mf, oracle_mod):
    rng = np.random.default_rng(5)
    fps = [(mf.Footprint.ellipse(9, 3, 30), OF.ellipse(9, 3, 30)),
           (mf.Footprint.regular_polygon(6, 7), OF.regular_polygon(6, 7)),
           (mf.Footprint.disc(20), OF.disc(20)),
           (mf.Footprint.disc_limit(6), OF.disc_limit(6))]
    items, exp = [], []
    for i, dt in enumerate(["u8", "u16", "f32", "u16"]):
        img = workloads.uniform(int(rng.integers(40, 200)), int(rng.integers(40, 200)), dt, i)
        d = dev(img)
        items.append((d, torch.empty_like(d), fps[i][0], "mirror"))
        exp.append(oracle_mod.filter(img, fps[i][1], "mirror"))
    mf.median_filter_batched(items)
    torch.cuda.synchronize()
    for (d, out, fp, b), e in zip(items, exp):
        got = out.cpu().numpy()
        plain = mf.median_filter(d, fp, b)
        torch.cuda.synchronize()
        assert np.array_equal(got.view(np.uint8), e.view(np.uint8))
        assert np.array_equal(plain.cpu().numpy().view(np.uint8), e.view(np.uint8))


def test_batched_graph_replays(mf, oracle_mod):
    items, hosts = small_batch(mf, seed=11, n=8, size_hi=200, r_hi=40)
    plan = mf.BatchPlan(items)
    s = torch.cuda.Stream()
    plan.capture(s)
    for rep in range(3):
        for _, out, _, _ in items:
            out.zero_()
        torch.cuda.synchronize()
        plan.replay(s)
        s.synchronize()
        check(items, hosts, oracle_mod, f"replay {rep}")
    # eager launches between replays keep working (queue counters reset)
    plan.launch()
    torch.cuda.synchronize()
    check(items, hosts, oracle_mod, "eager after replay")
    plan.close()


def test_batched_groups_on_forked_streams(mf, oracle_mod):
    """Tiles needing different kernel variants (8-bit small window, 16-bit
    window large enough for global scratch, float32, several register
    capacities) run as separate groups spread over forked streams: eager
    launches on a side stream and on the current stream, and graph replays
    with eager work between them, all equal the oracle."""
    cases = [("u8", 90, 64, 3), ("u16", 150, 120, 64), ("f32", 100, 70, 12),
             ("u16", 200, 40, 20), ("u8", 33, 250, 30), ("f32", 64, 64, 40)]
    items, hosts = [], []
    for i, (dt, w, h, r) in enumerate(cases):
        img = workloads.uniform(w, h, dt, 40 + i)
        d = dev(img)
        items.append((d, torch.empty_like(d), mf.Footprint.disc(r), "mirror"))
        hosts.append((img, r, "mirror"))
    plan = mf.BatchPlan(items)
    info = plan.info()
    assert info["groups"] >= 3 and info["streams"] >= 2, info
    assert info["scratch_bytes"] > 0, info
    side = torch.cuda.Stream()
    plan.launch(side)
    side.synchronize()
    check(items, hosts, oracle_mod, "launch on a side stream")
    for _, out, _, _ in items:
        out.zero_()
    plan.launch()
    torch.cuda.synchronize()
    check(items, hosts, oracle_mod, "launch on the current stream")
    plan.capture(side)
    for rep in range(3):
        for _, out, _, _ in items:
            out.zero_()
        torch.cuda.synchronize()
        plan.replay(side)
        side.synchronize()
        check(items, hosts, oracle_mod, f"replay {rep}")
    plan.close()


def test_batched_single_group_plan(mf, oracle_mod):
    """A batch whose images all use one kernel variant runs as one group on
    the caller's stream."""
    items, hosts = [], []
    for i, (w, h) in enumerate([(70, 50), (130, 90), (64, 64)]):
        img = workloads.uniform(w, h, "u8", 60 + i)
        d = dev(img)
        items.append((d, torch.empty_like(d), mf.Footprint.disc(2), "clamp"))
        hosts.append((img, 2, "clamp"))
    plan = mf.BatchPlan(items)
    info = plan.info()
    assert info["groups"] == 1 and info["streams"] == 1, info
    plan.launch()
    torch.cuda.synchronize()
    check(items, hosts, oracle_mod, "single group")
    plan.close()


def test_batched_rejects_aliasing(mf):
    a = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    b = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    fp = mf.Footprint.disc(2)
    with pytest.raises(mf.MedianFilterError):
        mf.BatchPlan([(a, b, fp, "clamp"), (b, a, fp, "clamp")])


def test_batched_full_mixed_batch_sampled(mf, oracle_mod):
    """The full 64-image mixed batch (w, h in 128..2048, u8/u16/f32, disc
    radius 1..64, clamp) in one captured launch: every pixel equals the
    plain filter's and 48 seeded pixels per image equal the oracle's."""
    batch = workloads.mixed_batch(64, 3)
    fps, items, plain = {}, [], []
    for img_np, s in batch:
        r = s["radius"]
        if r not in fps:
            fps[r] = mf.Footprint.disc(r)
        d = dev(img_np)
        items.append((d, torch.empty_like(d), fps[r], "clamp"))
        plain.append(mf.median_filter(d, fps[r], "clamp"))
    plan = mf.BatchPlan(items)
    s = torch.cuda.Stream()
    plan.capture(s)
    plan.replay(s)
    s.synchronize()
    torch.cuda.synchronize()
    for i, ((img_np, sp), it, p) in enumerate(zip(batch, items, plain)):
        got = it[1].cpu().numpy()
        assert np.array_equal(got.view(np.uint8), p.cpu().numpy().view(np.uint8)), i
        rng = np.random.default_rng(i)
        h, w = img_np.shape
        xs, ys = rng.integers(0, w, 48), rng.integers(0, h, 48)
        exp = oracle_mod.filter_points(img_np, OF.disc(sp["radius"]), xs, ys, "clamp")
        assert np.array_equal(got[ys, xs].view(np.uint8), exp.view(np.uint8)), (i, sp)
    plan.close()


def test_batched_degenerate_images(mf, oracle_mod):
    """Empty planes, 1-pixel planes and single rows/columns beside ordinary
    ones in one plan: the empty ones are skipped, the rest equal the oracle."""
    shapes = [(0, 7), (5, 0), (1, 1), (1, 9), (13, 1), (40, 33)]
    items, exp = [], []
    for i, (w, h) in enumerate(shapes):
        img = workloads.uniform(max(w, 1), max(h, 1), "u16", 70 + i)[:h, :w]
        d = torch.from_numpy(np.ascontiguousarray(img)).cuda() if w and h else \
            torch.empty((h, w), dtype=torch.uint16, device="cuda")
        items.append((d, torch.empty_like(d), mf.Footprint.disc(3), "mirror"))
        exp.append(oracle_mod.filter(img, OF.disc(3), "mirror") if w and h else None)
    plan = mf.BatchPlan(items)
    assert plan.info()["tiles"] > 0
    plan.launch()
    torch.cuda.synchronize()
    for (d, out, _, _), e in zip(items, exp):
        if e is not None:
            assert np.array_equal(out.cpu().numpy(), e), d.shape
    plan.close()


def test_batch_aware_tuning_keeps_results_exact(mf, oracle_mod):
    """mf_plan_autotune: per-image tuned shapes are recorded first, then the
    batch tuner keeps each only where the whole batch runs faster.  The
    batch time never gets worse, and plans built afterwards (whatever
    shapes the table holds) still match the oracle bit for bit."""
    items, hosts = small_batch(mf, seed=11, n=10, size_hi=400, r_hi=40)
    seen = set()
    for (d, out, fp, b), (img, r, _) in zip(items, hosts):
        key = (str(img.dtype), r)
        if key not in seen:
            seen.add(key)
            mf.autotune(d, fp, b, out=out, reps=1)
    before, after, dropped = mf.plan_autotune(items, reps=2)
    assert before > 0 and after > 0 and after <= before
    assert 0 <= dropped <= len(seen)
    plan = mf.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    check(items, hosts, oracle_mod, "after batch tuning")
    plan.close()
    with pytest.raises(mf.MedianFilterError):
        mf.lib()  # library loaded; bad arguments are rejected on the host
        import ctypes
        rc = mf.lib().mf_plan_autotune(None, 3, None, 1, None, None, None)
        mf._check("mf_plan_autotune", rc)
