"""The allocation-free entry point ripk_compute_K_noalloc against
ripk_compute_K, through the C ABI: two calls in a row (the second on a smaller
set and another grid, so the shared scratch array holds the first call's
contents), results bit for bit equal to a plan of the same descriptor, and the
size limit reported as an error before anything runs."""
import numpy as np
import pytest

from paper_1912_04753_amd import ripk, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def plain_K(desc, x, y, t, n_centres=0):
    plan = ripk.ripk_plan(desc)
    try:
        return ripk.ripk_compute_K(plan, x, y, t, n_centres=n_centres)
    finally:
        plan.destroy()


def noalloc_K(desc, x, y, t, n_centres=0):
    import torch
    nb = desc.n_s * desc.n_t
    out = {"C": torch.full((nb,), -1, dtype=torch.int64, device="cuda"),
           "W": torch.full((nb,), -1.0, dtype=torch.float64, device="cuda"),
           "K": torch.full((nb,), -1.0, dtype=torch.float64, device="cuda"),
           "L": torch.full((nb,), -1.0, dtype=torch.float64, device="cuda")}
    ripk.ripk_compute_K_noalloc(desc, x, y, t, out, n_centres=n_centres)
    torch.cuda.synchronize()
    shp = (desc.n_s, desc.n_t)
    return {"C": out["C"].cpu().numpy().view(np.uint64).reshape(shp),
            **{k: out[k].cpu().numpy().reshape(shp) for k in ("W", "K", "L")}}


def same(a, b, where):
    assert np.array_equal(a["C"], b["C"]), f"{where}: counts differ"
    for k in ("W", "K", "L"):
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{where}: {k} differs"


def cfg_desc(c, n, **kw):
    return ripk.make_desc(c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"], n_max=n, **kw)


def test_two_calls_match_plan_path():
    import torch
    torch.cuda.set_device(0)
    big = workloads.workload("uniform-100k-99csr")
    x, y, t = workloads.make_points(big)
    dx, dy, dt = (torch.from_numpy(a).cuda() for a in (x, y, t))
    d1 = cfg_desc(big, len(x), cell_div=2)
    say("noalloc call 1: uniform-100k device input n=%d" % len(x))
    g1 = noalloc_K(d1, dx, dy, dt)
    r1 = plain_K(d1, x, y, t)
    same(g1, r1, "call 1")
    assert int(g1["C"][-1, -1]) > 0
    small = workloads.workload("uniform-2k")
    xs, ys, ts = workloads.make_points(small)
    d2 = cfg_desc(small, len(xs))
    say("noalloc call 2: uniform-2k host input n=%d" % len(xs))
    g2 = noalloc_K(d2, xs, ys, ts)
    r2 = plain_K(d2, xs, ys, ts)
    same(g2, r2, "call 2")
    # ordered pairs and a centre subset, after the larger call
    d3 = cfg_desc(small, len(xs), flags=ripk.RIPK_PLAN_ORDERED)
    say("noalloc call 3: ordered, 700 centres")
    same(noalloc_K(d3, xs, ys, ts, n_centres=700), plain_K(d3, xs, ys, ts, n_centres=700),
         "call 3")


def test_thomas200k_matches_plan_path():
    c = workloads.workload("thomas-200k")
    x, y, t = workloads.make_points(c)
    d = cfg_desc(c, len(x), flags=ripk.RIPK_PLAN_SPLIT_RUNS)
    say("noalloc thomas-200k n=%d" % len(x))
    same(noalloc_K(d, x, y, t), plain_K(d, x, y, t), "thomas-200k")


def test_limits_and_errors():
    import torch
    c = workloads.workload("uniform-2k")
    x, y, t = workloads.make_points(c)
    nb = c["n_s"] * c["n_t"]
    out = {"C": torch.full((nb,), 7, dtype=torch.int64, device="cuda")}
    # 2M points exceed the 64 MiB scratch array: refused before any launch
    n = 2_000_000
    rng = np.random.default_rng(5)
    bx = rng.integers(0, 10_000, n).astype(np.int32)
    d = cfg_desc(c, n)
    with pytest.raises(ripk.RipkError) as e:
        ripk.ripk_compute_K_noalloc(d, bx, bx, bx, out)
    assert e.value.status == ripk.RIPK_E2BIG
    # a point outside the window: ERANGE, output untouched
    xb = x.copy()
    xb[5] = 10_001
    with pytest.raises(ripk.RipkError) as e:
        ripk.ripk_compute_K_noalloc(cfg_desc(c, len(x)), xb, y, t, out)
    assert e.value.status == ripk.RIPK_ERANGE
    assert bool((out["C"] == 7).all())
    # flags and study areas outside its scope
    for kw in (dict(flags=ripk.RIPK_PLAN_AUTOTUNE), dict(flags=ripk.RIPK_PLAN_CROSS),
               dict(poly=np.array([[0, 0], [9000, 0], [0, 9000]]))):
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_compute_K_noalloc(cfg_desc(c, len(x), **kw), x, y, t, out)
        assert e.value.status == ripk.RIPK_EINVAL
    # still correct after the refused calls
    same(noalloc_K(cfg_desc(c, len(x)), x, y, t), plain_K(cfg_desc(c, len(x)), x, y, t), "after")
