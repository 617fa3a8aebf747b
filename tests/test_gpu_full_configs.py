"""GPU parity at the full sizes of the large workloads, and of the histogram
flush that only they reach otherwise.

* Mid-set flush: with ``ripk_plan_set_flush_bound`` lowered to a few thousand
  candidates, every workgroup flushes its LDS bins after each group of work
  items, as workgroups of the 2M-point set do after 2^29 candidates; the
  oracle-compared cases (2k uniform, 200k clustered, the largest grids,
  sparse request windows, polygon and inhomogeneous launches) must stay
  bit-identical to the default runs and within tolerance of the oracle.
* The 2M mixed workload at full size: the symmetric launch (the one the
  benchmark times) against the ordered launch with 64-bit split counts, which
  share no bin layout, flush bound or candidate order, and against itself
  with mid-set flushes every 2^20 candidates; and the
  observed set plus simulations 0, 9 and 18 of the autotuned 19-simulation
  call against the oracle's values in ``tests/golden/mixed2m_19csr_oracle.npz``
  (written by ``tests/golden/make_mixed2m_golden.py``, oracle only).
* The 5,000-request serving stream: every request with n <= 20,000 (observed
  set and its first min(sims, 3) CSR simulations) against the oracle run here,
  and a seeded sample of 50 larger requests against
  ``tests/golden/stream50_oracle.npz`` (``make_stream_golden.py``).
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1912_04753_amd import ripk, workloads
from parity import compare, grid_values

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DAY = workloads.DAY
FLUSH = 4096


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _args(c):
    return (c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"])


def _run(args, x, y, t, flush=0, m=0, seed=0, lam=None, poly=None, **kw):
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=len(x), m_max=max(m, 0), poly=poly, **kw))
    try:
        if flush:
            ripk.ripk_plan_set_flush_bound(plan, flush)
        r = ripk.ripk_compute_K(plan, x, y, t, lam=lam) if lam is not None else \
            ripk.ripk_compute_K(plan, x, y, t)
        r["stats"] = ripk.ripk_plan_stats(plan)
        if m:
            r["env"] = ripk.ripk_simulate_envelope(plan, len(x), m, seed, per_sim=True)
        return r
    finally:
        plan.destroy()


def _flush_case(name):
    if name in ("uniform2k", "thomas200k"):
        c = workloads.workload({"uniform2k": "uniform-2k", "thomas200k": "thomas-200k"}[name])
        x, y, t = workloads.make_points(c)
        return _args(c), x, y, t, {}
    if name == "max_grid":
        rng = np.random.default_rng(21)
        win = (0, 0, 30_000, 30_000, 0, 400 * DAY)
        n = 24_000
        x = rng.integers(0, 30_001, n); y = rng.integers(0, 30_001, n)
        t = rng.integers(0, 400 * DAY + 1, n)
        return (win, 3_000, 40 * DAY, 64, 64), *(np.asarray(a, np.int32) for a in (x, y, t)), {}
    if name == "sparse":
        r = [r for r in workloads.serving_requests(num=300) if r["parts"][0][1] <= 7000][5]
        x, y, t = workloads.request_points(r)
        return (r["window"], r["s_max"], r["t_max"], r["n_s"], r["n_t"]), x, y, t, {}
    if name == "polygon":
        c = workloads.workload("polygon-100k-99csr")
        P = workloads.polygon_of(c)
        x, y, t = workloads.polygon_points(np.random.default_rng(61), 3000, c["window"], P)
        return (c["window"], 2000, 30 * DAY, 25, 15), x, y, t, {"poly": P}
    if name == "inhom":
        win = (0, 0, 10_000, 10_000, 0, 365 * DAY)
        x, y, t = workloads.uniform_points(np.random.default_rng(7), 4000, win)
        lam = (4000 / (1e8 * 365 * DAY)) * (0.5 + x / 10_000.0)
        return (win, 1_000, 30 * DAY, 10, 10), x, y, t, {"lam": lam, "flags": ripk.RIPK_PLAN_INHOM}
    raise KeyError(name)


@pytest.mark.parametrize("name", ["uniform2k", "thomas200k", "max_grid", "sparse", "polygon", "inhom"])
@pytest.mark.parametrize("ordered", [False, True])
def test_mid_set_flush_matches_default_and_oracle(name, ordered):
    args, x, y, t, kw = _flush_case(name)
    if ordered:
        kw = dict(kw, flags=kw.get("flags", 0) | ripk.RIPK_PLAN_ORDERED)
    m = 0 if name in ("thomas200k", "inhom") else 2
    say("flush", name, "ordered" if ordered else "symmetric", "n=%d" % len(x))
    a = _run(args, x, y, t, m=m, seed=31, **kw)
    b = _run(args, x, y, t, flush=FLUSH, m=m, seed=31, **kw)
    # the lowered bound flushes after every group: far more flushes, same sums
    for k in ("C", "W", "K", "L"):
        assert np.array_equal(a[k], b[k]), k
    if m:
        for k in ("C_sims", "W_sims", "K_sims"):
            assert np.array_equal(a["env"][k], b["env"][k]), k
    d = oracle.desc(*args, poly=kw.get("poly"))
    if "lam" in kw:
        r = oracle.estimate_inhom(d, x, y, t, kw["lam"])
    else:
        r = oracle.estimate(d, x, y, t)
    compare(b, r, *args[1:], where="flush " + name)
    if m:
        xs, ys, ts = oracle.csr_points(d, len(x), 1, 31)
        rs = oracle.estimate(d, xs, ys, ts)
        assert np.array_equal(b["env"]["C_sims"][1], rs["C"].astype(np.uint64))
        np.testing.assert_allclose(b["env"]["K_sims"][1], rs["K"], rtol=1e-6, atol=0)


def test_flush_bound_arguments():
    c = workloads.workload("uniform-2k")
    plan = ripk.ripk_plan(ripk.make_desc(*_args(c), n_max=10))
    try:
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_plan_set_flush_bound(plan, -1)
        assert e.value.status == ripk.RIPK_EINVAL
        for v in (0, 1, 1 << 40):
            ripk.ripk_plan_set_flush_bound(plan, v)
    finally:
        plan.destroy()


# ------------------------------------------------------------------ 2M -------
def test_mixed2m_symmetric_equals_ordered_wide_and_mid_set_flushes():
    """The whole 2M set and one simulation: the benchmark's launch (symmetric,
    32-bit counts) against the ordered launch with 64-bit split counts (every
    ordered pair found from its own centre, another bin layout and flush
    bound), and against the benchmark's launch with the flush bound lowered to
    2^20 candidates, so that its workgroups flush mid-set dozens of times:
    all bit-identical."""
    c = workloads.workload("mixed-2M-19csr")
    x, y, t = workloads.make_points(c)
    n = len(x)
    say("mixed2m symmetric vs ordered wide vs mid-set flushes, n=%d" % n)
    a = _run(_args(c), x, y, t, m=1, seed=c["seed"])
    b = _run(_args(c), x, y, t, m=1, seed=c["seed"],
             flags=ripk.RIPK_PLAN_ORDERED | ripk.RIPK_PLAN_WIDE_COUNTS)
    f = _run(_args(c), x, y, t, flush=1 << 20, m=1, seed=c["seed"])
    assert a["stats"]["bin_layout"] in (0, 1) and a["stats"]["symmetric"] == 1
    assert b["stats"]["bin_layout"] == 2 and b["stats"]["symmetric"] == 0
    for o in (b, f):
        for k in ("C", "W", "K", "L"):
            assert np.array_equal(a[k], o[k]), k
        for k in ("C_sims", "W_sims"):
            assert np.array_equal(a["env"][k], o["env"][k]), k
    # the symmetric launch examines about half the candidates
    assert b["stats"]["n_eval"] > 1.9 * a["stats"]["n_eval"]


def test_mixed2m_full_against_oracle_golden():
    """The autotuned combined call on all 2M points with its 19 CSR
    simulations, as the benchmark runs it: the observed set and simulations 0,
    9 and 18 against the oracle's C (exact) and W, K, L (Z12 tolerances)."""
    path = os.path.join(GOLDEN, "mixed2m_19csr_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/make_mixed2m_golden.py has not written its file")
    gold = np.load(path)
    c = workloads.workload("mixed-2M-19csr")
    x, y, t = workloads.make_points(c)
    n, m = len(x), c["sims"]
    assert int(gold["n"]) == n and int(gold["seed"]) == c["seed"]
    say("mixed2m golden: autotuned combined call, n=%d m=%d" % (n, m))
    plan = ripk.ripk_plan(ripk.make_desc(*_args(c), n_max=n, m_max=m,
                                         flags=ripk.RIPK_PLAN_AUTOTUNE))
    try:
        h = ripk.ripk_compute_K_envelope(plan, x, y, t, m, seed=c["seed"], per_sim=True)
        st = ripk.ripk_plan_stats(plan)
    finally:
        plan.destroy()
    assert st["n_sets"] == m + 1
    compare(h, {k: gold["obs_" + k] for k in ("C", "W", "K", "L")}, *_args(c)[1:],
            where="mixed2m observed")
    for s in gold["sims"]:
        g = {"C": h["C_sims"][s], "W": h["W_sims"][s], "K": h["K_sims"][s]}
        compare(g, {k: gold["sim%d_%s" % (s, k)] for k in ("C", "W", "K")}, *_args(c)[1:],
                where="mixed2m sim %d" % s)


# --------------------------------------------------------------- stream -----
def _stream_check(r, x, y, t, m, ref_sets):
    """One request through the combined call (observed + m simulations);
    ref_sets[k] = (C, K) of set k (observed first)."""
    args = (r["window"], r["s_max"], r["t_max"], r["n_s"], r["n_t"])
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=len(x), m_max=max(m, 1)))
    try:
        if m:
            h = ripk.ripk_compute_K_envelope(plan, x, y, t, m, seed=r["seed"], per_sim=True)
        else:
            h = ripk.ripk_compute_K(plan, x, y, t)
    finally:
        plan.destroy()
    s, tt = grid_values(*args[1:])
    for k, (C, K) in enumerate(ref_sets):
        Lr = np.sqrt(K / (2 * np.pi * tt)) - s   # Eq. 4 of the reference K
        if k == 0:
            g = {"C": h["C"], "K": h["K"], "L": h["L"]}
        else:
            Kg = h["K_sims"][k - 1]
            g = {"C": h["C_sims"][k - 1], "K": Kg, "L": np.sqrt(Kg / (2 * np.pi * tt)) - s}
        compare(g, {"C": C, "K": K, "L": Lr}, *args[1:], where="request %d set %d" % (r["id"], k))


def test_stream_small_requests_against_oracle():
    """Every request of the 5,000-request stream with n <= 20,000 (about 2,340):
    its observed set and its first min(sims, 3) simulations, through the
    combined call, against the oracle run here on the host cores."""
    reqs = [r for r in workloads.serving_requests(num=5000) if r["parts"][0][1] <= 20_000]
    assert len(reqs) > 2000
    say("stream: %d requests with n <= 20000" % len(reqs))
    for i, r in enumerate(reqs):
        x, y, t = workloads.request_points(r)
        n, m = len(x), min(r["sims"], 3)
        d = oracle.desc(r["window"], r["s_max"], r["t_max"], r["n_s"], r["n_t"])
        ref = []
        for s in range(-1, m):
            pts = (x, y, t) if s < 0 else oracle.csr_points(d, n, s, r["seed"])
            o = oracle.estimate(d, *pts)
            ref.append((o["C"], o["K"]))
        _stream_check(r, x, y, t, m, ref)
        if i % 250 == 0:
            say("stream small: %d of %d" % (i, len(reqs)))


def test_stream_sampled_large_requests_against_golden():
    """50 seeded requests of the stream with n > 20,000 (up to 442,172 points),
    observed set and first min(sims, 3) simulations, against the oracle's
    values stored by make_stream_golden.py."""
    path = os.path.join(GOLDEN, "stream50_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/make_stream_golden.py has not written its file")
    gold = np.load(path)
    reqs = workloads.serving_requests(num=5000)
    ids = [int(i) for i in gold["ids"]]
    assert len(ids) == 50
    for i in ids:
        r = reqs[i]
        x, y, t = workloads.request_points(r)
        C, K = gold["r%d_C" % i], gold["r%d_K" % i]
        m = len(C) - 1
        assert m == min(r["sims"], 3) and len(x) > 20_000
        say("stream large: request %d n=%d sims=%d" % (i, len(x), m))
        _stream_check(r, x, y, t, m, list(zip(C, K)))


@pytest.mark.parametrize("name", ["uniform2k", "thomas200k", "sparse", "polygon", "inhom"])
def test_cost_ordered_work_list_matches_default(name):
    """RIPK_PLAN_COST_ORDER hands the groups of a split launch out costliest
    first: the same sums bit for bit, in symmetric and ordered plans, and the
    workgroups of the 200k clustered set end close together."""
    args, x, y, t, kw = _flush_case(name)
    flags = kw.pop("flags", 0)
    for extra in (0, ripk.RIPK_PLAN_ORDERED):
        a = _run(args, x, y, t, flags=flags | extra | ripk.RIPK_PLAN_TIMING, **kw)
        b = _run(args, x, y, t, flags=flags | extra | ripk.RIPK_PLAN_TIMING |
                 ripk.RIPK_PLAN_COST_ORDER, **kw)
        say("cost order", name, extra, a["stats"]["split"], b["stats"]["cost_ordered"],
            "ends (median, p90, max) us", b["stats"]["us_wg_end_median"],
            b["stats"]["us_wg_end_p90"], b["stats"]["us_wg_end_max"])
        assert a["stats"]["cost_ordered"] == 0
        # (the order needs a split launch whose groups fit the point buffers)
        if name in ("thomas200k", "polygon"):
            assert b["stats"]["cost_ordered"] == 1
        for k in ("C", "W", "K", "L"):
            assert np.array_equal(a[k], b[k]), k
        assert a["stats"]["n_eval"] == b["stats"]["n_eval"]


def test_cost_ordered_clustered_set_ends_together():
    """The 200k clustered set on half-s_max, half-t_max cells with run
    fractions: handed out costliest first, its workgroups end within 15% of
    the median one (unordered, the dense clusters' groups end the launch)."""
    c = workloads.workload("thomas-200k")
    x, y, t = workloads.make_points(c)
    kw = dict(cell_div=2, tcell_div=2)
    fl = ripk.RIPK_PLAN_TIMING | ripk.RIPK_PLAN_SPLIT_RUNS
    for _ in range(2):   # (first launches warm the device up)
        a = _run(_args(c), x, y, t, flags=fl, **kw)
        b = _run(_args(c), x, y, t, flags=fl | ripk.RIPK_PLAN_COST_ORDER, **kw)
    sa, sb = a["stats"], b["stats"]
    say("clustered ends: default", sa["us_wg_end_median"], sa["us_wg_end_max"],
        "cost ordered", sb["us_wg_end_median"], sb["us_wg_end_max"])
    assert sb["cost_ordered"] == 1 and np.array_equal(a["W"], b["W"])
    assert sb["us_wg_end_max"] <= 1.15 * sb["us_wg_end_median"]
