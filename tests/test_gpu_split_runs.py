"""GPU tests of run fractions (RIPK_PLAN_SPLIT_RUNS): a single-set launch that
wants more work items than stencil rows cuts each row's neighbour run into
equal fractions.  Counts and fixed-point weights must not change, and the
candidates examined (n_eval, counted per fraction, including the triangular
home row of symmetric mode) must equal the whole-run count exactly.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04753_amd import ripk, workloads
from parity import compare

pytestmark = pytest.mark.gpu
DAY = workloads.DAY
WIN = (0, 0, 20_000, 20_000, 0, 200 * DAY)
ARGS = (WIN, 1_500, 20 * DAY, 10, 8)


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _clustered(n=30_000, seed=81):
    return workloads.thomas_points(np.random.default_rng(seed), n, WIN, 60, 150.0, 3.0 * DAY)


def _run(x, y, t, flags=0, n_centres=0, lam=None, **kw):
    plan = ripk.ripk_plan(ripk.make_desc(*ARGS, n_max=len(x), flags=flags, **kw))
    try:
        r = ripk.ripk_compute_K(plan, x, y, t, n_centres=n_centres, lam=lam)
        r["stats"] = ripk.ripk_plan_stats(plan)
        return r
    finally:
        plan.destroy()


@pytest.mark.parametrize("mode", ["symmetric", "ordered", "polygon", "cross"])
def test_split_runs_match_whole_runs(mode):
    x, y, t = _clustered()
    kw, flags, nc = {}, 0, 0
    if mode == "ordered":
        flags = ripk.RIPK_PLAN_ORDERED
    elif mode == "polygon":
        kw["poly"] = [(0, 0), (20_000, 0), (20_000, 12_000), (9_000, 20_000), (0, 20_000)]
        keep = workloads._strictly_inside(kw["poly"], x, y)  # the area holds every point
        x, y, t = x[keep], y[keep], t[keep]
    elif mode == "cross":
        flags, nc = ripk.RIPK_PLAN_CROSS, 12_000
    say("split runs", mode)
    a = _run(x, y, t, flags=flags, n_centres=nc, **kw)
    b = _run(x, y, t, flags=flags | ripk.RIPK_PLAN_SPLIT_RUNS, n_centres=nc, **kw)
    assert b["stats"]["split"] > a["stats"]["split"], (a["stats"]["split"], b["stats"]["split"])
    assert np.array_equal(a["C"], b["C"]) and np.array_equal(a["W"], b["W"])
    assert a["stats"]["n_eval"] == b["stats"]["n_eval"]
    if mode == "symmetric":
        compare(b, oracle.estimate(oracle.desc(*ARGS), x, y, t), *ARGS[1:], where="split runs")


def test_split_runs_inhomogeneous():
    x, y, t = _clustered(20_000, 82)
    lam = np.full(len(x), len(x) / (20_000.0 * 20_000.0 * 200 * DAY))
    a = _run(x, y, t, flags=ripk.RIPK_PLAN_INHOM, lam=lam)
    b = _run(x, y, t, flags=ripk.RIPK_PLAN_INHOM | ripk.RIPK_PLAN_SPLIT_RUNS, lam=lam)
    say("split runs inhomogeneous")
    assert b["stats"]["split"] > a["stats"]["split"]
    assert np.array_equal(a["C"], b["C"]) and a["stats"]["n_eval"] == b["stats"]["n_eval"]
    np.testing.assert_allclose(b["K"], a["K"], rtol=1e-12, atol=0)


def test_autotuned_clustered_set_matches_fixed_cells():
    """The autotuner also times run fractions for observed single sets; the
    result equals a fixed-cell plan whatever it picks."""
    x, y, t = _clustered(40_000, 83)
    a = _run(x, y, t)
    b = _run(x, y, t, flags=ripk.RIPK_PLAN_AUTOTUNE)
    say("autotuned clustered, split", b["stats"]["split"])
    assert np.array_equal(a["C"], b["C"]) and np.array_equal(a["W"], b["W"])


@pytest.mark.parametrize("n", [2, 65, 64 * 37 + 29])
@pytest.mark.parametrize("ordered", [False, True])
def test_split_runs_small_and_ragged_sets_match_oracle(n, ordered):
    """Small sets want far more parts than rows, so most fractions hold empty
    or one-point runs; a ragged last chunk and points on the window's sides
    and corners are included."""
    win = (0, 0, 6_000, 6_000, 0, 90 * DAY)
    args = (win, 900, 15 * DAY, 9, 7)
    x, y, t = workloads.uniform_points(np.random.default_rng(1000 + n), n, win)
    x[:2], y[:2], t[:2] = (0, 6_000), (6_000, 0), (0, 90 * DAY)  # corners and period ends
    flags = ripk.RIPK_PLAN_SPLIT_RUNS | (ripk.RIPK_PLAN_ORDERED if ordered else 0)
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=n, flags=flags))
    try:
        g = ripk.ripk_compute_K(plan, x, y, t)
        st = ripk.ripk_plan_stats(plan)
    finally:
        plan.destroy()
    say("split runs small n=%d ordered=%d split=%d" % (n, ordered, st["split"]))
    compare(g, oracle.estimate(oracle.desc(*args), x, y, t), *args[1:], where="split runs n=%d" % n)
    rows = 9 if ordered else 5  # stencil rows at one cell per s_max and t_max
    assert st["split"] >= 2 * rows, st["split"]  # at least two fractions per row
    nn = n * (n - 1)
    assert st["n_eval"] <= nn if ordered else st["n_eval"] <= nn // 2
