"""GPU tests of ripk_compute_K_envelope: the observed set and its simulations
in one call.

With CSR simulations the observed set is set 0 of the simulations' launch; the
results must equal ripk_compute_K followed by ripk_simulate_envelope (with the
observed L) bit for bit, and the simulations must be the oracle's draws.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04753_amd import ripk, workloads

pytestmark = pytest.mark.gpu
DAY = workloads.DAY
K_KEYS = ("C", "W", "K", "L")
ENV_KEYS = ("K_lo", "K_hi", "L_lo", "L_hi", "dL_hi")
SIM_KEYS = ("C_sims", "W_sims", "K_sims")


def say(*a):
    print("[gpu-case]", *a, flush=True)


def two_calls(desc, x, y, t, m, seed, n_centres=0):
    plan = ripk.ripk_plan(desc)
    try:
        k = ripk.ripk_compute_K(plan, x, y, t, n_centres=n_centres)
        e = ripk.ripk_simulate_envelope(plan, len(x), m, seed, L_obs=k["L"], per_sim=True)
    finally:
        plan.destroy()
    return {**k, **e}


def combined(desc, x, y, t, m, seed, n_centres=0, reps=1):
    plan = ripk.ripk_plan(desc)
    try:
        out = [ripk.ripk_compute_K_envelope(plan, x, y, t, m, seed, n_centres=n_centres,
                                            per_sim=True) for _ in range(reps)]
        stats = ripk.ripk_plan_stats(plan)
    finally:
        plan.destroy()
    return out, stats


def same(a, b, where):
    for k in K_KEYS + ENV_KEYS + SIM_KEYS:
        assert np.array_equal(a[k], b[k]), (where, k)


def _uniform(seed, n, win):
    return workloads.uniform_points(np.random.default_rng(seed), n, win)


def test_rectangle_matches_two_calls_and_oracle():
    win = (0, 0, 10_000, 10_000, 0, 365 * DAY)
    args = (win, 1_000, 30 * DAY, 10, 10)
    n, m, seed = 3_000, 4, 123
    x, y, t = _uniform(1, n, win)
    desc = ripk.make_desc(*args, n_max=n, m_max=m)
    say("combined rectangle n=%d m=%d" % (n, m))
    (g,), st = combined(desc, x, y, t, m, seed)
    same(g, two_calls(desc, x, y, t, m, seed), "rectangle")
    assert st["n_sets"] == m + 1
    d = oracle.desc(*args)
    r = oracle.estimate(d, x, y, t)
    assert np.array_equal(g["C"], r["C"].astype(np.uint64))
    np.testing.assert_allclose(g["K"], r["K"], rtol=1e-6, atol=0)
    ref = oracle.envelope(d, n, m, seed)
    assert np.array_equal(g["C_sims"], ref["C_sims"].astype(np.uint64))
    np.testing.assert_allclose(g["K_sims"], ref["K_sims"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(g["dL_hi"], g["L"] - g["L_hi"], rtol=0, atol=1e-9)


def test_full_size_workload_matches_two_calls():
    """The 100k workload with all 99 simulations (m = m_max: the plan holds
    m_max + 1 sets), autotuned."""
    c = workloads.workload("uniform-100k-99csr")
    x, y, t = workloads.make_points(c)
    m = c["sims"]
    desc = ripk.make_desc(c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"], n_max=len(x),
                          m_max=m, flags=ripk.RIPK_PLAN_AUTOTUNE)
    say("combined 100k x 99")
    (g,), st = combined(desc, x, y, t, m, c["seed"])
    plain = ripk.make_desc(c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"], n_max=len(x),
                           m_max=m)
    same(g, two_calls(plain, x, y, t, m, c["seed"]), "100k")
    assert st["n_sets"] == m + 1 and st["symmetric"] == 1


def test_polygon_and_cross_match_two_calls():
    c = workloads.workload("polygon-100k-99csr")
    star = workloads.polygon_of(c)
    args = (c["window"], 1_500, 20 * DAY, 10, 6)
    n, n1, m, seed = 2_500, 900, 3, 44
    x, y, t = workloads.polygon_points(np.random.default_rng(70), n, c["window"], star)
    say("combined polygon")
    desc = ripk.make_desc(*args, n_max=n, m_max=m, poly=star)
    (g,), _ = combined(desc, x, y, t, m, seed)
    same(g, two_calls(desc, x, y, t, m, seed), "polygon")
    say("combined polygon cross")
    desc = ripk.make_desc(*args, n_max=n, m_max=m, poly=star, flags=ripk.RIPK_PLAN_CROSS)
    (g,), st = combined(desc, x, y, t, m, seed, n_centres=n1)
    same(g, two_calls(desc, x, y, t, m, seed, n_centres=n1), "polygon cross")
    assert st["symmetric"] == 0
    ref = oracle.envelope_cross(oracle.desc(*args, poly=star), x, y, t, n1, m, seed, oracle.SIM_CSR)
    assert np.array_equal(g["C_sims"], ref["C_sims"].astype(np.uint64))


def test_cross_keeps_the_split_for_later_simulations():
    win = (0, 0, 12_000, 9_000, 0, 200 * DAY)
    args = (win, 1_500, 20 * DAY, 12, 9)
    n, n1, m, seed = 3_000, 1_100, 2, 9
    x, y, t = _uniform(3, n, win)
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=n, m_max=m, flags=ripk.RIPK_PLAN_CROSS))
    try:
        g = ripk.ripk_compute_K_envelope(plan, x, y, t, m, seed, n_centres=n1)
        e = ripk.ripk_simulate_envelope(plan, n, m, seed, L_obs=g["L"])
    finally:
        plan.destroy()
    say("combined cross split")
    for k in ENV_KEYS:
        assert np.array_equal(e[k], g[k]), k


@pytest.mark.parametrize("method", [ripk.RIPK_SIM_PERMUTE, ripk.RIPK_SIM_BOOTSTRAP])
def test_resampled_methods_run_the_two_calls(method):
    win = (0, 0, 10_000, 10_000, 0, 365 * DAY)
    args = (win, 1_000, 30 * DAY, 10, 10)
    n, m, seed = 2_000, 3, 5
    x, y, t = _uniform(4, n, win)
    desc = ripk.make_desc(*args, n_max=n, m_max=m, sim_method=method)
    say("combined resampled", method)
    (g,), _ = combined(desc, x, y, t, m, seed)
    same(g, two_calls(desc, x, y, t, m, seed), "resampled")


def test_device_inputs_graph_replays():
    """Device-resident points on a side stream through a graph plan: every
    replay equals the eager two-call result."""
    import torch
    win = (0, 0, 10_000, 10_000, 0, 365 * DAY)
    args = (win, 1_000, 30 * DAY, 10, 10)
    n, m, seed = 4_000, 3, 77
    x, y, t = _uniform(5, n, win)
    ref = two_calls(ripk.make_desc(*args, n_max=n, m_max=m), x, y, t, m, seed)
    dx, dy, dt = (torch.from_numpy(a).cuda() for a in (x, y, t))
    s = torch.cuda.Stream()
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=n, m_max=m, flags=ripk.RIPK_PLAN_GRAPH))
    try:
        for rep in range(3):
            with torch.cuda.stream(s):
                g = ripk.ripk_compute_K_envelope(plan, dx, dy, dt, m, seed, stream=s.cuda_stream,
                                                 per_sim=True)
            torch.cuda.synchronize()
            (dx + 1).sum().item()  # eager work between replays
            same(g, ref, "graph replay %d" % rep)
    finally:
        plan.destroy()
    say("combined graph replays")


def test_errors():
    win = (0, 0, 5_000, 5_000, 0, 100 * DAY)
    args = (win, 800, 20 * DAY, 8, 8)
    x, y, t = _uniform(6, 500, win)
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=500, m_max=2))
    try:
        for m in (0, 3):
            with pytest.raises(ripk.RipkError) as e:
                ripk.ripk_compute_K_envelope(plan, x, y, t, m, 1)
            assert e.value.status == ripk.RIPK_EINVAL, m
        bad = x.copy()
        bad[7] = 6_000  # outside the window
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_compute_K_envelope(plan, bad, y, t, 2, 1)
        assert e.value.status == ripk.RIPK_ERANGE
        g = ripk.ripk_compute_K_envelope(plan, x, y, t, 2, 1)  # the plan still works
        assert g["C"][-1, -1] > 0
    finally:
        plan.destroy()
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=500, m_max=2, flags=ripk.RIPK_PLAN_INHOM))
    try:
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_compute_K_envelope(plan, x, y, t, 2, 1)
        assert e.value.status == ripk.RIPK_EINVAL
    finally:
        plan.destroy()
    say("combined errors")
