"""GPU parity of the two-type (cross) K estimator against the FP64 oracle.

Type 1 = points [0, n_centres), type 2 = the rest; the library runs the pair
kernel with type-1 records marked as no neighbour.  Counts bit for bit, W, K and
L within the tolerances of ``tests/parity.py``.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04753_amd import ripk, workloads
from parity import compare

pytestmark = pytest.mark.gpu
DAY = workloads.DAY


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _two_types(seed, n, n1, win, cluster=False):
    rng = np.random.default_rng(seed)
    x0, y0, x1, y1, t0, t1 = win
    x = rng.integers(x0, x1 + 1, n)
    y = rng.integers(y0, y1 + 1, n)
    t = rng.integers(t0, t1 + 1, n)
    if cluster:  # type 1 in a few space-time clusters, type 2 uniform
        c = rng.integers(0, 5, n1)
        cx = rng.integers(x0, x1, 5)[c]; cy = rng.integers(y0, y1, 5)[c]; ct = rng.integers(t0, t1, 5)[c]
        x[:n1] = np.clip(cx + rng.normal(0, (x1 - x0) / 40, n1), x0, x1)
        y[:n1] = np.clip(cy + rng.normal(0, (y1 - y0) / 40, n1), y0, y1)
        t[:n1] = np.clip(ct + rng.normal(0, (t1 - t0) / 40, n1), t0, t1)
    k = min(5, n1, n - n1)  # coincident points across the types
    x[n1:n1 + k] = x[:k]; y[n1:n1 + k] = y[:k]; t[n1:n1 + k] = t[:k]
    return tuple(np.asarray(a, np.int32) for a in (x, y, t))


def _cross(args, x, y, t, n1, flags=0, edge=3, m_max=0, **kw):
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=len(x), m_max=m_max, edge=edge,
                                         flags=flags | ripk.RIPK_PLAN_CROSS, **kw))
    try:
        r = ripk.ripk_compute_K(plan, x, y, t, n_centres=n1)
        r["stats"] = ripk.ripk_plan_stats(plan)
        r["info"] = ripk.ripk_plan_get_info(plan)
        return r
    finally:
        plan.destroy()


CASES = {
    # name: (window, s_max, t_max, n_s, n_t, n, n1, cluster, edge, flags)
    "uniform": ((0, 0, 10_000, 10_000, 0, 365 * DAY), 1_000, 30 * DAY, 10, 10, 4_000, 1_500, False, 3, 0),
    "clustered": ((0, 0, 20_000, 15_000, 0, 200 * DAY), 2_000, 20 * DAY, 16, 12, 12_000, 5_000, True, 3, 0),
    "no_correction": ((0, 0, 10_000, 10_000, 0, 365 * DAY), 1_000, 30 * DAY, 10, 10, 3_000, 1_000, False, 0, 0),
    "spatial_only": ((0, 0, 10_000, 10_000, 0, 365 * DAY), 1_000, 30 * DAY, 7, 9, 3_000, 1_000, True, 1, 0),
    "temporal_only": ((0, 0, 10_000, 10_000, 0, 365 * DAY), 1_000, 30 * DAY, 9, 7, 3_000, 2_000, False, 2, 0),
    "one_type1": ((0, 0, 5_000, 5_000, 0, 100 * DAY), 800, 20 * DAY, 8, 8, 2_000, 1, False, 3, 0),
    "one_type2": ((0, 0, 5_000, 5_000, 0, 100 * DAY), 800, 20 * DAY, 8, 8, 2_000, 1_999, False, 3, 0),
    "u32": ((0, 0, 100_000, 80_000, 0, 400 * DAY), 10_000, 40 * DAY, 12, 10, 6_000, 2_500, True, 3, 0),
    "wide": ((0, 0, 400_000, 300_000, 0, 400 * DAY), 60_000, 40 * DAY, 12, 10, 5_000, 2_000, True, 3, 0),
    "ordered_flag": ((0, 0, 10_000, 10_000, 0, 365 * DAY), 1_000, 30 * DAY, 10, 10, 3_000, 1_200, True, 3,
                     ripk.RIPK_PLAN_ORDERED),
    "autotune": ((0, 0, 20_000, 15_000, 0, 200 * DAY), 2_000, 20 * DAY, 16, 12, 12_000, 5_000, True, 3,
                 ripk.RIPK_PLAN_AUTOTUNE),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_cross_k_matches_oracle(name):
    win, s_max, t_max, n_s, n_t, n, n1, cluster, edge, flags = CASES[name]
    x, y, t = _two_types(len(name) * 7 + n, n, n1, win, cluster)
    say("cross", name, "n=%d n1=%d" % (n, n1))
    args = (win, s_max, t_max, n_s, n_t)
    g = _cross(args, x, y, t, n1, flags=flags, edge=edge)
    d = oracle.desc(*args, edge=edge)
    r = oracle.estimate_cross(d, x, y, t, n1)
    compare(g, r, s_max, t_max, n_s, n_t, where="cross " + name)
    assert g["stats"]["n_in"] == int(r["C"][-1, -1])
    if name in ("u32", "wide"):
        assert g["info"]["dist_mode"] == (1 if name == "u32" else 2)


@pytest.mark.parametrize("method", [ripk.RIPK_SIM_CSR, ripk.RIPK_SIM_PERMUTE,
                                    ripk.RIPK_SIM_BOOTSTRAP])
def test_cross_simulations_match_oracle(method):
    """Simulations keep the type split of the last observed set: CSR sets with
    their first n1 points as type 1, permuted time labels, per-type bootstrap."""
    win = (0, 0, 12_000, 9_000, 0, 200 * DAY)
    args = (win, 1_500, 20 * DAY, 12, 9)
    n, n1, m, seed = 3_000, 1_100, 4, 808
    x, y, t = _two_types(40 + method, n, n1, win, cluster=True)
    d = oracle.desc(*args)
    ref = oracle.envelope_cross(d, x, y, t, n1, m, seed, method)
    plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=n, m_max=m, sim_method=method,
                                         flags=ripk.RIPK_PLAN_CROSS))
    try:
        with pytest.raises(ripk.RipkError) as e:   # no observed split yet
            ripk.ripk_simulate_envelope(plan, n, m, seed)
        assert e.value.status == ripk.RIPK_EINVAL
        with pytest.raises(ripk.RipkError):        # a cross plan needs the split
            ripk.ripk_compute_K(plan, x, y, t)
        obs = ripk.ripk_compute_K(plan, x, y, t, n_centres=n1)
        g = ripk.ripk_simulate_envelope(plan, n, m, seed, L_obs=obs["L"], per_sim=True)
    finally:
        plan.destroy()
    say("cross sims", method)
    assert np.array_equal(g["C_sims"], ref["C_sims"].astype(np.uint64))
    np.testing.assert_allclose(g["K_sims"], ref["K_sims"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(g["K_lo"], ref["K_lo"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(g["K_hi"], ref["K_hi"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(g["dL_hi"], obs["L"] - g["L_hi"], rtol=0, atol=1e-9)


def _uniform100k():
    c = workloads.workload("uniform-100k-99csr")
    return c, workloads.make_points(c)


def test_cross_terms_partition_full_size():
    """At the 100k workload split 40k / 60k: the univariate counts and fixed-point
    weight sums equal the sum of the two within-type and the two cross terms
    (each pair's weight depends only on its centre, d and u)."""
    c, (x, y, t) = _uniform100k()
    n, n1 = len(x), 40_000
    args = (c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"])
    say("cross partition 100k")

    def uni(xs, ys, ts):
        plan = ripk.ripk_plan(ripk.make_desc(*args, n_max=len(xs)))
        try:
            return ripk.ripk_compute_K(plan, xs, ys, ts)
        finally:
            plan.destroy()

    full = uni(x, y, t)
    aa = uni(x[:n1], y[:n1], t[:n1])
    bb = uni(x[n1:], y[n1:], t[n1:])
    ab = _cross(args, x, y, t, n1)
    sw = np.concatenate([np.arange(n1, n), np.arange(n1)])
    ba = _cross(args, x[sw], y[sw], t[sw], n - n1)
    assert np.array_equal(aa["C"] + bb["C"] + ab["C"] + ba["C"], full["C"])
    np.testing.assert_allclose(aa["W"] + bb["W"] + ab["W"] + ba["W"], full["W"], rtol=1e-14, atol=0)
    assert np.array_equal(ab["C"], ba["C"])


def test_cross_sampled_type1_at_full_size():
    """800 sampled type-1 points against the other 99,200 points of the 100k set
    as type 2: the whole cross grid against the oracle."""
    c, (x, y, t) = _uniform100k()
    n, n1 = len(x), 800
    rng = np.random.default_rng(12)
    pick = rng.choice(n, n1, replace=False)
    rest = np.setdiff1d(np.arange(n), pick)
    order = np.concatenate([pick, rest])
    xs, ys, ts = x[order], y[order], t[order]
    args = (c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"])
    say("cross sampled 100k")
    g = _cross(args, xs, ys, ts, n1)
    r = oracle.estimate_cross(oracle.desc(*args), xs, ys, ts, n1)
    compare(g, r, c["s_max"], c["t_max"], c["n_s"], c["n_t"], where="cross sampled")


def test_cross_request_through_server():
    """A cross-K request with simulations through the server equals the direct calls."""
    win = (0, 0, 12_000, 9_000, 0, 200 * DAY)
    args = (win, 1_500, 20 * DAY, 12, 9)
    n, n1, m, seed = 2_500, 900, 3, 17
    x, y, t = _two_types(77, n, n1, win, cluster=True)
    desc = ripk.make_desc(*args, n_max=n, m_max=m, flags=ripk.RIPK_PLAN_CROSS)
    plan = ripk.ripk_plan(desc)
    try:
        obs = ripk.ripk_compute_K(plan, x, y, t, n_centres=n1)
        env = ripk.ripk_simulate_envelope(plan, n, m, seed)
    finally:
        plan.destroy()
    srv = ripk.ripk_server_create(slots=2)
    try:
        tk = ripk.ripk_submit(srv, desc, x, y, t, m=m, seed=seed, n_centres=n1)
        res = ripk.ripk_poll(srv, tk, timeout_ms=-1)
    finally:
        ripk.ripk_server_destroy(srv)
    say("cross server")
    assert np.array_equal(res["C"], obs["C"]) and np.array_equal(res["W"], obs["W"])
    assert np.array_equal(res["L_lo"], env["L_lo"]) and np.array_equal(res["L_hi"], env["L_hi"])
