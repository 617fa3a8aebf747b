"""The request server (continuous batching) against the plain single-request
path and the oracle, through the C ABI.

Each request's outputs must be bit-identical to ripk_compute_K +
ripk_simulate_envelope on a plan of the same descriptor: the sums are exact
integers, so sharing the device with other requests changes nothing.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1912_04753_amd import ripk, workloads
from parity import compare

pytestmark = pytest.mark.gpu

DAY = workloads.DAY


def say(*a):
    print("[server]", *a, flush=True)
    sys.stdout.flush()


def make_requests(count, seed, n_lo=500, n_hi=40_000, m_hi=8):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        side = int(rng.integers(8_000, 40_000))
        dur = int(rng.integers(60, 400)) * DAY
        s_max = int(min(rng.integers(300, 3_000), side // 4))
        t_max = int(min(int(rng.integers(5, 60)) * DAY, dur // 4))
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        cfg = dict(seed=int(rng.integers(1 << 30)), window=(0, 0, side, side, 0, dur),
                   parts=[("uniform", n, {})] if rng.random() < 0.5 else
                   [("thomas", n, dict(parents=int(rng.integers(20, 200)),
                                       sigma_xy=float(rng.uniform(100, 400)),
                                       sigma_t=float(rng.uniform(2, 8)) * DAY))])
        x, y, t = workloads.make_points(cfg)
        reqs.append(dict(window=cfg["window"], s_max=s_max, t_max=t_max,
                         n_s=int(rng.integers(5, 65)), n_t=int(rng.integers(5, 65)),
                         m=int(rng.integers(0, m_hi + 1)), seed=(7 << 32) + r, x=x, y=y, t=t))
    return reqs


def desc_of(q, **kw):
    return ripk.make_desc(q["window"], q["s_max"], q["t_max"], q["n_s"], q["n_t"],
                          n_max=len(q["x"]), m_max=q["m"], **kw)


def plain(q, keep_sims=False):
    plan = ripk.ripk_plan(desc_of(q))
    try:
        r = ripk.ripk_compute_K(plan, q["x"], q["y"], q["t"])
        r["n_in"] = ripk.ripk_plan_stats(plan)["n_in"]
        if q["m"] > 0:
            e = ripk.ripk_simulate_envelope(plan, len(q["x"]), q["m"], q["seed"], L_obs=r["L"],
                                            per_sim=keep_sims)
            r.update(e)
            r["n_in"] += ripk.ripk_plan_stats(plan)["n_in"]
    finally:
        plan.destroy()
    return r


def same(a, b, where):
    for k in a:
        if k in b and isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), f"{where}: {k} differs"
    if "n_in" in a and "n_in" in b:
        assert a["n_in"] == b["n_in"], f"{where}: n_in differs"


def run_server(reqs, keep_sims=False, **kw):
    sv = ripk.ripk_server_create(**kw)
    try:
        tickets = [ripk.ripk_submit(sv, desc_of(q), q["x"], q["y"], q["t"], m=q["m"],
                                    seed=q["seed"], keep_sims=keep_sims) for q in reqs]
        out = [ripk.ripk_poll(sv, tk, timeout_ms=-1) for tk in tickets]
        state = ripk.ripk_server_status(sv)
    finally:
        sv.destroy()
    return out, state


def test_size_admission_sharing_and_slices_equal_alone():
    """Size-ordered admission (most requests large, one large at a time, aging)
    with device sharing at half the grid and pair launches cut into 50 us
    slices (several slices per request): every result bit-identical to the
    plain path, since slices and shares only change which workgroup takes
    which group of work items."""
    reqs = make_requests(16, seed=13)
    say("16 requests, sharing and slices")
    served, state = run_server(reqs, slots=4, admission=ripk.RIPK_ADMIT_SIZE, large_work=1e7,
                               age_ms=200.0, max_large=1, device_share=0.5, slice_ms=0.05)
    assert state["queued"] == 0 and state["unpolled"] == 0
    for i, (q, r) in enumerate(zip(reqs, served)):
        same(r, plain(q), f"request {i}")


def test_mix_equals_alone_and_oracle():
    reqs = make_requests(24, seed=11)
    say("24 requests, n", [len(q["x"]) for q in reqs])
    served, state = run_server(reqs, slots=4)
    assert state["queued"] == 0 and state["unpolled"] == 0
    slots_used = {r["slot"] for r in served}
    say("slots used", sorted(slots_used))
    assert len(slots_used) > 1
    overlaps = sum(1 for a in served for b in served
                   if a is not b and a["t_admit"] < b["t_admit"] < a["t_done"])
    say("overlapping admissions", overlaps)
    assert overlaps > 0
    for i, (q, r) in enumerate(zip(reqs, served)):
        same(r, plain(q), f"request {i}")
    # small ones against the oracle as well
    for i, (q, r) in enumerate(zip(reqs, served)):
        if len(q["x"]) > 6000:
            continue
        d = oracle.desc(q["window"], q["s_max"], q["t_max"], q["n_s"], q["n_t"])
        ref = oracle.estimate(d, q["x"], q["y"], q["t"])
        compare(r, ref, q["s_max"], q["t_max"], q["n_s"], q["n_t"], where=f"request {i}")
        assert r["n_in"] >= int(ref["C"][-1, -1])


def test_per_simulation_outputs_and_envelopes():
    reqs = [q for q in make_requests(6, seed=12, n_hi=8000, m_hi=6) if q["m"] > 0][:3]
    served, _ = run_server(reqs, keep_sims=True, slots=2)
    for i, (q, r) in enumerate(zip(reqs, served)):
        p = plain(q, keep_sims=True)
        same(r, p, f"request {i}")
        assert np.array_equal(r["K_lo"], p["K_sims"].min(axis=0))
        assert np.array_equal(r["dL_hi"], r["L"] - r["L_hi"])


def test_tight_budget_admits_by_footprint():
    reqs = make_requests(10, seed=13, n_lo=5_000, n_hi=30_000, m_hi=4)
    foot = [ripk.ripk_plan_check(desc_of(q))["device_bytes"] for q in reqs]
    budget = int(max(foot) * 1.2)
    say("footprints MB", [round(f / 1e6, 1) for f in foot], "budget", budget / 1e6)
    sv = ripk.ripk_server_create(slots=4, hbm_budget_bytes=budget)
    try:
        tickets = [ripk.ripk_submit(sv, desc_of(q), q["x"], q["y"], q["t"], m=q["m"], seed=q["seed"])
                   for q in reqs]
        peak = 0
        done = {}
        while len(done) < len(tickets):
            peak = max(peak, ripk.ripk_server_status(sv)["device_bytes"])
            for tk in tickets:
                if tk not in done:
                    r = ripk.ripk_poll(sv, tk, timeout_ms=0)
                    if r is not None:
                        done[tk] = r
            time.sleep(0.001)
    finally:
        sv.destroy()
    say("peak device bytes", peak)
    assert 0 < peak <= budget
    served = [done[tk] for tk in tickets]
    for i, (q, r) in enumerate(zip(reqs, served)):
        same(r, plain(q), f"request {i}")


def test_server_errors():
    q = make_requests(1, seed=14, n_lo=2000, n_hi=2001)[0]
    sv = ripk.ripk_server_create(slots=1, queue_cap=1, hbm_budget_bytes=1 << 20)
    try:
        with pytest.raises(ripk.RipkError) as e:   # footprint above the budget
            ripk.ripk_submit(sv, desc_of(q), q["x"], q["y"], q["t"], m=50)
        assert e.value.status == ripk.RIPK_E2BIG
        st = ripk.lib().ripk_poll(sv.handle, ripk._u64(12345), ripk.ctypes.byref(ripk.Result()), 0)
        assert st == ripk.RIPK_ENOTFOUND
    finally:
        sv.destroy()
    sv = ripk.ripk_server_create(slots=2, queue_cap=64)
    try:
        bad = dict(q)
        bad["x"] = q["x"].copy()
        bad["x"][5] = q["window"][2] + 10          # outside the window
        tb = ripk.ripk_submit(sv, desc_of(bad), bad["x"], bad["y"], bad["t"])
        tg = ripk.ripk_submit(sv, desc_of(q), q["x"], q["y"], q["t"], m=2, seed=q["seed"])
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_poll(sv, tb)
        assert e.value.status == ripk.RIPK_ERANGE
        q2 = dict(q, m=2)
        same(ripk.ripk_poll(sv, tg), plain(q2), "after an error")
        st = ripk.lib().ripk_poll(sv.handle, ripk._u64(tb), ripk.ctypes.byref(ripk.Result()), 0)
        assert st == ripk.RIPK_ENOTFOUND
    finally:
        sv.destroy()


def test_queue_full_and_shutdown_cancels():
    big = make_requests(1, seed=15, n_lo=60_000, n_hi=60_001)[0]
    sv = ripk.ripk_server_create(slots=1, queue_cap=1)
    statuses = []
    try:
        for _ in range(4):
            try:
                ripk.ripk_submit(sv, desc_of(dict(big, m=4)), big["x"], big["y"], big["t"], m=4,
                                 seed=1)
                statuses.append(0)
            except ripk.RipkError as e:
                statuses.append(e.status)
    finally:
        sv.destroy()          # cancels what is queued, waits for the running one
    say("submit statuses", statuses)
    assert statuses[0] == 0 and ripk.RIPK_EAGAIN in statuses
