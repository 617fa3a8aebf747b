"""Benchmark: space-time Ripley's K pair range count on one MI355X.

One step = the whole path over the batched-envelope workload: K/L of the
observed set (100,000 uniform points in 20 km x 20 km x 180 d, 25 x 15 grid to
2 km / 30 d, isotropic spatial + temporal correction) and the envelope of 99
Monte Carlo CSR simulations of the same size drawn on the device, in one
``ripk_compute_K_envelope`` call (the observed set is one more set of the
simulations' launch).  Inputs are resident in device memory before timing
starts.  ``two_calls`` times the same step as ``ripk_compute_K`` followed by
``ripk_simulate_envelope``.

Printed: one JSON line.  ``value`` = ordered in-range pair tests per second
(N_in over the step, in units of 1e9/s); ``sims_per_s``; ``roofline`` for the
pair kernel (integer ALU bound: 9 lane-ops per candidate pair against
compute units x 64 lanes x peak engine clock, read from the device), with HBM
traffic per launch from the stored counter summary while the pair kernel is
unchanged, and the same fraction for every other leg; ``cpu_baseline`` = the
FP64 oracle on the host cores over the observed set and as many of its
simulations as fit in about 12 s, plus one thread on the 2k set and on a
sample of centres of the 200k clustered set.
"""
import argparse
import json
import os
import subprocess
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G space-time pair tests/s + sims/s at 1 GPU; served p50/p99 latency vs plain path"
OPS_PER_EVAL = 9            # minimal integer test of one candidate pair (lane-ops)
OPS_PER_IN = 10             # bin (6) + fast-path weight (4) of one in-range ordered pair
PEAK = {"lane_ops": 256 * 64 * 2.4e9}   # CUs x lanes x clock, replaced by the device's figures


def leg_roof(stats, us_pair):
    """Candidates, mean pair-kernel time and roofline fraction of a leg."""
    ev = int(stats["n_eval"])
    return {"n_eval": ev, "pair_kernel_us": round(us_pair, 2),
            "frac": round(OPS_PER_EVAL * ev / (us_pair * 1e-6) / PEAK["lane_ops"], 4)
            if us_pair > 0 else None}


def cpu_baseline(cfg, x, y, t, target_s):
    """The FP64 oracle on the host cores: the observed set, then CSR simulations
    drawn by the oracle's own Philox, until about target_s seconds of work."""
    import oracle
    d = oracle.desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"])
    n = len(x)
    threads = oracle.max_threads()
    t0 = oracle.now()
    r = oracle.estimate(d, x, y, t, threads=threads)
    n_in = int(r["C"][-1, -1])
    sets = 1
    while oracle.now() - t0 < target_s and sets <= cfg["sims"]:
        xs, ys, ts = oracle.csr_points(d, n, sets - 1, cfg["seed"])
        r = oracle.estimate(d, xs, ys, ts, threads=threads)
        n_in += int(r["C"][-1, -1])
        sets += 1
    dt = oracle.now() - t0
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # one thread: the 2k set whole, and 4,000 centres of the 200k clustered set
    # against all its points
    from paper_1912_04753_amd import workloads
    one = {}
    for wname, nc in (("uniform-2k", None), ("thomas-200k", 4000)):
        wc = workloads.workload(wname)
        wx, wy, wt = workloads.make_points(wc)
        wd = oracle.desc(wc["window"], wc["s_max"], wc["t_max"], wc["n_s"], wc["n_t"])
        t1 = oracle.now()
        r1 = oracle.estimate(wd, wx, wy, wt, n_centres=nc, threads=1)
        d1 = oracle.now() - t1
        one[wname] = {"value": round(int(r1["C"][-1, -1]) / d1 / 1e9, 6),
                      "seconds": round(d1, 3),
                      "sample": "every ordered pair" if nc is None else
                                f"the first {nc} of {len(wx)} points as centres, every point "
                                f"as neighbour"}
    return {"value": n_in / dt / 1e9, "unit": "G pair tests/s", "cores": threads,
            "kind": "oracle", "cpu": cpu,
            "sample": f"observed set of the workload plus {sets - 1} of its {cfg['sims']} CSR "
                      f"simulations ({sets} sets of {n} points, every ordered pair); "
                      f"{n_in} in-range ordered pairs in {dt:.2f} s",
            "one_thread": one}


# the server configuration the serving leg reports (ripk_server_desc fields)
SERVER = {"admission": 1, "large_work": 2e10, "age_ms": 1000.0, "max_large": 2,
          "device_share": 0.9375, "slice_ms": 20.0}


def serving(ripk, workloads, n_req, slots, load, cap_n=200, variants=()):
    """The request stream served two ways on the same arrival schedule: the plain
    path (one request at a time, in arrival order: a plan, ripk_compute_K and
    ripk_simulate_envelope each) and the server (continuous batching over
    `slots` streams).  Arrivals are Poisson at `load` x the plain path's
    capacity, measured on the first `cap_n` requests; latency = completion -
    scheduled arrival.  The server's own capacity is the first `cap_n`
    requests submitted at once."""
    import numpy as np
    reqs = workloads.serving_requests(num=n_req)
    cap_n = min(cap_n, n_req)
    pts = [workloads.request_points(r) for r in reqs]
    descs = [ripk.make_desc(r["window"], r["s_max"], r["t_max"], r["n_s"], r["n_t"],
                            n_max=len(p[0]), m_max=r["sims"]) for r, p in zip(reqs, pts)]

    def plain_one(i):
        r, (x, y, t) = reqs[i], pts[i]
        plan = ripk.ripk_plan(descs[i])
        try:
            k = ripk.ripk_compute_K(plan, x, y, t)
            n_in = ripk.ripk_plan_stats(plan)["n_in"]
            if r["sims"] > 0:
                ripk.ripk_simulate_envelope(plan, len(x), r["sims"], r["seed"], L_obs=k["L"])
                n_in += ripk.ripk_plan_stats(plan)["n_in"]
        finally:
            plan.destroy()
        return n_in

    plain_one(0)  # warm-up
    t0 = time.monotonic()
    for i in range(cap_n):
        plain_one(i)
    capacity = cap_n / (time.monotonic() - t0)
    print(f"serving: plain capacity {capacity:.2f} requests/s on {cap_n}", file=sys.stderr,
          flush=True)
    rate = load * capacity
    gaps = np.random.Generator(np.random.PCG64(55)).exponential(1.0 / rate, n_req)
    offs = np.cumsum(gaps) - gaps[0]

    def wait_until(a):
        d = a - time.monotonic()
        if d > 0:
            time.sleep(d)

    # plain path on the arrival schedule
    start = time.monotonic() + 0.05
    lat_plain, end_plain, n_in_total = [], start, 0
    for i in range(n_req):
        a = start + offs[i]
        wait_until(a)
        n_in_total += plain_one(i)
        end_plain = time.monotonic()
        lat_plain.append(end_plain - a)
        if (i + 1) % 250 == 0:
            print(f"serving: plain {i + 1}/{n_req}", file=sys.stderr, flush=True)
    span_plain = end_plain - start

    def replay(cfg, burst):
        """The server with configuration cfg on the same schedule; with burst,
        its capacity on the first cap_n requests submitted at once."""
        sv = ripk.ripk_server_create(slots=slots, queue_cap=n_req, hbm_budget_bytes=64 << 30,
                                     **cfg)
        tickets = [None] * n_req
        ready = [threading.Event() for _ in range(n_req)]
        start = time.monotonic() + 0.05

        def submitter():
            for i in range(n_req):
                wait_until(start + offs[i])
                r, (x, y, t) = reqs[i], pts[i]
                tickets[i] = ripk.ripk_submit(sv, descs[i], x, y, t, m=r["sims"], seed=r["seed"])
                ready[i].set()

        th = threading.Thread(target=submitter)
        th.start()
        lat_srv, end_srv, n_in_srv = [], start, 0
        for i in range(n_req):
            ready[i].wait()
            res = ripk.ripk_poll(sv, tickets[i], timeout_ms=-1)
            lat_srv.append(res["t_done"] - (start + offs[i]))
            end_srv = max(end_srv, res["t_done"])
            n_in_srv += res["n_in"]
            if (i + 1) % 250 == 0:
                print(f"serving: served {i + 1}/{n_req}", file=sys.stderr, flush=True)
        th.join()
        assert n_in_srv == n_in_total
        cap = None
        if burst:
            t_burst = time.monotonic()
            tks = [ripk.ripk_submit(sv, descs[i], *pts[i], m=reqs[i]["sims"],
                                    seed=reqs[i]["seed"]) for i in range(cap_n)]
            end_burst = max(ripk.ripk_poll(sv, tk, timeout_ms=-1)["t_done"] for tk in tks)
            cap = cap_n / (end_burst - t_burst)
        sv.destroy()
        return lat_srv, end_srv - start, cap

    lat_srv, span_srv, served_capacity = replay(SERVER, True)

    def summary(lat, span):
        lat = np.sort(np.asarray(lat)) * 1e3
        return {"p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "pair_tests_per_s_G": round(n_in_total / span / 1e9, 3)}

    plain, served = summary(lat_plain, span_plain), summary(lat_srv, span_srv)
    others = []
    for cfg in variants:
        lat_v, span_v, _ = replay(cfg, False)
        sm = summary(lat_v, span_v)
        others.append({"server": cfg, **sm,
                       "over_plain": {"p50": round(sm["p50_ms"] / plain["p50_ms"], 3),
                                      "p99": round(sm["p99_ms"] / plain["p99_ms"], 3)}})
    return {"requests": n_req, "of_stream": 5000, "load": load, "rate_per_s": round(rate, 3),
            "plain_capacity_per_s": round(capacity, 3),
            "served_capacity_per_s": round(served_capacity, 3), "capacity_requests": cap_n,
            "slots": slots, "n_in": int(n_in_total), "server": SERVER,
            "plain": plain, "served": served, "variants": others,
            "served_over_plain": {"p50": round(served["p50_ms"] / plain["p50_ms"], 3),
                                  "p99": round(served["p99_ms"] / plain["p99_ms"], 3)},
            "note": "request stream: n log-uniform [1e3, 5e5], uniform or Thomas, own window "
                    "and grid, 0-99 CSR sims; host points in, H2D included; plain path "
                    "creates a plan per request; capacities on the first capacity_requests"}


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    from paper_1912_04753_amd.profiling import COPY_BYTES
    src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def polygon_leg(ripk, workloads, torch, stream, steps=3):
    """Polygon study area: 100k points uniform inside an 85-vertex boundary of
    the 20 km window, observed K + 99 CSR simulations (rejection inside the
    polygon) in one call, autotuned cells."""
    pc = workloads.workload("polygon-100k-99csr")
    poly = workloads.polygon_of(pc)
    px, py, pt = (torch.from_numpy(a).cuda() for a in workloads.make_points(pc))
    pn, pm = len(px), pc["sims"]
    pplan = ripk.ripk_plan(ripk.make_desc(pc["window"], pc["s_max"], pc["t_max"], pc["n_s"],
                                          pc["n_t"], n_max=pn, m_max=pm, poly=poly,
                                          flags=ripk.RIPK_PLAN_AUTOTUNE | ripk.RIPK_PLAN_TIMING))

    def pstep():
        t1 = time.perf_counter()
        ripk.ripk_compute_K_envelope(pplan, px, py, pt, pm, pc["seed"], stream=stream)
        b = ripk.ripk_plan_stats(pplan)
        return b["n_in"], time.perf_counter() - t1, b["us_pair"], b

    pstep()  # tuning
    pstep()
    torch.cuda.synchronize()
    t_p = time.perf_counter()
    ps = [pstep() for _ in range(steps)]
    torch.cuda.synchronize()
    p_ms = 1e3 * (time.perf_counter() - t_p) / steps
    pi_ = ripk.ripk_plan_get_info(pplan)
    polygon = {"ms_per_step": round(p_ms, 3),
               "pair_tests_per_s_G": round(ps[0][0] / (p_ms * 1e-3) / 1e9, 3),
               "sims_per_s": round(pm / (sum(v[1] for v in ps) / steps), 3),
               "pair_kernel_us": round(sum(v[2] for v in ps) / steps, 2),
               "phases_us": {k: round(sum(v[3][k] for v in ps) / steps, 1)
                             for k in ("us_gen", "us_grid", "us_pair", "us_finalize")},
               "cells_m_s": [pi_["cell_s"], pi_["cell_t"]],
               "roofline": leg_roof(ps[0][3], sum(v[2] for v in ps) / steps),
               "note": "100k uniform points inside an 85-vertex star-shaped boundary "
                       "(46% of the 20 km x 20 km window), 180 d, 25x15 grid to 2 km/30 d, "
                       "observed K + 99 CSR simulations"}
    pplan.destroy()
    return polygon


def larger_leg(ripk, workloads, torch, stream, wname, reps):
    """One of the larger workloads, autotuned: its step time from an untimed plan
    (median call), its phases and roofline from a timed plan."""
    wc = workloads.workload(wname)
    wx, wy, wt = (torch.from_numpy(a).cuda() for a in workloads.make_points(wc))
    wn, wm = len(wx), wc["sims"]
    wplan = ripk.ripk_plan(ripk.make_desc(wc["window"], wc["s_max"], wc["t_max"], wc["n_s"],
                                          wc["n_t"], n_max=wn, m_max=wm,
                                          flags=ripk.RIPK_PLAN_AUTOTUNE | ripk.RIPK_PLAN_TIMING))

    def wstep():
        t1 = time.perf_counter()
        if wm == 0:
            ripk.ripk_compute_K(wplan, wx, wy, wt, stream=stream)
        else:
            ripk.ripk_compute_K_envelope(wplan, wx, wy, wt, wm, wc["seed"], stream=stream)
        b = ripk.ripk_plan_stats(wplan)
        return b["n_in"], time.perf_counter() - t1, dict(b)

    wstep()  # tuning
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    ws = [wstep() for _ in range(reps)]
    torch.cuda.synchronize()
    w_ms_timed = 1e3 * (time.perf_counter() - t_w) / reps
    wi = ripk.ripk_plan_get_info(wplan)
    w_split = ripk.ripk_plan_stats(wplan)["split"]
    wplan.destroy()  # one plan at a time on the device
    # the same calls through an autotuned plan without per-phase timing (its
    # events and the workgroup-time read-back are diagnostics): the step time
    uplan = ripk.ripk_plan(ripk.make_desc(wc["window"], wc["s_max"], wc["t_max"], wc["n_s"],
                                          wc["n_t"], n_max=wn, m_max=wm,
                                          flags=ripk.RIPK_PLAN_AUTOTUNE))

    def ustep():
        if wm == 0:
            ripk.ripk_compute_K(uplan, wx, wy, wt, stream=stream)
        else:
            ripk.ripk_compute_K_envelope(uplan, wx, wy, wt, wm, wc["seed"], stream=stream)

    for _ in range(3):  # tuning, warm-up
        ustep()
    torch.cuda.synchronize()
    # each call returns its results to the host (it ends synchronised), so
    # calls are timed one by one; the step time is their median (a single
    # host-side stall would otherwise dominate a mean of ~1 ms calls)
    u_ms = []
    for _ in range(reps):
        t_u = time.perf_counter()
        ustep()
        u_ms.append(1e3 * (time.perf_counter() - t_u))
    torch.cuda.synchronize()
    w_ms = sorted(u_ms)[len(u_ms) // 2]
    ui = ripk.ripk_plan_get_info(uplan)
    u_stats = ripk.ripk_plan_stats(uplan)
    uplan.destroy()
    res = {"ms_per_step": round(w_ms, 3),
           "pair_tests_per_s_G": round(ws[0][0] / (w_ms * 1e-3) / 1e9, 3),
           "n_in_per_step": ws[0][0],
           "sims_per_s": round(wm / (w_ms * 1e-3), 3) if wm else None,
           "cells_m_s": [ui["cell_s"], ui["cell_t"]],
           "ms_per_call_mean": round(sum(u_ms) / len(u_ms), 3),
           "ms_per_call": [round(v, 3) for v in u_ms],
           "split_untimed": u_stats["split"], "cost_ordered_untimed": u_stats["cost_ordered"],
           "timed_plan": {"ms_per_step": round(w_ms_timed, 3),
                          "cells_m_s": [wi["cell_s"], wi["cell_t"]],
                          "phases_us": {k: round(sum(v[2][k] for v in ws) / reps, 1)
                                        for k in ("us_gen", "us_grid", "us_pair",
                                                  "us_finalize")}},
           "split": w_split,
           "roofline": leg_roof(ws[0][2], sum(v[2]["us_pair"] for v in ws) / reps),
           "cost_ordered": ws[0][2]["cost_ordered"],
           "workgroup_end_us": {k: round(ws[-1][2]["us_wg_end_" + k], 1)
                                for k in ("median", "p90", "max")}}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the 5,000-request serving stream (0 = skip the serving "
                         "leg)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run the serving leg alone and print its JSON object")
    ap.add_argument("--serve-variants", default="",
                    help="--serve-only: JSON list of further server configurations "
                         "(ripk_server_desc fields) replayed on the same schedule")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed cells (one per s_max and t_max) instead of the tuned grid")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain device copy of known size first (counter runs)")
    ap.add_argument("--clustered-only", action="store_true",
                    help="run the 200k clustered-set leg alone and print its JSON object")
    ap.add_argument("--polygon-only", action="store_true",
                    help="run the polygon leg alone (--steps timed calls) and print its JSON object")
    ap.add_argument("--main-only", action="store_true",
                    help="stop after the timed steps: no host-input, graph or resampled legs, so "
                         "the last pair-kernel launches of a trace are the timed steps")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding is a design note); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import gc
    import numpy as np
    import torch
    from paper_1912_04753_amd import ripk, workloads

    # the objects of the imports go to the collector's permanent generation, so
    # that a full collection during a timed call does not walk them (one took
    # tens of milliseconds in the middle of a ~1 ms call)
    gc.collect()
    gc.freeze()
    torch.cuda.set_device(0)
    if args.serve_only:
        variants = json.loads(args.serve_variants) if args.serve_variants else ()
        print(json.dumps({"serving": serving(ripk, workloads, args.serve_requests,
                                             args.serve_slots, args.serve_load,
                                             variants=variants)}), flush=True)
        return
    dev = ripk.ripk_device_query(0)
    PEAK["lane_ops"] = dev["compute_units"] * 64 * dev["clock_khz"] * 1e3
    if args.copy_calibration:
        copy_calibration(torch)
    if args.clustered_only:
        st = torch.cuda.current_stream().cuda_stream
        print(json.dumps({"thomas-200k": larger_leg(ripk, workloads, torch, st, "thomas-200k",
                                                    args.steps)}), flush=True)
        return
    if args.polygon_only:
        st = torch.cuda.current_stream().cuda_stream
        print(json.dumps({"polygon": polygon_leg(ripk, workloads, torch, st, steps=args.steps)}),
              flush=True)
        return
    cfg = workloads.workload("uniform-100k-99csr")
    x, y, t = workloads.make_points(cfg)
    n, m = len(x), cfg["sims"]
    dx, dy, dt = (torch.from_numpy(a).cuda() for a in (x, y, t))
    torch.cuda.synchronize()
    flags = ripk.RIPK_PLAN_TIMING | (0 if args.no_autotune else ripk.RIPK_PLAN_AUTOTUNE)
    desc = ripk.make_desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"],
                          n_max=n, m_max=m, flags=flags)
    t_cold = time.perf_counter()
    plan = ripk.ripk_plan(desc)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t_cold)
    stream = torch.cuda.current_stream().cuda_stream

    cells = {}

    def step():
        t0 = time.perf_counter()
        ripk.ripk_compute_K_envelope(plan, dx, dy, dt, m, cfg["seed"], stream=stream)
        st_ = ripk.ripk_plan_stats(plan)
        i = ripk.ripk_plan_get_info(plan)
        cells["step"] = [i["cell_s"], i["cell_t"]]
        return st_, time.perf_counter() - t0

    def step2():
        # the same step as two calls: observed set, then the simulations
        t0 = time.perf_counter()
        r = ripk.ripk_compute_K(plan, dx, dy, dt, stream=stream)
        s_obs = ripk.ripk_plan_stats(plan)
        t1 = time.perf_counter()
        ripk.ripk_simulate_envelope(plan, n, m, cfg["seed"], L_obs=r["L"], stream=stream)
        s_sim = ripk.ripk_plan_stats(plan)
        return s_obs, s_sim, t1 - t0, time.perf_counter() - t1

    t_tune = time.perf_counter()
    if not args.no_autotune:
        step()  # plan set-up: the first calls time the candidate cell grids
    torch.cuda.synchronize()
    first_step_ms = 1e3 * (time.perf_counter() - t_tune)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        recs.append(step())
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    if args.main_only:
        plan.destroy()
        ms = 1e3 * t_total / args.steps
        n_in = recs[0][0]["n_in"]
        print(json.dumps({"metric": METRIC, "value": round(n_in / (t_total / args.steps) / 1e9, 4),
                          "unit": "G pair tests/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": round(ms, 4),
                          "pair_kernel_us": [r[0]["us_pair"] for r in recs],
                          "n_eval": recs[0][0]["n_eval"], "cells_m_s": cells["step"],
                          "note": "main steps only"}), flush=True)
        return
    # the same step as two calls
    step2()  # tunes the observed call's cells
    torch.cuda.synchronize()
    t_2 = time.perf_counter()
    recs2 = [step2() for _ in range(args.steps)]
    torch.cuda.synchronize()
    two_ms = 1e3 * (time.perf_counter() - t_2) / args.steps
    two_calls = {"ms_per_step": round(two_ms, 4),
                 "pair_tests_per_s_G": round((recs2[0][0]["n_in"] + recs2[0][1]["n_in"]) /
                                             (two_ms * 1e-3) / 1e9, 3),
                 "sims_per_s": round(m / (sum(r[3] for r in recs2) / len(recs2)), 3),
                 "pair_kernel_us": {"observed": round(sum(r[0]["us_pair"] for r in recs2) / len(recs2), 2),
                                    "simulations": round(sum(r[1]["us_pair"] for r in recs2) / len(recs2), 2)},
                 "roofline_simulations": leg_roof(recs2[0][1], sum(r[1]["us_pair"] for r in recs2) / len(recs2))}
    # end to end with the observed points in host memory (H2D copy inside the call)
    t_h = time.perf_counter()
    for _ in range(3):
        ripk.ripk_compute_K(plan, x, y, t)
    host_obs_ms = 1e3 * (time.perf_counter() - t_h) / 3
    n_in_obs = ripk.ripk_plan_stats(plan)["n_in"]
    # the same step through a plan that replays captured HIP graphs (no per-phase
    # timing), on a stream of its own, with the tuned cells of the timed plan
    cd = max(1, round(cfg["s_max"] / cells["step"][0]))
    td = max(1, round(cfg["t_max"] / cells["step"][1]))
    gdesc = ripk.make_desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"],
                           n_max=n, m_max=m, flags=ripk.RIPK_PLAN_GRAPH, cell_div=cd, tcell_div=td)
    gplan = ripk.ripk_plan(gdesc)
    gs = torch.cuda.Stream()
    gsp = gs.cuda_stream

    def gstep():
        ripk.ripk_compute_K_envelope(gplan, dx, dy, dt, m, cfg["seed"], stream=gsp)

    for _ in range(2):
        gstep()
    torch.cuda.synchronize()
    t_g = time.perf_counter()
    for _ in range(args.steps):
        gstep()
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t_g) / args.steps
    gplan.destroy()
    # simulations drawn from the observed set: random permutation and bootstrap
    resampled = {}
    for name, method in (("permutation", ripk.RIPK_SIM_PERMUTE), ("bootstrap", ripk.RIPK_SIM_BOOTSTRAP)):
        rdesc = ripk.make_desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"],
                               n_max=n, m_max=m, cell_div=cd, tcell_div=td, sim_method=method,
                               flags=ripk.RIPK_PLAN_TIMING)
        rplan = ripk.ripk_plan(rdesc)
        ripk.ripk_compute_K(rplan, dx, dy, dt, stream=stream)
        ripk.ripk_simulate_envelope(rplan, n, m, cfg["seed"], stream=stream)
        torch.cuda.synchronize()
        t_r = time.perf_counter()
        for _ in range(3):
            ripk.ripk_simulate_envelope(rplan, n, m, cfg["seed"], stream=stream)
        torch.cuda.synchronize()
        dt_r = (time.perf_counter() - t_r) / 3
        rst = ripk.ripk_plan_stats(rplan)
        resampled[name] = {"sims_per_s": round(m / dt_r, 3),
                           "pair_tests_per_s_G": round(rst["n_in"] / dt_r / 1e9, 3),
                           "roofline": leg_roof(rst, rst["us_pair"])}
        rplan.destroy()
    # cross (two-type) K: the same set read as two types of n/2 points each,
    # observed cross K + m CSR simulations keeping the split, autotuned cells
    n1 = n // 2
    xplan = ripk.ripk_plan(ripk.make_desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"],
                                          cfg["n_t"], n_max=n, m_max=m,
                                          flags=ripk.RIPK_PLAN_CROSS | ripk.RIPK_PLAN_AUTOTUNE |
                                          ripk.RIPK_PLAN_TIMING))

    def xstep():
        t1 = time.perf_counter()
        ripk.ripk_compute_K_envelope(xplan, dx, dy, dt, m, cfg["seed"], n_centres=n1, stream=stream)
        b = ripk.ripk_plan_stats(xplan)
        return b["n_in"], time.perf_counter() - t1, b

    xstep()  # tuning
    xstep()
    torch.cuda.synchronize()
    t_x = time.perf_counter()
    xs = [xstep() for _ in range(3)]
    torch.cuda.synchronize()
    x_ms = 1e3 * (time.perf_counter() - t_x) / 3
    xi = ripk.ripk_plan_get_info(xplan)
    cross = {"ms_per_step": round(x_ms, 3),
             "pair_tests_per_s_G": round(xs[0][0] / (x_ms * 1e-3) / 1e9, 3),
             "sims_per_s": round(m / (sum(v[1] for v in xs) / 3), 3),
             "cells_m_s": [xi["cell_s"], xi["cell_t"]],
             "roofline": leg_roof(xs[0][2], sum(v[2]["us_pair"] for v in xs) / 3),
             "note": "types = first and second half of the set; ordered cross pairs"}
    xplan.destroy()
    polygon = polygon_leg(ripk, workloads, torch, stream)
    # inhomogeneous K: the same 100k points with an intensity per point (a smooth
    # bump about the window centre, mean n/(A*D)); observed K_I only
    AD = (cfg["window"][2] - cfg["window"][0]) * (cfg["window"][3] - cfg["window"][1]) * \
        float(cfg["window"][5] - cfg["window"][4])
    fx = 0.3 + 2.0 * np.exp(-((x - 10_000.0) ** 2 + (y - 10_000.0) ** 2) / (2 * 4_000.0 ** 2))
    dlam = torch.from_numpy((n / AD) * fx / fx.mean()).cuda()
    iplan = ripk.ripk_plan(ripk.make_desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"],
                                          cfg["n_t"], n_max=n,
                                          flags=ripk.RIPK_PLAN_INHOM | ripk.RIPK_PLAN_AUTOTUNE |
                                          ripk.RIPK_PLAN_TIMING))
    for _ in range(2):
        ripk.ripk_compute_K(iplan, dx, dy, dt, stream=stream, lam=dlam)
    torch.cuda.synchronize()
    t_i = time.perf_counter()
    ius = []
    for _ in range(5):
        ripk.ripk_compute_K(iplan, dx, dy, dt, stream=stream, lam=dlam)
        ius.append(ripk.ripk_plan_stats(iplan)["us_pair"])
    torch.cuda.synchronize()
    i_ms = 1e3 * (time.perf_counter() - t_i) / 5
    ist = ripk.ripk_plan_stats(iplan)
    inhom = {"ms_per_call": round(i_ms, 3),
             "pair_tests_per_s_G": round(ist["n_in"] / (i_ms * 1e-3) / 1e9, 3),
             "roofline": leg_roof(ist, sum(ius) / len(ius)),
             "note": "observed K_I of the 100k set, intensity per point (device), autotuned cells"}
    iplan.destroy()
    # the two larger workloads, autotuned: 200k clustered points (observed K), and
    # 1M uniform + 1M clustered points with 19 CSR simulations
    larger = {wname: larger_leg(ripk, workloads, torch, stream, wname, reps)
              for wname, reps in (("thomas-200k", 10), ("mixed-2M-19csr", 2))}
    plan.destroy()

    ms = 1e3 * t_total / args.steps
    n_in = recs[0][0]["n_in"]
    value = n_in / (t_total / args.steps) / 1e9
    t_step = sum(r[1] for r in recs) / len(recs)
    # dominant kernel: the persistent pair kernel, one launch per step (the
    # observed set and the simulations)
    pair_us = [r[0]["us_pair"] for r in recs]
    evals = recs[0][0]["n_eval"]
    avg_us = sum(pair_us) / len(pair_us)
    achieved = OPS_PER_EVAL * evals / (avg_us * 1e-6) / 1e12
    # the same with the binning work of the in-range pairs counted as well
    achieved_all = (OPS_PER_EVAL * evals + OPS_PER_IN * n_in) / (avg_us * 1e-6) / 1e12
    peak = PEAK["lane_ops"] / 1e12
    from paper_1912_04753_amd.profiling import load_traffic
    tr = load_traffic(os.path.join(ROOT, "profiles", "k_pair_uniform100k_99csr_traffic.json"))
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "G pair tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f32",
        "data": "synthetic",
        "config": {"workload": "100k uniform points, 20km x 20km x 180d, "
                               "25x15 grid to 2km/30d, observed K + 99 CSR simulations",
                   "n": n, "sims": m, "n_s": cfg["n_s"], "n_t": cfg["n_t"],
                   "cells_m_s": cells, "autotune": not args.no_autotune},
        "sims_per_s": round(m / t_step, 3),
        "two_calls": two_calls,
        "graph_ms_per_step": round(graph_ms, 4),
        "resampled_simulations": resampled,
        "cross_k": cross,
        "polygon": polygon,
        "inhomogeneous_k": inhom,
        "larger_workloads": larger,
        "cold_ms": {"plan": round(plan_ms, 2),
                    "first_step_with_tuning": round(first_step_ms, 2) if not args.no_autotune else None},
        "observed_host_input": {"ms": round(host_obs_ms, 3),
                                "pair_tests_per_s_G": round(n_in_obs / (host_obs_ms * 1e-3) / 1e9, 3),
                                "note": "ripk_compute_K on host arrays: PCIe copy of 1.2 MB inside the call"},
        "device": {"compute_units": dev["compute_units"], "clock_mhz": dev["clock_khz"] / 1e3,
                   "lds_per_cu_kib": dev["lds_per_cu_bytes"] / 1024, "arch": dev["arch"],
                   "note": "read with hipGetDeviceProperties; the roofline peak is "
                           "compute_units x 64 lanes x clock"},
        "n_in_per_step": n_in,
        "n_eval_per_step": evals,
        "pair_kernel_us": round(avg_us, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": round(peak, 4),
                     "unit": "T int lane-ops/s", "frac": round(achieved / peak, 4),
                     "traffic": (round(tr["bytes_per_launch"]) if tr else None),
                     "frac_with_binning": round(achieved_all / peak, 4),
                     "note": f"{OPS_PER_EVAL} lane-ops per candidate pair x candidates per "
                             f"launch / mean pair-kernel launch time ({avg_us:.1f} us); "
                             f"frac_with_binning adds {OPS_PER_IN} lane-ops per in-range "
                             f"ordered pair (bin + weight)"},
    }
    if args.serve_requests > 0:
        # in a process of its own: the plans and cached device memory of the
        # legs above would otherwise stay with the serving measurement
        torch.cuda.synchronize()
        cmd = [sys.executable, os.path.abspath(__file__), "--serve-only",
               "--serve-requests", str(args.serve_requests), "--serve-slots", str(args.serve_slots),
               "--serve-load", str(args.serve_load)]
        res = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
        lines = [ln for ln in res.stdout.splitlines() if ln.startswith("{")]
        if res.returncode == 0 and lines:
            out["serving"] = json.loads(lines[-1])["serving"]
            out["serving"]["process"] = "own process (bench.py --serve-only)"
        else:
            out["serving"] = {"error": f"serving process exited with status {res.returncode}"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, x, y, t, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
