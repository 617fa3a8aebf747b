"""Host-side tools without a GPU: the seeded input generators and the
rocprofv3 summary arithmetic used by the benchmark."""
import csv
import math
import os

import numpy as np
import pytest

from paper_1912_04753_amd import profiling, workloads


@pytest.mark.parametrize("name", ["uniform-2k", "thomas-200k", "uniform-100k-99csr"])
def test_workloads_are_seeded_and_inside_the_window(name):
    c = workloads.workload(name)
    x1, y1, t1 = workloads.make_points(c)
    x2, y2, t2 = workloads.make_points(c)
    assert all(np.array_equal(a, b) for a, b in ((x1, x2), (y1, y2), (t1, t2)))
    n = sum(p[1] for p in c["parts"])
    assert len(x1) == len(y1) == len(t1) == n and x1.dtype == np.int32
    X0, Y0, X1, Y1, T0, T1 = c["window"]
    assert x1.min() >= X0 and x1.max() <= X1 and y1.min() >= Y0 and y1.max() <= Y1
    assert t1.min() >= T0 and t1.max() <= T1
    # spatial correction needs s_max <= half the shorter side; temporal t_max <= duration
    assert 2 * c["s_max"] <= min(X1 - X0, Y1 - Y0) and c["t_max"] <= T1 - T0


def test_thomas_points_cluster():
    rng = np.random.Generator(np.random.PCG64(7))
    win = (0, 0, 50_000, 50_000, 0, 365 * workloads.DAY)
    x, y, t = workloads.thomas_points(rng, 20_000, win, parents=20, sigma_xy=100.0,
                                      sigma_t=2.0 * workloads.DAY)
    # 20 parents with sigma 100 m: a few dozen occupied 1 km cells out of 2500
    # (a uniform set of this size occupies all of them)
    cells = np.unique((x // 1000).astype(np.int64) * 100 + y // 1000)
    assert len(cells) < 200
    u = workloads.uniform_points(rng, 20_000, win)
    assert len(np.unique((u[0] // 1000).astype(np.int64) * 100 + u[1] // 1000)) > 2400


def test_serving_requests_follow_the_stream_recipe():
    reqs = workloads.serving_requests(num=200, rate=10.0)
    arr = [r["arrival"] for r in reqs]
    assert all(b >= a for a, b in zip(arr, arr[1:]))
    assert 10.0 / 2 < len(reqs) / arr[-1] < 10.0 * 2  # Poisson rate
    for r in reqs:
        n = r["parts"][0][1]
        side, dur = r["window"][2], r["window"][5]
        assert 1000 <= n <= 500_000
        assert 10_000 <= side <= 100_000 and 180 * workloads.DAY <= dur <= 730 * workloads.DAY
        assert r["s_max"] <= side / 4 and r["t_max"] <= dur / 4
        assert 10 <= r["n_s"] <= 50 and 10 <= r["n_t"] <= 50 and 0 <= r["sims"] <= 99
        assert r["seed"] == (5 << 32) + r["id"]


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, v in rows:
            # two instances per dispatch, summed by the reader
            w.writerow(dict(Dispatch_Id=d, Kernel_Name=name, Counter_Name=counter, Counter_Value=v / 2))
            w.writerow(dict(Dispatch_Id=d, Kernel_Name=name, Counter_Name=counter, Counter_Value=v / 2))


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    copy_kib = profiling.COPY_BYTES / 1024
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    # FETCH counts half the copy's bytes, WRITE all of them
    _counter_csv(f, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", copy_kib / 2),
                                   (2, "void ripk::k_pair<true, 0>(ripk::PairArgs)", 100.0),
                                   (3, "void ripk::k_pair<true, 0>(ripk::PairArgs)", 1000.0),
                                   (4, "void ripk::k_pair<true, 0>(ripk::PairArgs)", 3000.0)])
    _counter_csv(w, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", copy_kib),
                                   (2, "void ripk::k_pair<true, 0>(ripk::PairArgs)", 10.0),
                                   (3, "void ripk::k_pair<true, 0>(ripk::PairArgs)", 20.0),
                                   (4, "void ripk::k_pair<true, 0>(ripk::PairArgs)", 40.0)])
    tr = profiling.traffic(str(f), str(w), last=2)
    assert math.isclose(tr["fetch_scale"], 2.0) and math.isclose(tr["write_scale"], 1.0)
    assert tr["fetch_pair_kib_per_launch"] == [1000.0, 3000.0]       # the last two launches
    assert math.isclose(tr["fetch_bytes"], 2000.0 * 1024 * 2.0)
    assert math.isclose(tr["write_bytes"], 30.0 * 1024)
    assert math.isclose(tr["bytes_per_launch"], tr["fetch_bytes"] + tr["write_bytes"])
    assert tr["kernel_source_sha256"] == profiling.pair_source_hash()


def test_stored_traffic_is_dropped_when_the_kernel_changes(tmp_path):
    import json
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"kernel_source_sha256": "0" * 16, "bytes_per_launch": 1.0}))
    assert profiling.load_traffic(str(p)) is None
    p.write_text(json.dumps({"kernel_source_sha256": profiling.pair_source_hash(), "bytes_per_launch": 1.0}))
    assert profiling.load_traffic(str(p))["bytes_per_launch"] == 1.0
    assert profiling.load_traffic(str(tmp_path / "missing.json")) is None


def test_kernel_names_are_shortened():
    assert profiling._short_name("void ripk::(anonymous namespace)::k_pair<true, 0>(ripk::PairArgs)") \
        == "k_pair<true, 0>"
    assert profiling._short_name("ripk::(anonymous namespace)::k_gather(unsigned int const*, int)") \
        == "k_gather"


def test_kernel_resources_table(tmp_path):
    """Per-variant rows: launch count, min / median / max duration, scratch
    bytes and the distinct workgroup counts, longest total first."""
    path = tmp_path / "trace.csv"
    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Scratch_Size", "Workgroup_Size_X",
            "Grid_Size_X"]
    rows = [("void ripk::(anonymous namespace)::k_pair<true, 0, false, false>(ripk::PairArgs)", 0, 3000, 0, 256, 1536 * 256),
            ("void ripk::(anonymous namespace)::k_pair<true, 0, false, false>(ripk::PairArgs)", 5000, 6000, 0, 256, 1024 * 256),
            ("void ripk::(anonymous namespace)::k_pair<true, 0, false, false>(ripk::PairArgs)", 7000, 9000, 0, 256, 1536 * 256),
            ("void ripk::(anonymous namespace)::k_pair<true, 0, true, false>(ripk::PairArgs)", 0, 500, 16, 256, 1024 * 256),
            ("ripk::k_csr(unsigned int)", 0, 100000, 0, 256, 256)]
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        w.writerows(rows)
    lines = profiling.kernel_resources(str(path)).splitlines()
    assert len(lines) == 4  # header, rule, two pair variants (k_csr filtered out)
    assert lines[2] == "| `k_pair<true, 0, false, false>` | 3 | 1.0 | 2.0 | 3.0 | 0 | 256 | 1024, 1536 |"
    assert lines[3] == "| `k_pair<true, 0, true, false>` | 1 | 0.5 | 0.5 | 0.5 | 16 | 256 | 1024 |"
    assert "k_csr" in profiling.kernel_resources(str(path), "k_")
