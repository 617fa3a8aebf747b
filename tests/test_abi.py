"""The C-ABI library loads and exports what include/ripk.h declares; host-side
plan validation and geometry (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1912_04753_amd import ripk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ripk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ripk_[a-z_A-Z0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "ripk_plan" in names and "ripk_compute_K" in names
    lib = ctypes.CDLL(ripk.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(ripk._SIGS) | {"ripk_plan_destroy"}


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every field offset and struct size of the binding equals what the C
    compiler makes of include/ripk.h."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    structs = {"ripk_plan_desc": ripk.PlanDesc, "ripk_points": ripk.Points,
               "ripk_plan_info": ripk.PlanInfo, "ripk_stats": ripk.Stats,
               "ripk_server_desc": ripk.ServerDesc, "ripk_request": ripk.Request,
               "ripk_result": ripk.Result, "ripk_server_state": ripk.ServerState,
               "ripk_K_out": ripk.KOut, "ripk_env_out": ripk.EnvOut,
               "ripk_device_props": ripk.DeviceProps}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ripk.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, field, val = line.split()
        py = structs[cname]
        want = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(val) == want, (cname, field, int(val), want)


def desc(**kw):
    base = dict(window=(0, 0, 20_000, 20_000, 0, 15_552_000), s_max=2000, t_max=2_592_000,
                n_s=25, n_t=15, n_max=100_000, m_max=99)
    base.update(kw)
    w = base.pop("window")
    return ripk.make_desc(w, **base)


def test_plan_geometry_uniform100k():
    info = ripk.ripk_plan_check(desc())
    assert (info["nx"], info["ny"], info["nt"]) == (10, 10, 6)
    assert info["reach_s"] == 1 and info["reach_t"] == 1
    assert info["dist_mode"] == 0          # packed 16-bit differences
    assert info["n_bins"] == 375
    # exact floors: d <= s_k <=> d2 <= S2[k] (Eq. 3)
    for k, v in enumerate(info["S2"], 1):
        assert v * 25 * 25 <= (k * 2000) ** 2 < (v + 1) * 25 * 25
    for l, v in enumerate(info["T"], 1):
        assert v * 15 <= l * 2_592_000 < (v + 1) * 15


def test_plan_geometry_finer_cells_and_wide():
    info = ripk.ripk_plan_check(desc(cell_div=2, tcell_div=3))
    assert info["cell_s"] == 1000 and info["cell_t"] == 864_000
    assert info["reach_s"] == 2 and info["reach_t"] == 3
    w = ripk.ripk_plan_check(ripk.make_desc((0, 0, 200_000, 150_000, 0, 3_000_000), 40_000,
                                            600_000, 20, 12, n_max=10))
    assert w["dist_mode"] == 2


@pytest.mark.parametrize("bad", [
    dict(n_s=0), dict(n_t=65), dict(s_max=10_001), dict(t_max=15_552_001),
    dict(edge=1, window=(0, 0, 20_000, 20_000, 0, 2**31 - 1), t_max=2**30),
    dict(window=(0, 0, 0, 10, 0, 10)), dict(window=(0, 0, 2**24, 10**6, 0, 10**8), s_max=10),
    dict(n_max=1), dict(m_max=-1), dict(n_max=2**26, m_max=64), dict(edge=4),
    dict(norm=2), dict(cell_div=9), dict(s_max=0),
])
def test_plan_rejects_bad_descriptors(bad):
    with pytest.raises(ripk.RipkError) as e:
        ripk.ripk_plan_check(desc(**bad))
    assert e.value.status == ripk.RIPK_EINVAL
    assert ripk.ripk_last_error()


def test_plan_allows_large_s_without_spatial_correction():
    info = ripk.ripk_plan_check(desc(s_max=30_000, edge=ripk.RIPK_EDGE_TEMPORAL))
    assert info["nx"] == 1


def test_status_strings():
    assert ripk.ripk_status_str(ripk.RIPK_ERANGE) == "point outside the study window"
    assert ripk.ripk_status_str(0) == "ok"


def test_server_structs_and_argument_checks():
    assert ctypes.sizeof(ripk.ServerDesc) == 4 * 4 + 8 + 2 * 8 + 4 * 4
    assert ctypes.sizeof(ripk.Request) == ctypes.sizeof(ripk.PlanDesc) + ctypes.sizeof(ripk.Points) + 16
    assert ctypes.sizeof(ripk.Result) == 4 * 8 + 8 * 8 + 4 + 4 + 3 * 8 + 8
    for slots in (0, 17):
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_server_create(slots=slots)
        assert e.value.status == ripk.RIPK_EINVAL
    with pytest.raises(ripk.RipkError) as e:
        ripk.ripk_server_create(hbm_budget_bytes=0)
    assert e.value.status == ripk.RIPK_EINVAL
    for bad in (dict(admission=2), dict(device_share=1.5), dict(device_share=-0.5),
                dict(slice_ms=-1.0), dict(max_large=-1), dict(age_ms=-1.0),
                dict(large_work=float("nan"))):
        with pytest.raises(ripk.RipkError) as e:
            ripk.ripk_server_create(**bad)
        assert e.value.status == ripk.RIPK_EINVAL, bad


def _simple_brute(P):
    """Independent check that a closed polygon is simple: non-adjacent edges do
    not meet, adjacent edges share only their common vertex."""
    n = len(P)

    def orient(a, b, c):
        v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        return (v > 0) - (v < 0)

    def on_seg(a, b, c):
        return min(a[0], b[0]) <= c[0] <= max(a[0], b[0]) and min(a[1], b[1]) <= c[1] <= max(a[1], b[1])

    def meet(a, b, c, d):
        o1, o2, o3, o4 = orient(a, b, c), orient(a, b, d), orient(c, d, a), orient(c, d, b)
        if o1 * o2 < 0 and o3 * o4 < 0:
            return True
        return ((o1 == 0 and on_seg(a, b, c)) or (o2 == 0 and on_seg(a, b, d)) or
                (o3 == 0 and on_seg(c, d, a)) or (o4 == 0 and on_seg(c, d, b)))

    E = [(P[k], P[(k + 1) % n]) for k in range(n)]
    if any(a == b for a, b in E):
        return False
    for i in range(n):
        for j in range(i + 1, n):
            a, b = E[i]
            c, d = E[j]
            if j == i + 1 or (j + 1) % n == i:
                # shared vertex s; the other ends must not fold back onto it
                s, p, q = (b, a, d) if j == i + 1 else (a, b, c)
                dot = (p[0] - s[0]) * (q[0] - s[0]) + (p[1] - s[1]) * (q[1] - s[1])
                if orient(s, p, q) == 0 and dot > 0:
                    return False
                continue
            if meet(a, b, c, d):
                return False
    return True


def test_polygon_validation_matches_brute_force():
    """Random polygons on a coarse lattice (many self-intersecting, touching or
    degenerate): the plan accepts exactly the simple ones with enough area."""
    rng = np.random.default_rng(9)
    win = (0, 0, 1000, 1000, 0, 100)
    seen = {True: 0, False: 0}
    for trial in range(400):
        k = int(rng.integers(3, 9))
        P = [tuple(int(v) for v in rng.integers(0, 11, 2) * 100) for _ in range(k)]
        area2 = abs(sum(P[i][0] * P[(i + 1) % k][1] - P[(i + 1) % k][0] * P[i][1] for i in range(k)))
        want = _simple_brute(P) and area2 * 512 >= 1000 * 1000
        try:
            ripk.ripk_plan_check(ripk.make_desc(win, 100, 10, 2, 2, n_max=10, poly=P))
            got = True
        except ripk.RipkError as e:
            assert e.status == ripk.RIPK_EINVAL
            got = False
        assert got == want, (trial, P)
        seen[want] += 1
    assert seen[True] > 30 and seen[False] > 30


def test_polygon_edge_lists_reported():
    """ripk_plan_check builds a polygon plan's per-cell edge lists on the host:
    the 85-vertex boundary lists a few edges per cell near it; a comb whose
    teeth crowd one cell lists more than 32 there (every edge is scanned)."""
    from paper_1912_04753_amd import workloads
    c = workloads.workload("polygon-100k-99csr")
    P = workloads.polygon_of(c)
    info = ripk.ripk_plan_check(ripk.make_desc(c["window"], c["s_max"], c["t_max"], c["n_s"],
                                               c["n_t"], n_max=10, poly=P))
    assert 1 <= info["near_edges_max"] <= 32
    assert 0 < info["near_cells"] < info["nx"] * info["ny"]
    comb = [(0, 0), (4000, 0)] + [p for k in range(40)
                                  for p in ((4000 - 50 * k, 3000), (3975 - 50 * k, 3000),
                                            (3975 - 50 * k, 100), (3950 - 50 * k, 100))][:-1] + \
           [(0, 3000)]
    info = ripk.ripk_plan_check(ripk.make_desc((0, 0, 4000, 4000, 0, 1000), 400, 100, 4, 2,
                                               n_max=10, poly=comb))
    assert info["near_edges_max"] == 33
    rect = ripk.ripk_plan_check(ripk.make_desc(c["window"], c["s_max"], c["t_max"], c["n_s"],
                                               c["n_t"], n_max=10))
    assert rect["near_edges_max"] == 0 and rect["near_cells"] == 0
