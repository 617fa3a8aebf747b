"""Summaries of rocprofv3 output for the pair kernel (measurement tooling).

``traffic`` turns two counter passes (``--pmc FETCH_SIZE`` and ``--pmc
WRITE_SIZE``, CSV output) into HBM bytes per launch of the pair kernel, scaled
by what the same counters read for a plain device copy of known size run in the
same process (``bench.py --copy-calibration``).  ``kernel_stats`` condenses a
``--kernel-trace --stats`` CSV into a short text table.  The results are
written as small text files under ``profiles/``; ``bench.py`` reads the traffic
file back and reports it only while the pair kernel source is unchanged.
"""
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
PAIR_SRC = os.path.join(HERE, "csrc", "pair.hip")
COPY_BYTES = 256 << 20  # the calibration copy moves this many bytes each way


def pair_source_hash():
    with open(PAIR_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _dispatches(csv_path, counter):
    out = []
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    agg = {}
    for d, name, v in out:
        agg.setdefault(d, [name, 0.0])[1] += v
    return [(d, n, v) for d, (n, v) in sorted(agg.items())]


# pair-kernel launches per benchmark step: the observed set and the
# simulations share one launch
LAUNCHES_PER_STEP = 1


def traffic(fetch_csv, write_csv, last=LAUNCHES_PER_STEP):
    """HBM bytes per pair-kernel launch (mean over the run's last `last` launches,
    i.e. one benchmark step after the plan's tuning calls, as the roofline's
    achieved rate is) from two counter passes."""
    res = {"kernel_source_sha256": pair_source_hash()}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _dispatches(path, counter)
        copies = [v for d, n, v in rows if "copy" in n.lower() or "elementwise" in n.lower()]
        pair = [v for d, n, v in rows if "k_pair" in n][-last:]
        if not copies or not pair:
            raise ValueError(f"{path}: need a copy kernel and a pair kernel in the trace")
        kib_copy = max(copies)
        scale = COPY_BYTES / (kib_copy * 1024.0)
        mean_kib = sum(pair) / len(pair)
        res[f"{key}_copy_kib"] = kib_copy
        res[f"{key}_scale"] = scale
        res[f"{key}_pair_kib_per_launch"] = [round(v, 1) for v in pair]
        res[f"{key}_bytes"] = mean_kib * 1024.0 * scale
    res["bytes_per_launch"] = res["fetch_bytes"] + res["write_bytes"]
    return res


def _short_name(full):
    """'void ns::(anonymous namespace)::k_pair<true, 0>(ripk::PairArgs)' -> 'k_pair<true, 0>'."""
    name = full.replace("void ", "").replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += (ch == "<") - (ch == ">")
        if ch == "(" and depth == 0:
            name = name[:i]
            break
    head, sep, args = name.partition("<")
    return head.split("::")[-1] + sep + args


def pair_launches(trace_csv):
    """Durations (us) of the pair-kernel dispatches in a kernel trace, in order."""
    out = []
    for r in csv.DictReader(open(trace_csv)):
        if "k_pair" in r["Kernel_Name"]:
            out.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return out


def kernel_stats(stats_csv, top=12):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        name = _short_name(r["Name"])
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def kernel_resources(trace_csv, match="k_pair"):
    """Per kernel variant of a kernel trace: launch count, duration spread,
    scratch (spill) bytes and the workgroup counts it was launched with.  The
    trace's register and LDS columns are left out: they are not the compiler's
    VGPR count, and LDS sized at launch is not in them."""
    agg = {}
    for r in csv.DictReader(open(trace_csv)):
        if match not in r["Kernel_Name"]:
            continue
        a = agg.setdefault(_short_name(r["Kernel_Name"]), {"us": [], "grids": set(), "r": r})
        a["us"].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        a["grids"].add(int(r["Grid_Size_X"]) // max(int(r["Workgroup_Size_X"]), 1))
    lines = ["| kernel | calls | min us | median us | max us | scratch bytes | threads per WG | workgroups |",
             "|---|---|---|---|---|---|---|---|"]
    for name, a in sorted(agg.items(), key=lambda kv: -sum(kv[1]["us"])):
        us, r = sorted(a["us"]), a["r"]
        wg = ", ".join(str(g) for g in sorted(a["grids"]))
        lines.append(f"| `{name}` | {len(us)} | {us[0]:.1f} | {us[len(us) // 2]:.1f} | {us[-1]:.1f} | "
                     f"{r['Scratch_Size']} | {r['Workgroup_Size_X']} | {wg} |")
    return "\n".join(lines)


PROFILE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d $R/gpurun_out/prof -o run -- "
               "python3 $R/bench.py --steps {steps} --warmup 1 --main-only")
PMC_CMD = ("timeout -s KILL 120 rocprofv3 --pmc {counter} --output-format csv -d $R/gpurun_out/{d} -o {o} "
           "-- python3 $R/bench.py --steps 1 --warmup 0 --main-only "
           "--copy-calibration")


def summary(title, stats_csv, trace_csv, steps, tr, bench_line=None):
    """Markdown summary of one profiled benchmark run: the kernel table, the pair
    kernel's launches of the timed steps, and the traffic record."""
    launches = pair_launches(trace_csv)
    timed = launches[-LAUNCHES_PER_STEP * steps:]
    lines = [f"# {title}", "",
             f"Pair-kernel source hash (sha256 of `paper_1912_04753_amd/csrc/pair.hip`, first 16 hex): "
             f"`{tr['kernel_source_sha256']}`.", "",
             "## Kernel trace (`--kernel-trace --stats`)", "",
             "Command (from `/tmp`, `TMPDIR=/tmp`, `R` = repository root):", "", "```",
             PROFILE_CMD.format(steps=steps), "```", "",
             "The table covers every launch of the run: the plan's tuning calls (each candidate cell grid "
             "once), the warm-up step and the timed steps.", "", kernel_stats(stats_csv), "",
             f"Pair-kernel launches of the {steps} timed steps, in order (us; one per step, the "
             f"observed set and the simulations together): {' '.join(f'{v:.1f}' for v in timed)}.",
             f"Mean {sum(timed) / len(timed):.1f} us per launch.", ""]
    if bench_line:
        lines += [f"`bench.py`'s own HIP-event mean for the same launches (its timed steps): "
                  f"{bench_line}.", ""]
    lines += ["## HBM traffic (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "", "```",
              PMC_CMD.format(counter="FETCH_SIZE", d="pmcF", o="f"),
              PMC_CMD.format(counter="WRITE_SIZE", d="pmcW", o="w"),
              "python paper_1912_04753_amd/profiling.py traffic $R/gpurun_out/pmcF/f_counter_collection.csv "
              "$R/gpurun_out/pmcW/w_counter_collection.csv", "```", "",
              f"Calibration: a 256 MiB device copy (`--copy-calibration`) reads {tr['fetch_copy_kib']:.0f} KiB "
              f"of FETCH_SIZE (scale {tr['fetch_scale']:.4f}) and {tr['write_copy_kib']:.0f} KiB of WRITE_SIZE "
              f"(scale {tr['write_scale']:.4f}).", "",
              "| launch (last step) | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|"] + [
              f"| {i + 1} | {f} | {w} |" for i, (f, w) in enumerate(
                  zip(tr['fetch_pair_kib_per_launch'], tr['write_pair_kib_per_launch']))] + ["",
              f"Mean scaled bytes per launch: fetch {tr['fetch_bytes'] / 1e6:.1f} MB + write "
              f"{tr['write_bytes'] / 1e6:.1f} MB = {tr['bytes_per_launch'] / 1e6:.1f} MB.", ""]
    return "\n".join(lines)


def load_traffic(path):
    """Stored traffic record, or None when the pair kernel changed since it was taken."""
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256") != pair_source_hash():
        return None
    return d


if __name__ == "__main__":
    import sys
    if sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3]), indent=1))
    elif sys.argv[1] == "stats":
        print(kernel_stats(sys.argv[2]))
    elif sys.argv[1] == "resources":
        print(kernel_resources(sys.argv[2], *(sys.argv[3:4] or ["k_pair"])))
    elif sys.argv[1] == "launches":
        print(" ".join(f"{v:.1f}" for v in pair_launches(sys.argv[2])))
    elif sys.argv[1] == "summary":
        # summary <title> <prof dir> <fetch csv> <write csv> <steps> <traffic json out> [bench note]
        title, prof, fcsv, wcsv, steps, out = sys.argv[2:8]
        tr = traffic(fcsv, wcsv)
        with open(out, "w") as f:
            json.dump(tr, f, indent=1)
        note = sys.argv[8] if len(sys.argv) > 8 else None
        print(summary(title, os.path.join(prof, "run_kernel_stats.csv"),
                      os.path.join(prof, "run_kernel_trace.csv"), int(steps), tr, note))
