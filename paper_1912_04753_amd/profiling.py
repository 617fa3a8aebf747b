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


def traffic(fetch_csv, write_csv):
    """HBM bytes per pair-kernel launch (mean over the launches of the run, as the
    roofline's achieved rate is) from two counter passes."""
    res = {"kernel_source_sha256": pair_source_hash()}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _dispatches(path, counter)
        copies = [v for d, n, v in rows if "copy" in n.lower() or "elementwise" in n.lower()]
        pair = [v for d, n, v in rows if "k_pair" in n]
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
    elif sys.argv[1] == "launches":
        print(" ".join(f"{v:.1f}" for v in pair_launches(sys.argv[2])))
