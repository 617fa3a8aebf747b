"""Writes ``mixed2m_19csr_oracle.npz``: the oracle's C, W, K and L for the
2,000,000-point mixed workload (1M uniform + 1M Thomas-clustered points in
100 km x 100 km x 730 d, 50 x 30 grid to 10 km / 90 d, isotropic spatial and
temporal correction) -- the observed set and CSR simulations 0, 9 and 18 of the
19 the workload draws with its seed.

Only ``oracle`` (the plain O(n^2) FP64 loop of Eq. 2-4, Sec. 3) and the seeded
input generator ``workloads.make_points`` are used; nothing here touches the
HIP library.  Simulation s is drawn by the oracle's own Philox4x64-10 with
counter (point, s, 0, 0) and key (seed, 0) (Sec. 3, Monte Carlo under CSR).

Each set is 4e12 ordered pair evaluations: about 20-30 minutes on 8 cores.
Results of finished sets are kept in ``<output>.partial.npz`` so that an
interrupted run resumes.

    python tests/golden/make_mixed2m_golden.py [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1912_04753_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "mixed2m_19csr_oracle.npz")
SIMS = (0, 9, 18)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    c = workloads.workload("mixed-2M-19csr")
    d = oracle.desc(c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"])
    x, y, t = workloads.make_points(c)
    n = len(x)
    part = a.out + ".partial.npz"
    done = dict(np.load(part)) if os.path.exists(part) else {}
    jobs = [("obs", None)] + [("sim%d" % s, s) for s in SIMS]
    for name, s in jobs:
        if name + "_C" in done:
            print("%s: cached" % name, flush=True)
            continue
        pts = (x, y, t) if s is None else oracle.csr_points(d, n, s, c["seed"])
        t0 = time.time()
        r = oracle.estimate(d, *pts, threads=a.threads)
        for k in ("C", "W", "K", "L"):
            done["%s_%s" % (name, k)] = r[k]
        np.savez(part, **done)
        print("%s: n=%d N_in=%d in %.0f s" % (name, n, int(r["C"][-1, -1]), time.time() - t0),
              flush=True)
    done["sims"] = np.array(SIMS, np.int64)
    done["n"] = np.array(n, np.int64)
    done["seed"] = np.array(c["seed"], np.int64)
    np.savez_compressed(a.out, **done)
    os.remove(part)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
