"""Writes ``stream50_oracle.npz``: the oracle's C and K for a seeded sample of
50 requests with n > 20,000 from the 5,000-request serving stream
(``workloads.serving_requests``), each request's observed set and its CSR
simulations 0 .. min(sims, 3) - 1.  The GPU test compares every request of
the stream with n <= 20,000 against the oracle directly and these 50 larger
ones against this file.

Only ``oracle`` (the plain O(n^2) FP64 loop of Eq. 2-4, Sec. 3) and the seeded
input generators of ``workloads`` are used; nothing here touches the HIP
library.  Simulation s of request r is drawn by the oracle's own Philox4x64-10
with counter (point, s, 0, 0) and key (5 * 2^32 + r, 0) (Sec. 3, Monte Carlo
under CSR).  L follows from K by Eq. 4 and is not stored.

Results of finished requests are kept in ``<output>.partial.npz`` so that an
interrupted run resumes.

    python tests/golden/make_stream_golden.py [--threads N]
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

OUT = os.path.join(HERE, "stream50_oracle.npz")
N_SMALL = 20_000      # requests up to this size are compared directly
SAMPLE = 50
SAMPLE_SEED = 505
MAX_SIMS = 3


def sample_ids(reqs):
    """The seeded sample of larger requests (sorted ids)."""
    big = [r["id"] for r in reqs if r["parts"][0][1] > N_SMALL]
    rng = np.random.default_rng(SAMPLE_SEED)
    return sorted(int(i) for i in rng.choice(big, SAMPLE, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    reqs = workloads.serving_requests(num=5000)
    ids = sample_ids(reqs)
    part = a.out + ".partial.npz"
    done = dict(np.load(part)) if os.path.exists(part) else {}
    for i in ids:
        r = reqs[i]
        if "r%d_C" % i in done:
            continue
        d = oracle.desc(r["window"], r["s_max"], r["t_max"], r["n_s"], r["n_t"])
        x, y, t = workloads.request_points(r)
        n, m = len(x), min(r["sims"], MAX_SIMS)
        t0 = time.time()
        Cs, Ks = [], []
        for s in range(-1, m):
            pts = (x, y, t) if s < 0 else oracle.csr_points(d, n, s, r["seed"])
            res = oracle.estimate(d, *pts, threads=a.threads)
            Cs.append(res["C"])
            Ks.append(res["K"])
        done["r%d_C" % i] = np.stack(Cs).astype(np.uint64)
        done["r%d_K" % i] = np.stack(Ks)
        np.savez(part, **done)
        print("request %d: n=%d sims=%d in %.0f s" % (i, n, m, time.time() - t0), flush=True)
    done["ids"] = np.array(ids, np.int64)
    np.savez_compressed(a.out, **done)
    os.remove(part)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
