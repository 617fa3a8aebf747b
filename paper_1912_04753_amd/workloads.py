"""Seeded synthetic point sets for the benchmark and the tests.

This module holds input generation only -- no part of the estimator's
arithmetic -- so that the HIP library and the CPU oracle can be fed the very
same points.  Everything is drawn from ``numpy.random.Generator(PCG64(seed))``.

The paper's own data (enterprise registrations in Hubei, 1949-2015, and a
synthetic US set; Sec. 6.1 and the appendix) are not available, so these
recipes stand in for them:

* ``uniform``  -- integer coordinates uniform on the half-open window
  [x0, x1) x [y0, y1) x [t0, t1) (complete spatio-temporal randomness).
* ``thomas``   -- a space-time Thomas-type cluster process: P parents uniform in
  the window; every point picks a parent uniformly at random and is displaced
  by independent N(0, sigma_xy) in x and y and N(0, sigma_t) in t; displaced
  points falling outside the closed window are drawn again; coordinates are
  floored to integers.  It stands in for the strongly skewed POI data the
  paper describes (Sec. 6.2).

* ``polygon``  -- a seeded star-shaped simple polygon with dents (concave
  vertices) standing in for the administrative boundaries of the paper's
  experiments (a Hubei province boundary and an 85-vertex simplified US
  boundary, Sec. 6 and the appendix), with points uniform strictly inside it.

Sizes and grids bracket the paper's experiments (10k-500k points, 10-20 grid
steps per axis; Sec. 6.1, Table 5, appendix Table A).  Units: metres and
seconds; a day is 86,400 s.
"""
import math

import numpy as np

DAY = 86400


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(rng, n, window):
    x0, y0, x1, y1, t0, t1 = window
    x = rng.integers(x0, x1, size=n, dtype=np.int64)
    y = rng.integers(y0, y1, size=n, dtype=np.int64)
    t = rng.integers(t0, t1, size=n, dtype=np.int64)
    return x.astype(np.int32), y.astype(np.int32), t.astype(np.int32)


def thomas_points(rng, n, window, parents, sigma_xy, sigma_t):
    x0, y0, x1, y1, t0, t1 = window
    px = rng.uniform(x0, x1, size=parents)
    py = rng.uniform(y0, y1, size=parents)
    pt = rng.uniform(t0, t1, size=parents)
    par = rng.integers(0, parents, size=n)
    x = np.empty(n, np.float64)
    y = np.empty(n, np.float64)
    t = np.empty(n, np.float64)
    todo = np.arange(n)
    while todo.size:
        p = par[todo]
        cx = px[p] + rng.normal(0.0, sigma_xy, size=todo.size)
        cy = py[p] + rng.normal(0.0, sigma_xy, size=todo.size)
        ct = pt[p] + rng.normal(0.0, sigma_t, size=todo.size)
        ok = (cx >= x0) & (cx <= x1) & (cy >= y0) & (cy <= y1) & (ct >= t0) & (ct <= t1)
        x[todo[ok]] = cx[ok]
        y[todo[ok]] = cy[ok]
        t[todo[ok]] = ct[ok]
        todo = todo[~ok]
    return (np.floor(x).astype(np.int32), np.floor(y).astype(np.int32),
            np.floor(t).astype(np.int32))


def star_polygon(rng, window, n_vertices, dent=0.45):
    """Integer vertices (n_vertices, 2) of a simple polygon, star-shaped about
    the window centre: vertex k at angle 2*pi*(k + jitter_k)/v (jitter in
    (-0.3, 0.3), so angles increase) and radius R*(1 - dent*f_k), where
    R = 0.48*min(W, H) and f in [0, 1] is a sum of six random Fourier modes
    rescaled to [0, 1]."""
    x0, y0, x1, y1 = window[:4]
    cx, cy = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    R = 0.48 * min(x1 - x0, y1 - y0)
    v = int(n_vertices)
    th = 2 * math.pi * (np.arange(v) + rng.uniform(-0.3, 0.3, v)) / v
    f = np.zeros(v)
    for h in range(1, 7):
        f += rng.normal(0, 1.0 / h) * np.cos(h * th + rng.uniform(0, 2 * math.pi))
    f = (f - f.min()) / max(f.max() - f.min(), 1e-12)
    r = R * (1.0 - dent * f)
    px = np.clip(np.rint(cx + r * np.cos(th)), x0, x1).astype(np.int64)
    py = np.clip(np.rint(cy + r * np.sin(th)), y0, y1).astype(np.int64)
    return np.stack([px, py], axis=1).astype(np.int32)


def _strictly_inside(poly, x, y):
    """Crossing number along +x with the half-open rule, on integers; points on
    an edge are not inside.  For drawing inputs only."""
    P = np.asarray(poly, np.int64)
    ax, ay = P[:, 0][None, :], P[:, 1][None, :]
    bx, by = np.roll(P[:, 0], -1)[None, :], np.roll(P[:, 1], -1)[None, :]
    X = np.asarray(x, np.int64)[:, None]
    Y = np.asarray(y, np.int64)[:, None]
    cr = (bx - ax) * (Y - ay) - (by - ay) * (X - ax)
    on = ((cr == 0) & (X >= np.minimum(ax, bx)) & (X <= np.maximum(ax, bx)) &
          (Y >= np.minimum(ay, by)) & (Y <= np.maximum(ay, by))).any(axis=1)
    straddle = (ay > Y) != (by > Y)
    den = by - ay
    lhs = (X - ax) * den
    num = (Y - ay) * (bx - ax)
    left = np.where(den > 0, lhs < num, lhs > num)
    inside = (np.count_nonzero(straddle & left, axis=1) % 2) == 1
    return inside & ~on


def polygon_points(rng, n, window, poly):
    """n points uniform on the integer grid strictly inside the polygon (by
    rejection from the window), times uniform on [t0, t1)."""
    xs, ys = [], []
    got = 0
    while got < n:
        k = max(1024, 2 * (n - got))
        x, y, _ = uniform_points(rng, k, window)
        ok = np.zeros(k, bool)
        for a in range(0, k, 8192):
            ok[a:a + 8192] = _strictly_inside(poly, x[a:a + 8192], y[a:a + 8192])
        xs.append(x[ok]); ys.append(y[ok])
        got += int(ok.sum())
    x = np.concatenate(xs)[:n]
    y = np.concatenate(ys)[:n]
    t = rng.integers(window[4], window[5], size=n, dtype=np.int64).astype(np.int32)
    return x, y, t


# The five workloads.  ``window`` = (x0, y0, x1, y1, t0, t1); isotropic spatial
# and temporal edge correction (edge = 3) throughout.
WORKLOADS = {
    "uniform-2k": dict(name="uniform-2k", seed=1, window=(0, 0, 10_000, 10_000, 0, 365 * DAY),
            s_max=1_000, n_s=10, t_max=30 * DAY, n_t=10, sims=0,
            parts=[("uniform", 2_000, {})]),
    "thomas-200k": dict(name="thomas-200k", seed=2, window=(0, 0, 50_000, 50_000, 0, 365 * DAY),
            s_max=5_000, n_s=20, t_max=60 * DAY, n_t=20, sims=0,
            parts=[("thomas", 200_000, dict(parents=500, sigma_xy=200.0,
                                            sigma_t=5.0 * DAY))]),
    "uniform-100k-99csr": dict(name="uniform-100k-99csr", seed=3, window=(0, 0, 20_000, 20_000, 0, 180 * DAY),
            s_max=2_000, n_s=25, t_max=30 * DAY, n_t=15, sims=99,
            parts=[("uniform", 100_000, {})]),
    "polygon-100k-99csr": dict(name="polygon-100k-99csr", seed=6,
            window=(0, 0, 20_000, 20_000, 0, 180 * DAY), s_max=2_000, n_s=25, t_max=30 * DAY, n_t=15,
            sims=99, polygon=85, parts=[("polygon", 100_000, {})]),
    "mixed-2M-19csr": dict(name="mixed-2M-19csr", seed=4, window=(0, 0, 100_000, 100_000, 0, 730 * DAY),
            s_max=10_000, n_s=50, t_max=90 * DAY, n_t=30, sims=19,
            parts=[("uniform", 1_000_000, {}),
                   ("thomas", 1_000_000, dict(parents=2_000, sigma_xy=500.0,
                                              sigma_t=10.0 * DAY))]),
}


def make_points(cfg):
    """Observed point set of a workload dict: three int32 arrays (x, y, t)."""
    rng = _rng(cfg["seed"])
    xs, ys, ts = [], [], []
    for kind, n, kw in cfg["parts"]:
        if kind == "polygon":
            x, y, t = polygon_points(rng, n, cfg["window"], polygon_of(cfg))
        elif kind == "uniform":
            x, y, t = uniform_points(rng, n, cfg["window"])
        elif kind == "thomas":
            x, y, t = thomas_points(rng, n, cfg["window"], **kw)
        else:
            raise ValueError(kind)
        xs.append(x); ys.append(y); ts.append(t)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ts)


def polygon_of(cfg):
    """The workload's study polygon (None for a rectangle): drawn from its own
    stream (seed + 1000) so the points do not depend on how it was drawn."""
    if not cfg.get("polygon"):
        return None
    return star_polygon(_rng(cfg["seed"] + 1000), cfg["window"], cfg["polygon"])


def workload(name):
    """A copy of one of the named workload dicts above."""
    return dict(WORKLOADS[name])


def serving_requests(num=5000, rate=None, seed=5):
    """The request stream: one dict per request with its own window, grid and points.

    n is log-uniform in [1e3, 5e5]; each set is uniform or Thomas with equal
    odds (P log-uniform in [500, 2000], sigma_xy in [200, 500] m, sigma_t in
    [5, 10] d); window side U[10, 100] km, duration U[180, 730] d; s_max =
    min(U[1, 10] km, side/4) with U{10..50} steps; t_max = min(U[30, 90] d,
    D/4) with U{10..50} steps; U{0..99} CSR simulations with Philox key
    5*2^32 + request id.  Arrival times are Poisson at ``rate`` per second
    (None: all at t = 0).  Points are generated lazily by ``request_points``.
    """
    rng = _rng(seed)
    t_arr = 0.0
    out = []
    for r in range(num):
        if rate:
            t_arr += rng.exponential(1.0 / rate)
        n = int(math.floor(math.exp(rng.uniform(math.log(1e3), math.log(5e5)))))
        side = int(rng.uniform(10_000, 100_000))
        dur = int(rng.uniform(180, 730) * DAY)
        s_max = int(min(rng.uniform(1_000, 10_000), side / 4))
        t_max = int(min(rng.uniform(30, 90) * DAY, dur / 4))
        kind = "uniform" if rng.random() < 0.5 else "thomas"
        kw = {}
        if kind == "thomas":
            kw = dict(parents=int(math.exp(rng.uniform(math.log(500), math.log(2000)))),
                      sigma_xy=float(rng.uniform(200, 500)),
                      sigma_t=float(rng.uniform(5, 10) * DAY))
        out.append(dict(id=r, arrival=t_arr, seed=(5 << 32) + r, point_seed=seed * 1_000_003 + r,
                        window=(0, 0, side, side, 0, dur), s_max=s_max,
                        n_s=int(rng.integers(10, 51)), t_max=t_max,
                        n_t=int(rng.integers(10, 51)), sims=int(rng.integers(0, 100)),
                        parts=[(kind, n, kw)]))
    return out


def request_points(req):
    cfg = dict(req)
    cfg["seed"] = req["point_seed"]
    return make_points(cfg)
