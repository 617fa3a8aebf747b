"""Pins for the CPU oracle against facts the paper and the mathematics fix.

Citations are to Wang et al., arXiv 1912.04753, Sec. 3 (Eqs. 1-4 and the
isotropic / temporal edge-correction rules) unless stated otherwise.  None of
these tests re-types an oracle formula: each compares it with a closed form, a
hand-derived case, a different construction (arc-union, 50-digit mpmath, dense
sampling of the circle, literal per-(s,t) evaluation of Eq. 2), an invariant,
or an independent library (numpy's Philox).
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import literal, omega_ref
from paper_1912_04753_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ----
def test_philox_known_answers():
    """Philox4x64-10 equals the published known-answer vectors (Salmon et al., SC'11)."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x64_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(w, 16) for w in r]
        out = oracle.philox4x64_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_philox_matches_numpy_stream():
    """numpy's Philox advances the counter before generating: block c+1 comes first."""
    for key in ([0, 0], [3, 0], [0x0123456789ABCDEF, 7]):
        for c0 in (0, 5, 2**64 - 3):
            ctr = [c0, 11, 0, 9]
            bg = np.random.Philox(key=np.array(key, np.uint64),
                                  counter=np.array(ctr, np.uint64))
            raw = bg.random_raw(8)
            nxt = list(ctr)
            for blk in range(2):
                # carry-propagating increment of the 256-bit counter
                for w in range(4):
                    nxt[w] = (nxt[w] + 1) % 2**64
                    if nxt[w] != 0:
                        break
                mine = oracle.philox4x64_10(nxt, key)
                assert [int(v) for v in mine] == [int(v) for v in raw[4 * blk:4 * blk + 4]]


def test_csr_points_range_and_uniformity():
    """CSR draws stay in the half-open window and are uniform (Sec. 3, Monte Carlo CSTR)."""
    d = oracle.desc((-500, 100, 1500, 2100, 1000, 101000), 100, 1000, 4, 4)
    x, y, t = oracle.csr_points(d, 200_000, 3, 42)
    assert x.min() >= -500 and x.max() < 1500
    assert y.min() >= 100 and y.max() < 2100
    assert t.min() >= 1000 and t.max() < 101000
    for a, lo, hi in ((x, -500, 1500), (y, 100, 2100), (t, 1000, 101000)):
        h, _ = np.histogram(a, bins=20, range=(lo, hi))
        e = len(a) / 20
        chi2 = float(((h - e) ** 2 / e).sum())
        assert chi2 < 60.0  # 19 dof; p < 1e-5 otherwise
    # distinct simulations and distinct seeds differ
    x2, _, _ = oracle.csr_points(d, 1000, 4, 42)
    x3, _, _ = oracle.csr_points(d, 1000, 3, 43)
    assert not np.array_equal(x[:1000], x2) and not np.array_equal(x[:1000], x3)


# ------------------------------------------------------------ thresholds ----
def test_thresholds_are_exact_floors():
    """d <= s_k  <=>  d2 <= S2_k for integer d2 needs S2_k = floor(s_k^2) (Eq. 3)."""
    for s_max, n_s, t_max, n_t in ((1000, 10, 2592000, 10), (1001, 7, 999, 13),
                                   (8388607, 64, 2**31 - 1, 64), (3, 64, 5, 64)):
        d = oracle.desc((0, 0, 10**7, 10**7, 0, 2**31 - 1), s_max, t_max, n_s, n_t)
        S2, T = oracle.thresholds(d)
        for k in range(1, n_s + 1):
            v = int(S2[k - 1])
            assert v * n_s * n_s <= (k * s_max) ** 2 < (v + 1) * n_s * n_s
        for l in range(1, n_t + 1):
            v = int(T[l - 1])
            assert v * n_t <= l * t_max < (v + 1) * n_t


# ----------------------------------------------------------------- omega ----
RECT = (0, 0, 20_000, 15_000)


def _od(rect=RECT):
    return oracle.desc((rect[0], rect[1], rect[2], rect[3], 0, 10**6), 5000, 1000, 10, 10)


@pytest.mark.parametrize("x,y,d2,want", [
    (10_000, 7_500, 0, 1.0),                    # zero radius
    (10_000, 7_500, 7_000**2, 1.0),             # circle inside the area
    (10_000, 7_500, 7_500**2, 1.0),             # tangent to two sides, touching only
    (0, 7_500, 1000**2, 0.5),                   # centre on a side
    (20_000, 7_500, 4321**2, 0.5),
    (10_000, 15_000, 77**2, 0.5),
    (0, 0, 1000**2, 0.25),                      # centre on a corner
    (20_000, 15_000, 4999**2, 0.25),
    (500, 7_500, 1000**2, 2.0 / 3.0),           # one side at r/2: arc 2*pi/3 lost
    (500, 500, 1000**2, 5.0 / 12.0),            # two sides at r/2, corner inside
    (600, 800, 1000**2, 0.5),                   # corner exactly on the circle
    (19_400, 14_200, 1000**2, 0.5),             # same, opposite corner (600, 800 away)
])
def test_omega_closed_forms(x, y, d2, want):
    """Hand-derived shares of the circle inside the rectangle (Sec. 3, isotropic correction)."""
    assert oracle.omega(x, y, d2, _od()) == pytest.approx(want, abs=1e-14)


def test_omega_textbook_one_side():
    """One cut side at distance e < r: share 1 - arccos(e/r)/pi (classical Ripley weight)."""
    d = _od()
    for e, r in ((1, 2), (3, 5), (999, 1000), (0, 7), (4000, 4999)):
        want = 1.0 - math.acos(e / r) / math.pi
        assert oracle.omega(e, 7_500, r * r, d) == pytest.approx(want, abs=1e-14)


def test_omega_matches_arc_union_random():
    """Arc-subtraction form == arc-union construction to 1e-12 over random cases."""
    rng = np.random.default_rng(7)
    d = _od()
    worst = 0.0
    for _ in range(3000):
        x = int(rng.integers(0, RECT[2] + 1))
        y = int(rng.integers(0, RECT[3] + 1))
        r = int(rng.integers(1, 7_500 + 1))      # r <= min(W, H)/2
        a = oracle.omega(x, y, r * r, d)
        b = omega_ref.omega_arc(x, y, float(r), RECT)
        worst = max(worst, abs(a - b))
    assert worst < 1e-12


def test_omega_near_corners_and_tangency():
    """Corner-touching and nearly tangent circles, where cancellation is worst."""
    d = _od()
    cases = []
    for ea in range(0, 40, 3):
        for eb in range(0, 40, 5):
            for d2 in (ea * ea + eb * eb - 1, ea * ea + eb * eb, ea * ea + eb * eb + 1,
                       ea * ea + 1, eb * eb + 1):
                if d2 > 0:
                    cases.append((ea, eb, d2))
    for ea, eb, d2 in cases:
        a = oracle.omega(ea, eb, d2, d)
        b = float(omega_ref.omega_arc_mp(ea, eb, d2, RECT, dps=40))
        assert abs(a - b) < 1e-12, (ea, eb, d2, a, b)


def test_omega_against_mpmath_and_sampling():
    """50-digit arc-union pins the FP64 forms; dense circle sampling pins the arc-union."""
    rng = np.random.default_rng(11)
    d = _od()
    for _ in range(25):
        x = int(rng.integers(0, 3000))
        y = int(rng.integers(0, 3000))
        r = int(rng.integers(1, 6000))
        hi = float(omega_ref.omega_arc_mp(x, y, r * r, RECT, dps=50))
        assert abs(oracle.omega(x, y, r * r, d) - hi) < 1e-13
        assert abs(omega_ref.omega_arc(x, y, r, RECT) - hi) < 1e-12
        n = 1 << 18
        assert abs(omega_ref.omega_sampled(x, y, r, RECT, n) - hi) <= 8.0 / n


def test_omega_continuous_at_corner_touch():
    """No jump where the corner enters the circle: the steps of omega per unit
    of d2 across the switch are as small as the steps next to it."""
    d = _od()
    for ea, eb in ((300, 400), (5, 12), (2000, 2100)):
        c = ea * ea + eb * eb
        vals = [oracle.omega(ea, eb, c + k, d) for k in (-2, -1, 0, 1, 2)]
        steps = np.abs(np.diff(vals))
        assert steps.max() < 3.0 * steps.min()
        assert np.all(np.diff(vals) <= 1e-15)    # non-increasing in r here


def test_omega_off_switch():
    d = oracle.desc((0, 0, 100, 100, 0, 100), 10, 10, 2, 2, edge=oracle.EDGE_TEMPORAL)
    assert oracle.omega(0, 0, 50, d) == 1.0


# ------------------------------------------------------------------ v -------
def test_temporal_weight_cases():
    """v = 1 when t-u and t+u both lie in the period, else 1/2 (Sec. 3)."""
    d = oracle.desc((0, 0, 100, 100, 1000, 2000), 10, 500, 2, 2)
    assert oracle.vt(1500, 0, d) == 1.0
    assert oracle.vt(1500, 500, d) == 1.0          # both ends exactly on the bounds
    assert oracle.vt(1500, 501, d) == 0.5
    assert oracle.vt(1000, 1, d) == 0.5            # centre at the start
    assert oracle.vt(1000, 0, d) == 1.0
    assert oracle.vt(1999, 2, d) == 0.5
    assert oracle.vt(1200, 200, d) == 1.0
    assert oracle.vt(1200, 201, d) == 0.5
    d0 = oracle.desc((0, 0, 100, 100, 1000, 2000), 10, 500, 2, 2, edge=oracle.EDGE_SPATIAL)
    assert oracle.vt(1000, 1, d0) == 1.0


# --------------------------------------------------------- hand examples ----
def test_two_points_hand_derived():
    """Two points, weights derived by hand from Sec. 3 and K from Eq. 2.

    Window [0,100]^2 x [0,100].  Points (2, 50, 10) and (2, 54, 30): d = 4,
    u = 20.  Both centres sit 2 from the left side, so one side cuts each
    circle at e = r/2 and omega = 2/3 for both.  Centre 1 (t=10): 10-20 < 0,
    so v = 1/2 and w = 3; centre 2 (t=30): [10, 50] inside, v = 1, w = 3/2.
    For every grid point with s >= 4 and t >= 20: W = 4.5 and
    K = A*D*W/(n(n-1)) = 1e6*4.5/2; elsewhere 0.
    """
    win = (0, 0, 100, 100, 0, 100)
    d = oracle.desc(win, 8, 40, 4, 4)            # s = 2,4,6,8 ; t = 10,20,30,40
    r = oracle.estimate(d, [2, 2], [50, 54], [10, 30])
    on = np.zeros((4, 4), bool)
    on[1:, 1:] = True
    assert np.array_equal(r["C"], np.where(on, 2, 0).astype(np.uint64))
    assert np.allclose(r["W"], np.where(on, 4.5, 0.0), rtol=1e-15, atol=0)
    assert np.allclose(r["K"], np.where(on, 1e6 * 4.5 / 2, 0.0), rtol=1e-15, atol=0)
    s = np.array([2, 4, 6, 8.0])[:, None]
    t = np.array([10, 20, 30, 40.0])[None, :]
    Lwant = np.sqrt(np.where(on, 1e6 * 4.5 / 2, 0.0) / (2 * np.pi * t)) - s
    assert np.allclose(r["L"], Lwant, rtol=1e-14, atol=1e-12)
    # literal n^2 normalisation (Eq. 2 as printed) scales K by (n-1)/n = 1/2
    d2 = oracle.desc(win, 8, 40, 4, 4, norm=oracle.NORM_N2)
    r2 = oracle.estimate(d2, [2, 2], [50, 54], [10, 30])
    assert np.allclose(r2["K"], r["K"] / 2, rtol=1e-15)


def test_coincident_points_count():
    """Coincident points (d = 0, u = 0) with i != j are counted (Eq. 2, j != i)."""
    win = (0, 0, 1000, 1000, 0, 1000)
    d = oracle.desc(win, 100, 100, 2, 2)
    r = oracle.estimate(d, [500] * 3, [500] * 3, [500] * 3)
    assert np.all(r["C"] == 6)
    assert np.allclose(r["W"], 6.0)


def test_normalisation_closed_form():
    """No edge correction, s_max past the diagonal, t_max >= D: every ordered pair
    counts with weight 1, so K = A*D exactly for N = n(n-1) (Eqs. 1-2)."""
    rng = np.random.default_rng(3)
    win = (0, 0, 300, 200, 0, 5000)
    n = 257
    x = rng.integers(0, 301, n); y = rng.integers(0, 201, n); t = rng.integers(0, 5001, n)
    d = oracle.desc(win, 361, 5000, 3, 4, edge=0)
    r = oracle.estimate(d, x, y, t)
    assert int(r["C"][-1, -1]) == n * (n - 1)
    assert r["K"][-1, -1] == pytest.approx(300 * 200 * 5000, rel=1e-14)
    dn = oracle.desc(win, 361, 5000, 3, 4, edge=0, norm=oracle.NORM_N2)
    rn = oracle.estimate(dn, x, y, t)
    assert rn["K"][-1, -1] == pytest.approx(300 * 200 * 5000 * (n - 1) / n, rel=1e-14)


# ------------------------------------------------------ literal Eq. 2 -------
def _tiny_sets():
    rng = np.random.default_rng(2024)
    win = (0, 0, 1000, 800, 0, 10_000)
    out = []
    n = 60
    out.append(("uniform", win, rng.integers(0, 1001, n), rng.integers(0, 801, n),
                rng.integers(0, 10_001, n)))
    # clusters plus exact duplicates and points on sides and corners
    cx = np.clip(rng.normal(100, 40, n), 0, 1000).astype(int)
    cy = np.clip(rng.normal(700, 40, n), 0, 800).astype(int)
    ct = np.clip(rng.normal(9000, 500, n), 0, 10_000).astype(int)
    cx[:6] = [0, 0, 1000, 1000, 0, 500]
    cy[:6] = [0, 800, 0, 800, 400, 0]
    ct[:6] = [0, 10_000, 5000, 0, 10_000, 1]
    cx[6:9] = cx[9]; cy[6:9] = cy[9]; ct[6:9] = ct[9]
    out.append(("clustered+edges", win, cx, cy, ct))
    return out


@pytest.mark.parametrize("edge", [3, 1, 2, 0])
@pytest.mark.parametrize("norm", [0, 1])
def test_literal_eq2_matches_oracle(edge, norm):
    """Eq. 2 evaluated literally per (s_k, t_l) equals histogram + 2-D prefix:
    counts exactly, K to 1e-12 (P1 brute force on tiny inputs)."""
    for name, win, x, y, t in _tiny_sets():
        s_max, n_s, t_max, n_t = 400, 7, 4_000, 5          # s_max <= min(W, H)/2
        Craw, Klit, Llit = literal.literal_K(win, s_max, t_max, n_s, n_t, x, y, t,
                                             edge=edge, norm=norm)
        d = oracle.desc(win, s_max, t_max, n_s, n_t, edge=edge, norm=norm)
        r = oracle.estimate(d, x, y, t)
        assert np.array_equal(r["C"].astype(np.int64), Craw), name
        assert np.allclose(r["K"], Klit, rtol=1e-12, atol=0), name
        ok = Klit > 0
        assert np.allclose(r["L"][ok], Llit[ok], rtol=0, atol=1e-9), name


def test_literal_larger_grid_non_divisible():
    """A grid whose steps do not divide s_max / t_max exactly (floor thresholds)."""
    rng = np.random.default_rng(99)
    win = (100, -50, 1300, 950, 7, 20_007)
    n = 90
    x = rng.integers(100, 1301, n); y = rng.integers(-50, 951, n); t = rng.integers(7, 20_008, n)
    s_max, n_s, t_max, n_t = 497, 9, 6_001, 11
    Craw, Klit, _ = literal.literal_K(win, s_max, t_max, n_s, n_t, x, y, t)
    d = oracle.desc(win, s_max, t_max, n_s, n_t)
    r = oracle.estimate(d, x, y, t)
    assert np.array_equal(r["C"].astype(np.int64), Craw)
    assert np.allclose(r["K"], Klit, rtol=1e-12, atol=0)


# ------------------------------------------------------------ invariants ----
def test_symmetry_and_monotonicity():
    """Unweighted ordered counts are symmetric in i<->j (all even); C and W are
    non-decreasing in s and t (Eq. 3 is monotone)."""
    cfg = workloads.workload("uniform-2k")
    x, y, t = workloads.make_points(cfg)
    d = oracle.desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"])
    r = oracle.estimate(d, x, y, t)
    C = r["C"].astype(np.int64)
    assert np.all(C % 2 == 0)
    assert np.all(np.diff(C, axis=0) >= 0) and np.all(np.diff(C, axis=1) >= 0)
    W = r["W"]
    assert np.all(np.diff(W, axis=0) >= 0) and np.all(np.diff(W, axis=1) >= 0)
    # weights lie in [1, 8]: W between C and 8C
    assert np.all(W >= C - 1e-9) and np.all(W <= 8 * C + 1e-9)


def test_centre_subset_additivity():
    """Sum over a split of the centres equals the full estimate (Eq. 2 sums over i)."""
    rng = np.random.default_rng(5)
    win = (0, 0, 2000, 2000, 0, 100_000)
    n = 700
    x = rng.integers(0, 2000, n); y = rng.integers(0, 2000, n); t = rng.integers(0, 100_000, n)
    d = oracle.desc(win, 300, 20_000, 6, 5)
    full = oracle.hist(d, x, y, t)
    perm = rng.permutation(n)
    a = oracle.hist(d, x[perm], y[perm], t[perm], n_centres=250)
    rev = np.concatenate([perm[250:], perm[:250]])
    b = oracle.hist(d, x[rev], y[rev], t[rev], n_centres=n - 250)
    assert np.array_equal(a[0] + b[0], full[0])
    assert np.allclose(a[1] + b[1], full[1], rtol=1e-13)


def test_csr_expectation():
    """Under CSR with n(n-1) normalisation and both edge corrections,
    E[K(s,t)] = 2*pi*s^2*t (Sec. 3, Eq. 1 and the CSTR expectation); checked as the
    mean of 160 simulated sets within 4 standard errors.  Also L ~ 0."""
    win = (0, 0, 2000, 2000, 0, 1_000_000)
    s_max, n_s, t_max, n_t = 400, 4, 200_000, 4
    d = oracle.desc(win, s_max, t_max, n_s, n_t)
    m = 160
    env = oracle.envelope(d, 900, m, seed=77)
    Ks = env["K_sims"]
    mean = Ks.mean(axis=0)
    se = Ks.std(axis=0, ddof=1) / math.sqrt(m)
    s = (np.arange(1, n_s + 1) * s_max / n_s)[:, None]
    t = (np.arange(1, n_t + 1) * t_max / n_t)[None, :]
    want = 2 * np.pi * s ** 2 * t
    z = (mean - want) / se
    assert np.all(np.abs(z) < 4.0), z
    # the envelope brackets every simulation and the theoretical value mostly
    assert np.all(env["K_lo"] <= Ks.min(axis=0) + 0) and np.all(env["K_hi"] >= Ks.max(axis=0))
    assert np.all((env["K_lo"] < want) & (want < env["K_hi"]))


def test_csr_expectation_detects_missing_temporal_correction():
    """Planted mistake, on the CPU: dropping the temporal correction biases the
    CSR mean low by a clear margin -- so the check above has teeth."""
    win = (0, 0, 2000, 2000, 0, 1_000_000)
    d = oracle.desc(win, 400, 200_000, 4, 4, edge=oracle.EDGE_SPATIAL)
    env = oracle.envelope(d, 900, 60, seed=77)
    mean = env["K_sims"].mean(axis=0)
    want = 2 * np.pi * (400.0 ** 2) * 200_000
    assert mean[-1, -1] < 0.95 * want


def test_envelope_min_max_semantics():
    """Envelopes are the pointwise min/max over the simulations only (Sec. 3)."""
    cfg = workloads.workload("uniform-2k")
    d = oracle.desc(cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"])
    env = oracle.envelope(d, 400, 7, seed=1)
    Ks = env["K_sims"]
    assert np.array_equal(env["K_lo"], Ks.min(axis=0))
    assert np.array_equal(env["K_hi"], Ks.max(axis=0))
    # L is increasing in K at fixed (s, t), so its envelope follows K's
    s = (np.arange(1, 11) * 100.0)[:, None]
    t = (np.arange(1, 11) * 259200.0)[None, :]
    assert np.allclose(env["L_lo"], np.sqrt(env["K_lo"] / (2 * np.pi * t)) - s, rtol=0, atol=1e-9)
    # each simulation is reproducible from (seed, sim) alone
    x, y, tt = oracle.csr_points(d, 400, 5, 1)
    r = oracle.estimate(d, x, y, tt)
    assert np.array_equal(r["C"], env["C_sims"][5])
    assert np.allclose(r["K"], Ks[5], rtol=1e-15, atol=0)


# ------------------------------------------------- resampled simulations ----
def _numpy_block(key, ctr):
    """Philox4x64-10 block at counter ``ctr`` from numpy's generator (which
    increments its 256-bit counter before generating, so start one below)."""
    c = [int(v) for v in ctr]
    for w in range(4):  # 256-bit decrement with borrow
        c[w] = (c[w] - 1) % 2**64
        if c[w] != 2**64 - 1:
            break
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(c, np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def test_permutation_is_the_argsort_of_philox_keys():
    """Random permutation (Sec. 3): locations kept, time labels exchanged; point i
    takes the time of the point ranked i-th by the high 32 bits of Philox word 0
    (key (seed, 1), counter (j, sim, 0, 0)), ties by index."""
    rng = np.random.default_rng(3)
    n, seed = 300, 77
    x = rng.integers(0, 1000, n).astype(np.int32)
    y = rng.integers(0, 1000, n).astype(np.int32)
    t = rng.integers(0, 10**6, n).astype(np.int32)
    for sim in (0, 5):
        u = np.array([_numpy_block([seed, 1], [j, sim, 0, 0])[0] >> 32 for j in range(n)], np.uint64)
        order = np.argsort(u, kind="stable")
        xs, ys, ts = oracle.resampled_points(x, y, t, sim, seed, oracle.SIM_PERMUTE)
        assert np.array_equal(xs, x) and np.array_equal(ys, y)
        assert np.array_equal(ts, t[order])
        assert np.array_equal(np.sort(ts), np.sort(t))


def test_bootstrap_indices_follow_philox():
    """Bootstrap (Sec. 3): point i of simulation sim is observed point
    floor(r0 * n / 2^64), r = Philox(key (seed, 2), counter (i, sim, 0, 0))."""
    rng = np.random.default_rng(4)
    n, seed, sim = 257, 9, 3
    x = rng.integers(0, 1000, n).astype(np.int32)
    y = rng.integers(0, 1000, n).astype(np.int32)
    t = np.arange(n, dtype=np.int32) * 7
    idx = np.array([(_numpy_block([seed, 2], [i, sim, 0, 0])[0] * n) >> 64 for i in range(n)])
    xs, ys, ts = oracle.resampled_points(x, y, t, sim, seed, oracle.SIM_BOOTSTRAP)
    assert np.array_equal(xs, x[idx]) and np.array_equal(ys, y[idx]) and np.array_equal(ts, t[idx])
    assert len(np.unique(idx)) < n  # with replacement


def test_permutation_labels_are_uniform():
    """Over many simulations each position receives each label equally often."""
    n, sims = 6, 6000
    x = np.zeros(n, np.int32); y = np.zeros(n, np.int32); t = np.arange(n, dtype=np.int32)
    counts = np.zeros((n, n))
    for s in range(sims):
        _, _, ts = oracle.resampled_points(x, y, t, s, 123, oracle.SIM_PERMUTE)
        counts[np.arange(n), ts] += 1
    e = sims / n
    chi2 = float(((counts - e) ** 2 / e).sum())
    assert chi2 < 80.0  # 25 dof; p < 1e-6 otherwise


def test_permuted_set_keeps_spatial_counts():
    """With the temporal threshold covering the whole period, exchanging time
    labels cannot change which pairs are within s: the last column of C (all u)
    equals the observed one, while inner columns differ."""
    rng = np.random.default_rng(5)
    win = (0, 0, 4000, 4000, 0, 100_000)
    n = 400
    x = rng.integers(0, 4001, n).astype(np.int32)
    y = rng.integers(0, 4001, n).astype(np.int32)
    t = rng.integers(0, 100_001, n).astype(np.int32)
    d = oracle.desc(win, 800, 100_000, 8, 5, edge=0)
    obs = oracle.estimate(d, x, y, t)
    env = oracle.envelope_resampled(d, x, y, t, 3, 11, oracle.SIM_PERMUTE)
    for s in range(3):
        assert np.array_equal(env["C_sims"][s][:, -1], obs["C"][:, -1])
        assert not np.array_equal(env["C_sims"][s][:, :-1], obs["C"][:, :-1])
    assert np.all(env["K_lo"] <= env["K_hi"])


# ------------------------------------------------------- cross (bivariate) K ----
def _two_types(seed, n, n1, win):
    rng = np.random.default_rng(seed)
    x0, y0, x1, y1, t0, t1 = win
    x = rng.integers(x0, x1 + 1, n).astype(np.int32)
    y = rng.integers(y0, y1 + 1, n).astype(np.int32)
    t = rng.integers(t0, t1 + 1, n).astype(np.int32)
    # a few type-2 points on top of type-1 points (coincident pairs across types)
    k = min(3, n1, n - n1)
    x[n1:n1 + k] = x[:k]; y[n1:n1 + k] = y[:k]; t[n1:n1 + k] = t[:k]
    return x, y, t


@pytest.mark.parametrize("edge", [3, 1, 2, 0])
def test_cross_literal_matches_oracle(edge):
    """Two-type estimator evaluated literally per (s_k, t_l), with the arc-union
    omega and exact rational indicators, equals the oracle's cross histogram +
    prefix: counts exactly, K12 to 1e-12, N = n1 * n2."""
    win = (0, 0, 1000, 1200, 0, 50_000)
    for n, n1 in ((40, 13), (25, 1), (25, 24)):
        x, y, t = _two_types(n + n1, n, n1, win)
        s_max, n_s, t_max, n_t = 450, 6, 9_000, 5
        Craw, Klit, Llit = literal.literal_K(win, s_max, t_max, n_s, n_t, x, y, t, edge=edge,
                                             n1=n1)
        d = oracle.desc(win, s_max, t_max, n_s, n_t, edge=edge)
        r = oracle.estimate_cross(d, x, y, t, n1)
        assert np.array_equal(r["C"].astype(np.int64), Craw), (n, n1)
        assert np.allclose(r["K"], Klit, rtol=1e-12, atol=0), (n, n1)
        ok = Klit > 0
        assert np.allclose(r["L"][ok], Llit[ok], rtol=0, atol=1e-9)


def test_cross_terms_partition_the_univariate_sum():
    """The ordered pairs of a two-type set split into type 1 x type 1, type 2 x
    type 2 and the two cross terms, with weights centred on i in each: the
    univariate histogram equals the sum of the four (counts exactly)."""
    win = (0, 0, 3000, 3000, 0, 200_000)
    n, n1 = 900, 340
    x, y, t = _two_types(17, n, n1, win)
    d = oracle.desc(win, 500, 30_000, 8, 6)
    full = oracle.hist(d, x, y, t)
    aa = oracle.hist(d, x[:n1], y[:n1], t[:n1])
    bb = oracle.hist(d, x[n1:], y[n1:], t[n1:])
    ab = oracle.hist_cross(d, x, y, t, n1)
    sw = np.concatenate([np.arange(n1, n), np.arange(n1)])
    ba = oracle.hist_cross(d, x[sw], y[sw], t[sw], n - n1)
    assert np.array_equal(aa[0] + bb[0] + ab[0] + ba[0], full[0])
    assert np.allclose(aa[1] + bb[1] + ab[1] + ba[1], full[1], rtol=1e-12)
    # the indicator is symmetric, the weights are not (centred on type 1 / type 2)
    assert np.array_equal(ab[0], ba[0])
    assert not np.allclose(ab[1], ba[1], rtol=1e-6)


def test_cross_without_correction_counts_pairs():
    """With no edge correction every cross weight is 1: W12 = C12 and K12 equals
    A*D*C12/(n1*n2) exactly as written."""
    win = (0, 0, 2000, 2000, 0, 100_000)
    n, n1 = 500, 200
    x, y, t = _two_types(8, n, n1, win)
    d = oracle.desc(win, 300, 20_000, 5, 4, edge=0)
    r = oracle.estimate_cross(d, x, y, t, n1)
    assert np.array_equal(r["W"], r["C"].astype(np.float64))
    want = 2000.0 * 2000.0 * 100_000.0 * r["C"].astype(np.float64) / (n1 * (n - n1))
    assert np.allclose(r["K"], want, rtol=1e-15, atol=0)


def test_cross_expectation_independent_types():
    """Two independent CSR types: E[K12(s,t)] = 2*pi*s^2*t as for one CSR
    process (the cross pairs of independent uniform sets are uniform)."""
    win = (0, 0, 2000, 2000, 0, 1_000_000)
    s_max, n_s, t_max, n_t = 400, 4, 200_000, 4
    d = oracle.desc(win, s_max, t_max, n_s, n_t)
    m = 120
    env = oracle.envelope_cross(d, np.zeros(900, np.int32), np.zeros(900, np.int32),
                                np.zeros(900, np.int32), 300, m, 21, oracle.SIM_CSR)
    Ks = env["K_sims"]
    se = Ks.std(axis=0, ddof=1) / math.sqrt(m)
    s = (np.arange(1, n_s + 1) * s_max / n_s)[:, None]
    tt = (np.arange(1, n_t + 1) * t_max / n_t)[None, :]
    z = (Ks.mean(axis=0) - 2 * np.pi * s ** 2 * tt) / se
    assert np.all(np.abs(z) < 4.0), z


def test_typed_bootstrap_draws_each_type_from_itself():
    """Bootstrap with two types: point i < n1 is observed point floor(r0*n1/2^64),
    point i >= n1 is n1 + floor(r0*(n-n1)/2^64), r from Philox (key (seed, 2))."""
    n, n1, seed, sim = 120, 45, 6, 2
    x = np.arange(n, dtype=np.int32); y = x * 2; t = x * 3
    xs, ys, ts = oracle.resampled_points(x, y, t, sim, seed, oracle.SIM_BOOTSTRAP, n1=n1)
    r0 = [_numpy_block([seed, 2], [i, sim, 0, 0])[0] for i in range(n)]
    idx = np.array([(r0[i] * n1) >> 64 if i < n1 else n1 + ((r0[i] * (n - n1)) >> 64)
                    for i in range(n)])
    assert np.array_equal(xs, x[idx]) and np.array_equal(ts, t[idx])
    assert np.all(idx[:n1] < n1) and np.all(idx[n1:] >= n1)
    # one type spanning the set is the untyped bootstrap
    a = oracle.resampled_points(x, y, t, sim, seed, oracle.SIM_BOOTSTRAP, n1=n)
    b = oracle.resampled_points(x, y, t, sim, seed, oracle.SIM_BOOTSTRAP)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))


# ----------------------------------------------------- polygon study area ----
L_SHAPE = [(0, 0), (2000, 0), (2000, 1000), (1000, 1000), (1000, 2000), (0, 2000)]


def _inside_np(poly, px, py):
    """Crossing number of real points (vectorised), written for these tests."""
    P = np.asarray(poly, np.float64)
    ax, ay = P[:, 0], P[:, 1]
    bx, by = np.roll(ax, -1), np.roll(ay, -1)
    X, Y = px[:, None], py[:, None]
    st = (ay > Y) != (by > Y)
    with np.errstate(divide="ignore", invalid="ignore"):
        xc = ax + (Y - ay) * (bx - ax) / (by - ay)
    return (np.count_nonzero(st & (X < xc), axis=1) % 2) == 1


def test_polygon_rectangle_reduces_to_rectangle():
    """A polygon that is the window rectangle (either orientation) gives the
    rectangle's closed-form omega, area and whole estimate."""
    win = (0, 0, 3000, 2000, 0, 100_000)
    rect = [(0, 0), (3000, 0), (3000, 2000), (0, 2000)]
    dr = oracle.desc(win, 900, 20_000, 6, 4)
    rng = np.random.default_rng(21)
    for poly in (rect, rect[::-1]):
        dp = oracle.desc(win, 900, 20_000, 6, 4, poly=poly)
        assert oracle.poly_area(dp) == 6e6
        for _ in range(400):
            x, y = int(rng.integers(1, 3000)), int(rng.integers(1, 2000))
            d2 = int(rng.integers(0, 1000 ** 2))
            assert abs(oracle.omega(x, y, d2, dp) - oracle.omega(x, y, d2, dr)) < 1e-12
    n = 400
    x = rng.integers(1, 3000, n); y = rng.integers(1, 2000, n); t = rng.integers(0, 100_001, n)
    a = oracle.estimate(dr, x, y, t)
    b = oracle.estimate(oracle.desc(win, 900, 20_000, 6, 4, poly=rect), x, y, t)
    assert np.array_equal(a["C"], b["C"])
    assert np.allclose(a["K"], b["K"], rtol=1e-12, atol=0)


def test_polygon_omega_hand_derived_reflex_corner():
    """L-shaped area, centre (1100, 900) at distance 100 from both lines of the
    reflex corner (1000, 1000).  The circle of radius r leaves the area where
    x > 1000 and y > 1000, i.e. sin(th) > a and cos(th) > -a with a = 100/r:
    th from arcsin(a) to min(pi - arcsin(a), pi/2 + arcsin(a)).  For
    r >= 100*sqrt(2) that is an arc of pi/2 (omega = 3/4, until the sides 900
    away are reached); for 100 < r < 100*sqrt(2) it is pi - 2*arcsin(a); below
    r = 100 the circle stays inside (omega = 1)."""
    d = oracle.desc((0, 0, 2000, 2000, 0, 1000), 600, 100, 3, 2, poly=L_SHAPE)
    for r2 in (2 * 100 ** 2, 200 ** 2, 400 ** 2, 890 ** 2):
        assert abs(oracle.omega(1100, 900, r2, d) - 0.75) < 1e-12, r2
    for r2 in (101 ** 2, 120 ** 2, 141 ** 2):
        want = 1 - (math.pi - 2 * math.asin(100 / math.sqrt(r2))) / (2 * math.pi)
        assert abs(oracle.omega(1100, 900, r2, d) - want) < 1e-12, r2
    assert oracle.omega(1100, 900, 99 ** 2, d) == 1.0
    # a convex corner of the L: quarter of the circle inside at the vertex limit
    assert abs(oracle.omega(1, 1, 500 ** 2, d) - 0.25) < 2e-3
    assert oracle.poly_area(d) == 3e6


def test_polygon_omega_against_angle_sampling():
    """The 85-vertex synthetic boundary: omega against the share of 200,000
    equally spaced points of the circle that lie inside (an independent
    crossing-number test); the sampling error is a few crossings / 200,000."""
    c = workloads.workload("polygon-100k-99csr")
    P = workloads.polygon_of(c)
    d = oracle.desc(c["window"], c["s_max"], c["t_max"], c["n_s"], c["n_t"], poly=P)
    rng = np.random.default_rng(8)
    x, y, _ = workloads.polygon_points(rng, 60, c["window"], P)
    th = (np.arange(200_000) + 0.5) * (2 * np.pi / 200_000)
    checked = 0
    for i in range(60):
        d2 = int(rng.integers(1, 3_000 ** 2))
        r = math.sqrt(d2)
        share = _inside_np(P, x[i] + r * np.cos(th), y[i] + r * np.sin(th)).mean()
        om = oracle.omega(int(x[i]), int(y[i]), d2, d)
        assert abs(om - share) < 1e-4, (i, om, share)
        checked += om < 1.0
    assert checked >= 10  # many circles actually cross the boundary


def test_polygon_containment_and_area():
    d = oracle.desc((0, 0, 2000, 2000, 0, 1000), 600, 100, 3, 2, poly=L_SHAPE)
    pts = [(500, 500, 1), (1500, 500, 1), (1500, 1500, 0), (0, 500, 0), (1000, 1500, 0),
           (1000, 1000, 0), (999, 1500, 1), (2000, 2000, 0), (1999, 999, 1), (1999, 1000, 0)]
    got = oracle.poly_contains(d, [p[0] for p in pts], [p[1] for p in pts])
    assert got.tolist() == [p[2] for p in pts]
    d2 = oracle.desc((0, 0, 2000, 2000, 0, 1000), 600, 100, 3, 2, poly=L_SHAPE[::-1])
    assert oracle.poly_area(d2) == 3e6


def test_polygon_csr_rejection_follows_philox():
    """CSR in a polygon: attempt a of point i uses Philox counter (i, sim, a, 0)
    (key (seed, 0)); the first attempt strictly inside is kept."""
    win = (0, 0, 2000, 2000, 0, 1000)
    d = oracle.desc(win, 600, 100, 3, 2, poly=L_SHAPE)
    n, sim, seed = 300, 2, 13
    x, y, t = oracle.csr_points(d, n, sim, seed)
    assert oracle.poly_contains(d, x, y).all()
    for i in range(n):
        for a in range(64):
            r = _numpy_block([seed, 0], [i, sim, a, 0])
            px, py = (r[0] * 2000) >> 64, (r[1] * 2000) >> 64
            if oracle.poly_contains(d, px, py)[0]:
                assert (x[i], y[i], t[i]) == (px, py, (r[2] * 1000) >> 64), i
                break


def test_polygon_csr_expectation():
    """CSR inside the L-shaped area with the polygon correction and area:
    mean K over 120 simulations within 4 standard errors of 2*pi*s^2*t."""
    win = (0, 0, 2000, 2000, 0, 1_000_000)
    s_max, n_s, t_max, n_t = 300, 3, 200_000, 4
    d = oracle.desc(win, s_max, t_max, n_s, n_t, poly=L_SHAPE)
    m = 120
    env = oracle.envelope(d, 700, m, seed=5)
    Ks = env["K_sims"]
    se = Ks.std(axis=0, ddof=1) / math.sqrt(m)
    s = (np.arange(1, n_s + 1) * s_max / n_s)[:, None]
    tt = (np.arange(1, n_t + 1) * t_max / n_t)[None, :]
    z = (Ks.mean(axis=0) - 2 * np.pi * s ** 2 * tt) / se
    assert np.all(np.abs(z) < 4.0), z


def test_polygon_weight_uncapped_spike():
    """Sec. 3's spatial weight 1/omega has no bound: on the thin arm of an L
    (y in [0, w], x in [1000, 4000]) a circle of radius r about a centre at
    height w/2 stays inside only where |sin(th)| <= (w/2)/r and x lies on the
    arm.  Centre (3990, w/2), r = 1390: one such arc (near th = pi), so
    omega = asin(w/2r)/pi (1/omega = 87.3 for w = 100, 873 for w = 10); centre
    (2600, w/2): two arcs, omega = 2 asin(w/2r)/pi.  The two-point set weighs
    exactly the sum of both inverses, far beyond 64; angle sampling of the
    circle agrees."""
    win = (0, 0, 4000, 4000, 0, 1000)
    for w in (100, 10):
        spike = [(0, 0), (4000, 0), (4000, w), (1000, w), (1000, 4000), (0, 4000)]
        d = oracle.desc(win, 1500, 100, 1, 1, edge=oracle.EDGE_SPATIAL, poly=spike)
        a = math.asin((w / 2) / 1390)
        om_i = oracle.omega(3990, w // 2, 1390 ** 2, d)
        om_j = oracle.omega(2600, w // 2, 1390 ** 2, d)
        assert abs(om_i - a / math.pi) < 1e-13 * (a / math.pi) + 1e-15, (w, om_i)
        assert abs(om_j - 2 * a / math.pi) < 1e-13 * (a / math.pi) + 1e-15, (w, om_j)
        assert 1 / om_i > 64
        th = (np.arange(2_000_000) + 0.5) * (2 * np.pi / 2_000_000)
        share = _inside_np(spike, 3990 + 1390 * np.cos(th), w / 2 + 1390 * np.sin(th)).mean()
        assert abs(share - om_i) < 2e-6, (w, share, om_i)
        x = np.array([3990, 2600], np.int32); y = np.array([w // 2, w // 2], np.int32)
        t = np.array([10, 10], np.int32)
        Hc, Hw = oracle.hist(d, x, y, t)
        assert Hc[0, 0] == 2
        want = math.pi / a * 1.5
        assert abs(Hw[0, 0] - want) < 1e-12 * want, (w, Hw[0, 0], want)


# -------------------------------------------------------- inhomogeneous K ----
def test_inhom_constant_intensity_is_the_n2_estimate():
    """With lambda_i = n/(A*D) for every point the inhomogeneous estimator is
    Eq. 2 with N = n^2; any constant c*lambda scales K by 1/c^2."""
    cfg = workloads.workload("uniform-2k")
    x, y, t = workloads.make_points(cfg)
    n = len(x)
    args = (cfg["window"], cfg["s_max"], cfg["t_max"], cfg["n_s"], cfg["n_t"])
    AD = 10_000.0 * 10_000.0 * 365 * 86400
    r2 = oracle.estimate(oracle.desc(*args, norm=oracle.NORM_N2), x, y, t)
    ri = oracle.estimate_inhom(oracle.desc(*args), x, y, t, np.full(n, n / AD))
    assert np.array_equal(ri["C"], r2["C"])
    assert np.allclose(ri["K"], r2["K"], rtol=1e-12, atol=0)
    r3 = oracle.estimate_inhom(oracle.desc(*args), x, y, t, np.full(n, 3.0 * n / AD))
    assert np.allclose(r3["K"], r2["K"] / 9.0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("edge", [3, 0])
def test_inhom_literal_matches_oracle(edge):
    """Literal per-step evaluation with 1/(lambda_i lambda_j) weights."""
    rng = np.random.default_rng(71)
    win = (0, 0, 1500, 1200, 0, 60_000)
    n = 45
    x = rng.integers(0, 1501, n); y = rng.integers(0, 1201, n); t = rng.integers(0, 60_001, n)
    lam = rng.uniform(0.5, 4.0, n) * n / (1500 * 1200 * 60_000)
    args = (win, 500, 9_000, 5, 4)
    Craw, Klit, _ = literal.literal_K(*args, x, y, t, edge=edge, lam=lam)
    r = oracle.estimate_inhom(oracle.desc(*args, edge=edge), x, y, t, lam)
    assert np.array_equal(r["C"].astype(np.int64), Craw)
    assert np.allclose(r["K"], Klit, rtol=1e-12, atol=0)


def test_inhom_expectation_under_inhomogeneous_poisson():
    """A Poisson process with intensity lambda(x) = lam0 * (0.2 + 1.6 x/W)
    (drawn by thinning, Poisson count): with the true intensity, the mean of
    K_I over 150 draws is 2*pi*s^2*t within 4 standard errors; the homogeneous
    estimator of the same draws is biased upwards."""
    win = (0, 0, 2000, 2000, 0, 1_000_000)
    s_max, n_s, t_max, n_t = 300, 3, 200_000, 4
    d = oracle.desc(win, s_max, t_max, n_s, n_t)
    AD = 2000.0 * 2000.0 * 1_000_000
    lam0 = 800 / AD
    rng = np.random.default_rng(72)
    Ks, Kh = [], []
    for _ in range(150):
        m = rng.poisson(800 * 1.8)   # candidates at the peak intensity, thinned
        x = rng.integers(0, 2000, m); y = rng.integers(0, 2000, m); t = rng.integers(0, 1_000_000, m)
        f = 0.2 + 1.6 * x / 2000.0
        keep = rng.uniform(0, 1.8, m) < f
        x, y, t = x[keep], y[keep], t[keep]
        Ks.append(oracle.estimate_inhom(d, x, y, t, lam0 * (0.2 + 1.6 * x / 2000.0))["K"])
        Kh.append(oracle.estimate(d, x, y, t)["K"])
    Ks, Kh = np.array(Ks), np.array(Kh)
    se = Ks.std(axis=0, ddof=1) / math.sqrt(len(Ks))
    s = (np.arange(1, n_s + 1) * s_max / n_s)[:, None]
    tt = (np.arange(1, n_t + 1) * t_max / n_t)[None, :]
    want = 2 * np.pi * s ** 2 * tt
    z = (Ks.mean(axis=0) - want) / se
    assert np.all(np.abs(z) < 4.0), z
    assert Kh.mean(axis=0)[-1, -1] > 1.1 * want[-1, -1]
