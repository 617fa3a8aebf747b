"""Eq. 2 of the paper evaluated literally, one grid point at a time -- test infrastructure.

For every grid point (s_k, t_l) this sums I_{s_k,t_l}(d_ij, u_ij)/(omega_ij*v_ij)
over every ordered pair i != j and scales by A*D/N (Wang et al., Sec. 3,
Eqs. 2-3), then takes L = sqrt(K/(2*pi*t)) - s (Eq. 4).  It uses none of the
histogram/prefix reformulation of ``oracle.c``:

  * the indicator d_ij <= s_k and u_ij <= t_l is decided in exact rational
    arithmetic (d2 * n_s^2 <= (k*s_max)^2, u * n_t <= l*t_max);
  * omega_ij comes from the arc-union construction in ``omega_ref``;
  * v_ij is the end-point rule of Sec. 3 written out.

With ``lam`` (an intensity per point) it evaluates the inhomogeneous
estimator: each pair weighs 1/(omega v lambda_i lambda_j) and K = W/(A*D).
With ``n1`` it evaluates the two-type (cross) estimator instead: only ordered
pairs with i < n1 (type 1) and j >= n1 (type 2) count, and N = n1 * (n - n1).

Cost is O(n_s * n_t * n^2) numpy work plus n^2 arc-union calls, so it is for
tiny inputs only (n up to a few hundred).
"""
import math

import numpy as np

from .omega_ref import omega_arc

EDGE_SPATIAL = 1
EDGE_TEMPORAL = 2


def literal_K(window, s_max, t_max, n_s, n_t, x, y, t, edge=3, norm=0, n1=None, lam=None):
    """Return (Craw, K, L): Craw[k, l] = number of ordered pairs counted at (s_k, t_l)."""
    x0, y0, x1, y1, t0, t1 = (int(v) for v in window)
    x = [int(v) for v in x]
    y = [int(v) for v in y]
    t = [int(v) for v in t]
    n = len(x)
    # pairwise integer quantities and weights, ordered pairs, diagonal excluded
    D2 = np.zeros((n, n), dtype=object)
    U = np.zeros((n, n), dtype=object)
    Wt = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d2 = (x[i] - x[j]) ** 2 + (y[i] - y[j]) ** 2
            u = abs(t[i] - t[j])
            D2[i, j] = d2
            U[i, j] = u
            if d2 > s_max * s_max or u * n_t > n_t * t_max:
                continue    # outside every grid point: the weight is never used
            om = 1.0
            if edge & EDGE_SPATIAL:
                om = omega_arc(x[i], y[i], math.sqrt(d2), (x0, y0, x1, y1))
            v = 1.0
            if edge & EDGE_TEMPORAL:
                v = 1.0 if (t[i] - u >= t0 and t[i] + u <= t1) else 0.5
            Wt[i, j] = 1.0 / (om * v)
            if lam is not None:
                Wt[i, j] /= float(lam[i]) * float(lam[j])
    off = ~np.eye(n, dtype=bool)
    A = (x1 - x0) * (y1 - y0)
    Dur = t1 - t0
    N = n * n if norm == 1 else n * (n - 1)
    if lam is not None:
        N = (A * Dur) ** 2   # K_I = W/(A*D)
    if n1 is not None:
        idx = np.arange(n)
        off = (idx[:, None] < n1) & (idx[None, :] >= n1)
        N = n1 * (n - n1)
    Craw = np.zeros((n_s, n_t), dtype=np.int64)
    K = np.zeros((n_s, n_t), dtype=np.float64)
    L = np.zeros((n_s, n_t), dtype=np.float64)
    d2n = D2 * (n_s * n_s)
    un = U * n_t
    for k in range(1, n_s + 1):
        sk2 = (k * s_max) ** 2
        in_s = (d2n <= sk2).astype(bool) & off
        for l in range(1, n_t + 1):
            in_st = in_s & (un <= l * t_max).astype(bool)
            Craw[k - 1, l - 1] = int(in_st.sum())
            acc = math.fsum(Wt[in_st].tolist())
            Kv = A * Dur * acc / N
            K[k - 1, l - 1] = Kv
            s_k = k * s_max / n_s
            t_l = l * t_max / n_t
            L[k - 1, l - 1] = math.sqrt(Kv / (2.0 * math.pi * t_l)) - s_k
    return Craw, K, L
