"""Comparison helpers shared by the GPU parity tests.

Tolerances (FP64 oracle vs the library):
  * counts C: bit-exact (integer decisions on exact int64 distances, Eq. 3);
  * weight sums W and K: |dK| <= 1e-6 * K_ref, and K = 0 exactly where K_ref = 0
    (FP32 weights summed exactly in fixed point: each weight carries a few ulp of
    FP32 error, about 3e-7 relative at most, and sums of positive terms keep it);
  * L = sqrt(K/(2 pi t)) - s: |dL| <= 1e-6 * sqrt(K_ref/(2 pi t)), i.e. the K
    bound carried through the square root (L itself cancels near CSR).
"""
import numpy as np

RTOL = 1e-6


def grid_values(s_max, t_max, n_s, n_t):
    s = (np.arange(1, n_s + 1) * (s_max / n_s))[:, None]
    t = (np.arange(1, n_t + 1) * (t_max / n_t))[None, :]
    return s, t


def compare(gpu, ref, s_max, t_max, n_s, n_t, rtol=RTOL, where=""):
    """Assert parity of one grid; returns the worst relative K error."""
    Cg = np.asarray(gpu["C"]).astype(np.uint64)
    Cr = np.asarray(ref["C"]).astype(np.uint64)
    bad = np.argwhere(Cg != Cr)
    assert bad.size == 0, f"{where}: counts differ at {bad[:5].tolist()}: {Cg[tuple(bad[0])]} vs {Cr[tuple(bad[0])]}"
    worst = 0.0
    for key in ("W", "K"):
        if key not in gpu or key not in ref:
            continue
        g = np.asarray(gpu[key], np.float64)
        r = np.asarray(ref[key], np.float64)
        zero = r == 0
        assert np.all(g[zero] == 0), f"{where}: {key} nonzero where the oracle is 0"
        rel = np.abs(g[~zero] - r[~zero]) / np.abs(r[~zero])
        if rel.size:
            worst = max(worst, float(rel.max()))
            assert rel.max() <= rtol, f"{where}: {key} rel err {rel.max():.3g} > {rtol}"
    if "L" in gpu and "L" in ref and "K" in ref:
        s, t = grid_values(s_max, t_max, n_s, n_t)
        Kr = np.asarray(ref["K"], np.float64)
        tol = rtol * np.sqrt(Kr / (2 * np.pi * t)) + 1e-9
        dL = np.abs(np.asarray(gpu["L"]) - np.asarray(ref["L"]))
        assert np.all(dL <= tol), f"{where}: L err {dL.max():.3g}"
    return worst
