"""Isotropic spatial edge-correction weight by direct arc-union -- test infrastructure.

The paper's spatial weight omega_ij is the share of the circumference of the
circle centred on point i with radius d_ij that lies inside the study area
(Wang et al., Sec. 3, isotropic edge correction).  This module measures that
share geometrically, with no closed form: it splits the circle at every angle
where it crosses one of the four lines bounding the rectangle, tests the
midpoint of every piece for being inside the (closed) rectangle, and adds up
the inside pieces.  It is a different route from the arc-subtraction formula
in ``oracle.c`` and serves to pin it.

``omega_arc``       FP64 version.
``omega_arc_mp``    the same construction in mpmath at ``dps`` digits.
``omega_sampled``   share of N equally spaced points of the circle inside the
                    rectangle (error below (number of crossings)/N).
"""
import math

import mpmath


def _split_angles(px, py, r, rect, acos, asin, pi):
    x0, y0, x1, y1 = rect
    angs = [0 * pi, 2 * pi]
    for c in (x0, x1):          # vertical sides: cos(theta) = (c - px)/r
        a = (c - px) / r
        if -1 < a < 1:
            th = acos(a)
            angs += [th, 2 * pi - th]
    for c in (y0, y1):          # horizontal sides: sin(theta) = (c - py)/r
        b = (c - py) / r
        if -1 < b < 1:
            th = asin(b)
            angs += [th % (2 * pi), pi - th]
    return sorted(angs)


def _inside(x, y, rect):
    x0, y0, x1, y1 = rect
    return x0 <= x <= x1 and y0 <= y <= y1


def omega_arc(px, py, r, rect):
    """Share of the circle (centre (px, py), radius r) inside ``rect`` = (x0, y0, x1, y1)."""
    if r <= 0:
        return 1.0
    px, py, r = float(px), float(py), float(r)
    rect = tuple(float(v) for v in rect)
    angs = _split_angles(px, py, r, rect, math.acos, math.asin, math.pi)
    inside = 0.0
    for a, b in zip(angs[:-1], angs[1:]):
        if b <= a:
            continue
        m = 0.5 * (a + b)
        if _inside(px + r * math.cos(m), py + r * math.sin(m), rect):
            inside += b - a
    return inside / (2.0 * math.pi)


def omega_arc_mp(px, py, r2, rect, dps=50):
    """Arc-union share in mpmath; ``r2`` is the (integer) squared radius."""
    with mpmath.workdps(dps):
        if r2 <= 0:
            return mpmath.mpf(1)
        px, py = mpmath.mpf(px), mpmath.mpf(py)
        r = mpmath.sqrt(mpmath.mpf(r2))
        rect_m = tuple(mpmath.mpf(v) for v in rect)
        angs = _split_angles(px, py, r, rect_m, mpmath.acos, mpmath.asin, mpmath.pi)
        inside = mpmath.mpf(0)
        for a, b in zip(angs[:-1], angs[1:]):
            if b <= a:
                continue
            m = (a + b) / 2
            if _inside(px + r * mpmath.cos(m), py + r * mpmath.sin(m), rect_m):
                inside += b - a
        return inside / (2 * mpmath.pi)


def omega_sampled(px, py, r, rect, n=1 << 20):
    """Share of n equally spaced circle points (half-step offset) inside ``rect``."""
    import numpy as np
    th = (np.arange(n, dtype=np.float64) + 0.5) * (2.0 * np.pi / n)
    x = px + r * np.cos(th)
    y = py + r * np.sin(th)
    x0, y0, x1, y1 = rect
    ok = (x >= x0) & (x <= x1) & (y >= y0) & (y <= y1)
    return float(ok.mean())
