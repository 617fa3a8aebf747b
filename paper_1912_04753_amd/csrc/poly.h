// Polygon study areas on the device: strict containment (ingest and CSR
// rejection), a lower bound of the distance to the boundary (the interior fast
// path of the pair kernel), and the share of a circle inside the polygon (the
// isotropic weight of Sec. 3 for a general study area).
//
// Vertices are window-relative int32 (coordinates below 2^24), so every vector
// product below is an integer below 2^52, exact in FP64, and the circle-edge
// discriminant is exact in 128-bit integers where its sign is in doubt.
// Edges are (V[k], V[k+1 mod n]), one int4 {a, b} each.  Each xy-cell of the
// grid lists the edges within s_max of the cell ({count, index...}, kNearMax +
// 1 u16 words; count kNearAll = every edge): a circle of radius <= s_max
// centred in the cell meets no other edge.  Each horizontal band of the window
// lists the edges whose y-range meets it (containment), and each sorted point
// record has a row of distance ranges to its cell's edges (poly_row).
#pragma once
#include "ripk_internal.h"

namespace ripk {

// Strictly inside: crossing number along +x with the half-open rule; a point
// on an edge is not inside.  Only the edges of the point's horizontal band can
// straddle its y or hold it.  The products are integers below 2^49, exact in
// FP64.
__device__ __forceinline__ bool poly_inside(const Geom &g, int px, int py) {
  const uint32_t b = (uint32_t)py >> g.band_shift;
  const uint32_t i1 = g.band_off[b + 1];
  bool in = false;
  for (uint32_t i = g.band_off[b]; i < i1; ++i) {
    const int4 e = g.poly[g.band_idx[i]];  // a = (e.x, e.y), b = (e.z, e.w)
    const double ex = (double)(e.z - e.x), ey = (double)(e.w - e.y);
    const double qx = (double)(px - e.x), qy = (double)(py - e.y);
    const double lhs = qx * ey, num = qy * ex;
    if (lhs == num && px >= min(e.x, e.z) && px <= max(e.x, e.z) && py >= min(e.y, e.w) &&
        py <= max(e.y, e.w))
      return false;
    // px left of the edge's crossing with the line y = py
    if (((e.y > py) != (e.w > py)) && (ey > 0.0 ? lhs < num : lhs > num)) in = !in;
  }
  return in;
}

// the xy-cell of a window-relative point, and the list of edges near it
__device__ __forceinline__ uint32_t poly_cell(const Geom &g, int px, int py) {
  const uint32_t cx = min((uint32_t)px / (uint32_t)g.cell_s, (uint32_t)g.nx - 1u);
  const uint32_t cy = min((uint32_t)py / (uint32_t)g.cell_s, (uint32_t)g.ny - 1u);
  return cy * (uint32_t)g.nx + cx;
}

__device__ __forceinline__ const uint16_t *poly_list(const Geom &g, int px, int py) {
  return g.near + (size_t)poly_cell(g, px, py) * (kNearMax + 1);
}

template <typename F>
__device__ __forceinline__ void poly_for_near(const Geom &g, int px, int py, F f) {
  const uint16_t *lst = poly_list(g, px, py);
  const uint32_t cnt = lst[0];
  if (cnt == kNearAll) {
    for (int k = 0; k < g.poly_n; ++k) f(k);
  } else {
    for (uint32_t i = 0; i < cnt; ++i) f((int)lst[1 + i]);
  }
}

// An integer e with e^2 no larger than the squared distance from the point to
// the boundary, capped at `cap` (edges beyond the cell's list are farther than
// s_max >= cap).  The FP64 distance is rounded down with a margin well above
// its error, so a pair with d2 <= e^2 has its whole circle inside.
__device__ __forceinline__ int32_t poly_edist(const Geom &g, int px, int py, int32_t cap) {
  double best = (double)cap * (double)cap;
  const int4 *__restrict__ E = g.poly;
  poly_for_near(g, px, py, [&](int k) {
    const int4 e = E[k];
    const double ex = (double)e.z - e.x, ey = (double)e.w - e.y;
    const double qx = (double)px - e.x, qy = (double)py - e.y;
    const double ee = ex * ex + ey * ey;
    const double s = fmin(fmax(ee > 0.0 ? (qx * ex + qy * ey) / ee : 0.0, 0.0), 1.0);
    const double dx = qx - s * ex, dy = qy - s * ey;
    best = fmin(best, dx * dx + dy * dy);
  });
  if (best >= (double)cap * (double)cap) return cap;
  return (int32_t)fmax(floor(sqrt(best * (1.0 - 1e-12))) - 1.0, 0.0);
}

// The row of a point for the weight: a 4-word head holding its xy-cell and the
// length of that cell's list, then from word 4, for each edge of the list, the
// range [lo, hi] of distances from the point to the edge's points, in units of
// 2^-row_shift metres as 16-bit integers (lo | hi << 16; (s_max + 2)
// 2^row_shift < 2^16), lo rounded down and hi up by a unit beyond the FP64
// error: a circle about the point meets the edge only if lo <= radius <= hi.
// Entries up to the next multiple of 4 hold an empty range (lo > hi).  Cells
// with more than kRowEdges edges listed, or that scan every edge, keep only the
// head.
__device__ __forceinline__ void poly_row(const Geom &g, int px, int py, uint32_t *__restrict__ row) {
  const uint32_t cell = poly_cell(g, px, py);
  const uint16_t *lst = g.near + (size_t)cell * (kNearMax + 1);
  const uint32_t cnt = lst[0];
  row[0] = cell;
  row[1] = cnt;
  if (cnt > (uint32_t)kRowEdges) return;  // (kNearAll included)
  for (uint32_t i = cnt; i < ((cnt + 3u) & ~3u); ++i) row[4 + i] = 0xFFFFu;
  const double u = ldexp(1.0, g.row_shift);
  for (uint32_t i = 0; i < cnt; ++i) {
    const int4 e = g.poly[lst[1 + i]];
    const double ax = (double)(e.x - px), ay = (double)(e.y - py);
    const double bx = (double)(e.z - px), by = (double)(e.w - py);
    const double ex = bx - ax, ey = by - ay;
    const double ee = ex * ex + ey * ey;
    const double s = fmin(fmax(ee > 0.0 ? -(ax * ex + ay * ey) / ee : 0.0, 0.0), 1.0);
    const double dx = ax + s * ex, dy = ay + s * ey;
    const double lo = fmax(floor(sqrt(dx * dx + dy * dy) * u * (1.0 - 1e-12)) - 1.0, 0.0);
    const double hi = ceil(sqrt(fmax(ax * ax + ay * ay, bx * bx + by * by)) * u * (1.0 + 1e-12)) + 1.0;
    row[4 + i] = (uint32_t)fmin(lo, 65535.0) | ((uint32_t)fmin(hi, 65535.0) << 16);
  }
}

// a / b from the hardware reciprocal, one Newton step on it and one on the
// quotient (equal to the IEEE quotient on 2^20 random pairs with exponents in
// +-60): a few instructions instead of the IEEE division sequence
__device__ __forceinline__ double poly_div(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// Angle of (x, y) in [0, 2 pi), FP64, within a few ulp (depends only on the
// direction of (x, y)): octant reduction to z = min/max in [0, 1], then
// atan z = pi/6 + atan((sqrt(3) z - 1)/(z + sqrt(3))) for z > tan(pi/12) (one
// quotient of min and max either way), and the Taylor series of atan to z^25
// on [0, tan(pi/12)] (remainder below 2e-16 there).  Light on registers,
// unlike a general-purpose atan2.
__device__ __forceinline__ double poly_angle(double x, double y) {
  const double ax = fabs(x), ay = fabs(y);
  const double lo = fmin(ax, ay), hi = fmax(ax, ay);
  if (hi == 0.0) return 0.0;
  const bool red = lo > 0.26794919243112270 * hi;  // tan(pi/12)
  const double z = red ? poly_div(lo * 1.7320508075688772 - hi, lo + hi * 1.7320508075688772)
                       : poly_div(lo, hi);
  const double base = red ? 0.52359877559829887 : 0.0;  // pi/6
  const double w = z * z;
  double p = 1.0 / 25.0;
  p = fma(p, w, -1.0 / 23.0);
  p = fma(p, w, 1.0 / 21.0);
  p = fma(p, w, -1.0 / 19.0);
  p = fma(p, w, 1.0 / 17.0);
  p = fma(p, w, -1.0 / 15.0);
  p = fma(p, w, 1.0 / 13.0);
  p = fma(p, w, -1.0 / 11.0);
  p = fma(p, w, 1.0 / 9.0);
  p = fma(p, w, -1.0 / 7.0);
  p = fma(p, w, 1.0 / 5.0);
  p = fma(p, w, -1.0 / 3.0);
  p = fma(p, w, 1.0);
  double a = fma(z, p, base);
  if (ay > ax) a = 1.5707963267948966 - a;
  if (x < 0.0) a = 3.1415926535897932 - a;
  if (y < 0.0) a = 6.2831853071795865 - a;
  return a;
}

// Square root of x > 0 to a few ulp (4e-15 relative measured over 1 .. 2^104):
// the hardware reciprocal square root and one Newton step.  It only places a
// crossing's direction; which edges cross is decided on integers.
__device__ __forceinline__ double poly_sqrt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double s = x * r;
  return fma(fma(-s, s, x), 0.5 * r, s);
}

// 1/omega, omega the share of the circle centred on the window-relative point
// (px, py), strictly inside the polygon, with radius sqrt(d2) inside the
// polygon; rec is the point's sorted record (its row, see poly_row).  The
// circle passes through the pair's other point, also strictly inside, so a
// circle that crosses the boundary nowhere lies inside (1/omega = 1).
//
// Walking the circle counter-clockwise, the inside length is the sum of the
// exit angles minus the sum of the entry angles, plus 2 pi when the walk
// starts inside (angles in [0, 2 pi)); the sum alone is then negative, so its
// sign decides, and with any crossing the length is that sum modulo 2 pi.
// The crossings enter as a product of their direction vectors (conjugated for
// subtracted angles) kept at unit scale by powers of two, whose angle is taken
// once at the end: the lanes of a wave hold different circles, so some lane
// crosses at almost every edge and a per-crossing arctangent would cost every
// lane that much.  Which edges the circle crosses, and where, is decided on
// exact integers: with A = a - c, E = b - a, the crossing parameters solve
// |A + s E|^2 = d2, i.e. ee s^2 + 2 ae s + (aa - d2) = 0, and the root
// conditions 0 < s < 1 reduce to signs of ae, ae + ee and to comparisons of
// aa = |a - c|^2 and bb = |b - c|^2 with d2.  The larger root has E.(X - c) > 0:
// an entry when the polygon is counter-clockwise (its inside on the left), an
// exit otherwise.  A vertex on the circle counts half for each of its two
// edges, so a circle through a vertex crossing the boundary counts once and one
// only touching it cancels (an edge tangent at the vertex counts as leaving the
// disk); the two halves are added at the edge the vertex starts, so a vertex
// is one crossing or none.  An edge tangent inside its span (zero
// discriminant) counts nothing.  Only the angles are floating point (FP64);
// the integer quantities are carried in FP64 registers, where they are exact.
//
// The edges go in chunks of 32 list entries.  A first pass keeps, in a bit
// mask, the entries whose distance range from the point holds the radius
// (two integer compares per entry on the point's row); the exact work above
// then runs only for those.  The lanes of a wave hold different circles, so a
// single pass paid for the crossing work at almost every entry, while a
// circle meets few of them (two, near a smooth boundary).  Cells that scan
// every edge (more than 32 near it), or that list more than kRowEdges, take the
// first pass on exact integers.
__device__ __forceinline__ double poly_inv_omega(const Geom &g, int px, int py, uint64_t d2u,
                                                 uint32_t rec) {
  if (d2u == 0) return 1.0;
  const int4 *__restrict__ E = g.poly;
  const int nv = g.poly_n;
  // every quantity below is an integer of at most 52 bits, exact in FP64
  const double d2 = (double)d2u;
  const double sg = (double)g.poly_sign;
  double Px = 1.0, Py = 0.0;   // product of the crossings' directions
  bool crossed = false;
  // P <- P (x + i y), rescaled so that its larger component lies in [1, 2)
  auto turn = [&](double x, double y) {
    const double nx = fma(Px, x, -Py * y), ny = fma(Px, y, Py * x);
    const int e = ilogb(fmax(fabs(nx), fabs(ny)));
    Px = ldexp(nx, -e);
    Py = ldexp(ny, -e);
    crossed = true;
  };
  const uint32_t *__restrict__ row = g.prow + (size_t)rec * kRowWords;
  const uint2 head = *(const uint2 *)row;  // the cell and its list length, one load
  const uint16_t *__restrict__ lst = g.near + (size_t)head.x * (kNearMax + 1);
  const bool all = head.y == kNearAll;
  const uint32_t len = all ? (uint32_t)nv : head.y;
  const bool rows = len <= (uint32_t)kRowEdges && !all;
  // the squared radius in the row's units: d2 <= s_max^2, so below 2^32
  const uint32_t d2s = (uint32_t)d2u << (2 * g.row_shift);
  for (uint32_t base = 0; base < len; base += 32) {
    const uint32_t m = min(len - base, 32u);
    uint32_t keep = 0;
    if (rows) {
      // four entries per load, the next load issued before the current
      // entries are tested
      const uint4 *__restrict__ rw = (const uint4 *)(row + 4);
      const uint32_t nq = (m + 3u) >> 2;
      uint4 w = rw[0];
      for (uint32_t q = 0; q < nq; ++q) {
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        if (q + 1u < nq) w = rw[q + 1u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t lo = ws[u] & 0xFFFFu, hi = ws[u] >> 16;
          const bool k = __umul24(lo, lo) <= d2s && d2s <= __umul24(hi, hi);
          keep |= (uint32_t)k << (4u * q + (uint32_t)u);
        }
      }
    } else {
      for (uint32_t i = 0; i < m; ++i) {
        const int4 e = E[all ? base + i : (uint32_t)lst[1 + i]];
        const double ax = (double)(e.x - px), ay = (double)(e.y - py);
        const double bx = (double)(e.z - px), by = (double)(e.w - py);
        const double ex = bx - ax, ey = by - ay;
        const double ee = fma(ex, ex, ey * ey), ae = fma(ax, ex, ay * ey);
        const double aa = fma(ax, ax, ay * ay), bb = fma(bx, bx, by * by);
        // a root strictly inside the edge, or vertex a on the circle: from
        // inside only if b is outside; from outside to inside always; with
        // both ends on or outside, only if the line's closest point lies
        // strictly inside the edge and the discriminant is not negative
        // beyond its rounding bound (the test below)
        const double t1 = ae * ae, t2 = ee * (aa - d2);
        const bool k = aa == d2 || (aa < d2 && bb > d2) || (aa > d2 && bb < d2) ||
                       (aa > d2 && ae < 0.0 && ae + ee > 0.0 &&
                        (bb == d2 || t1 - t2 >= -0x1p-50 * (t1 + t2)));
        keep |= (uint32_t)k << i;
      }
    }
    // the next kept edge is loaded while the current one is worked
    auto edge_at = [&](uint32_t i) { return all ? (int)(base + i) : (int)lst[1 + i]; };
    int kn = keep ? edge_at((uint32_t)__builtin_ctz(keep)) : 0;
    int4 en = keep ? E[kn] : make_int4(0, 0, 0, 0);
    while (keep) {
      keep &= keep - 1u;
      const int kk = kn;
      const int4 e = en;
      if (keep) {
        kn = edge_at((uint32_t)__builtin_ctz(keep));
        en = E[kn];
      }
      const double ax = (double)(e.x - px), ay = (double)(e.y - py);
      const double bx = (double)(e.z - px), by = (double)(e.w - py);
      const double ex = bx - ax, ey = by - ay;
      const double ee = fma(ex, ex, ey * ey), ae = fma(ax, ex, ay * ey);
      const double aa = fma(ax, ax, ay * ay), bb = fma(bx, bx, by * by);
      if (ee == 0.0) continue;
      // vertex a on the circle: its halves from this edge (a-end) and from the
      // previous one (b-end), each signed by the side of the circle the edge
      // lies on next to the vertex (this edge: E.A > 0 lies outside beyond a;
      // the previous edge, F = a - prev: F.A > 0 lies inside before a), an
      // edge tangent there (zero product) lying outside the disk; +-1/2 each,
      // exact integer products
      if (aa == d2) {
        const int4 pe = E[kk == 0 ? nv - 1 : kk - 1];
        const double fx = (double)(e.x - pe.x), fy = (double)(e.y - pe.y);
        const int h = (ae >= 0.0 ? -1 : 1) + (fma(fx, ax, fy * ay) > 0.0 ? -1 : 1);
        if (h != 0) turn(ax, (h > 0 ? sg : -sg) * ay);
      }
      // discriminant ae^2 - ee (aa - d2): its sign from FP64 when clear of the
      // rounding bound, else from exact 128-bit integers
      const double t1 = ae * ae, t2 = ee * (aa - d2);
      double disc = t1 - t2;
      if (fabs(disc) <= 0x1p-50 * (fabs(t1) + fabs(t2))) {
        const long long iae = (long long)ae, iee = (long long)ee, iad = (long long)(aa - d2);
        const __int128 q = (__int128)iae * iae - (__int128)iee * iad;
        disc = q > 0 ? (double)q : 0.0;
      }
      if (disc > 0.0) {
        // the crossing A + s E with s = (-ae -+ sq)/ee, scaled by ee > 0 (the
        // angle depends on the direction only).  Smaller root strictly inside
        // the edge: an exit (counter-clockwise), its angle added with the
        // orientation's sign (direction (x, sg y)); larger root strictly
        // inside: an entry, its angle subtracted.
        const bool out = ae < 0.0 && aa > d2 && (ae + ee > 0.0 || bb < d2);
        const bool in = (ae < 0.0 || aa < d2) && ae + ee > 0.0 && bb > d2;
        if (out || in) {
          const double sq = poly_sqrt(disc);
          const double s1 = out ? -ae - sq : -ae + sq;
          turn(fma(s1, ex, ee * ax), (out ? sg : -sg) * fma(s1, ey, ee * ay));
          if (out && in) {
            const double s2 = -ae + sq;
            turn(fma(s2, ex, ee * ax), -sg * fma(s2, ey, ee * ay));
          }
        }
      }
    }
  }
  if (!crossed) return 1.0;
  return poly_div(6.283185307179586476925, poly_angle(Px, Py));
}

}  // namespace ripk
