// Polygon study areas on the device: strict containment (ingest and CSR
// rejection), a lower bound of the distance to the boundary (the interior fast
// path of the pair kernel), and the share of a circle inside the polygon (the
// isotropic weight of Sec. 3 for a general study area).
//
// Vertices are window-relative int32 (coordinates below 2^24), so every vector
// product below is exact in 64 bits and the circle-edge discriminant in 128.
// Edges are (V[k], V[k+1 mod n]).  Each xy-cell of the grid lists the edges
// within s_max of the cell ({count, index...}, kNearMax + 1 u16 words; count
// kNearAll = every edge): a circle of radius <= s_max centred in the cell meets
// no other edge.
#pragma once
#include "ripk_internal.h"

namespace ripk {

// Strictly inside: crossing number along +x with the half-open rule, exact
// integers; a point on an edge is not inside.
__device__ __forceinline__ bool poly_inside(const int2 *__restrict__ V, int nv, int px, int py) {
  bool in = false;
  int2 a = V[nv - 1];
  for (int k = 0; k < nv; ++k) {
    const int2 b = V[k];
    const long long ex = (long long)b.x - a.x, ey = (long long)b.y - a.y;
    const long long qx = (long long)px - a.x, qy = (long long)py - a.y;
    if (ex * qy == ey * qx && px >= min(a.x, b.x) && px <= max(a.x, b.x) &&
        py >= min(a.y, b.y) && py <= max(a.y, b.y))
      return false;
    if ((a.y > py) != (b.y > py)) {
      // px left of the edge's crossing with the line y = py
      const long long num = qy * ex, lhs = qx * ey;
      if (ey > 0 ? lhs < num : lhs > num) in = !in;
    }
    a = b;
  }
  return in;
}

// the list of edges near the xy-cell of a window-relative point
__device__ __forceinline__ const uint16_t *poly_list(const Geom &g, int px, int py) {
  const uint32_t cx = min((uint32_t)px / (uint32_t)g.cell_s, (uint32_t)g.nx - 1u);
  const uint32_t cy = min((uint32_t)py / (uint32_t)g.cell_s, (uint32_t)g.ny - 1u);
  return g.near + (size_t)(cy * (uint32_t)g.nx + cx) * (kNearMax + 1);
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
  const int2 *__restrict__ V = g.poly;
  const int nv = g.poly_n;
  poly_for_near(g, px, py, [&](int k) {
    const int2 a = V[k], b = V[k + 1 == nv ? 0 : k + 1];
    const double ex = (double)b.x - a.x, ey = (double)b.y - a.y;
    const double qx = (double)px - a.x, qy = (double)py - a.y;
    const double ee = ex * ex + ey * ey;
    const double s = fmin(fmax(ee > 0.0 ? (qx * ex + qy * ey) / ee : 0.0, 0.0), 1.0);
    const double dx = qx - s * ex, dy = qy - s * ey;
    best = fmin(best, dx * dx + dy * dy);
  });
  if (best >= (double)cap * (double)cap) return cap;
  return (int32_t)fmax(floor(sqrt(best * (1.0 - 1e-12))) - 1.0, 0.0);
}

__device__ __forceinline__ double poly_angle(double x, double y) {
  const double a = atan2(y, x);
  return a < 0.0 ? a + 6.283185307179586476925 : a;
}

// Share of the circle centred on the window-relative point (px, py), strictly
// inside the polygon, with radius sqrt(d2) inside the polygon.
//
// Walking the circle counter-clockwise, the inside length is the sum of the
// exit angles minus the sum of the entry angles, plus 2 pi when the walk
// starts inside (angles in [0, 2 pi)); the sum alone is then negative, so its
// sign decides.  Which edges the circle crosses, and where, is decided on
// exact integers: with A = a - c, E = b - a, the crossing parameters solve
// |A + s E|^2 = d2, i.e. ee s^2 + 2 ae s + (aa - d2) = 0, and the root
// conditions 0 < s < 1 reduce to signs of ae, ae + ee and to comparisons of
// aa = |a - c|^2 and bb = |b - c|^2 with d2.  The larger root has E.(X - c) > 0:
// an entry when the polygon is counter-clockwise (its inside on the left), an
// exit otherwise.  A vertex on the circle counts half for each of its two
// edges, so a circle through a vertex crossing the boundary counts once and one
// only touching it cancels (an edge tangent at the vertex counts as leaving the
// disk); an edge tangent inside its span (zero discriminant) counts nothing.
// With no net crossing the circle is wholly inside unless the polygon lies
// within it (some vertex strictly inside the disk).  Only the angles are
// floating point (FP64).
__device__ __forceinline__ double poly_omega(const Geom &g, int px, int py, uint64_t d2u) {
  if (d2u == 0) return 1.0;
  const int2 *__restrict__ V = g.poly;
  const int nv = g.poly_n;
  const long long d2 = (long long)d2u;
  const double sg = (double)g.poly_sign;
  double S = 0.0;
  bool vin = false;
  poly_for_near(g, px, py, [&](int k) {
    const int2 a = V[k], b = V[k + 1 == nv ? 0 : k + 1];
    const long long Ax = (long long)a.x - px, Ay = (long long)a.y - py;
    const long long Bx = (long long)b.x - px, By = (long long)b.y - py;
    const long long Ex = Bx - Ax, Ey = By - Ay;
    const long long ee = Ex * Ex + Ey * Ey, ae = Ax * Ex + Ay * Ey;
    const long long aa = Ax * Ax + Ay * Ay, bb = Bx * Bx + By * By;
    vin = vin || aa < d2 || bb < d2;
    if (ee == 0) return;
    // a vertex on the circle: half a crossing, signed by the side of the
    // circle the edge lies on next to the vertex (E.(vertex - c) > 0: outside
    // beyond a, inside before b); an edge tangent there (zero product) lies
    // outside the disk
    if (aa == d2) S += (ae >= 0 ? -0.5 : 0.5) * sg * poly_angle((double)Ax, (double)Ay);
    if (bb == d2) S += (ae + ee > 0 ? -0.5 : 0.5) * sg * poly_angle((double)Bx, (double)By);
    const __int128 disc = (__int128)ae * ae - (__int128)ee * (aa - d2);
    if (disc > 0) {
      const double sq = sqrt((double)disc);
      const double dae = (double)ae, dee = (double)ee;
      // smaller root strictly inside the edge: an exit (counter-clockwise)
      if (ae < 0 && aa > d2 && (ae + ee > 0 || bb < d2)) {
        const double s = (-dae - sq) / dee;
        S += sg * poly_angle((double)Ax + s * (double)Ex, (double)Ay + s * (double)Ey);
      }
      // larger root strictly inside the edge: an entry
      if ((ae < 0 || aa < d2) && ae + ee > 0 && bb > d2) {
        const double s = (-dae + sq) / dee;
        S -= sg * poly_angle((double)Ax + s * (double)Ex, (double)Ay + s * (double)Ey);
      }
    }
  });
  const double two_pi = 6.283185307179586476925;
  const double L = S > 0.0 ? S : (S < 0.0 ? S + two_pi : (vin ? 0.0 : two_pi));
  return L / two_pi;
}

}  // namespace ripk
