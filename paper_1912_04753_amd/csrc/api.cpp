// Host runtime of the ripk C ABI: plan validation and geometry, device buffer
// pool, the launch sequence of one evaluation, and the exported entry points.
//
// One evaluation of S point sets of n points each (S = 1 for an observed set,
// S = m for Monte Carlo simulations, Sec. 3, S = m + 1 for an observed set and
// its simulations together) runs, on the caller's stream:
//   keys (or on-device CSR / resampling draw) -> radix sort by (set, cell,
//   halo) or, for two-type sets, (set, type, cell) -> cell bounds -> sorted
//   point records -> work items -> pair kernel (persistent) -> per-set prefix
//   sums, K (Eq. 2) and L (Eq. 4) -> envelopes -> copies out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ripk.h"
#include "ripk_internal.h"

using namespace ripk;

namespace {

// detail of the calling thread's last error (a fixed buffer: recording an
// error allocates nothing)
thread_local char g_err[512];

ripk_status fail(ripk_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ripk_status fail(ripk_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(RIPK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

constexpr int64_t kI32Min = -2147483648LL, kI32Max = 2147483647LL;

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((1ull << b) < v) ++b;
  return b;
}

struct Layout {
  ripk_plan_info info;
  Geom g;
  int32_t clamp_e;
  Caps caps;
  double area = 0;          // study area A of Eq. 2 (rectangle or polygon)
  std::vector<int2> V;      // polygon vertices, window-relative (empty: rectangle)
};

int64_t orient(int2 p, int2 q, int2 r) {
  const int64_t v = (int64_t)(q.x - p.x) * (r.y - p.y) - (int64_t)(q.y - p.y) * (r.x - p.x);
  return v > 0 ? 1 : (v < 0 ? -1 : 0);
}

bool on_segment(int2 p, int2 q, int2 r) {  // r on the closed segment pq (collinear given)
  return r.x >= std::min(p.x, q.x) && r.x <= std::max(p.x, q.x) && r.y >= std::min(p.y, q.y) &&
         r.y <= std::max(p.y, q.y);
}

bool segments_meet(int2 a, int2 b, int2 c, int2 d) {
  const int64_t o1 = orient(a, b, c), o2 = orient(a, b, d), o3 = orient(c, d, a),
                o4 = orient(c, d, b);
  if (o1 * o2 < 0 && o3 * o4 < 0) return true;
  return (o1 == 0 && on_segment(a, b, c)) || (o2 == 0 && on_segment(a, b, d)) ||
         (o3 == 0 && on_segment(c, d, a)) || (o4 == 0 && on_segment(c, d, b));
}

// Polygon of a descriptor: window-relative vertices, exact doubled signed
// area; checks that it is simple and inside the rectangle.
ripk_status read_polygon(const ripk_plan_desc *d, std::vector<int2> *V, int64_t *area2) {
  const int n = d->poly_n;
  if (n < 3 || n > kMaxPoly || !d->poly)
    return fail(RIPK_EINVAL, "a polygon needs 3 to %d vertices and a vertex array", kMaxPoly);
  V->resize((size_t)n);
  for (int k = 0; k < n; ++k) {
    const int64_t x = d->poly[2 * k], y = d->poly[2 * k + 1];
    if (x < d->x0 || x > d->x1 || y < d->y0 || y > d->y1)
      return fail(RIPK_EINVAL, "polygon vertex %d lies outside the rectangle", k);
    (*V)[(size_t)k] = make_int2((int)(x - d->x0), (int)(y - d->y0));
  }
  int64_t a2 = 0;
  for (int k = 0; k < n; ++k) {
    const int2 a = (*V)[(size_t)k], b = (*V)[(size_t)((k + 1) % n)];
    if (a.x == b.x && a.y == b.y) return fail(RIPK_EINVAL, "polygon edge %d has zero length", k);
    a2 += (int64_t)a.x * b.y - (int64_t)b.x * a.y;
  }
  // simple: edges that do not share a vertex do not meet; edges that do share
  // one do not fold back onto each other
  for (int i = 0; i < n; ++i) {
    const int2 a = (*V)[(size_t)i], b = (*V)[(size_t)((i + 1) % n)];
    for (int j = i + 1; j < n; ++j) {
      const int2 c = (*V)[(size_t)j], e = (*V)[(size_t)((j + 1) % n)];
      const bool next = j == i + 1, prev = (j + 1) % n == i;
      if (next || prev) {
        // shared vertex s, other ends p (of edge i) and q (of edge j)
        const int2 sv = next ? b : a, pv = next ? a : b, qv = next ? e : c;
        if (orient(sv, pv, qv) == 0 &&
            (int64_t)(pv.x - sv.x) * (qv.x - sv.x) + (int64_t)(pv.y - sv.y) * (qv.y - sv.y) > 0)
          return fail(RIPK_EINVAL, "polygon edges %d and %d overlap", i, j);
        continue;
      }
      if (segments_meet(a, b, c, e))
        return fail(RIPK_EINVAL, "polygon edges %d and %d intersect (not a simple polygon)", i, j);
    }
  }
  *area2 = a2;
  return RIPK_OK;
}

// squared distance from a point to a closed segment (FP64)
double seg_point_d2(double ax, double ay, double bx, double by, double px, double py) {
  const double ex = bx - ax, ey = by - ay, ee = ex * ex + ey * ey;
  const double s = ee > 0 ? std::min(std::max(((px - ax) * ex + (py - ay) * ey) / ee, 0.0), 1.0) : 0.0;
  const double dx = px - ax - s * ex, dy = py - ay - s * ey;
  return dx * dx + dy * dy;
}

// Edges by horizontal band of height 2^band_shift (the containment test's
// lists): band b holds every edge whose closed y-range meets the band.
void build_bands(const Layout &L, std::vector<uint32_t> *off, std::vector<uint16_t> *idx) {
  const Geom &g = L.g;
  const int nv = (int)L.V.size();
  const uint32_t nb = ((uint32_t)(g.y1 - g.y0) >> g.band_shift) + 1u;
  off->assign((size_t)nb + 1, 0);
  auto span = [&](int k, uint32_t *b0, uint32_t *b1) {
    const int2 a = L.V[(size_t)k], b = L.V[(size_t)((k + 1) % nv)];
    *b0 = (uint32_t)std::min(a.y, b.y) >> g.band_shift;
    *b1 = (uint32_t)std::max(a.y, b.y) >> g.band_shift;
  };
  for (int k = 0; k < nv; ++k) {
    uint32_t b0, b1;
    span(k, &b0, &b1);
    for (uint32_t b = b0; b <= b1; ++b) ++(*off)[b + 1];
  }
  for (uint32_t b = 0; b < nb; ++b) (*off)[b + 1] += (*off)[b];
  idx->assign((*off)[nb], 0);
  std::vector<uint32_t> fill(off->begin(), off->end() - 1);
  for (int k = 0; k < nv; ++k) {
    uint32_t b0, b1;
    span(k, &b0, &b1);
    for (uint32_t b = b0; b <= b1; ++b) (*idx)[fill[b]++] = (uint16_t)k;
  }
}

// Per xy-cell lists of the edges within s_max (plus a margin) of the cell's
// rectangle (the last cell of an axis reaches the window's side).
void build_near(const Layout &L, int64_t s_max, std::vector<uint16_t> *out) {
  const Geom &g = L.g;
  const int nv = (int)L.V.size();
  const int64_t W = (int64_t)g.x1 - g.x0, H = (int64_t)g.y1 - g.y0, cs = g.cell_s;
  out->assign((size_t)g.nx * g.ny * (kNearMax + 1), 0);
  const double reach = (double)s_max + 2.0;
  for (int k = 0; k < nv; ++k) {
    const int2 a = L.V[(size_t)k], b = L.V[(size_t)((k + 1) % nv)];
    const double lox = std::min(a.x, b.x) - reach, hix = std::max(a.x, b.x) + reach;
    const double loy = std::min(a.y, b.y) - reach, hiy = std::max(a.y, b.y) + reach;
    const int cx0 = (int)std::max<int64_t>(0, (int64_t)std::floor(lox / cs));
    const int cx1 = (int)std::min<int64_t>(g.nx - 1, (int64_t)std::floor(hix / cs));
    const int cy0 = (int)std::max<int64_t>(0, (int64_t)std::floor(loy / cs));
    const int cy1 = (int)std::min<int64_t>(g.ny - 1, (int64_t)std::floor(hiy / cs));
    for (int cy = cy0; cy <= cy1; ++cy)
      for (int cx = cx0; cx <= cx1; ++cx) {
        const double x0 = (double)cx * cs, x1 = cx == g.nx - 1 ? (double)W : (double)(cx + 1) * cs;
        const double y0 = (double)cy * cs, y1 = cy == g.ny - 1 ? (double)H : (double)(cy + 1) * cs;
        // distance between the segment and the cell rectangle
        double d2;
        const bool a_in = a.x >= x0 && a.x <= x1 && a.y >= y0 && a.y <= y1;
        const bool b_in = b.x >= x0 && b.x <= x1 && b.y >= y0 && b.y <= y1;
        if (a_in || b_in) {
          d2 = 0.0;
        } else {
          auto pr = [&](double px, double py) {
            const double dx = std::max({x0 - px, 0.0, px - x1}), dy = std::max({y0 - py, 0.0, py - y1});
            return dx * dx + dy * dy;
          };
          d2 = std::min(pr(a.x, a.y), pr(b.x, b.y));
          const double cxs[4] = {x0, x1, x1, x0}, cys[4] = {y0, y0, y1, y1};
          for (int q = 0; q < 4; ++q) d2 = std::min(d2, seg_point_d2(a.x, a.y, b.x, b.y, cxs[q], cys[q]));
          // a segment crossing the rectangle with both ends outside: it meets
          // one of the rectangle's sides
          const int2 r0 = make_int2((int)x0, (int)y0), r1 = make_int2((int)x1, (int)y0),
                     r2 = make_int2((int)x1, (int)y1), r3 = make_int2((int)x0, (int)y1);
          if (segments_meet(a, b, r0, r1) || segments_meet(a, b, r1, r2) ||
              segments_meet(a, b, r2, r3) || segments_meet(a, b, r3, r0))
            d2 = 0.0;
        }
        if (d2 > reach * reach) continue;
        uint16_t *lst = out->data() + ((size_t)cy * g.nx + cx) * (kNearMax + 1);
        if (lst[0] == kNearAll) continue;
        if (lst[0] == kNearMax) {
          lst[0] = kNearAll;
          continue;
        }
        lst[1 + lst[0]] = (uint16_t)k;
        ++lst[0];
      }
  }
}

// The longest list (kNearMax + 1 for "every edge") and the cells with a list.
void near_summary(const std::vector<uint16_t> &near, ripk_plan_info *info) {
  int mx = 0, cells = 0;
  for (size_t c = 0; c < near.size(); c += kNearMax + 1) {
    const int k = near[c] == kNearAll ? kNearMax + 1 : (int)near[c];
    mx = std::max(mx, k);
    cells += k > 0 ? 1 : 0;
  }
  info->near_edges_max = mx;
  info->near_cells = cells;
}

}  // namespace

namespace ripk {

Caps caps_for(int64_t S, int64_t n_max, int64_t n_cells, int64_t n_bins, int64_t V,
              int64_t NXY, int64_t R) {
  Caps c;
  c.V = V;
  c.NXY = NXY;
  c.R = R;
  c.S = S;
  c.N = S * n_max;
  c.SNC = S * n_cells;
  // room for items split kSplitMax ways when a launch holds few sets
  c.items = std::max<int64_t>(S, kSplitMax) * (n_max / kChunk + n_cells + kItemsPerGroup);
  c.SNB = S * n_bins;
  c.NB = n_bins;
  c.P = n_max;
  return c;
}

int64_t caps_bytes(const Caps &c) {
  int64_t bytes = 0;
  bytes += 3 * 4 * c.N;                       // x, y, t staging / simulated points
  bytes += 4 * 4 * c.N;                       // keys, vals (double buffered)
  bytes += (int64_t)radix_sort_temp_bytes((uint32_t)c.N, (uint32_t)c.S);
  bytes += 4 * (2 * c.SNC + 1);               // cell starts
  bytes += 16 * c.N;                          // sorted point records
  bytes += 4 * c.SNC * 2 + 4 * (c.S + 1) + (int64_t)scan_temp_bytes((uint32_t)c.SNC) + 256;
  bytes += 16 * c.items;                      // work items
  bytes += 8 * (1 + kBinWords) * c.SNB;       // bins
  bytes += 8 * 4 * c.SNB;                     // C, W, K, L
  bytes += 8 * 6 * c.NB + 8 * 2 * kMaxSteps;  // envelopes, L_obs, thresholds
  bytes += 8 * (kQueues + 1) * kQueueStride;   // scalars and work-queue blocks
  bytes += 8 * (kScalWords + kPackRows * c.NB);  // result staging
  bytes += 3 * 4 * c.P;                       // copy of the observed set (resampling)
  bytes += 16 * c.V + 2 * (kNearMax + 1) * c.NXY;  // polygon edges and per-cell edge lists
  if (c.V > 0) bytes += 4 * kRowWords * c.N;       // per-record edge distance ranges
  if (c.V > 0) bytes += 4 * (kBandsMax + 1) + 2 * c.V * kBandsMax;  // edges by band
  bytes += 16 * c.R;                          // intensities and their sorted reciprocals
  return bytes;
}

bool caps_fit(const Caps &have, const Caps &need) {
  return need.S <= have.S && need.N <= have.N && need.SNC <= have.SNC &&
         need.items <= have.items && need.SNB <= have.SNB && need.NB <= have.NB &&
         need.P <= have.P && need.V <= have.V && need.NXY <= have.NXY && need.R <= have.R;
}

Caps caps_max(const Caps &a, const Caps &b) {
  Caps c;
  c.S = std::max(a.S, b.S);
  c.N = std::max(a.N, b.N);
  c.SNC = std::max(a.SNC, b.SNC);
  c.items = std::max(a.items, b.items);
  c.SNB = std::max(a.SNB, b.SNB);
  c.NB = std::max(a.NB, b.NB);
  c.P = std::max(a.P, b.P);
  c.V = std::max(a.V, b.V);
  c.NXY = std::max(a.NXY, b.NXY);
  c.R = std::max(a.R, b.R);
  return c;
}

}  // namespace ripk

namespace {

// Validation and derived geometry; no device access.
ripk_status derive(const ripk_plan_desc *d, Layout *L) {
  if (!d || !L) return fail(RIPK_EINVAL, "null descriptor");
  *L = Layout{};  // every field zero, the polygon vertices released
  ripk_plan_info &I = L->info;
  const int64_t W = d->x1 - d->x0, H = d->y1 - d->y0, D = d->t1 - d->t0;
  if (d->x0 < kI32Min || d->x1 > kI32Max || d->y0 < kI32Min || d->y1 > kI32Max ||
      d->t0 < kI32Min || d->t1 > kI32Max)
    return fail(RIPK_EINVAL, "window must lie within int32");
  if (W < 1 || H < 1 || D < 1) return fail(RIPK_EINVAL, "empty window (x1<=x0, y1<=y0 or t1<=t0)");
  if (W >= (1LL << 24) || H >= (1LL << 24))
    return fail(RIPK_EINVAL, "window sides must be below 2^24 m");
  if (D >= (1LL << 31)) return fail(RIPK_EINVAL, "period must be below 2^31 s");
  if (d->n_s < 1 || d->n_s > kMaxSteps || d->n_t < 1 || d->n_t > kMaxSteps)
    return fail(RIPK_EINVAL, "n_s and n_t must be in [1, 64]");
  if (d->s_max < 1 || d->t_max < 1) return fail(RIPK_EINVAL, "s_max and t_max must be >= 1");
  if (d->s_max >= (1LL << 23)) return fail(RIPK_EINVAL, "s_max must be below 2^23");
  if (d->t_max >= (1LL << 30)) return fail(RIPK_EINVAL, "t_max must be below 2^30");
  if (d->edge & ~RIPK_EDGE_ISO) return fail(RIPK_EINVAL, "unknown edge-correction bits");
  if (d->reserved != 0) return fail(RIPK_EINVAL, "reserved descriptor field must be 0");
  int64_t area2 = 0;
  L->V.clear();
  if (d->poly_n != 0) {
    ripk_status ps = read_polygon(d, &L->V, &area2);
    if (ps != RIPK_OK) return ps;
    if (std::llabs(area2) * 512 < W * H)
      return fail(RIPK_EINVAL, "polygon area must be at least 1/1024 of the rectangle's");
  }
  if ((d->edge & RIPK_EDGE_SPATIAL_ISO) && d->poly_n == 0 && 2 * d->s_max > std::min(W, H))
    return fail(RIPK_EINVAL,
                "isotropic spatial correction needs 2*s_max <= min(width, height) "
                "(the weight would reach 0 beyond that)");
  if ((d->edge & RIPK_EDGE_TEMPORAL) && d->t_max > D)
    return fail(RIPK_EINVAL, "temporal correction needs t_max <= t1-t0");
  if (d->norm > RIPK_NORM_N2) return fail(RIPK_EINVAL, "unknown normalisation");
  if (d->flags & ~(RIPK_PLAN_ORDERED | RIPK_PLAN_TIMING | RIPK_PLAN_WIDE_COUNTS |
                   RIPK_PLAN_AUTOTUNE | RIPK_PLAN_GRAPH | RIPK_PLAN_CROSS | RIPK_PLAN_INHOM |
                   RIPK_PLAN_SPLIT_RUNS | RIPK_PLAN_COST_ORDER))
    return fail(RIPK_EINVAL, "unknown plan flags");
  if ((d->flags & RIPK_PLAN_INHOM) && ((d->flags & RIPK_PLAN_CROSS) || d->poly_n != 0))
    return fail(RIPK_EINVAL, "inhomogeneous K plans take one point type and the rectangle");
  // polygon weights and inhomogeneous weights are summed in wide fixed point,
  // whose LDS piece sums are bounded for sets below kWidePoints
  if (((d->poly_n != 0 && (d->edge & RIPK_EDGE_SPATIAL_ISO)) || (d->flags & RIPK_PLAN_INHOM)) &&
      d->n_max >= kWidePoints)
    return fail(RIPK_EINVAL,
                "polygon (with spatial correction) and inhomogeneous plans take n_max below 2^22");
  if (d->sim_method != RIPK_SIM_CSR && d->sim_method != RIPK_SIM_PERMUTE &&
      d->sim_method != RIPK_SIM_BOOTSTRAP)
    return fail(RIPK_EINVAL, "unknown simulation method");
  if (d->n_max < 2) return fail(RIPK_EINVAL, "n_max must be >= 2");
  if (d->m_max < 0) return fail(RIPK_EINVAL, "m_max must be >= 0");
  // sets per launch: the simulations, plus the observed set that
  // ripk_compute_K_envelope evaluates in the same launch
  const int64_t S = d->m_max > 0 ? (int64_t)d->m_max + 1 : 1;
  if ((int64_t)(d->m_max + 1) * d->n_max >= (1LL << 31))
    return fail(RIPK_EINVAL, "(m_max + 1)*n_max must be below 2^31");
  if (d->cell_div < 0 || d->cell_div > 8 || d->tcell_div < 0 || d->tcell_div > 8)
    return fail(RIPK_EINVAL, "cell_div and tcell_div must be in [0, 8]");

  for (int k = 1; k <= d->n_s; ++k) {
    __int128 a = (__int128)k * d->s_max;
    I.S2[k - 1] = (int64_t)(a * a / ((__int128)d->n_s * d->n_s));
  }
  for (int l = 1; l <= d->n_t; ++l) I.T[l - 1] = (int64_t)l * d->t_max / d->n_t;

  // cells: edge ceil(s_max/alpha) so that the stencil reaches alpha cells; grown
  // when the grid would be too large for 32-bit keys.
  const int alpha = d->cell_div ? d->cell_div : 1;
  const int beta = d->tcell_div ? d->tcell_div : 1;
  int64_t cs = (d->s_max + alpha - 1) / alpha, ct = (d->t_max + beta - 1) / beta;
  int64_t nx, ny, nt;
  for (;;) {
    nx = std::max<int64_t>(1, W / cs);
    ny = std::max<int64_t>(1, H / cs);
    nt = std::max<int64_t>(1, D / ct);
    if (nx * ny * nt * S * 2 < (1LL << 31) && nx * ny * nt <= (1LL << 24)) break;
    if (nx * ny >= nt) cs *= 2; else ct *= 2;
  }
  I.cell_s = cs;
  I.cell_t = ct;
  I.nx = (int32_t)nx;
  I.ny = (int32_t)ny;
  I.nt = (int32_t)nt;
  I.reach_s = (int32_t)((d->s_max + cs - 1) / cs);
  I.reach_t = (int32_t)((d->t_max + ct - 1) / ct);
  I.n_cells = nx * ny * nt;
  // Strict bound on |dx| and |dy| between a centre and any candidate: the
  // stencil spans reach+1 cells beyond the centre's cell, a row item's centres
  // span up to kItemExtent more x-cells, and the last cell of an axis also
  // holds the remainder of the side.
  const int64_t span = (I.reach_s + 1 + kItemExtent) * cs + std::max(W % cs, H % cs);
  if (span <= 32768)
    I.dist_mode = kModePacked;  // |dx|, |dy| <= 32767 and dx^2 + dy^2 < 2^31
  else if (2 * (span - 1) * (span - 1) < (1LL << 32))
    I.dist_mode = kModeU32;
  else
    I.dist_mode = kModeWide;
  I.n_bins = d->n_s * d->n_t;

  Geom &g = L->g;
  g.x0 = (int32_t)d->x0; g.y0 = (int32_t)d->y0; g.x1 = (int32_t)d->x1; g.y1 = (int32_t)d->y1;
  g.t0 = (int32_t)d->t0; g.t1 = (int32_t)d->t1;
  g.cell_s = (int32_t)cs; g.cell_t = (int32_t)ct;
  g.nx = I.nx; g.ny = I.ny; g.nt = I.nt;
  g.rs = I.reach_s; g.rt = I.reach_t;
  g.n_cells = (uint32_t)I.n_cells;
  g.n_s = d->n_s; g.n_t = d->n_t;
  g.edge = d->edge;
  g.mode = I.dist_mode;
  g.s2max = (uint64_t)I.S2[d->n_s - 1];
  g.tmax = (uint32_t)I.T[d->n_t - 1];
  // scaled down by 2^-20 so that the pair kernel's FP32 step estimates never
  // exceed the exact step (it then corrects upward by at most one)
  g.inv_ds = (float)((double)d->n_s / (double)d->s_max * (1.0 - 0x1p-20));
  g.inv_dt = (float)((double)d->n_t / (double)d->t_max * (1.0 - 0x1p-20));
  L->clamp_e = (int32_t)d->s_max;
  g.poly = nullptr;
  g.near = nullptr;
  g.prow = nullptr;
  g.row_shift = 0;
  while ((((int64_t)d->s_max + 2) << (g.row_shift + 1)) <= 65535 && g.row_shift < 8) ++g.row_shift;
  g.band_off = nullptr;
  g.band_idx = nullptr;
  g.band_shift = 0;
  while ((H >> g.band_shift) >= kBandsMax) ++g.band_shift;
  g.poly_n = (int32_t)L->V.size();
  g.poly_sign = area2 < 0 ? -1 : 1;
  L->area = L->V.empty() ? (double)W * (double)H : 0.5 * (double)std::llabs(area2);

  L->caps = caps_for(S, d->n_max, I.n_cells, I.n_bins, (int64_t)L->V.size(),
                     L->V.empty() ? 0 : nx * ny, (d->flags & RIPK_PLAN_INHOM) ? d->n_max : 0);
  I.device_bytes = caps_bytes(L->caps);
  return RIPK_OK;
}

}  // namespace

// Candidate cell subdivisions (spatial cells per s_max, temporal cells per
// t_max) the autotuner times.
constexpr int kTuneCand[][2] = {{1, 1}, {2, 1}, {1, 2}, {2, 2}, {3, 1}, {3, 2}};
constexpr int kTuneN = (int)(sizeof kTuneCand / sizeof kTuneCand[0]);
constexpr int kTuneSims = 32;  // simulations per timed candidate

// (observed single sets also time every cell grid with run fractions)
struct TuneState {
  bool done = false;
  int32_t cd = 1, td = 1;
  bool split_runs = false;
  bool cost_order = false;
  double us[2 * kTuneN] = {};
};

struct ripk_plan_s {
  ripk_plan_desc desc;       // descriptor of the bound geometry
  ripk_plan_desc user_desc;  // descriptor as given (autotuning varies the cells)
  TuneState tune[2];         // [0] observed sets, [1] simulations
  hipEvent_t tev[2] = {};    // autotuner timing
  bool tuning = false;       // autotuner trials in progress (eager launches)
  Layout lay;
  int32_t bound_cd = 1, bound_td = 1;  // cell subdivisions of the bound geometry
  bool split_runs = false;             // run fractions for this call's launch
  bool cost_order = false;             // cost-ordered work list for this call's launch
  uint64_t flush_evals = 0;            // ripk_plan_set_flush_bound (0: default)
  // served plans (plan_set_sharing): host-visible count of busy slots, the
  // share of the pair kernel's grid kept while others are busy, and the
  // slice length of long pair launches
  const int32_t *share_word = nullptr;
  double share_frac = 1.0;
  double slice_us = 0.0;
  uint64_t bind_gen = 0;               // bumped whenever a geometry is bound
  // RIPK_PLAN_GRAPH: the captured launch sequence of the last call shape
  hipGraphExec_t gexec = nullptr;
  uint64_t gkey[15] = {};
  int device = 0;
  int cus = 0;
  size_t lds_max = 0;  // LDS bytes a workgroup may use on this device
  Caps caps{};         // capacities the device buffers were allocated for
  uint64_t S2h[kMaxSteps] = {};  // host copies of the threshold tables
  uint32_t Th[kMaxSteps] = {};
  // device buffers
  int32_t *x = nullptr, *y = nullptr, *t = nullptr;
  int32_t *ox = nullptr, *oy = nullptr, *ot = nullptr;  // last observed set (resampling)
  int64_t obs_n = 0;
  int64_t split_n = 0, split_n1 = 0;  // cross K: n and n1 of the last observed set
  uint32_t *keys[2] = {nullptr, nullptr}, *vals[2] = {nullptr, nullptr};
  void *sort_temp = nullptr;
  uint32_t *cs = nullptr;
  int4 *P = nullptr;
  uint32_t *chunks = nullptr, *offs = nullptr, *set_base = nullptr;
  void *scan_temp = nullptr;
  Item *items = nullptr;
  unsigned long long *binC = nullptr, *binW = nullptr;
  unsigned long long *outC = nullptr;
  double *outW = nullptr, *outK = nullptr, *outL = nullptr;
  double *env = nullptr, *Lobs = nullptr;
  uint64_t *S2 = nullptr;
  uint32_t *T = nullptr;
  double *lam = nullptr;       // intensities of the observed set (host input staged here)
  double *rho = nullptr;       // 1/lambda per sorted record
  const double *cur_lam = nullptr;  // intensities of the current call (device)
  int4 *poly = nullptr;        // polygon edges {V[k], V[k+1 mod n]} (window-relative)
  uint32_t *prow = nullptr;    // per-record polygon rows (kRowWords words each)
  uint32_t *band_off = nullptr;  // polygon edges by horizontal band (see Geom)
  uint16_t *band_idx = nullptr;
  std::vector<uint32_t> band_offh;  // host copies (sources of the upload)
  std::vector<uint16_t> band_idxh;
  uint16_t *near = nullptr;    // per xy-cell edge lists of the bound geometry
  std::vector<uint16_t> nearh; // host copy of the lists (source of the upload)
  std::vector<int4> edgeh;     // host copy of the edges (source of the upload)
  // [0] n_eval, [1] n_in, [2] err|n_items (u32s); from word kQueueStride on,
  // the pair kernel's kQueues work-queue blocks
  unsigned long long *scal = nullptr;
  // a call's scalars and result rows, packed on the device and brought to
  // pinned host memory in one copy (kScalWords + kPackRows * n_bins words)
  unsigned long long *dstage = nullptr;
  // RIPK_PLAN_TIMING: start and end of every pair-kernel workgroup (2 words
  // each, up to kMaxWgPerCu per compute unit)
  unsigned long long *wg_times = nullptr;
  unsigned long long *hstage = nullptr;
  hipEvent_t ev[6] = {};
  ripk_stats stats{};
};

namespace {

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  return hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}

void release(ripk_plan_s *p) {
  if (!p) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(p->device);
  void *bufs[] = {p->x, p->y, p->t, p->ox, p->oy, p->ot, p->keys[0], p->keys[1], p->vals[0],
                  p->vals[1],
                  p->sort_temp, p->cs, p->P, p->chunks, p->offs, p->set_base, p->scan_temp,
                  p->items, p->binC, p->binW, p->outC, p->outW, p->outK, p->outL, p->env,
                  p->Lobs, p->S2, p->T, p->poly, p->near, p->prow, p->band_off, p->band_idx,
                  p->lam, p->rho, p->scal, p->dstage, p->wg_times};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (p->hstage) (void)hipHostFree(p->hstage);
  for (auto &e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : p->tev)
    if (e) (void)hipEventDestroy(e);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  (void)hipSetDevice(prev);
  delete p;
}

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

// Bit budget of one pair's fixed-point weight in an inhomogeneous launch of
// sets of n points: below 2^93 (three 32-bit pieces per side with room), and
// n(n-1) ordered pairs below 2^budget each sum below 2^126.
int wide_budget(uint32_t n) {
  const uint64_t pairs = (uint64_t)n * (n > 0 ? n - 1 : 0);
  int lg = 0;
  while (lg < 64 && (1ull << lg) < pairs) ++lg;  // ceil(log2(pairs))
  return std::min(93, 126 - lg);
}

// Enqueues the launch sequence of one evaluation of S sets of n points each on
// st (kernels only, and event records when timing): capturable into a graph.
// With `simulate` the points are drawn on the device; otherwise keys come from
// (x, y, t).
// with_obs (CSR simulations only): set 0 is the observed set, already in
// p->x, p->y, p->t [0, n), and sets 1..S-1 are the simulations; the envelope
// covers those and takes set 0's L as L_obs.
ripk_status enqueue_sets(ripk_plan_s *p, uint32_t S, uint32_t n, uint32_t n_centres,
                         const int32_t *x, const int32_t *y, const int32_t *t, bool simulate,
                         uint64_t seed, bool has_Lobs, hipStream_t st, bool symmetric,
                         bool timing, uint32_t S_split, bool with_obs = false) {
  const Geom &g = p->lay.g;
  const uint32_t NB = (uint32_t)p->lay.info.n_bins;
  const uint32_t N = S * n;
  if (timing) HIPCHK(hipEventRecord(p->ev[0], st));
  uint32_t *err = (uint32_t *)(p->scal + 2);
  uint32_t *n_items = err + 1;
  unsigned long long *queues = p->scal + kQueueStride;
  // the scalars and work queue, and every set's bins
  HIPCHK(launch_zero3(Zero3{{p->scal, p->binC, p->binW},
                            {(size_t)(kQueues + 1) * kQueueStride, (size_t)S * NB,
                             (size_t)S * NB * kBinWords}},
                      st));
  const bool cross = (p->desc.flags & RIPK_PLAN_CROSS) != 0;
  const uint32_t so = with_obs ? 1u : 0u;  // sets before the first simulation
  if (simulate) {
    if (with_obs)
      HIPCHK(launch_keys(p->x, p->y, p->t, n, n_centres, 0, 1, g, cross, p->keys[0], p->vals[0],
                         err, st));
    if (p->desc.sim_method == RIPK_SIM_CSR)
      HIPCHK(launch_csr(n, n_centres, S - so, seed, g, cross, p->x, p->y, p->t, p->keys[0],
                        p->vals[0], err, so, st));
    else
      HIPCHK(launch_resample(p->desc.sim_method == RIPK_SIM_PERMUTE ? 1 : 2, n, n_centres, S,
                             seed, cross, p->ox, p->oy, p->ot, g, p->x, p->y, p->t, p->keys, p->vals,
                             p->sort_temp, st));
    x = p->x; y = p->y; t = p->t;
  } else {
    HIPCHK(launch_keys(x, y, t, n, n_centres, 0, 1, g, cross, p->keys[0], p->vals[0], err, st));
  }
  if (timing) HIPCHK(hipEventRecord(p->ev[1], st));
  const uint64_t n_keys = (uint64_t)S * g.n_cells * 2;
  int alt = 0;
  // every set's entries are contiguous and its keys span 2 * n_cells values
  // (interleaved: (set * n_cells + cell) * 2 + halo; blocked: (2 * set + type)
  // * n_cells + cell), so each set is sorted on its own
  const uint32_t set_keys = 2u * (uint32_t)g.n_cells;
  HIPCHK(radix_sort(p->keys[0], p->vals[0], p->keys[1], p->vals[1], N, ceil_log2(set_keys),
                    p->sort_temp, st, &alt, S, set_keys));
  // (cross K sets are sorted in blocked order, each type one cell-sorted block:
  // centres come from the type-1 block and neighbour runs from the type-2 block)
  HIPCHK(launch_bounds_gather(p->keys[alt], p->vals[alt], N, (uint32_t)n_keys, p->cs, x, y, t, g,
                              p->lay.clamp_e, p->P, p->prow, st));
  const bool inhom = (p->desc.flags & RIPK_PLAN_INHOM) != 0 && !simulate;
  // (scal[3]: the largest 1/lambda of an inhomogeneous launch, as its bits)
  unsigned long long *rho_max = p->scal + 3;
  if (inhom) HIPCHK(launch_gather_rho(p->vals[alt], N, p->cur_lam, p->rho, err, rho_max, st));
  // row items need rows without halo entries: every point a centre, or the
  // type-1 block of a cross-K set
  const bool row_items = n_centres == n || cross;
  // bin layout: wide for polygon weights and inhomogeneous K; otherwise packed
  // (one LDS atomic per pair) unless the set is large or the extra 4 bytes
  // per bin would lower the occupancy
  const int var = inhom ? 2 : (pair_poly(g) ? 1 : 0);
  int bins = pair_bins_for_var(
      var, ((int64_t)n >= kWideCountPoints || (p->desc.flags & RIPK_PLAN_WIDE_COUNTS))
               ? kBinsSplit64
               : kBinsSplit32);
  int per_cu = 0;
  HIPCHK(pair_occupancy(g.n_s, g.n_t, bins, symmetric ? 1 : 0, g.mode, var, &per_cu));
  if (bins == kBinsSplit32 && (int64_t)n < kPackedPoints) {
    int per_cu_packed = 0;
    HIPCHK(pair_occupancy(g.n_s, g.n_t, kBinsPacked, symmetric ? 1 : 0, g.mode, var,
                          &per_cu_packed));
    if (per_cu_packed >= per_cu) bins = kBinsPacked;
  }
  if (per_cu < 1) return fail(RIPK_EINVAL, "pair kernel does not fit on a compute unit (n_bins=%u)", NB);
  // A launch with fewer groups than about 16 times the resident workgroups
  // splits every item's stencil rows into `split` parts taken by different
  // waves: a single set's items then come in pieces small enough for the
  // queue to even out dense clusters.
  const int64_t slots = (int64_t)per_cu * p->cus;
  const int64_t items_bound = (int64_t)S * (n / kChunk + g.n_cells + kItemsPerGroup);
  // (sized for S_split sets: the autotuner times a few sets of a larger call)
  const int64_t items_est = (int64_t)S_split * (n / kChunk + 1);
  const uint32_t n_rows = symmetric ? (uint32_t)((g.rs + 1) + g.rt * (2 * g.rs + 1))
                                    : (uint32_t)((2 * g.rt + 1) * (2 * g.rs + 1));
  // With run fractions (RIPK_PLAN_SPLIT_RUNS, or chosen by the autotuner), a
  // launch that wants more parts than rows cuts each row's run into k equal
  // fractions: n_rows * k parts.
  const int64_t want = (16 * slots * kItemsPerGroup + items_est - 1) / items_est;
  const int64_t room = std::min<int64_t>(kSplitMax, p->caps.items / std::max<int64_t>(items_bound, 1));
  int64_t split = std::min<int64_t>({want, (int64_t)n_rows, room});
  if (p->split_runs && want > (int64_t)n_rows) {
    const int64_t k = std::min<int64_t>({(want + n_rows - 1) / n_rows, kMaxFractions, room / n_rows});
    if (k >= 2) split = (int64_t)n_rows * k;
  }
  split = std::max<int64_t>(split, 1);
  // (with split items, each item is written once into the free point-sort key
  // buffer and expanded in parallel, when it has room for every item)
  Item *tmp_items = nullptr;
  uint32_t max_slots = 0;
  if (split > 1 && items_bound <= (int64_t)N / 4) {
    tmp_items = (Item *)p->keys[0];
    max_slots = (uint32_t)std::min<int64_t>(p->caps.items, items_bound * split);
  }
  HIPCHK(launch_items(p->cs, S, g, row_items, cross, (uint32_t)split, n_rows, p->chunks, p->offs,
                      p->set_base, p->items, n_items, p->scan_temp, st, tmp_items, max_slots));

  if (timing) HIPCHK(hipEventRecord(p->ev[2], st));

  PairArgs a;
  a.g = g;
  a.P = p->P;
  a.cs = p->cs;
  a.items = p->items;
  a.n_items = n_items;
  a.queues = queues;
  a.S2 = p->S2;
  a.T = p->T;
  a.binC = p->binC;
  a.binW = p->binW;
  a.symmetric = symmetric ? 1 : 0;
  a.row_items = row_items ? 1 : 0;
  a.blocked = cross ? 1 : 0;
  a.rho = inhom ? p->rho : nullptr;
  a.rho_max = inhom ? rho_max : nullptr;
  a.wbudget = inhom ? wide_budget(n) : 0;
  a.bins = bins;
  a.flush_evals = p->flush_evals;
  a.share_word = p->share_word;
  a.share_grid = (int32_t)std::max<int64_t>(1, (int64_t)(p->share_frac * (double)slots));
  a.slice_ticks = 0;
  a.perm = nullptr;
  a.wg_times = timing ? p->wg_times : nullptr;
  const int64_t groups_cap = items_bound * split / kItemsPerGroup + 1;
  // A launch whose items are split (few sets) hands its groups out costliest
  // first, dealt over the queue partitions, so that the long groups of dense
  // clusters do not start last.  The sort reuses the point-sort buffers, free
  // once the records are gathered.
  p->stats.cost_ordered = 0;
  if (p->cost_order && split > 1) {
    const uint64_t mg = ordered_slots((uint32_t)std::min<int64_t>(groups_cap, 1LL << 30));
    if (mg <= (uint64_t)N && radix_sort_temp_bytes((uint32_t)mg) <= radix_sort_temp_bytes(N, S)) {
      HIPCHK(launch_order_groups(a, (uint32_t)mg, p->keys[0], p->vals[0], p->keys[1], p->vals[1],
                                 p->sort_temp, &a.perm, st));
      p->stats.cost_ordered = 1;
    }
  }
  const int grid = (int)std::min<int64_t>(slots, groups_cap);
  // A served plan cuts a long pair launch into slices: workgroups leave after
  // slice_us, the next launch on the stream carries on with the same work
  // queue, and the last launch runs to the end.  Between slices the other
  // requests' kernels get the device.  The launch time is estimated from the
  // candidates a uniform set would have (full stencil rows, symmetric half).
  int slices = 1;
  if (p->slice_us > 0.0) {
    const double W = (double)(g.x1 - g.x0), H = (double)(g.y1 - g.y0), D = (double)(g.t1 - g.t0);
    const double reach = std::min(1.0, (2.0 * g.rs + 1) * g.cell_s / W) *
                         std::min(1.0, (2.0 * g.rs + 1) * g.cell_s / H) *
                         std::min(1.0, (2.0 * g.rt + 1) * g.cell_t / D);
    const double est_us = 0.5 * (double)S * (double)n * (double)n * reach / 1.0e6;
    slices = (int)std::min(64.0, std::floor(est_us / p->slice_us)) + 1;
  }
  for (int sl = 0; sl < slices; ++sl) {
    a.slice_ticks = sl + 1 < slices ? (uint32_t)(p->slice_us * 100.0) : 0u;  // 100 MHz ticks
    HIPCHK(launch_pair(a, grid, st));
  }
  if (timing) HIPCHK(hipEventRecord(p->ev[3], st));

  // K = AD * W / Nn; inhomogeneous K is W / (A D)
  const double vol = p->lay.area * (double)(p->desc.t1 - p->desc.t0);
  const double AD = inhom ? 1.0 : vol;
  const double Nn = inhom ? vol
                    : cross ? (double)n_centres * (double)(n - n_centres)
                    : p->desc.norm == RIPK_NORM_N2 ? (double)n * (double)n
                                                   : (double)n * (double)(n - 1);
  HIPCHK(launch_finalize(p->binC, p->binW, S, g.n_s, g.n_t, (double)p->desc.s_max,
                         (double)p->desc.t_max, AD, Nn, p->outC, p->outW, p->outK, p->outL,
                         queues, p->scal, st, a.rho_max, a.wbudget));
  if (simulate && with_obs)
    HIPCHK(launch_envelope(p->outK + NB, p->outL + NB, S - 1, (int)NB, p->outL, p->env, st));
  else if (simulate)
    HIPCHK(launch_envelope(p->outK, p->outL, S, (int)NB, has_Lobs ? p->Lobs : nullptr, p->env, st));
  if (timing) HIPCHK(hipEventRecord(p->ev[4], st));
  p->stats.pair_grid = grid;
  p->stats.split = (int32_t)split;
  p->stats.bin_layout = bins;
  p->stats.symmetric = symmetric ? 1 : 0;
  return RIPK_OK;
}

// One evaluation of S sets: eager launches, or with RIPK_PLAN_GRAPH (on a
// non-null stream, without per-phase timing) the replay of a graph captured
// for this call shape -- sizes, inputs, seed and bound geometry; any change
// captures afresh.
ripk_status run_sets(ripk_plan_s *p, uint32_t S, uint32_t n, uint32_t n_centres, const int32_t *x,
                     const int32_t *y, const int32_t *t, bool simulate, uint64_t seed,
                     const double *L_obs, hipStream_t st, bool symmetric, uint32_t S_split = 0,
                     bool with_obs = false) {
  if (S_split == 0) S_split = S;
  const uint32_t NB = (uint32_t)p->lay.info.n_bins;
  const bool has_Lobs = simulate && L_obs != nullptr;
  if (has_Lobs) HIPCHK(hipMemcpyAsync(p->Lobs, L_obs, sizeof(double) * NB, hipMemcpyHostToDevice, st));
  const bool timing = (p->desc.flags & RIPK_PLAN_TIMING) != 0;
  // (autotuner trials run eager: a capture inside a timed trial would count)
  const bool graph = (p->desc.flags & RIPK_PLAN_GRAPH) && !timing && st != nullptr && !p->tuning;
  if (!graph)
    return enqueue_sets(p, S, n, n_centres, x, y, t, simulate, seed, has_Lobs, st, symmetric, timing,
                        S_split, with_obs);
  const uint64_t key[15] = {S, n, n_centres, (uint64_t)simulate, (uint64_t)symmetric,
                            (uint64_t)(uintptr_t)x, (uint64_t)(uintptr_t)y, (uint64_t)(uintptr_t)t,
                            seed, (uint64_t)has_Lobs, p->bind_gen, S_split,
                            (uint64_t)(uintptr_t)p->cur_lam, (uint64_t)with_obs,
                            (uint64_t)p->split_runs | ((uint64_t)p->cost_order << 1)};
  if (!p->gexec || std::memcmp(key, p->gkey, sizeof key) != 0) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const ripk_status s =
        enqueue_sets(p, S, n, n_centres, x, y, t, simulate, seed, has_Lobs, st, symmetric, false,
                     S_split, with_obs);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &gr);
    if (s != RIPK_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return s;
    }
    if (e != hipSuccess) return fail(RIPK_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&p->gexec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) {
      p->gexec = nullptr;
      return fail(RIPK_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    std::memcpy(p->gkey, key, sizeof key);
  }
  HIPCHK(hipGraphLaunch(p->gexec, st));
  return RIPK_OK;
}

// Waits for the call and reads its scalars; with `rows`, those result rows of
// n_bins words come along in the same copy, at p->hstage + kScalWords + r*n_bins.
ripk_status collect_stats(ripk_plan_s *p, hipStream_t st, uint32_t S, uint32_t n,
                          uint32_t *err_out, const PackRows *rows = nullptr) {
  const int NB = (int)p->lay.info.n_bins;
  PackRows none = {};
  int last = -1;
  if (rows)
    for (int r = 0; r < kPackRows; ++r)
      if (rows->p[r]) last = r;
  HIPCHK(launch_pack(p->scal, rows ? *rows : none, NB, p->dstage, st));
  const size_t words = kScalWords + (size_t)(last + 1) * NB;
  HIPCHK(hipMemcpyAsync(p->hstage, p->dstage, sizeof(unsigned long long) * words,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const unsigned long long *sc = p->hstage;
  const uint32_t *w = (const uint32_t *)(sc + 2);
  *err_out = w[0];
  p->stats.n_eval = (int64_t)sc[0];
  p->stats.n_in = (int64_t)sc[1];
  p->stats.n_items = (int64_t)w[1];
  p->stats.n_sets = S;
  p->stats.n_points = (int64_t)S * n;
  if (p->desc.flags & RIPK_PLAN_TIMING) {
    float ms[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) HIPCHK(hipEventElapsedTime(&ms[i], p->ev[i], p->ev[i + 1]));
    p->stats.us_gen = 1e3 * ms[0];
    p->stats.us_grid = 1e3 * ms[1];
    p->stats.us_pair = 1e3 * ms[2];
    p->stats.us_finalize = 1e3 * ms[3];
    // workgroup end times of the last pair launch, after the earliest start
    // (100 MHz ticks); workgroups that took no work left zeros
    p->stats.us_wg_end_median = p->stats.us_wg_end_p90 = p->stats.us_wg_end_max = 0.0;
    const int grid = p->stats.pair_grid;
    if (p->wg_times && grid > 0 && grid <= std::max(p->cus, 1) * kMaxWgPerCu) {
      std::vector<unsigned long long> tw(2 * (size_t)grid);
      HIPCHK(hipMemcpy(tw.data(), p->wg_times, sizeof(unsigned long long) * tw.size(),
                       hipMemcpyDeviceToHost));
      unsigned long long t0 = ~0ull;
      for (int w = 0; w < grid; ++w)
        if (tw[2 * w]) t0 = std::min(t0, tw[2 * w]);
      std::vector<double> ends;
      for (int w = 0; w < grid; ++w)
        if (tw[2 * w] && tw[2 * w + 1] >= t0) ends.push_back(0.01 * (double)(tw[2 * w + 1] - t0));
      if (!ends.empty()) {
        std::sort(ends.begin(), ends.end());
        p->stats.us_wg_end_median = ends[ends.size() / 2];
        p->stats.us_wg_end_p90 = ends[std::min(ends.size() - 1, ends.size() * 9 / 10)];
        p->stats.us_wg_end_max = ends.back();
      }
    }
  }
  return RIPK_OK;
}

// the device error word: bit 0 a point outside the study area, bit 1 a CSR
// point that found no attempt inside the polygon
ripk_status err_status(uint32_t err) {
  if (err & 1u) return fail(RIPK_ERANGE, "a point lies outside the study area");
  if (err & 4u) return fail(RIPK_ERANGE, "an intensity lies outside [2^-400, 2^400]");
  return fail(RIPK_EDEVICE, "rejection sampling found no point inside the polygon");
}

ripk_status sync_status(hipError_t e) {
  if (e != hipSuccess) return fail(RIPK_EDEVICE, "device synchronisation failed: %s", hipGetErrorString(e));
  return RIPK_OK;
}

}  // namespace

namespace ripk {

ripk_status plan_caps_all(const ripk_plan_desc *desc, Caps *caps);

ripk_status plan_validate(const ripk_plan_desc *desc, Caps *caps) {
  Caps c;
  ripk_status s = plan_caps_all(desc, &c);
  if (s == RIPK_OK && caps) *caps = c;
  return s;
}

// Device buffers for the capacities c on `device`; geometry is bound later.
ripk_status plan_create(int device, const Caps &c, ripk_plan_s **out) {
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(RIPK_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev)
    return fail(RIPK_EINVAL, "device %d out of range (have %d)", device, ndev);
  DeviceGuard dg(device);
  ripk_plan_s *p = new ripk_plan_s();
  p->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    release(p);
    return fail(RIPK_EDEVICE, "hipGetDeviceProperties failed");
  }
  p->cus = prop.multiProcessorCount;
  p->lds_max = prop.sharedMemPerBlock;
  p->caps = c;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, cnt) \
  if (e == hipSuccess) e = dalloc(&(ptr), (size_t)(cnt))
  ALLOC(p->x, c.N); ALLOC(p->y, c.N); ALLOC(p->t, c.N);
  ALLOC(p->ox, c.P); ALLOC(p->oy, c.P); ALLOC(p->ot, c.P);
  ALLOC(p->keys[0], c.N); ALLOC(p->keys[1], c.N); ALLOC(p->vals[0], c.N); ALLOC(p->vals[1], c.N);
  if (e == hipSuccess)
    e = hipMalloc(&p->sort_temp, radix_sort_temp_bytes((uint32_t)c.N, (uint32_t)c.S));
  ALLOC(p->cs, 2 * c.SNC + 1);
  ALLOC(p->P, c.N);
  ALLOC(p->chunks, c.SNC); ALLOC(p->offs, c.SNC + 1); ALLOC(p->set_base, c.S + 1);
  if (e == hipSuccess) e = hipMalloc(&p->scan_temp, scan_temp_bytes((uint32_t)c.SNC) + 256);
  ALLOC(p->items, c.items);
  ALLOC(p->binC, c.SNB); ALLOC(p->binW, kBinWords * c.SNB);
  ALLOC(p->outC, c.SNB); ALLOC(p->outW, c.SNB); ALLOC(p->outK, c.SNB); ALLOC(p->outL, c.SNB);
  ALLOC(p->env, 5 * c.NB); ALLOC(p->Lobs, c.NB);
  ALLOC(p->S2, kMaxSteps); ALLOC(p->T, kMaxSteps);
  ALLOC(p->poly, c.V); ALLOC(p->near, (kNearMax + 1) * c.NXY);
  if (c.V > 0) ALLOC(p->prow, (int64_t)kRowWords * c.N);
  if (c.V > 0) ALLOC(p->band_off, kBandsMax + 1);
  if (c.V > 0) ALLOC(p->band_idx, (int64_t)kBandsMax * c.V);
  ALLOC(p->lam, c.R); ALLOC(p->rho, c.R);
  ALLOC(p->scal, (kQueues + 1) * kQueueStride);
  ALLOC(p->dstage, kScalWords + kPackRows * c.NB);
  ALLOC(p->wg_times, 2 * (size_t)std::max(p->cus, 1) * kMaxWgPerCu);
#undef ALLOC
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&p->hstage, sizeof(unsigned long long) * (kScalWords + kPackRows * c.NB),
                      hipHostMallocDefault);
  if (e != hipSuccess) {
    release(p);
    return fail(e == hipErrorOutOfMemory ? RIPK_ENOMEM : RIPK_EDEVICE, "allocation failed: %s",
                hipGetErrorString(e));
  }
  for (auto &ev : p->ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  for (auto &ev : p->tev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e != hipSuccess) {
    release(p);
    return fail(RIPK_EDEVICE, "plan set-up failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return RIPK_OK;
}

ripk_status bind_geometry(ripk_plan_s *p, const ripk_plan_desc *desc, hipStream_t stream);

// Binds a descriptor to a plan whose buffers hold its capacities; the
// threshold tables are copied on `stream`.  With RIPK_PLAN_AUTOTUNE the cells
// are tuned afresh on the next calls.
void plan_set_sharing(ripk_plan_s *p, const int32_t *share_word, double share_frac,
                      double slice_us) {
  p->share_word = share_word;
  p->share_frac = share_frac;
  p->slice_us = slice_us;
  ++p->bind_gen;  // a captured graph holds the old launch sequence
}

ripk_status plan_bind(ripk_plan_s *p, const ripk_plan_desc *desc, hipStream_t stream) {
  ripk_status s = bind_geometry(p, desc, stream);
  if (s != RIPK_OK) return s;
  p->user_desc = *desc;
  p->tune[0] = TuneState();
  p->tune[1] = TuneState();
  p->obs_n = 0;  // no observed set for resampled simulations yet
  p->split_n = p->split_n1 = 0;
  return RIPK_OK;
}

// Capacities for every geometry a descriptor may be bound to (all autotuner
// candidates with RIPK_PLAN_AUTOTUNE).
ripk_status plan_caps_all(const ripk_plan_desc *desc, Caps *caps) {
  Layout L;
  ripk_status s = derive(desc, &L);
  if (s != RIPK_OK) return s;
  Caps c = L.caps;
  if (desc->flags & RIPK_PLAN_AUTOTUNE) {
    for (int i = 0; i < kTuneN; ++i) {
      ripk_plan_desc d = *desc;
      d.cell_div = kTuneCand[i][0];
      d.tcell_div = kTuneCand[i][1];
      s = derive(&d, &L);
      if (s != RIPK_OK) return s;
      c = caps_max(c, L.caps);
    }
  }
  *caps = c;
  return RIPK_OK;
}

ripk_status bind_geometry(ripk_plan_s *p, const ripk_plan_desc *desc, hipStream_t stream) {
  Layout L;
  ripk_status s = derive(desc, &L);
  if (s != RIPK_OK) return s;
  if (desc->device != p->device) return fail(RIPK_EINVAL, "descriptor device differs from the plan's");
  if (!caps_fit(p->caps, L.caps)) return fail(RIPK_E2BIG, "descriptor exceeds the plan's capacity");
  // (the split layout of the plan's largest sets; packed bins are taken only
  // where they fit as well)
  const bool inhom = (desc->flags & RIPK_PLAN_INHOM) != 0;
  const int var = inhom ? 2 : (pair_poly(L.g) ? 1 : 0);
  const int lds = pair_lds_bytes(
      desc->n_s, desc->n_t,
      pair_bins_for_var(var, desc->n_max >= kWideCountPoints ||
                                     (desc->flags & RIPK_PLAN_WIDE_COUNTS)
                                 ? kBinsSplit64
                                 : kBinsSplit32),
      inhom);
  if ((size_t)lds > p->lds_max)
    return fail(RIPK_EINVAL, "grid of %d bins needs %d B of LDS per workgroup, device has %zu",
                L.info.n_bins, lds, p->lds_max);
  DeviceGuard dg(p->device);
  p->desc = *desc;
  p->lay = L;
  p->bound_cd = desc->cell_div ? desc->cell_div : 1;
  p->bound_td = desc->tcell_div ? desc->tcell_div : 1;
  ++p->bind_gen;
  std::memset(p->S2h, 0, sizeof p->S2h);
  std::memset(p->Th, 0, sizeof p->Th);
  for (int k = 0; k < desc->n_s; ++k) p->S2h[k] = (uint64_t)L.info.S2[k];
  for (int l = 0; l < desc->n_t; ++l) p->Th[l] = (uint32_t)L.info.T[l];
  HIPCHK(hipMemcpyAsync(p->S2, p->S2h, sizeof p->S2h, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(p->T, p->Th, sizeof p->Th, hipMemcpyHostToDevice, stream));
  if (!p->lay.V.empty()) {
    build_near(p->lay, desc->s_max, &p->nearh);
    near_summary(p->nearh, &p->lay.info);
    const size_t nv = p->lay.V.size();
    p->edgeh.resize(nv);
    for (size_t k = 0; k < nv; ++k) {
      const int2 a = p->lay.V[k], b = p->lay.V[k + 1 == nv ? 0 : k + 1];
      p->edgeh[k] = make_int4(a.x, a.y, b.x, b.y);
    }
    HIPCHK(hipMemcpyAsync(p->poly, p->edgeh.data(), sizeof(int4) * nv, hipMemcpyHostToDevice,
                          stream));
    HIPCHK(hipMemcpyAsync(p->near, p->nearh.data(), sizeof(uint16_t) * p->nearh.size(),
                          hipMemcpyHostToDevice, stream));
    build_bands(p->lay, &p->band_offh, &p->band_idxh);
    HIPCHK(hipMemcpyAsync(p->band_off, p->band_offh.data(), sizeof(uint32_t) * p->band_offh.size(),
                          hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(p->band_idx, p->band_idxh.data(), sizeof(uint16_t) * p->band_idxh.size(),
                          hipMemcpyHostToDevice, stream));
    // the host sources are replaced by the next bind: let the copies finish
    HIPCHK(hipStreamSynchronize(stream));
    p->lay.g.poly = p->poly;
    p->lay.g.near = p->near;
    p->lay.g.prow = pair_poly(p->lay.g) ? p->prow : nullptr;
    p->lay.g.band_off = p->band_off;
    p->lay.g.band_idx = p->band_idx;
  }
  return RIPK_OK;
}

const Caps &plan_caps(const ripk_plan_s *p) { return p->caps; }

// Runs run_sets in the geometry tuned for `which` (0 observed sets, 1
// simulations).  On a plan made with RIPK_PLAN_AUTOTUNE the first such call
// times every candidate cell subdivision on S_tune sets of the same input
// (results do not depend on the cells) and keeps the fastest.
ripk_status run_tuned(ripk_plan_s *p, int which, uint32_t S, uint32_t S_tune, uint32_t n,
                      uint32_t nc, const int32_t *x, const int32_t *y, const int32_t *t,
                      bool simulate, uint64_t seed, const double *L_obs, hipStream_t st,
                      bool sym, bool with_obs = false) {
  if (p->user_desc.flags & RIPK_PLAN_AUTOTUNE) {
    TuneState &ts = p->tune[which];
    ripk_plan_desc d = p->user_desc;
    // observed single sets: every cell grid without and with run fractions
    // (with them only, when the plan forces them)
    const bool forced = (p->user_desc.flags & RIPK_PLAN_SPLIT_RUNS) != 0;
    const int n_cand = (which == 0 && S == 1 && !forced) ? 2 * kTuneN : kTuneN;
    if (!ts.done) {
      double best = 1e300;
      int bi = 0;
      struct Tuning {  // trials run eager, whatever way the tuning ends
        ripk_plan_s *p;
        ~Tuning() { p->tuning = false; }
      } tuning_scope{p};
      p->tuning = true;
      for (int i = 0; i < n_cand; ++i) ts.us[i] = 1e300;
      // three untimed runs first, then the candidates in two rounds, the
      // second in reverse order, each kept at its faster run: candidates can be
      // a few % apart, and a device still raising its clock at the start of the
      // call would otherwise favour the ones timed last
      for (int rep = -3; rep < 2; ++rep) {
        for (int j = 0; j < n_cand; ++j) {
          if (rep < 0 && j > 0) break;
          const int i = rep == 1 ? n_cand - 1 - j : j;
          d.cell_div = kTuneCand[i % kTuneN][0];
          d.tcell_div = kTuneCand[i % kTuneN][1];
          p->split_runs = forced || i >= kTuneN;
          ripk_status s = bind_geometry(p, &d, st);
          if (s != RIPK_OK) return s;
          HIPCHK(hipEventRecord(p->tev[0], st));
          s = run_sets(p, S_tune, n, nc, x, y, t, simulate, seed, nullptr, st, sym, S, with_obs);
          if (s != RIPK_OK) return s;
          HIPCHK(hipEventRecord(p->tev[1], st));
          uint32_t err = 0;
          s = collect_stats(p, st, S_tune, n, &err);
          if (s != RIPK_OK) return s;
          if (err) return err_status(err);
          float ms = 0;
          HIPCHK(hipEventElapsedTime(&ms, p->tev[0], p->tev[1]));
          if (rep >= 0) ts.us[i] = std::min(ts.us[i], 1e3 * (double)ms);
        }
      }
      for (int i = 0; i < n_cand; ++i)
        if (ts.us[i] < best) {
          best = ts.us[i];
          bi = i;
        }
      ts.done = true;
      ts.cd = kTuneCand[bi % kTuneN][0];
      ts.td = kTuneCand[bi % kTuneN][1];
      ts.split_runs = forced || bi >= kTuneN;
      ts.cost_order = (p->user_desc.flags & RIPK_PLAN_COST_ORDER) != 0;
      if (which == 0 && S == 1 && !ts.cost_order) {
        // the chosen geometry with and without the cost-ordered work list,
        // in turn (three runs each, the faster of each kept), so that both
        // see the same device state
        d.cell_div = ts.cd;
        d.tcell_div = ts.td;
        p->split_runs = ts.split_runs;
        ripk_status s = bind_geometry(p, &d, st);
        if (s != RIPK_OK) return s;
        double us[2] = {1e300, 1e300};
        for (int rep = 0; rep < 6; ++rep) {
          const int on = (rep & 1) ^ 1;
          p->cost_order = on != 0;
          HIPCHK(hipEventRecord(p->tev[0], st));
          s = run_sets(p, S_tune, n, nc, x, y, t, simulate, seed, nullptr, st, sym, S, with_obs);
          if (s != RIPK_OK) return s;
          HIPCHK(hipEventRecord(p->tev[1], st));
          uint32_t err = 0;
          s = collect_stats(p, st, S_tune, n, &err);
          if (s != RIPK_OK) return s;
          if (err) return err_status(err);
          float ms = 0;
          HIPCHK(hipEventElapsedTime(&ms, p->tev[0], p->tev[1]));
          us[on] = std::min(us[on], 1e3 * (double)ms);
        }
        ts.cost_order = us[1] < us[0];
      }
    }
    p->split_runs = ts.split_runs;
    p->cost_order = ts.cost_order;
    if (p->bound_cd != ts.cd || p->bound_td != ts.td) {
      d.cell_div = ts.cd;
      d.tcell_div = ts.td;
      ripk_status s = bind_geometry(p, &d, st);
      if (s != RIPK_OK) return s;
    }
  } else {
    p->split_runs = (p->user_desc.flags & RIPK_PLAN_SPLIT_RUNS) != 0;
    p->cost_order = (p->user_desc.flags & RIPK_PLAN_COST_ORDER) != 0;
  }
  return run_sets(p, S, n, nc, x, y, t, simulate, seed, L_obs, st, sym, 0, with_obs);
}

void plan_free(ripk_plan_s *p) { release(p); }

ripk_status set_error(ripk_status s, const char *msg) { return fail(s, "%s", msg); }

namespace {

// Hands out 256-byte aligned pieces of one region (base null: sizes only).
struct Carve {
  unsigned char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

// The device buffers one observed set needs, cut from `base` (plan buffers
// the call does not use stay null); returns the bytes taken.
size_t carve_observed(ripk_plan_s *p, const Caps &c, bool host_points, unsigned char *base) {
  Carve k{base};
  p->scal = k.take<unsigned long long>((size_t)(kQueues + 1) * kQueueStride);
  p->binC = k.take<unsigned long long>(c.SNB);
  p->binW = k.take<unsigned long long>(kBinWords * c.SNB);
  for (int b = 0; b < 2; ++b) {
    p->keys[b] = k.take<uint32_t>(c.N);
    p->vals[b] = k.take<uint32_t>(c.N);
  }
  p->sort_temp = k.take<unsigned char>(radix_sort_temp_bytes((uint32_t)c.N, (uint32_t)c.S));
  p->cs = k.take<uint32_t>(2 * c.SNC + 1);
  p->P = k.take<int4>(c.N);
  p->chunks = k.take<uint32_t>(c.SNC);
  p->offs = k.take<uint32_t>(c.SNC + 1);
  p->set_base = k.take<uint32_t>(c.S + 1);
  p->scan_temp = k.take<unsigned char>(scan_temp_bytes((uint32_t)c.SNC) + 256);
  p->items = k.take<Item>(c.items);
  p->outC = k.take<unsigned long long>(c.SNB);
  p->outW = k.take<double>(c.SNB);
  p->outK = k.take<double>(c.SNB);
  p->outL = k.take<double>(c.SNB);
  p->S2 = k.take<uint64_t>(kMaxSteps);
  p->T = k.take<uint32_t>(kMaxSteps);
  if (host_points) {
    p->x = k.take<int32_t>(c.N);
    p->y = k.take<int32_t>(c.N);
    p->t = k.take<int32_t>(c.N);
  }
  return k.off;
}

}  // namespace

// ripk_compute_K for a rectangle, one point type and no intensities, with
// every device buffer cut from the caller's region `scratch` (no allocation):
// the plan lives on the stack, the thresholds are copied from it, and the
// results go to the device buffers of `out` once the call has succeeded.
ripk_status compute_K_in_scratch(const ripk_plan_desc *desc, const ripk_points *pts,
                                 hipStream_t st, unsigned char *scratch, size_t scratch_bytes,
                                 ripk_K_out *out) {
  if (!desc || !pts) return fail(RIPK_EINVAL, "null descriptor or points");
  if (desc->poly_n != 0 || desc->poly)
    return fail(RIPK_EINVAL, "the allocation-free call takes the rectangle (no polygon)");
  if (desc->flags & ~(RIPK_PLAN_ORDERED | RIPK_PLAN_WIDE_COUNTS | RIPK_PLAN_SPLIT_RUNS |
                      RIPK_PLAN_COST_ORDER))
    return fail(RIPK_EINVAL,
                "the allocation-free call takes RIPK_PLAN_ORDERED, RIPK_PLAN_WIDE_COUNTS, "
                "RIPK_PLAN_SPLIT_RUNS and RIPK_PLAN_COST_ORDER only");
  const int64_t n = pts->n;
  const int64_t nc = pts->n_centres ? pts->n_centres : n;
  if (n < 2) return fail(RIPK_EINVAL, "need n >= 2 points (n(n-1) = 0 otherwise)");
  if (nc < 0 || nc > n) return fail(RIPK_EINVAL, "n_centres must be in [0, n]");
  if (n >= (1LL << 31)) return fail(RIPK_EINVAL, "n must be below 2^31");
  if (!pts->x || !pts->y || !pts->t) return fail(RIPK_EINVAL, "null coordinate array");
  // sized for this call's n; no simulations
  ripk_plan_desc d = *desc;
  d.n_max = n;
  d.m_max = 0;
  Layout L;
  ripk_status s = derive(&d, &L);
  if (s != RIPK_OK) return s;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || d.device < 0 || d.device >= ndev)
    return fail(RIPK_EINVAL, "device %d out of range", d.device);
  DeviceGuard dg(d.device);
  ripk_plan_s p;
  p.device = d.device;
  int cus = 0, lds = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d.device));
  HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, d.device));
  p.cus = cus;
  p.lds_max = (size_t)lds;
  p.caps = L.caps;
  const bool host_points = !pts->on_device;
  const size_t need = carve_observed(&p, p.caps, host_points, nullptr);
  if (need > scratch_bytes)
    return fail(RIPK_E2BIG,
                "%lld points on %lld cells need %zu bytes of scratch; the allocation-free call "
                "has %zu",
                (long long)n, (long long)L.info.n_cells, need, scratch_bytes);
  carve_observed(&p, p.caps, host_points, scratch);
  s = bind_geometry(&p, &d, st);
  if (s != RIPK_OK) return s;
  p.user_desc = d;
  p.split_runs = (d.flags & RIPK_PLAN_SPLIT_RUNS) != 0;
  p.cost_order = (d.flags & RIPK_PLAN_COST_ORDER) != 0;
  const int32_t *x = pts->x, *y = pts->y, *t = pts->t;
  if (host_points) {
    HIPCHK(hipMemcpyAsync(p.x, x, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p.y, y, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p.t, t, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    x = p.x; y = p.y; t = p.t;
  }
  const bool sym = !(d.flags & RIPK_PLAN_ORDERED) && nc == n;
  s = enqueue_sets(&p, 1, (uint32_t)n, (uint32_t)nc, x, y, t, false, 0, false, st, sym, false, 1);
  if (s != RIPK_OK) return s;
  unsigned long long sc[3] = {0, 0, 0};
  HIPCHK(hipMemcpyAsync(sc, p.scal, sizeof sc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const uint32_t err = (uint32_t)sc[2];
  if (err) return err_status(err);
  if (out) {
    const size_t bytes = 8 * (size_t)L.info.n_bins;
    void *dst[4] = {out->C, out->W, out->K, out->L};
    const void *src[4] = {p.outC, p.outW, p.outK, p.outL};
    for (int r = 0; r < 4; ++r)
      if (dst[r]) HIPCHK(hipMemcpyAsync(dst[r], src[r], bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return RIPK_OK;
}

}  // namespace ripk

extern "C" {

const char *ripk_status_str(ripk_status s) {
  switch (s) {
    case RIPK_OK: return "ok";
    case RIPK_PENDING: return "pending";
    case RIPK_EINVAL: return "invalid argument";
    case RIPK_ERANGE: return "point outside the study window";
    case RIPK_ENOMEM: return "out of memory";
    case RIPK_EDEVICE: return "device error";
    case RIPK_E2BIG: return "request exceeds capacity";
    case RIPK_EAGAIN: return "queue full";
    case RIPK_EOVERFLOW: return "accumulator overflow";
    case RIPK_ECANCELED: return "cancelled";
    case RIPK_ENOTFOUND: return "unknown ticket";
    default: return "unknown status";
  }
}

const char *ripk_last_error(void) { return g_err; }

ripk_status ripk_plan_check(const ripk_plan_desc *desc, ripk_plan_info *info) {
  Layout L;
  ripk_status s = derive(desc, &L);
  if (s != RIPK_OK) return s;
  if (!L.V.empty()) {
    // the per-cell edge lists a plan of this geometry builds (host only)
    std::vector<uint16_t> near;
    build_near(L, desc->s_max, &near);
    near_summary(near, &L.info);
  }
  if (info) *info = L.info;
  return RIPK_OK;
}

ripk_status ripk_plan(const ripk_plan_desc *desc, ripk_plan_t *out) {
  if (!out) return fail(RIPK_EINVAL, "null output handle");
  *out = nullptr;
  Caps caps;
  ripk_status s = plan_caps_all(desc, &caps);
  if (s != RIPK_OK) return s;
  ripk_plan_s *p = nullptr;
  s = plan_create(desc->device, caps, &p);
  if (s != RIPK_OK) return s;
  s = plan_bind(p, desc, nullptr);
  if (s == RIPK_OK) s = sync_status(hipStreamSynchronize(nullptr));
  if (s != RIPK_OK) {
    release(p);
    return s;
  }
  *out = p;
  return RIPK_OK;
}

void ripk_plan_destroy(ripk_plan_t plan) { release(plan); }

ripk_status ripk_compute_K(ripk_plan_t p, const ripk_points *pts, void *stream, ripk_K_out *out) {
  if (!p || !pts) return fail(RIPK_EINVAL, "null plan or points");
  const int64_t n = pts->n;
  const int64_t nc = pts->n_centres ? pts->n_centres : n;
  if (n < 2) return fail(RIPK_EINVAL, "need n >= 2 points (n(n-1) = 0 otherwise)");
  if (n > p->desc.n_max) return fail(RIPK_EINVAL, "n = %lld exceeds n_max = %lld", (long long)n, (long long)p->desc.n_max);
  if (nc < 0 || nc > n) return fail(RIPK_EINVAL, "n_centres must be in [0, n]");
  const bool cross = (p->desc.flags & RIPK_PLAN_CROSS) != 0;
  const bool inhom = (p->desc.flags & RIPK_PLAN_INHOM) != 0;
  if (inhom && !pts->lambda)
    return fail(RIPK_EINVAL, "an inhomogeneous K plan needs the intensity of every point");
  if (inhom && nc != n) return fail(RIPK_EINVAL, "inhomogeneous K takes every point as a centre");
  if (cross && (pts->n_centres < 1 || pts->n_centres >= n))
    return fail(RIPK_EINVAL, "cross K needs 1 <= n_centres < n (type 1 = points [0, n_centres))");
  if (!pts->x || !pts->y || !pts->t) return fail(RIPK_EINVAL, "null coordinate array");
  auto t0 = std::chrono::steady_clock::now();
  DeviceGuard dg(p->device);
  hipStream_t st = (hipStream_t)stream;
  const int32_t *x = pts->x, *y = pts->y, *t = pts->t;
  p->cur_lam = nullptr;
  if (inhom) {
    if (pts->on_device) {
      p->cur_lam = pts->lambda;
    } else {
      HIPCHK(hipMemcpyAsync(p->lam, pts->lambda, sizeof(double) * n, hipMemcpyHostToDevice, st));
      p->cur_lam = p->lam;
    }
  }
  if (!pts->on_device) {
    HIPCHK(hipMemcpyAsync(p->x, x, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->y, y, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->t, t, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    x = p->x; y = p->y; t = p->t;
  }
  if (p->desc.sim_method != RIPK_SIM_CSR) {
    // resampled simulations draw from this set: keep a copy
    HIPCHK(hipMemcpyAsync(p->ox, x, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p->oy, y, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p->ot, t, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    p->obs_n = 0;  // set once the call succeeds
  }
  p->split_n = p->split_n1 = 0;
  const bool sym = !(p->desc.flags & RIPK_PLAN_ORDERED) && nc == n;
  ripk_status s = run_tuned(p, 0, 1, 1, (uint32_t)n, (uint32_t)nc, x, y, t, false, 0, nullptr, st,
                            sym);
  if (s != RIPK_OK) return s;
  uint32_t err = 0;
  PackRows rows = {};
  if (out)
    rows = {{out->C ? p->outC : nullptr, out->W ? (const unsigned long long *)p->outW : nullptr,
             out->K ? (const unsigned long long *)p->outK : nullptr,
             out->L ? (const unsigned long long *)p->outL : nullptr, nullptr}};
  s = collect_stats(p, st, 1, (uint32_t)n, &err, &rows);
  if (s != RIPK_OK) return s;
  if (err) return err_status(err);
  if (p->desc.sim_method != RIPK_SIM_CSR) p->obs_n = n;
  if (cross) {
    p->split_n = n;
    p->split_n1 = nc;
  }
  const size_t NB = (size_t)p->lay.info.n_bins;
  if (out) {
    void *dst[4] = {out->C, out->W, out->K, out->L};
    for (int r = 0; r < 4; ++r)
      if (dst[r]) std::memcpy(dst[r], p->hstage + kScalWords + r * NB, 8 * NB);
  }
  p->stats.us_total = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  return RIPK_OK;
}

ripk_status ripk_simulate_envelope(ripk_plan_t p, int64_t n, int32_t m, uint64_t seed,
                                   const double *L_obs, void *stream, ripk_env_out *out) {
  if (!p) return fail(RIPK_EINVAL, "null plan");
  if (n < 2) return fail(RIPK_EINVAL, "need n >= 2 points");
  if (n > p->desc.n_max) return fail(RIPK_EINVAL, "n = %lld exceeds n_max = %lld", (long long)n, (long long)p->desc.n_max);
  if (m < 1 || m > p->desc.m_max) return fail(RIPK_EINVAL, "m = %d outside [1, m_max = %d]", m, p->desc.m_max);
  if (p->desc.sim_method != RIPK_SIM_CSR && p->obs_n != n)
    return fail(RIPK_EINVAL,
                "permutation and bootstrap simulations draw from the plan's last observed set: "
                "call ripk_compute_K on %lld points first", (long long)n);
  const bool cross = (p->desc.flags & RIPK_PLAN_CROSS) != 0;
  if (p->desc.flags & RIPK_PLAN_INHOM)
    return fail(RIPK_EINVAL,
                "inhomogeneous K plans take no simulations (the null model needs the "
                "intensity as a function)");
  if (cross && p->split_n != n)
    return fail(RIPK_EINVAL,
                "cross K simulations keep the type split of the plan's last observed set: "
                "call ripk_compute_K on %lld points first", (long long)n);
  auto t0 = std::chrono::steady_clock::now();
  DeviceGuard dg(p->device);
  hipStream_t st = (hipStream_t)stream;
  const bool sym = !(p->desc.flags & RIPK_PLAN_ORDERED) && !cross;
  const uint32_t nc = cross ? (uint32_t)p->split_n1 : (uint32_t)n;
  ripk_status s = run_tuned(p, 1, (uint32_t)m, (uint32_t)std::min(m, kTuneSims), (uint32_t)n,
                            nc, nullptr, nullptr, nullptr, true, seed, L_obs, st, sym);
  if (s != RIPK_OK) return s;
  uint32_t err = 0;
  const size_t NB = (size_t)p->lay.info.n_bins;
  double *dst[kPackRows] = {};
  PackRows rows = {};
  if (out) {
    double *d[kPackRows] = {out->K_lo, out->K_hi, out->L_lo, out->L_hi, L_obs ? out->dL_hi : nullptr};
    for (int r = 0; r < kPackRows; ++r) {
      dst[r] = d[r];
      rows.p[r] = d[r] ? (const unsigned long long *)(p->env + r * NB) : nullptr;
    }
  }
  s = collect_stats(p, st, (uint32_t)m, (uint32_t)n, &err, &rows);
  if (s != RIPK_OK) return s;
  if (err) return err_status(err);
  if (out) {
    for (int r = 0; r < kPackRows; ++r)
      if (dst[r]) std::memcpy(dst[r], p->hstage + kScalWords + r * NB, 8 * NB);
    if (out->C_sims) HIPCHK(hipMemcpyAsync(out->C_sims, p->outC, 8 * NB * m, hipMemcpyDeviceToHost, st));
    if (out->W_sims) HIPCHK(hipMemcpyAsync(out->W_sims, p->outW, 8 * NB * m, hipMemcpyDeviceToHost, st));
    if (out->K_sims) HIPCHK(hipMemcpyAsync(out->K_sims, p->outK, 8 * NB * m, hipMemcpyDeviceToHost, st));
    if (out->C_sims || out->W_sims || out->K_sims) HIPCHK(hipStreamSynchronize(st));
  }
  p->stats.us_total = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  return RIPK_OK;
}

ripk_status ripk_compute_K_envelope(ripk_plan_t p, const ripk_points *pts, int32_t m,
                                    uint64_t seed, void *stream, ripk_K_out *kout,
                                    ripk_env_out *eout) {
  if (!p || !pts) return fail(RIPK_EINVAL, "null plan or points");
  if (p->desc.flags & RIPK_PLAN_INHOM)
    return fail(RIPK_EINVAL,
                "inhomogeneous K plans take no simulations (the null model needs the "
                "intensity as a function)");
  if (m < 1 || m > p->desc.m_max) return fail(RIPK_EINVAL, "m = %d outside [1, m_max = %d]", m, p->desc.m_max);
  const int64_t n = pts->n;
  const int64_t nc = pts->n_centres ? pts->n_centres : n;
  const bool cross = (p->desc.flags & RIPK_PLAN_CROSS) != 0;
  const size_t NB = (size_t)p->lay.info.n_bins;
  if (p->desc.sim_method != RIPK_SIM_CSR || (!cross && nc != n)) {
    // simulations drawn from the observed set, or a centre subset: the two calls
    std::vector<double> Lh(NB);
    ripk_K_out ko = kout ? *kout : ripk_K_out{};
    if (!ko.L) ko.L = Lh.data();
    ripk_status s = ripk_compute_K(p, pts, stream, &ko);
    if (s != RIPK_OK) return s;
    return ripk_simulate_envelope(p, n, m, seed, ko.L, stream, eout);
  }
  if (n < 2) return fail(RIPK_EINVAL, "need n >= 2 points (n(n-1) = 0 otherwise)");
  if (n > p->desc.n_max) return fail(RIPK_EINVAL, "n = %lld exceeds n_max = %lld", (long long)n, (long long)p->desc.n_max);
  if (cross && (pts->n_centres < 1 || pts->n_centres >= n))
    return fail(RIPK_EINVAL, "cross K needs 1 <= n_centres < n (type 1 = points [0, n_centres))");
  if (!pts->x || !pts->y || !pts->t) return fail(RIPK_EINVAL, "null coordinate array");
  auto t0 = std::chrono::steady_clock::now();
  DeviceGuard dg(p->device);
  hipStream_t st = (hipStream_t)stream;
  // the observed points become set 0 of the simulation launch
  const hipMemcpyKind kind = pts->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(hipMemcpyAsync(p->x, pts->x, sizeof(int32_t) * n, kind, st));
  HIPCHK(hipMemcpyAsync(p->y, pts->y, sizeof(int32_t) * n, kind, st));
  HIPCHK(hipMemcpyAsync(p->t, pts->t, sizeof(int32_t) * n, kind, st));
  p->cur_lam = nullptr;
  p->split_n = p->split_n1 = 0;
  const bool sym = !(p->desc.flags & RIPK_PLAN_ORDERED) && !cross;
  ripk_status s = run_tuned(p, 1, (uint32_t)m + 1, (uint32_t)std::min(m + 1, kTuneSims),
                            (uint32_t)n, (uint32_t)nc, p->x, p->y, p->t, true, seed, nullptr, st,
                            sym, true);
  if (s != RIPK_OK) return s;
  // rows 0-3: C, W, K, L of the observed set; rows 4-8: the envelopes
  PackRows rows = {};
  double *dst[kPackRows] = {};
  if (kout) {
    void *k[4] = {kout->C, kout->W, kout->K, kout->L};
    const unsigned long long *src[4] = {p->outC, (const unsigned long long *)p->outW,
                                        (const unsigned long long *)p->outK,
                                        (const unsigned long long *)p->outL};
    for (int r = 0; r < 4; ++r) {
      dst[r] = (double *)k[r];
      rows.p[r] = k[r] ? src[r] : nullptr;
    }
  }
  if (eout) {
    double *e[5] = {eout->K_lo, eout->K_hi, eout->L_lo, eout->L_hi, eout->dL_hi};
    for (int r = 0; r < 5; ++r) {
      dst[4 + r] = e[r];
      rows.p[4 + r] = e[r] ? (const unsigned long long *)(p->env + r * NB) : nullptr;
    }
  }
  uint32_t err = 0;
  s = collect_stats(p, st, (uint32_t)m + 1, (uint32_t)n, &err, &rows);
  if (s != RIPK_OK) return s;
  if (err) return err_status(err);
  if (cross) {
    p->split_n = n;
    p->split_n1 = nc;
  }
  for (int r = 0; r < kPackRows; ++r)
    if (dst[r]) std::memcpy(dst[r], p->hstage + kScalWords + r * NB, 8 * NB);
  if (eout && (eout->C_sims || eout->W_sims || eout->K_sims)) {
    if (eout->C_sims)
      HIPCHK(hipMemcpyAsync(eout->C_sims, p->outC + NB, 8 * NB * m, hipMemcpyDeviceToHost, st));
    if (eout->W_sims)
      HIPCHK(hipMemcpyAsync(eout->W_sims, p->outW + NB, 8 * NB * m, hipMemcpyDeviceToHost, st));
    if (eout->K_sims)
      HIPCHK(hipMemcpyAsync(eout->K_sims, p->outK + NB, 8 * NB * m, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  p->stats.us_total = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  return RIPK_OK;
}

ripk_status ripk_plan_get_info(ripk_plan_t p, ripk_plan_info *out) {
  if (!p || !out) return fail(RIPK_EINVAL, "null plan or output");
  *out = p->lay.info;
  return RIPK_OK;
}

ripk_status ripk_plan_stats(ripk_plan_t p, ripk_stats *out) {
  if (!p || !out) return fail(RIPK_EINVAL, "null plan or output");
  *out = p->stats;
  return RIPK_OK;
}

ripk_status ripk_device_query(int32_t device, ripk_device_props *out) {
  if (!out) return fail(RIPK_EINVAL, "null output");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(RIPK_EDEVICE, "hipGetDeviceProperties failed for device %d", device);
  std::memset(out, 0, sizeof *out);
  out->compute_units = prop.multiProcessorCount;
  out->clock_khz = prop.clockRate;
  out->lds_per_cu_bytes = (int64_t)prop.maxSharedMemoryPerMultiProcessor;
  out->hbm_bytes = (int64_t)prop.totalGlobalMem;
  out->wavefront = prop.warpSize;
  std::strncpy(out->arch, prop.gcnArchName, sizeof out->arch - 1);
  return RIPK_OK;
}

ripk_status ripk_plan_set_flush_bound(ripk_plan_t p, int64_t candidates) {
  if (!p) return fail(RIPK_EINVAL, "null plan");
  if (candidates < 0) return fail(RIPK_EINVAL, "flush bound must be >= 0");
  // (a bound at or above the smallest default selects the layout's default)
  p->flush_evals = candidates >= (1LL << 29) ? 0u : (uint64_t)candidates;
  ++p->bind_gen;  // a captured graph holds the old bound
  return RIPK_OK;
}

}  // extern "C"
