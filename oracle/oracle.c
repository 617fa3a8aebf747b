/*
 * oracle.c -- plain FP64 CPU reference for the space-time Ripley's K estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the HIP implementation.
 *
 * What it computes (Wang et al., "Distributed space-time Ripley's K", Sec. 3):
 *   K^(s,t) = A*D/N * sum_i sum_{j!=i} I_{s,t}(d_ij,u_ij) / (omega_ij * v_ij)   (Eq. 2)
 *   I_{s,t} = 1 iff d_ij <= s and u_ij <= t                                      (Eq. 3)
 *   omega_ij = share of the circumference of the circle centred on point i with
 *              radius d_ij that lies inside the study area (isotropic correction)
 *   v_ij     = 1 if both ends of the interval [t_i-u_ij, t_i+u_ij] lie inside the
 *              study period, 1/2 otherwise                                      (Sec. 3)
 *   L^(s,t) = sqrt(K^(s,t)/(2*pi*t)) - s                                         (Eq. 4)
 *   N = n(n-1) by default, n^2 when the literal Eq. 2 normalisation is asked for.
 *
 * The grid is s_k = k*s_max/n_s (k=1..n_s) and t_l = l*t_max/n_t (l=1..n_t).
 * Coordinates are integers (metres, seconds), so d_ij <= s_k is decided exactly
 * as d2 <= floor(s_k^2) with d2 an exact int64, and u <= t_l as
 * u <= floor(l*t_max/n_t).
 *
 * Because omega_ij and v_ij do not depend on the threshold (s,t) and the
 * indicator is monotone in s and t (Eq. 3), the sum at every grid point equals a
 * 2-D inclusive prefix sum over a histogram indexed by the smallest grid step
 * that contains the pair.  The oracle builds that histogram with a plain loop
 * over every ordered pair (i, j), i != j -- no index, no cell grid, no symmetry
 * -- and cross-checks against the literal per-(s,t) evaluation of Eq. 2 in the
 * Python test suite.
 *
 * Cross (bivariate) K, the first extension named in the paper's outlook (Sec. 7),
 * read as the usual two-type estimator: with type 1 = points [0, n1) and type
 * 2 = points [n1, n),
 *   K12^(s,t) = A*D/(n1*n2) * sum_{i in 1} sum_{j in 2} I_{s,t}(d_ij,u_ij) / (omega_ij * v_ij)
 * with both corrections centred on the type-1 point i, and L12 from K12 as in
 * Eq. 4.  The histogram loop is the same, with i over type 1 and j over type 2.
 *
 * Inhomogeneous K, the second extension named in Sec. 7 (after Baddeley,
 * Moller and Waagepetersen's estimator, in its space-time form): with an
 * intensity lambda_i > 0 given for every point,
 *   K_I^(s,t) = 1/(A*D) * sum_i sum_{j!=i} I_{s,t}(d_ij,u_ij) / (omega_ij v_ij lambda_i lambda_j),
 * L_I from K_I as in Eq. 4.  With lambda_i = n/(A*D) for all i it is Eq. 2 with
 * N = n^2.
 *
 * Polygon study areas (the general case of the isotropic correction, Sec. 3 and
 * the boundary-vertex cost of Sec. 4.4): A is the polygon's area, points lie
 * strictly inside it, omega is the share of the circle's circumference inside
 * it (arcs between crossing points, each classified by its midpoint), and the
 * spatial weight is 1/omega with no bound: omega > 0 for every pair, since the
 * neighbour j lies strictly inside the area and on the circle, so an arc about
 * j is inside.  CSR points are drawn by rejection:
 * attempt a of point i uses counter (i, sim, a, 0) and the first attempt
 * strictly inside is kept.
 *
 * Simulations (Sec. 3, Monte Carlo under complete spatio-temporal randomness):
 * n points uniform over the window, drawn from Philox4x64-10 (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) with
 * key = (seed, 0) and counter = (point, simulation, 0, 0); the three first
 * output words give x, y, t by a 64x64->128-bit multiply-high onto the
 * half-open window.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EDGE_SPATIAL 1u
#define ORC_EDGE_TEMPORAL 2u

typedef struct {
  int64_t x0, y0, x1, y1; /* closed study rectangle                      */
  int64_t t0, t1;         /* closed study period                         */
  int64_t s_max, t_max;   /* largest spatial / temporal distance          */
  int32_t n_s, n_t;       /* grid steps                                   */
  uint32_t edge;          /* bit 0: isotropic spatial, bit 1: temporal    */
  uint32_t norm;          /* 0: n(n-1), 1: n^2                            */
  const int32_t *poly;    /* optional polygon study area: vertex k at     */
                          /* (poly[2k], poly[2k+1]), closed implicitly    */
  int32_t poly_n;         /* vertex count; below 3: the rectangle         */
} orc_desc;

/* ---------------------------------------------------------------- O1 -- */
/* Integer thresholds: S2[k-1] = floor((k*s_max)^2 / n_s^2), T[l-1] =
 * floor(l*t_max/n_t).  d <= s_k  <=>  d2 <= S2[k-1] for integer d2. (Eq. 3) */
void orc_thresholds(const orc_desc *q, int64_t *S2, int64_t *T) {
  for (int k = 1; k <= q->n_s; ++k) {
    __int128 a = (__int128)k * q->s_max;
    __int128 den = (__int128)q->n_s * q->n_s;
    S2[k - 1] = (int64_t)((a * a) / den);
  }
  for (int l = 1; l <= q->n_t; ++l) T[l - 1] = ((int64_t)l * q->t_max) / q->n_t;
}

/* ---------------------------------------------------------------- O3 -- */
/* Isotropic spatial correction on the rectangle, textbook arc form.
 * Distances from (x, y) to the four sides: left, right, bottom, top.  A side
 * at distance e < r cuts an arc of half-angle acos(e/r) out of the circle; two
 * adjacent cut sides whose corner lies strictly inside the circle overlap by
 * (a_p + a_q - pi/2), which is added back once.  Valid while no two opposite
 * sides are both cut, which holds for r <= min(W, H)/2.  A zero radius gives
 * omega = 1.  (Sec. 3, isotropic correction) */
double orc_omega_poly(int64_t x, int64_t y, int64_t d2, const orc_desc *q);

double orc_omega(int64_t x, int64_t y, int64_t d2, const orc_desc *q) {
  if (!(q->edge & ORC_EDGE_SPATIAL)) return 1.0;
  if (q->poly_n >= 3) return orc_omega_poly(x, y, d2, q);
  int64_t e[4] = {x - q->x0, q->x1 - x, y - q->y0, q->y1 - y};
  int cut[4];
  double a[4];
  double r = sqrt((double)d2);
  double excluded = 0.0;
  for (int s = 0; s < 4; ++s) {
    cut[s] = (e[s] * e[s] < d2);
    a[s] = cut[s] ? acos((double)e[s] / r) : 0.0;
    excluded += 2.0 * a[s];
  }
  /* adjacent side pairs: (left,bottom) (left,top) (right,bottom) (right,top) */
  static const int P[4][2] = {{0, 2}, {0, 3}, {1, 2}, {1, 3}};
  for (int c = 0; c < 4; ++c) {
    int p = P[c][0], s = P[c][1];
    if (cut[p] && cut[s] && e[p] * e[p] + e[s] * e[s] < d2)
      excluded -= (a[p] + a[s] - M_PI / 2.0);
  }
  return 1.0 - excluded / (2.0 * M_PI);
}

/* ------------------------------------------------------------ O3 poly -- */
/* Polygon study area.  Exact integer tests for points; FP64 for the circle. */
static void orc_vertex(const orc_desc *q, int k, int64_t *x, int64_t *y) {
  k %= q->poly_n;
  *x = q->poly[2 * k];
  *y = q->poly[2 * k + 1];
}

/* 1 if (px, py) lies strictly inside the polygon (crossing number along +x with
 * the half-open rule; a point on an edge is not inside), else 0. */
int orc_poly_contains(const orc_desc *q, int64_t px, int64_t py) {
  int inside = 0;
  for (int k = 0; k < q->poly_n; ++k) {
    int64_t ax, ay, bx, by;
    orc_vertex(q, k, &ax, &ay);
    orc_vertex(q, k + 1, &bx, &by);
    const int64_t cr = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
    if (cr == 0 && px >= (ax < bx ? ax : bx) && px <= (ax > bx ? ax : bx) &&
        py >= (ay < by ? ay : by) && py <= (ay > by ? ay : by))
      return 0; /* on the boundary */
    if ((ay > py) != (by > py)) {
      /* crossing x = ax + (py - ay)(bx - ax)/(by - ay); px < crossing ? */
      const int64_t num = (py - ay) * (bx - ax), den = by - ay;
      const int64_t lhs = (px - ax) * den;
      if (den > 0 ? lhs < num : lhs > num) inside ^= 1;
    }
  }
  return inside;
}

/* the same crossing-number rule for a point with real coordinates */
static int orc_poly_contains_f(const orc_desc *q, double px, double py) {
  int inside = 0;
  for (int k = 0; k < q->poly_n; ++k) {
    int64_t ax, ay, bx, by;
    orc_vertex(q, k, &ax, &ay);
    orc_vertex(q, k + 1, &bx, &by);
    if (((double)ay > py) != ((double)by > py)) {
      const double xc = (double)ax + (py - (double)ay) * (double)(bx - ax) / (double)(by - ay);
      if (px < xc) inside ^= 1;
    }
  }
  return inside;
}

/* area by the shoelace formula */
double orc_poly_area(const orc_desc *q) {
  int64_t x0, y0, acc = 0;
  orc_vertex(q, 0, &x0, &y0);
  for (int k = 0; k < q->poly_n; ++k) {
    int64_t ax, ay, bx, by;
    orc_vertex(q, k, &ax, &ay);
    orc_vertex(q, k + 1, &bx, &by);
    acc += (ax - x0) * (by - y0) - (bx - x0) * (ay - y0);
  }
  return 0.5 * (double)(acc < 0 ? -acc : acc);
}

static int orc_dbl_cmp(const void *a, const void *b) {
  const double u = *(const double *)a, v = *(const double *)b;
  return u < v ? -1 : (u > v ? 1 : 0);
}

/* Share of the circle centred on (x, y) with radius sqrt(d2) inside the
 * polygon: every crossing of the circle with an edge (closed segment; the
 * discriminant exact in 128-bit integers), sorted by angle; each arc between
 * consecutive crossings counts when its midpoint is inside. */
double orc_omega_poly(int64_t x, int64_t y, int64_t d2, const orc_desc *q) {
  if (d2 == 0) return 1.0;
  const double r = sqrt((double)d2);
  int cap = 2 * q->poly_n + 2, m = 0;
  double *ang = (double *)malloc(sizeof(double) * (size_t)cap);
  if (!ang) return -1.0;
  for (int k = 0; k < q->poly_n; ++k) {
    int64_t ax, ay, bx, by;
    orc_vertex(q, k, &ax, &ay);
    orc_vertex(q, k + 1, &bx, &by);
    const int64_t Ax = ax - x, Ay = ay - y, Ex = bx - ax, Ey = by - ay;
    /* |A + s E|^2 = d2:  ee s^2 + 2 ae s + (aa - d2) = 0 */
    const __int128 ee = (__int128)Ex * Ex + (__int128)Ey * Ey;
    const __int128 ae = (__int128)Ax * Ex + (__int128)Ay * Ey;
    const __int128 aa = (__int128)Ax * Ax + (__int128)Ay * Ay;
    if (ee == 0) continue;
    const __int128 disc = ae * ae - ee * (aa - d2);
    if (disc < 0) continue;
    const long double sq = sqrtl((long double)disc);
    for (int sg = -1; sg <= 1; sg += 2) {
      const long double sp = (-(long double)ae + sg * sq) / (long double)ee;
      if (sp < -1e-12L || sp > 1.0L + 1e-12L) continue;
      const double cx = (double)((long double)Ax + sp * (long double)Ex);
      const double cy = (double)((long double)Ay + sp * (long double)Ey);
      double th = atan2(cy, cx);
      if (th < 0) th += 2.0 * M_PI;
      ang[m++] = th;
      if (disc == 0) break;
    }
  }
  double inside = 0.0;
  if (m == 0) {
    inside = orc_poly_contains_f(q, (double)x + r, (double)y) ? 2.0 * M_PI : 0.0;
  } else {
    qsort(ang, (size_t)m, sizeof(double), orc_dbl_cmp);
    for (int k = 0; k < m; ++k) {
      const double a0 = ang[k], a1 = (k + 1 < m) ? ang[k + 1] : ang[0] + 2.0 * M_PI;
      if (a1 - a0 <= 0.0) continue;
      const double mid = 0.5 * (a0 + a1);
      if (orc_poly_contains_f(q, (double)x + r * cos(mid), (double)y + r * sin(mid)))
        inside += a1 - a0;
    }
  }
  free(ang);
  return inside / (2.0 * M_PI);
}

/* ---------------------------------------------------------------- O4 -- */
/* Temporal correction: 1 if t-u and t+u both lie in [t0, t1], else 1/2. */
double orc_vt(int64_t t, int64_t u, const orc_desc *q) {
  if (!(q->edge & ORC_EDGE_TEMPORAL)) return 1.0;
  return (t - u >= q->t0 && t + u <= q->t1) ? 1.0 : 0.5;
}

/* Neumaier-compensated accumulation of v into (sum, comp). */
static inline void neumaier(double *sum, double *comp, double v) {
  double s = *sum, t = s + v;
  if (fabs(s) >= fabs(v))
    *comp += (s - t) + v;
  else
    *comp += (v - t) + s;
  *sum = t;
}

/* ------------------------------------------------------------ O2, O5, O6 */
/* Histogram over every ordered pair (i, j), i != j, with i < n_centres acting
 * as the centre and j in [j_begin, n).  Hc[(k-1)*n_t + (l-1)] counts pairs
 * whose smallest containing grid step is (k, l); Hw holds the matching sum of
 * 1/(omega*v) in FP64 with Neumaier compensation (per thread, then merged).
 * Returns 0, or -1 on bad arguments / allocation failure. */
static int orc_hist_range(const orc_desc *q, const int32_t *x, const int32_t *y,
                          const int32_t *t, const double *rho, int64_t n, int64_t n_centres,
                          int64_t j_begin, int nthreads, uint64_t *Hc, double *Hw) {
  if (!q || q->n_s < 1 || q->n_t < 1 || n < 0 || n_centres < 0 || n_centres > n ||
      j_begin < 0 || j_begin > n)
    return -1;
  const int ns = q->n_s, nt = q->n_t, nb = ns * nt;
  int64_t S2[4096], T[4096];
  if (ns > 4096 || nt > 4096) return -1;
  orc_thresholds(q, S2, T);
  const int64_t s2max = S2[ns - 1], tmax = T[nt - 1];
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
  nthreads = 1;
#endif
  uint64_t *pc = (uint64_t *)calloc((size_t)nthreads * nb, sizeof(uint64_t));
  double *ps = (double *)calloc((size_t)nthreads * nb, sizeof(double));
  double *pe = (double *)calloc((size_t)nthreads * nb, sizeof(double));
  if (!pc || !ps || !pe) {
    free(pc); free(ps); free(pe);
    return -1;
  }
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    uint64_t *c = pc + (size_t)tid * nb;
    double *s = ps + (size_t)tid * nb;
    double *e = pe + (size_t)tid * nb;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < n_centres; ++i) {
      const int64_t xi = x[i], yi = y[i], ti = t[i];
      for (int64_t j = j_begin; j < n; ++j) {
        if (j == i) continue;
        int64_t dx = xi - x[j], dy = yi - y[j], dt = ti - t[j];
        int64_t d2 = dx * dx + dy * dy;
        int64_t u = dt < 0 ? -dt : dt;
        if (d2 > s2max || u > tmax) continue;
        int k = 0;
        while (d2 > S2[k]) ++k; /* smallest k with d2 <= S2[k] */
        int l = 0;
        while (u > T[l]) ++l;
        /* spatial weight 1/omega (Sec. 3; omega >= 1/4 on a rectangle) */
        const double om = orc_omega(xi, yi, d2, q);
        double w = 1.0 / (om * orc_vt(ti, u, q));
        if (rho) w *= rho[i] * rho[j]; /* inhomogeneous: 1/(lambda_i lambda_j) */
        c[k * nt + l] += 1;
        neumaier(&s[k * nt + l], &e[k * nt + l], w);
      }
    }
  }
  for (int b = 0; b < nb; ++b) {
    uint64_t cc = 0;
    double sum = 0.0, comp = 0.0;
    for (int th = 0; th < nthreads; ++th) {
      cc += pc[(size_t)th * nb + b];
      neumaier(&sum, &comp, ps[(size_t)th * nb + b]);
      neumaier(&sum, &comp, pe[(size_t)th * nb + b]);
    }
    Hc[b] = cc;
    Hw[b] = sum + comp;
  }
  free(pc); free(ps); free(pe);
  return 0;
}

/* every point a neighbour: the univariate histogram of Eq. 2 */
int orc_hist(const orc_desc *q, const int32_t *x, const int32_t *y, const int32_t *t,
             int64_t n, int64_t n_centres, int nthreads, uint64_t *Hc, double *Hw) {
  return orc_hist_range(q, x, y, t, NULL, n, n_centres, 0, nthreads, Hc, Hw);
}

/* cross histogram: centres i in [0, n1), neighbours j in [n1, n) */
int orc_hist_cross(const orc_desc *q, const int32_t *x, const int32_t *y, const int32_t *t,
                   int64_t n, int64_t n1, int nthreads, uint64_t *Hc, double *Hw) {
  return orc_hist_range(q, x, y, t, NULL, n, n1, n1, nthreads, Hc, Hw);
}

/* ---------------------------------------------------------------- O7 -- */
/* 2-D inclusive prefix sum in place: C[k][l] = sum_{k'<=k, l'<=l} H[k'][l']. */
void orc_cumulate(const orc_desc *q, uint64_t *C, double *W) {
  const int ns = q->n_s, nt = q->n_t;
  for (int k = 0; k < ns; ++k)
    for (int l = 1; l < nt; ++l) {
      C[k * nt + l] += C[k * nt + l - 1];
      W[k * nt + l] += W[k * nt + l - 1];
    }
  for (int k = 1; k < ns; ++k)
    for (int l = 0; l < nt; ++l) {
      C[k * nt + l] += C[(k - 1) * nt + l];
      W[k * nt + l] += W[(k - 1) * nt + l];
    }
}

/* ------------------------------------------------------------- O8, O9 -- */
/* K = A*D*W/N (Eq. 2) and L = sqrt(K/(2*pi*t_l)) - s_k (Eq. 4), for a given
 * pair-count normaliser N. */
static void orc_normalise_by(const orc_desc *q, double N, const double *W, double *K,
                             double *L) {
  const int ns = q->n_s, nt = q->n_t;
  const double A = q->poly_n >= 3 ? orc_poly_area(q)
                                  : (double)(q->x1 - q->x0) * (double)(q->y1 - q->y0);
  const double D = (double)(q->t1 - q->t0);
  for (int k = 0; k < ns; ++k) {
    const double sk = (double)(k + 1) * (double)q->s_max / (double)ns;
    for (int l = 0; l < nt; ++l) {
      const double tl = (double)(l + 1) * (double)q->t_max / (double)nt;
      const double Kv = A * D * W[k * nt + l] / N;
      if (K) K[k * nt + l] = Kv;
      if (L) L[k * nt + l] = sqrt(Kv / (2.0 * M_PI * tl)) - sk;
    }
  }
}

/* univariate: N = n(n-1), or n^2 with the literal Eq. 2 normalisation */
void orc_normalise(const orc_desc *q, int64_t n, const double *W, double *K, double *L) {
  orc_normalise_by(q, q->norm == 1 ? (double)n * (double)n : (double)n * (double)(n - 1), W, K,
                   L);
}

/* Whole estimator for one point set: cumulative counts C, cumulative weight
 * sums W, K and L (each n_s*n_t, s-major).  Any output may be NULL. */
int orc_estimate(const orc_desc *q, const int32_t *x, const int32_t *y, const int32_t *t,
                 int64_t n, int64_t n_centres, int nthreads, uint64_t *C, double *W,
                 double *K, double *L) {
  const int nb = q->n_s * q->n_t;
  uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * nb);
  double *w = (double *)malloc(sizeof(double) * nb);
  if (!c || !w) {
    free(c); free(w);
    return -1;
  }
  int rc = orc_hist(q, x, y, t, n, n_centres, nthreads, c, w);
  if (rc == 0) {
    orc_cumulate(q, c, w);
    orc_normalise(q, n, w, K, L);
    if (C) memcpy(C, c, sizeof(uint64_t) * nb);
    if (W) memcpy(W, w, sizeof(double) * nb);
  }
  free(c); free(w);
  return rc;
}

/* Cross estimator: type 1 = points [0, n1), type 2 = [n1, n); K12 = A*D*W/(n1*n2). */
int orc_estimate_cross(const orc_desc *q, const int32_t *x, const int32_t *y, const int32_t *t,
                       int64_t n, int64_t n1, int nthreads, uint64_t *C, double *W, double *K,
                       double *L) {
  if (n1 < 1 || n1 >= n) return -1;
  const int nb = q->n_s * q->n_t;
  uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * nb);
  double *w = (double *)malloc(sizeof(double) * nb);
  if (!c || !w) {
    free(c); free(w);
    return -1;
  }
  int rc = orc_hist_cross(q, x, y, t, n, n1, nthreads, c, w);
  if (rc == 0) {
    orc_cumulate(q, c, w);
    orc_normalise_by(q, (double)n1 * (double)(n - n1), w, K, L);
    if (C) memcpy(C, c, sizeof(uint64_t) * nb);
    if (W) memcpy(W, w, sizeof(double) * nb);
  }
  free(c); free(w);
  return rc;
}

/* Inhomogeneous estimator: every ordered pair weighted by 1/(lambda_i lambda_j);
 * K_I = W/(A*D) (Eq. 2 with A*D/N replaced by 1/(A*D)). */
int orc_estimate_inhom(const orc_desc *q, const int32_t *x, const int32_t *y, const int32_t *t,
                       const double *lambda, int64_t n, int nthreads, uint64_t *C, double *W,
                       double *K, double *L) {
  const int nb = q->n_s * q->n_t;
  uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * nb);
  double *w = (double *)malloc(sizeof(double) * nb);
  double *rho = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  int rc = (c && w && rho) ? 0 : -1;
  for (int64_t i = 0; rc == 0 && i < n; ++i) {
    if (!(lambda[i] > 0.0)) rc = -1;
    rho[i] = 1.0 / lambda[i];
  }
  if (rc == 0) rc = orc_hist_range(q, x, y, t, rho, n, n, 0, nthreads, c, w);
  if (rc == 0) {
    orc_cumulate(q, c, w);
    const double A = q->poly_n >= 3 ? orc_poly_area(q)
                                    : (double)(q->x1 - q->x0) * (double)(q->y1 - q->y0);
    const double AD = A * (double)(q->t1 - q->t0);
    orc_normalise_by(q, AD * AD, w, K, L);
    if (C) memcpy(C, c, sizeof(uint64_t) * nb);
    if (W) memcpy(W, w, sizeof(double) * nb);
  }
  free(c); free(w); free(rho);
  return rc;
}

/* ---------------------------------------------------------------- O10 - */
/* 64x64 -> 128-bit product, high word. */
static inline uint64_t mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

/* Philox4x64 with 10 rounds (Salmon et al., SC'11).  One round maps counter
 * (c0,c1,c2,c3) with key (k0,k1) to
 *   (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
 * and the key advances by the Weyl constants between rounds. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0 = mulhi64(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = mulhi64(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* CSR simulation `sim` of n points: point i takes Philox(counter=(i,sim,0,0),
 * key=(seed,0)); x = x0 + floor(r0*(x1-x0)/2^64), likewise y with r1 and t
 * with r2 over [t0, t1).  With a polygon, attempts a = 0, 1, ... use counter
 * (i, sim, a, 0) until the point lies strictly inside. */
void orc_csr_points(int64_t n, int64_t sim, uint64_t seed, const orc_desc *q, int32_t *x,
                    int32_t *y, int32_t *t) {
  const uint64_t W = (uint64_t)(q->x1 - q->x0), H = (uint64_t)(q->y1 - q->y0),
                 D = (uint64_t)(q->t1 - q->t0);
  const uint64_t key[2] = {seed, 0};
  for (int64_t i = 0; i < n; ++i) {
    for (uint64_t a = 0;; ++a) {
      uint64_t ctr[4] = {(uint64_t)i, (uint64_t)sim, a, 0}, r[4];
      orc_philox4x64_10(ctr, key, r);
      x[i] = (int32_t)(q->x0 + (int64_t)mulhi64(r[0], W));
      y[i] = (int32_t)(q->y0 + (int64_t)mulhi64(r[1], H));
      t[i] = (int32_t)(q->t0 + (int64_t)mulhi64(r[2], D));
      if (q->poly_n < 3 || orc_poly_contains(q, x[i], y[i])) break;
    }
  }
}

/* Random permutation (Sec. 3): a copy of the observed points whose temporal
 * labels are exchanged at random.  Simulation `sim` keeps every location and
 * gives point i the time of point order[i], where order lists the points by
 * increasing u_j = high 32 bits of word 0 of Philox(counter=(j,sim,0,0),
 * key=(seed,1)), equal u by index. */
typedef struct {
  uint32_t u;
  int64_t i;
} orc_rank;

static int orc_rank_cmp(const void *a, const void *b) {
  const orc_rank *p = (const orc_rank *)a, *q = (const orc_rank *)b;
  if (p->u != q->u) return p->u < q->u ? -1 : 1;
  return p->i < q->i ? -1 : (p->i > q->i ? 1 : 0);
}

int orc_permute_points(const int32_t *x, const int32_t *y, const int32_t *t, int64_t n,
                       int64_t sim, uint64_t seed, int32_t *xs, int32_t *ys, int32_t *ts) {
  orc_rank *r = (orc_rank *)malloc(sizeof(orc_rank) * (size_t)(n > 0 ? n : 1));
  if (!r) return -1;
  const uint64_t key[2] = {seed, 1};
  for (int64_t j = 0; j < n; ++j) {
    uint64_t ctr[4] = {(uint64_t)j, (uint64_t)sim, 0, 0}, w[4];
    orc_philox4x64_10(ctr, key, w);
    r[j].u = (uint32_t)(w[0] >> 32);
    r[j].i = j;
  }
  qsort(r, (size_t)n, sizeof(orc_rank), orc_rank_cmp);
  for (int64_t i = 0; i < n; ++i) {
    xs[i] = x[i];
    ys[i] = y[i];
    ts[i] = t[r[i].i];
  }
  free(r);
  return 0;
}

/* Bootstrap (Sec. 3): points sampled at random with replacement from the
 * observed points.  Point i of simulation `sim` is observed point
 * floor(r0 * n / 2^64), r = Philox(counter=(i,sim,0,0), key=(seed,2)).  With
 * two types (n1 < n) each type is resampled from itself: point i < n1 is
 * observed point floor(r0 * n1 / 2^64), point i >= n1 is observed point
 * n1 + floor(r0 * (n - n1) / 2^64). */
void orc_bootstrap_points_typed(const int32_t *x, const int32_t *y, const int32_t *t, int64_t n,
                                int64_t n1, int64_t sim, uint64_t seed, int32_t *xs,
                                int32_t *ys, int32_t *ts) {
  const uint64_t key[2] = {seed, 2};
  for (int64_t i = 0; i < n; ++i) {
    uint64_t ctr[4] = {(uint64_t)i, (uint64_t)sim, 0, 0}, w[4];
    orc_philox4x64_10(ctr, key, w);
    const int64_t j = i < n1 ? (int64_t)mulhi64(w[0], (uint64_t)n1)
                             : n1 + (int64_t)mulhi64(w[0], (uint64_t)(n - n1));
    xs[i] = x[j];
    ys[i] = y[j];
    ts[i] = t[j];
  }
}

void orc_bootstrap_points(const int32_t *x, const int32_t *y, const int32_t *t, int64_t n,
                          int64_t sim, uint64_t seed, int32_t *xs, int32_t *ys, int32_t *ts) {
  orc_bootstrap_points_typed(x, y, t, n, n, sim, seed, xs, ys, ts);
}

/* Simulation envelope: for sims 0..m-1, draw the CSR set, estimate K and L,
 * and keep the pointwise minimum and maximum over the simulations (Sec. 3).
 * Per-simulation C, W, K (m*n_s*n_t each) are returned when asked for. */
int orc_envelope(const orc_desc *q, int64_t n, int64_t m, uint64_t seed, int nthreads,
                 double *K_lo, double *K_hi, double *L_lo, double *L_hi, uint64_t *C_sims,
                 double *W_sims, double *K_sims) {
  const int nb = q->n_s * q->n_t;
  int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *y = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *t = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * nb);
  double *W = (double *)malloc(sizeof(double) * nb);
  double *K = (double *)malloc(sizeof(double) * nb);
  double *L = (double *)malloc(sizeof(double) * nb);
  int rc = (x && y && t && C && W && K && L) ? 0 : -1;
  for (int64_t s = 0; rc == 0 && s < m; ++s) {
    orc_csr_points(n, s, seed, q, x, y, t);
    rc = orc_estimate(q, x, y, t, n, n, nthreads, C, W, K, L);
    if (rc) break;
    for (int b = 0; b < nb; ++b) {
      if (s == 0 || K[b] < K_lo[b]) K_lo[b] = K[b];
      if (s == 0 || K[b] > K_hi[b]) K_hi[b] = K[b];
      if (s == 0 || L[b] < L_lo[b]) L_lo[b] = L[b];
      if (s == 0 || L[b] > L_hi[b]) L_hi[b] = L[b];
    }
    if (C_sims) memcpy(C_sims + (size_t)s * nb, C, sizeof(uint64_t) * nb);
    if (W_sims) memcpy(W_sims + (size_t)s * nb, W, sizeof(double) * nb);
    if (K_sims) memcpy(K_sims + (size_t)s * nb, K, sizeof(double) * nb);
  }
  free(x); free(y); free(t); free(C); free(W); free(K); free(L);
  return rc;
}

/* Wall-clock seconds (steady), for the CPU-baseline timing. */
double orc_now(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
