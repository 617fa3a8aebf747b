/*
 * ripk.h -- C ABI of the MI355X (gfx950) space-time Ripley's K library.
 *
 * The library evaluates the space-time K function of Wang et al.,
 * "Distributed space-time Ripley's K function" (arXiv 1912.04753), Sec. 3:
 *
 *   K(s,t) = A*D/N * sum_i sum_{j!=i} I(d_ij <= s, u_ij <= t) / (omega_ij v_ij)  (Eq. 2, 3)
 *   L(s,t) = sqrt(K(s,t) / (2 pi t)) - s                                          (Eq. 4)
 *
 * with Ripley's isotropic spatial correction omega_ij (share of the circle
 * centred on i with radius d_ij inside the study rectangle) and the temporal
 * correction v_ij (1 if [t_i-u_ij, t_i+u_ij] lies in the study period, else
 * 1/2), on the grid s_k = k*s_max/n_s, t_l = l*t_max/n_t (k, l >= 1), and the
 * Monte Carlo CSR simulation envelopes used to judge significance (Sec. 3).
 *
 * Conventions shared by every call
 *  - Every call returns a ripk_status and never throws.  On an error no
 *    output buffer is written; ripk_last_error() gives a detail string for the
 *    calling thread.
 *  - Coordinates are int32 metres (x, y) and int32 seconds (t).  d_ij^2 and u_ij
 *    are exact integers, so pair counts are exact; weights 1/(omega v) are
 *    computed in FP32 and summed in 128-bit fixed point with 23 fractional bits,
 *    so weighted sums do not depend on summation order.  K and L are FP64.
 *  - Grids are s-major: element (k, l) (0-based) sits at index k*n_t + l.
 *  - A plan is used by one thread at a time.  Handles are created and freed by
 *    the library; caller buffers are never retained after a call returns.
 *  - `stream` is a hipStream_t (NULL = the null stream of the plan's device).
 *    All calls return only after their results are in the caller's buffers.
 */
#ifndef RIPK_H
#define RIPK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ripk_status;
enum {
  RIPK_OK = 0,
  RIPK_PENDING = 1,       /* request not finished yet (ripk_poll)                    */
  RIPK_EINVAL = -1,       /* bad argument: see ripk_last_error()                     */
  RIPK_ERANGE = -2,       /* a point lies outside the closed study window            */
  RIPK_ENOMEM = -3,       /* device or host allocation failed                        */
  RIPK_EDEVICE = -4,      /* HIP runtime error                                       */
  RIPK_E2BIG = -5,        /* request larger than the plan's / server's capacity      */
  RIPK_EAGAIN = -6,       /* server queue full, try again                            */
  RIPK_EOVERFLOW = -7,    /* an accumulator bound would be exceeded                  */
  RIPK_ECANCELED = -8,    /* request cancelled by server shutdown                    */
  RIPK_ENOTFOUND = -9     /* unknown ticket                                          */
};

/* edge-correction bits (Sec. 3): omega_ij and v_ij can be switched on separately */
#define RIPK_EDGE_SPATIAL_ISO 1u
#define RIPK_EDGE_TEMPORAL 2u
#define RIPK_EDGE_ISO 3u

/* normalisation N of Eq. 2: n(n-1) (unbiased under CSR, default) or n^2 as printed */
#define RIPK_NORM_NN1 0u
#define RIPK_NORM_N2 1u

/* simulation methods (Sec. 3).  CSR: Monte Carlo under complete spatio-temporal
 * randomness, drawn on the device (see ripk_simulate_envelope).  PERMUTE: a copy
 * of the observed points with their time labels exchanged at random; set s
 * gives point k the time of observed point order_s[k], where order_s lists the
 * points by increasing high 32 bits of word 0 of Philox4x64-10(counter
 * (j, s, 0, 0), key (seed, 1)), equal values by index.  BOOTSTRAP: points drawn
 * with replacement; point k of set s is observed point floor(r0 * n / 2^64),
 * r = Philox4x64-10((k, s, 0, 0), (seed, 2)).  PERMUTE and BOOTSTRAP draw from
 * the observed set of the plan's last successful ripk_compute_K. */
/* With RIPK_PLAN_CROSS, BOOTSTRAP point k < n1 is observed point
 * floor(r0 * n1 / 2^64) and point k >= n1 is n1 + floor(r0 * (n - n1) / 2^64). */
#define RIPK_SIM_CSR 0u
#define RIPK_SIM_PERMUTE 1u
#define RIPK_SIM_BOOTSTRAP 2u

/* plan flags */
#define RIPK_PLAN_ORDERED (1u << 0) /* evaluate ordered pairs (full stencil) even when   */
                                    /* every point is a centre; default: each unordered */
                                    /* pair once, both weights added                    */
#define RIPK_PLAN_TIMING (1u << 1)  /* record per-phase device timings for stats         */
#define RIPK_PLAN_WIDE_COUNTS (1u << 2) /* 64-bit pair counters in the pair kernel's     */
                                        /* workgroup histograms (automatic for sets of  */
                                        /* 2^23 points or more; results are identical)  */
#define RIPK_PLAN_AUTOTUNE (1u << 3)    /* pick the cell grid by timing: the first      */
                                        /* ripk_compute_K times each candidate cell     */
                                        /* subdivision on its own input, the first      */
                                        /* ripk_simulate_envelope on up to 32 of its    */
                                        /* simulations; cell_div/tcell_div are ignored; */
                                        /* results do not depend on the cells            */
#define RIPK_PLAN_GRAPH (1u << 4)       /* on a non-null stream and without             */
                                        /* RIPK_PLAN_TIMING: capture a call's launch    */
                                        /* sequence into a HIP graph and replay it      */
                                        /* while the call shape (sizes, input pointers, */
                                        /* seed, geometry) repeats                      */
#define RIPK_PLAN_CROSS (1u << 5)       /* two-type (cross, bivariate) K, the first     */
                                        /* extension named in Sec. 7: see below         */
#define RIPK_PLAN_INHOM (1u << 6)       /* inhomogeneous K, the second extension named  */
                                        /* in Sec. 7: see below                         */
#define RIPK_PLAN_COST_ORDER (1u << 8)  /* a launch whose work items are split (few    */
                                        /* sets) hands out its groups of items in      */
                                        /* descending order of estimated candidates,   */
                                        /* dealt over the work-queue partitions, so    */
                                        /* that dense clusters do not end the launch   */
                                        /* (costs a sort of the groups; taken when     */
                                        /* they are fewer than the launch's points).   */
                                        /* Without this                                */
                                        /* flag an autotuned plan times its chosen     */
                                        /* single-set geometry with and without the    */
                                        /* order and keeps the faster; results do not  */
                                        /* depend on it                                */
#define RIPK_PLAN_SPLIT_RUNS (1u << 7)  /* a single-set launch that wants more work     */
                                        /* items than stencil rows also cuts each row's */
                                        /* neighbour run into equal fractions (uneven,  */
                                        /* clustered sets).  Without this flag, an      */
                                        /* autotuned plan times its first single-set    */
                                        /* ripk_compute_K with and without fractions    */
                                        /* and keeps the faster; results do not depend  */
                                        /* on it                                        */

/*
 * Inhomogeneous K.  With RIPK_PLAN_INHOM, ripk_compute_K reads an intensity
 * lambda_i > 0 (finite) for every point (ripk_points.lambda; RIPK_EINVAL when
 * NULL, RIPK_ERANGE when a value is not positive and finite) and computes
 *   K_I(s,t) = 1/(A*D) * sum_i sum_{j!=i} I(d_ij <= s, u_ij <= t) / (omega_ij v_ij lambda_i lambda_j),
 * which is Eq. 2 with N = n^2 when lambda is the constant n/(A*D); L_I follows
 * as in Eq. 4, and C counts pairs as usual.  The norm field is ignored.  Every
 * lambda must lie in [2^-400, 2^400] (RIPK_ERANGE otherwise).  Each side's
 * weight w/(lambda_i lambda_j) (w the FP32 weight of the homogeneous path) is
 * rounded in FP64 to a multiple of 2^-F and the multiples are summed exactly,
 * so W, K and L are bitwise identical across runs, launch shapes and symmetric
 * or ordered evaluation.  F is taken per call from the largest 1/lambda, so
 * that one pair stays below 2^B units with B = min(93, 126 - ceil(log2(n(n-1))))
 * (B >= 82 for n < 2^22): the rounding adds a relative error below
 * 2^(5-B) (lambda_max/lambda_min)^2 to a bin.  n_max must be below 2^22.
 * Such plans take a rectangle (no polygon), one point type (no
 * RIPK_PLAN_CROSS) and no simulations: the null model, a Poisson process of
 * intensity lambda, needs the intensity as a function, not at the points
 * (ripk_simulate_envelope returns RIPK_EINVAL).
 */

/*
 * Cross K.  With RIPK_PLAN_CROSS the points of ripk_compute_K carry two types:
 * type 1 = points [0, n_centres) (1 <= n_centres < n), type 2 = the rest, and
 *   K12(s,t) = A*D/(n1*n2) * sum_{i in 1} sum_{j in 2} I(d_ij <= s, u_ij <= t) / (omega_ij v_ij)
 * with both corrections centred on the type-1 point i (the weights of Eq. 2);
 * L12 follows from K12 as in Eq. 4 and C counts the ordered cross pairs.  The
 * norm field is ignored (the normaliser is n1*n2).  ripk_simulate_envelope
 * keeps the type split of the plan's last successful ripk_compute_K (RIPK_EINVAL
 * before one, or for another n): CSR sets take their first n1 points as type 1,
 * PERMUTE exchanges time labels over all points (types stay with locations),
 * BOOTSTRAP draws each type from itself (see RIPK_SIM_BOOTSTRAP).
 */

/*
 * Problem statement (the job parameters of Sec. 4.1 and the GUI of Sec. 5:
 * study area, period, spatial/temporal thresholds and steps, edge correction,
 * simulation method and count).
 *
 * Requirements (RIPK_EINVAL otherwise):
 *   x0 < x1, y0 < y1, t0 < t1, all within int32; x1-x0 and y1-y0 < 2^24;
 *   t1-t0 < 2^31;  1 <= n_s, n_t <= 64;  s_max >= 1;  1 <= t_max < 2^30;
 *   with RIPK_EDGE_SPATIAL_ISO: 2*s_max <= min(x1-x0, y1-y0) (so omega >= 1/4);
 *   with RIPK_EDGE_TEMPORAL:   t_max <= t1-t0;
 *   s_max < 2^23;  n_max >= 2;  0 <= m_max;  (m_max+1)*n_max < 2^31.
 */
typedef struct {
  int64_t x0, y0, x1, y1; /* closed study rectangle [x0,x1] x [y0,y1], metres     */
  int64_t t0, t1;         /* closed study period [t0,t1], seconds                 */
  int64_t s_max, t_max;   /* largest spatial / temporal distance of the grid      */
  int32_t n_s, n_t;       /* number of grid steps in s and in t                    */
  uint32_t edge;          /* RIPK_EDGE_* bits                                      */
  uint32_t norm;          /* RIPK_NORM_*                                           */
  uint32_t sim_method;    /* RIPK_SIM_CSR                                          */
  int64_t n_max;          /* capacity: largest point count per set                 */
  int32_t m_max;          /* capacity: largest simulation count per call           */
  uint32_t flags;         /* RIPK_PLAN_* bits                                      */
  int32_t device;         /* HIP device ordinal                                    */
  int32_t cell_div;       /* spatial cells per s_max (0 = library default)         */
  int32_t tcell_div;      /* temporal cells per t_max (0 = library default)        */
  const int32_t *poly;    /* optional polygon study area, see below (NULL: none)   */
  int32_t poly_n;         /* its vertex count (0: the rectangle is the study area) */
  int32_t reserved;       /* 0                                                     */
} ripk_plan_desc;

/*
 * Polygon study areas (Sec. 3 defines omega for any study area; the cost of a
 * weight grows with the boundary's vertex count, Sec. 4.4).  With poly_n >= 3,
 * vertex k is (poly[2k], poly[2k+1]), the boundary closes from the last vertex
 * to the first, and the polygon replaces the rectangle as the study area:
 *   - it must be simple (edges meet only at shared vertices), lie inside the
 *     rectangle [x0,x1] x [y0,y1], have at most 4096 vertices and an area of at
 *     least 1/1024 of the rectangle's (RIPK_EINVAL otherwise);
 *   - A in Eq. 2 is its area (shoelace); every point must lie strictly inside
 *     it (RIPK_ERANGE otherwise);
 *   - omega_ij is the share of the circle centred on point i with radius d_ij
 *     that lies inside the polygon, and the spatial weight is 1/omega_ij with
 *     no cap: j lies strictly inside and on the circle, so omega_ij > 0, and
 *     on the integer lattice 1/omega_ij < pi*|E|*s_max < 2^49.2 (|E| the
 *     longest edge); each side's weight is rounded to a multiple of 2^-23 and
 *     summed exactly in 128-bit fixed point; the rule
 *     2*s_max <= min(x1-x0, y1-y0) does not apply;
 *   - with RIPK_EDGE_SPATIAL_ISO, n_max must be below 2^22 (RIPK_EINVAL);
 *   - CSR simulations draw by rejection: attempt a of point k of set s uses the
 *     Philox counter (k, s, a, 0) and the first attempt strictly inside is kept;
 *   - device memory (in ripk_plan_info.device_bytes): besides the edges and
 *     their per-cell and per-band lists, a polygon plan keeps 80 bytes per
 *     point of its largest call (S * n_max points: each point's distance range
 *     to every nearby edge, which the weight reads).
 * The vertex array is read during ripk_plan_check, ripk_plan and ripk_submit
 * and copied; the caller keeps ownership.
 */

typedef struct ripk_plan_s *ripk_plan_t;

/* Geometry a plan derives from its descriptor; filled by ripk_plan_check
 * without touching any device. */
typedef struct {
  int64_t S2[64];          /* floor((k*s_max)^2/n_s^2), k = 1..n_s (Eq. 3 on integers)   */
  int64_t T[64];           /* floor(l*t_max/n_t), l = 1..n_t                             */
  int64_t cell_s, cell_t;  /* cell edge in metres / seconds                              */
  int32_t nx, ny, nt;      /* cells per axis                                             */
  int32_t reach_s, reach_t;/* stencil half-width in cells (space, time)                  */
  int64_t n_cells;         /* nx*ny*nt                                                   */
  int32_t dist_mode;       /* distance test: 0 packed 16-bit, 1 32-bit, 2 64-bit squares */
  int32_t n_bins;          /* n_s*n_t                                                    */
  int64_t device_bytes;    /* device memory a plan of this descriptor allocates          */
  int32_t near_edges_max;  /* polygon study areas: most boundary edges listed for one
                              xy-cell (edges within s_max of it; 33 = more than 32, and
                              such a cell scans every edge); 0 for the rectangle          */
  int32_t near_cells;      /* polygon study areas: xy-cells with a nonempty edge list    */
} ripk_plan_info;

/* A point set in structure-of-arrays form.  Points [0, n_centres) act as
 * centres i of Eq. 2; points [n_centres, n) are neighbours j only (a halo,
 * as when one shard of a larger set is evaluated).  n_centres = 0 means all.
 * on_device = 1: x, y, t (and lambda) are device pointers on the plan's
 * device, ordered on the call's stream; 0: host pointers.  lambda: the
 * intensity at every point (points per m^2 per s), read by plans made with
 * RIPK_PLAN_INHOM only (NULL otherwise). */
typedef struct {
  const int32_t *x, *y, *t;
  int64_t n;
  int64_t n_centres;
  int32_t on_device;
  const double *lambda;
} ripk_points;

/* Outputs of ripk_compute_K: host buffers of n_s*n_t elements each, any may
 * be NULL.  C: cumulative ordered-pair counts; W: cumulative sums of
 * 1/(omega v); K: Eq. 2; L: Eq. 4. */
typedef struct {
  uint64_t *C;
  double *W, *K, *L;
} ripk_K_out;

/* Outputs of ripk_simulate_envelope: host buffers, any may be NULL.
 * K_lo/K_hi/L_lo/L_hi: pointwise min/max over the m simulations (n_s*n_t);
 * dL_hi: L_obs - L_hi (needs L_obs);  C_sims/W_sims/K_sims: per simulation,
 * m*n_s*n_t, simulation-major. */
typedef struct {
  double *K_lo, *K_hi, *L_lo, *L_hi, *dL_hi;
  uint64_t *C_sims;
  double *W_sims, *K_sims;
} ripk_env_out;

/* Counters and timings of the last compute call on a plan. */
typedef struct {
  int64_t n_sets;          /* point sets evaluated                                      */
  int64_t n_points;        /* points over all sets                                      */
  int64_t n_in;            /* ordered in-range pairs, summed over sets                   */
  int64_t n_eval;          /* candidate pairs the pair kernel examined                   */
  int64_t n_items;         /* work items of the pair kernel                              */
  int32_t pair_grid;       /* workgroups of the persistent pair kernel                   */
  int32_t symmetric;       /* 1 if unordered pairs were evaluated once                   */
  int32_t split;           /* parts each work item's stencil rows were split into        */
  int32_t bin_layout;      /* LDS bins of the pair kernel: 0 count and interior weight
                              in one word, 1 weight + 32-bit count, 2 weight + 64-bit
                              count, 3 count + three words of 32-bit weight pieces
                              (polygon weights, inhomogeneous K)                         */
  double us_total;         /* wall time of the call, microseconds                        */
  double us_gen, us_grid, us_pair, us_finalize; /* device phases (RIPK_PLAN_TIMING)      */
  /* RIPK_PLAN_TIMING: when the pair kernel's workgroups ended, microseconds after
   * the first one started (the device's 100 MHz real-time counter): median, 90th
   * percentile and last; and the groups of the work list, 1 if they were handed
   * out in descending order of estimated cost                                    */
  double us_wg_end_median, us_wg_end_p90, us_wg_end_max;
  int32_t cost_ordered;
  int32_t reserved;
} ripk_stats;

/* Validate a descriptor and derive its geometry; host only, no device use.
 * Returns RIPK_OK or RIPK_EINVAL. */
ripk_status ripk_plan_check(const ripk_plan_desc *desc, ripk_plan_info *info);

/* Create a plan: validate, derive thresholds and the cell grid, and allocate
 * every device buffer for n_max points and m_max simulations on desc->device
 * (m_max + 1 sets when m_max > 0: ripk_compute_K_envelope evaluates the
 * observed set in the simulations' launch).
 * Errors: EINVAL, ENOMEM, EDEVICE.  Free with ripk_plan_destroy. */
ripk_status ripk_plan(const ripk_plan_desc *desc, ripk_plan_t *out);
void ripk_plan_destroy(ripk_plan_t plan);

/* K, L of one observed point set (Eq. 2-4).  Errors: EINVAL (n < 2,
 * n > n_max, n_centres > n, NULL coordinates), ERANGE (a point outside the
 * window), EDEVICE. */
ripk_status ripk_compute_K(ripk_plan_t plan, const ripk_points *pts, void *stream,
                           ripk_K_out *out);

/* m simulations of n points each, drawn on the device by the plan's method
 * and evaluated together, with pointwise min/max envelopes (Sec. 3).  CSR uses
 * Philox4x64-10 (key = (seed, 0), counter = (point, simulation, 0, 0), x from
 * the first output word by a 64x64 multiply-high onto [x0, x1), y and t
 * likewise from the second and third); PERMUTE and BOOTSTRAP see
 * RIPK_SIM_PERMUTE.  L_obs (host, n_s*n_t, optional) gives dL_hi.
 * Errors: EINVAL (n < 2, n > n_max, m < 1, m > m_max; PERMUTE or BOOTSTRAP
 * without a previous ripk_compute_K of n points), EDEVICE. */
ripk_status ripk_simulate_envelope(ripk_plan_t plan, int64_t n, int32_t m, uint64_t seed,
                                   const double *L_obs, void *stream, ripk_env_out *out);

/* One Monte Carlo test as the paper's job runs it (Sec. 3 and 4): K, L of the
 * observed set and the envelopes of m simulations of n = pts->n points, with
 * dL_hi against the observed L.  Results equal ripk_compute_K followed by
 * ripk_simulate_envelope(..., L_obs = the observed L, ...) bit for bit.  With
 * CSR simulations the observed set is set 0 of the simulations' launch (one
 * sort, one pair-kernel launch, one copy back); PERMUTE and BOOTSTRAP plans,
 * and centre subsets without RIPK_PLAN_CROSS, run the two calls.  Either
 * output may be NULL; C_sims, W_sims, K_sims of env_out cover the m
 * simulations.  The plan's stats cover the m + 1 sets (two-call cases: the
 * simulations).  Errors: those of the two calls; EINVAL for inhomogeneous
 * plans (no simulations). */
ripk_status ripk_compute_K_envelope(ripk_plan_t plan, const ripk_points *pts, int32_t m,
                                    uint64_t seed, void *stream, ripk_K_out *k_out,
                                    ripk_env_out *env_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the K and L
 * of one observed set, as ripk_compute_K computes them on a plan made from
 * `desc`, with no plan and no allocation.  Every device buffer of the call is
 * cut from one static device array of RIPK_NOALLOC_SCRATCH_BYTES bytes, which
 * each device the library runs on holds from the library's first use on it
 * until the process ends.  Its contents stay from one call to the next; the
 * call clears what it needs cleared.
 *
 *  - desc: a rectangle study area (poly_n = 0), one point type, no
 *    intensities: flags may hold RIPK_PLAN_ORDERED, RIPK_PLAN_WIDE_COUNTS,
 *    RIPK_PLAN_SPLIT_RUNS and RIPK_PLAN_COST_ORDER only; cell_div/tcell_div as in ripk_plan (no
 *    autotuning); n_max and m_max are ignored (the call is sized by pts->n).
 *  - pts: as for ripk_compute_K (host or device coordinates; n_centres as
 *    there; lambda ignored).
 *  - out: DEVICE buffers of n_s*n_t elements on desc->device (any may be
 *    NULL), written on `stream` only when the call succeeds; the call returns
 *    after they are written.
 *  - Results are bit-identical to ripk_compute_K on a plan of the same
 *    descriptor (exact integer sums; the same FP64 finalisation).
 *  - Errors: EINVAL (as ripk_compute_K, and for a polygon, intensities,
 *    RIPK_PLAN_CROSS or other flags), E2BIG when the call's buffers (about
 *    52 bytes per point plus 1 KiB per cell of the grid) exceed the scratch
 *    array, ERANGE, EDEVICE.  Nothing is allocated on any path.
 *  - Calls that overlap on one device (from several threads, or on several
 *    streams without ordering) share the array and race: serialise them.
 */
#define RIPK_NOALLOC_SCRATCH_BYTES (64ull << 20)
ripk_status ripk_compute_K_noalloc(const ripk_plan_desc *desc, const ripk_points *pts,
                                   void *stream, ripk_K_out *out);

/* Counters and timings of the plan's last compute call. */
ripk_status ripk_plan_stats(ripk_plan_t plan, ripk_stats *out);

/* Geometry the plan's last compute call used (with RIPK_PLAN_AUTOTUNE: the
 * tuned cells). */
ripk_status ripk_plan_get_info(ripk_plan_t plan, ripk_plan_info *out);

/* The device figures the pair kernel's integer-ALU roofline is priced on
 * (compute units x 64 lanes x peak engine clock), read with
 * hipGetDeviceProperties: multiProcessorCount, clockRate (kHz),
 * maxSharedMemoryPerMultiProcessor, totalGlobalMem, warpSize, gcnArchName.
 * RIPK_EINVAL for a null output, RIPK_EDEVICE when the query fails. */
typedef struct {
  int32_t compute_units;
  int32_t clock_khz;
  int64_t lds_per_cu_bytes;
  int64_t hbm_bytes;
  int32_t wavefront;
  char arch[68];
} ripk_device_props;
ripk_status ripk_device_query(int32_t device, ripk_device_props *out);

/* Test hook for the pair kernel's histogram flush (the merge of each
 * workgroup's LDS bins into a set's global bins).  A workgroup flushes when
 * it moves on to another point set and, within a set, once it has examined
 * more candidate pairs than a bound (checked before each group of work
 * items): 2^29 or 2^31 by default, set by the fields of the LDS bins.  This
 * call lowers that bound to `candidates` for the plan's later calls (0, or
 * 2^29 and more, select the default), so that small
 * sets run the mid-set flush that only sets of millions of points reach
 * otherwise.  Results do not depend on it.  RIPK_EINVAL for a null plan or a
 * negative bound. */
ripk_status ripk_plan_set_flush_bound(ripk_plan_t plan, int64_t candidates);

/* ---- Serving ---------------------------------------------------------------
 *
 * A server evaluates requests -- an observed set's K and L and, when m > 0, its
 * m CSR simulations and envelopes (Sec. 3) -- with continuous batching on one
 * device.  It runs `slots` requests at a time, each on its own HIP stream with
 * its own device workspace, so their kernels overlap.  Queued requests are
 * admitted in arrival order as soon as a slot is idle and the request's device
 * footprint (ripk_plan_info.device_bytes of its descriptor) fits in the HBM
 * budget beside the workspaces the slots hold; idle slots give their workspaces
 * back when the budget runs short.  Results are exact integer sums, so a
 * request's outputs are bit-identical to ripk_compute_K and
 * ripk_simulate_envelope on a plan of the same descriptor, alone or in a mix.
 * All server calls are thread-safe, except that ripk_server_destroy must not
 * overlap any other call on the same server.
 */
typedef struct ripk_server_s *ripk_server_t;

/* Admission orders.  FIFO: the oldest waiting request first.  SIZE: each
 * request's work is estimated at submit as (m + 1)(n^2 f + 64 n), f the share
 * of a uniform set's ordered pairs within the thresholds; a request above
 * large_work is large.  A free slot takes the oldest request that has waited
 * longer than age_ms, else the oldest large request while fewer than
 * max_large are running, else the smallest waiting request that is not
 * large.  Either way a request is admitted once its device footprint fits
 * the HBM budget. */
enum { RIPK_ADMIT_FIFO = 0, RIPK_ADMIT_SIZE = 1 };

typedef struct {
  int32_t device;            /* HIP device ordinal                                     */
  int32_t slots;             /* requests evaluated concurrently, 1..16                 */
  int32_t queue_cap;         /* requests that may wait for admission, >= 1             */
  uint32_t admission;        /* RIPK_ADMIT_*                                           */
  int64_t hbm_budget_bytes;  /* device bytes all slot workspaces may hold together     */
  double large_work;         /* SIZE: work above which a request is large (0: 2e10)    */
  double age_ms;             /* SIZE: wait after which a request goes first (0: none)  */
  int32_t max_large;         /* SIZE: large requests running at once (0: no limit)     */
  float device_share;        /* share of a pair launch's workgroups kept while other   */
                             /* slots are busy, in (0, 1] (0: 1, no sharing)           */
  float slice_ms;            /* pair launches of a request are cut into slices of this */
                             /* length (0: none); the other slots' kernels start       */
                             /* between slices                                         */
  int32_t reserved;          /* set to 0                                               */
} ripk_server_desc;

#define RIPK_REQ_KEEP_SIMS (1u << 0) /* keep per-simulation C, W, K for ripk_poll */

/* One request.  plan: window, grid, edge correction, normalisation, flags;
 * its n_max, m_max and device are ignored (the request's n and m and the
 * server's device are used).  pts: host points (on_device must be 0), copied
 * by ripk_submit, so the caller's arrays may be reused as soon as it returns.
 * m: CSR simulations (0 = K only); seed: Philox key as in
 * ripk_simulate_envelope.  dL_hi is computed against the request's own L. */
typedef struct {
  ripk_plan_desc plan;
  ripk_points pts;
  int32_t m;
  uint32_t flags;            /* RIPK_REQ_* bits                                        */
  uint64_t seed;
} ripk_request;

/* Result of ripk_poll.  k and env are input fields: host buffers the caller
 * provides (n_s*n_t elements, per-simulation arrays m*n_s*n_t and only with
 * RIPK_REQ_KEEP_SIMS; any may be NULL).  The rest are outputs.  Times are
 * seconds on the host's CLOCK_MONOTONIC. */
typedef struct {
  ripk_K_out k;
  ripk_env_out env;
  ripk_status status;        /* the request's status                                   */
  int32_t slot;              /* slot that evaluated it (-1 if never admitted)          */
  double t_submit, t_admit, t_done;
  int64_t n_in;              /* ordered in-range pairs over the observed and simulated sets */
} ripk_result;

/* Occupancy of a server. */
typedef struct {
  int64_t queued;            /* requests waiting for admission                          */
  int64_t unpolled;          /* requests submitted and not yet collected by ripk_poll   */
  int64_t device_bytes;      /* device bytes held by slot workspaces                    */
  int32_t busy_slots;
  int32_t reserved;
} ripk_server_state;

/* Create a server: starts `slots` worker threads.  Errors: EINVAL, EDEVICE. */
ripk_status ripk_server_create(const ripk_server_desc *desc, ripk_server_t *out);

/* Cancel queued requests (ECANCELED), let admitted ones finish, free all. */
void ripk_server_destroy(ripk_server_t server);

/* Queue a request; never blocks on the device.  *ticket identifies it.
 * Errors: EINVAL (bad descriptor or points), E2BIG (footprint above the
 * budget), EAGAIN (queue full), ECANCELED (server shutting down). */
ripk_status ripk_submit(ripk_server_t server, const ripk_request *req, uint64_t *ticket);

/* Wait up to timeout_ms (0 = do not wait, < 0 = until done) for a request.
 * Returns RIPK_PENDING if it is not done; otherwise fills *out, forgets the
 * ticket and returns the request's status (ERANGE, EDEVICE, ENOMEM, ...).
 * ENOTFOUND for an unknown or already collected ticket. */
ripk_status ripk_poll(ripk_server_t server, uint64_t ticket, ripk_result *out, int32_t timeout_ms);

ripk_status ripk_server_status(ripk_server_t server, ripk_server_state *out);

const char *ripk_status_str(ripk_status s);
const char *ripk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RIPK_H */
