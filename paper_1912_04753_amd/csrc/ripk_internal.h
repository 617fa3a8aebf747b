// Internal interfaces between the host runtime (api.cpp) and the gfx950
// kernels (*.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ripk.h"

namespace ripk {

constexpr int kMaxSteps = 64;      // n_s, n_t <= 64
constexpr int kChunk = 64;         // centres per work item = one wavefront
constexpr int kItemsPerGroup = 4;  // work items grabbed together by one workgroup
constexpr int kPairThreads = 256;  // workgroup size of the pair kernel (4 wavefronts)
constexpr int kFracBits = 23;      // fixed-point fraction bits of the weight sums
constexpr int kItemExtent = 2;     // a row item's centres lie in at most 1 + kItemExtent
                                   // consecutive x-cells (bounds the candidate |dx|)

// Arithmetic of the candidate distance test (chosen per plan from the largest
// coordinate difference a stencil can hold).
constexpr int kModePacked = 0;  // 16-bit packed x/y differences, |dx|, |dy| < 2^15
constexpr int kModeU32 = 1;     // 32-bit squared distances
constexpr int kModeWide = 2;    // 64-bit squared distances

// Geometry and thresholds shared by the grid and pair kernels (by value).
struct Geom {
  int32_t x0, y0, x1, y1, t0, t1;  // closed window; all coordinates are int32
  int32_t cell_s, cell_t;          // cell edge (metres, seconds)
  int32_t nx, ny, nt;              // cells per axis
  int32_t rs, rt;                  // stencil half-width in cells
  uint32_t n_cells;                // nx*ny*nt
  int32_t n_s, n_t;
  uint32_t edge;
  int32_t mode;                    // kModePacked / kModeU32 / kModeWide
  uint64_t s2max;                  // S2[n_s-1]
  uint32_t tmax;                   // T[n_t-1]
  float inv_ds;                    // n_s / s_max * (1 - 2^-20)
  float inv_dt;                    // n_t / t_max * (1 - 2^-20)
  // polygon study area (poly_n = 0: the rectangle): window-relative edges
  // {V[k], V[k+1 mod n]}, per xy-cell lists of the edges within s_max (see
  // poly.h), orientation sign
  const int4 *poly;
  const uint16_t *near;
  // per sorted record (spatial correction): its xy-cell, then the distance
  // range of each listed edge from the point (see poly_row); kRowWords words
  const uint32_t *prow;
  int32_t row_shift;  // rows hold distances in units of 2^-row_shift metres
  // edges by horizontal band of height 2^band_shift: band b lists the edges
  // whose y-range meets [b 2^shift, (b + 1) 2^shift), band_idx[band_off[b] ..
  // band_off[b + 1])
  const uint32_t *band_off;
  const uint16_t *band_idx;
  int32_t band_shift;
  int32_t poly_n;
  int32_t poly_sign;  // +1 counter-clockwise, -1 clockwise
};
constexpr int kMaxPoly = 4096;       // vertices of a polygon study area
constexpr int kNearMax = 32;         // edges listed per cell (more: every edge is scanned)
constexpr uint16_t kNearAll = 0xFFFF;
constexpr int kBandsMax = 1024;       // horizontal bands of the containment test
// per-record polygon row: a 4-word head and a word per listed edge, for lists
// of up to kRowEdges edges (longer lists take the exact first pass)
constexpr int kRowEdges = 16;
constexpr int kRowWords = 4 + kRowEdges;

// Work item of the pair kernel: up to kChunk consecutive centres of one unit
// of one set: a cell, or an x-row of cells (row items).
struct Item {
  uint32_t set;
  uint32_t cell;   // unit index within the set: cell, or row (t * ny + y)
  uint32_t begin;  // first centre, index into the sorted point array
  uint32_t count;  // bits 0-6: number of centres (0 = padding); bits 7-18 and
                   // 19-30: first and end index of the stencil rows this item
                   // covers (end 0 = all rows; items split for small launches);
                   // with bit 31 set, one row (bits 7-18) and fraction f (bits
                   // 19-24) of k (bits 25-30) of its neighbour run
};
constexpr int kSplitMax = 64;  // parts an item may be split into
constexpr int kMaxFractions = 8;  // fractions a row's run may be cut into
// The pair kernel's work queue is cut into kQueues contiguous partitions of
// item groups, one per XCD, each with its own counter kQueueStride words
// (4 KB) from the next: returning atomics on one address serialise across the
// chip, so one counter for every workgroup would cost tens of microseconds per
// launch.
constexpr int kQueues = 8;
constexpr int kQueueStride = 512;

struct PairArgs {
  Geom g;
  const int4 *P;          // sorted points: x, y, t, min(edge distance)
  const uint32_t *cs;     // cell starts: 2*n_cells*n_sets + 1 entries
  const Item *items;
  const uint32_t *n_items;  // device scalar
  // kQueues blocks of kQueueStride words, zeroed before launch: word 0 counts
  // the groups handed out of that partition of the work queue, word 1 sums
  // the candidates examined by the workgroups whose home it is
  unsigned long long *queues;
  const uint64_t *S2;       // n_s thresholds (device)
  const uint32_t *T;        // n_t thresholds (device)
  unsigned long long *binC;  // [sets][n_bins] counts
  // [sets][kBinWords][n_bins] fixed-point weight sums, split so that no flush
  // needs the old value: word k sums the k-th 32-bit pieces of the
  // workgroups' partial sums (each addend below 2^34), and the weight is
  // sum_k word_k * 2^(32 k) mod 2^128 times 2^-F (F = kFracBits, or the
  // launch's scale for inhomogeneous K)
  unsigned long long *binW;
  int symmetric;
  int row_items;               // items are chunks of x-rows (else of cells)
  int blocked;                 // two-type sets in blocked key order: centres from the
                               // type-1 block, neighbours from the type-2 block
  const double *rho;           // inhomogeneous K: 1/lambda per sorted record (else null)
  // inhomogeneous K: bit pattern of the largest rho of the launch (device
  // word) and the bit budget of one pair's fixed-point weight (see wide_fbits)
  const unsigned long long *rho_max;
  int wbudget;
  int bins;                    // LDS bin layout (kBinsPacked, kBinsSplit32, kBinsSplit64,
                               // kBinsWide)
  // candidates a workgroup examines before it flushes its LDS bins within a
  // set (0: the layout's own bound)
  unsigned long long flush_evals;
  // Sharing the device with other streams (a server's concurrent requests):
  // with share_word set, a workgroup whose index is share_grid or more exits
  // at once while the host-visible count *share_word exceeds 1, leaving those
  // slots to the other streams' kernels; with slice_ticks > 0 a workgroup
  // stops taking groups after that many ticks of the 100 MHz real-time
  // counter, so that a long launch can be cut into several (the work queue
  // persists between them; the last launch of a call runs without a slice).
  const int32_t *share_word;
  int32_t share_grid;
  uint32_t slice_ticks;
  // Cost-ordered work list: slot s of the work queue holds group perm[s]
  // (kEmptySlot: none); the queue then has (groups + 7) & ~7 slots.  Null:
  // slot s is group s.
  const uint32_t *perm;
  // RIPK_PLAN_TIMING: per workgroup its start and end on the 100 MHz
  // real-time counter (2 words per workgroup of the launch), else null
  unsigned long long *wg_times;
};
constexpr uint32_t kEmptySlot = 0xFFFFFFFEu;
constexpr int kMaxWgPerCu = 32;  // pair-kernel workgroups a compute unit can hold, at most
// Slots of the cost-ordered work list: the sorted groups dealt round-robin
// over the kQueues partitions, so that each partition hands out its groups
// in descending cost.
__host__ __device__ inline uint32_t ordered_slots(uint32_t groups) {
  return (groups + kQueues - 1) / kQueues * kQueues;
}

// Words per bin of the global weight sums (see PairArgs::binW).
constexpr int kBinWords = 4;

// Fraction bits of the fixed-point weight of an inhomogeneous launch: with
// rho_max < 2^e (frexp exponent) one ordered pair weighs at most
// 8 rho_max^2 (omega >= 1/4, v >= 1/2) and a symmetric pair twice that, so
// 2^F times it stays below 2^budget.  The host sets budget so that one pair
// fits three 32-bit pieces and the sum over n(n-1) ordered pairs fits 128
// bits.
__host__ __device__ inline int wide_fbits(unsigned long long rho_max_bits, int budget) {
  union {
    unsigned long long u;
    double d;
  } v;
  v.u = rho_max_bits;
  int e = 0;
  (void)frexp(v.d, &e);
  return budget - 4 - 2 * e;
}

// ---- host runtime (api.cpp) -------------------------------------------------

// Buffer capacities of a plan: S sets, N = S*n_max points, SNC = S*n_cells
// cells, work items, SNB = S*n_bins bins, NB = n_bins, P = n_max (one set),
// V polygon vertices, NXY xy-cells with edge lists (0 without a polygon), R
// intensities (inhomogeneous plans).
struct Caps {
  int64_t S = 0, N = 0, SNC = 0, items = 0, SNB = 0, NB = 0, P = 0, V = 0, NXY = 0, R = 0;
};
Caps caps_for(int64_t S, int64_t n_max, int64_t n_cells, int64_t n_bins, int64_t V = 0,
              int64_t NXY = 0, int64_t R = 0);
int64_t caps_bytes(const Caps &c);
bool caps_fit(const Caps &have, const Caps &need);
Caps caps_max(const Caps &a, const Caps &b);

// Plans with capacities apart from their geometry (the server keeps one per
// slot and rebinds it to each request that fits).
ripk_status plan_validate(const ripk_plan_desc *desc, Caps *caps);
ripk_status plan_create(int device, const Caps &c, ripk_plan_s **out);
ripk_status plan_bind(ripk_plan_s *p, const ripk_plan_desc *desc, hipStream_t stream);
const Caps &plan_caps(const ripk_plan_s *p);
void plan_free(ripk_plan_s *p);
ripk_status set_error(ripk_status s, const char *msg);  // sets ripk_last_error()
// Served plans: device sharing and launch slicing of the pair kernel (see
// PairArgs); slice_us = 0 turns slicing off, a null word sharing.
void plan_set_sharing(ripk_plan_s *p, const int32_t *share_word, double share_frac,
                      double slice_us);
// ripk_compute_K of one rectangle set with every device buffer cut from the
// region [scratch, scratch + scratch_bytes) of the descriptor's device;
// outputs are device buffers (api.cpp)
ripk_status compute_K_in_scratch(const ripk_plan_desc *desc, const ripk_points *pts,
                                 hipStream_t st, unsigned char *scratch, size_t scratch_bytes,
                                 ripk_K_out *out);

// launchers (kernels.hip) ----------------------------------------------
// Sort keys: interleaved ((set*n_cells + cell) << 1 | halo) or, with
// `blocked` (two-type sets), (2*set + type)*n_cells + cell.
hipError_t launch_keys(const int32_t *x, const int32_t *y, const int32_t *t, uint32_t n,
                       uint32_t n_centres, uint32_t set_base, uint32_t n_sets,
                       const Geom &g, int blocked, uint32_t *keys, uint32_t *vals,
                       uint32_t *err, hipStream_t s);
// m CSR sets of n points; points k >= n_centres of each set are type 2 of a
// cross-K plan (halo slot, or the type-2 block of blocked keys; n_centres = n
// otherwise)
// (polygon: rejection sampling; a point that finds no attempt inside sets bit 1
// of *err).  Simulation s is stored as set s + set_off: x, y, t, keys and vals
// are the arrays of all sets, written from entry set_off * n on.
hipError_t launch_csr(uint32_t n, uint32_t n_centres, uint32_t m, uint64_t seed, const Geom &g,
                      int blocked, int32_t *x, int32_t *y, int32_t *t, uint32_t *keys,
                      uint32_t *vals, uint32_t *err, uint32_t set_off, hipStream_t s);
// Simulated sets drawn from the observed points ox, oy, ot (n each): method 1
// random permutation of the time labels, 2 bootstrap (each of the types
// [0, n_centres) and [n_centres, n) from itself); writes x, y, t and the cell
// keys/values into keys[0], vals[0] (uses both sort buffers).
hipError_t launch_resample(int method, uint32_t n, uint32_t n_centres, uint32_t m, uint64_t seed,
                           int blocked, const int32_t *ox,
                           const int32_t *oy, const int32_t *ot, const Geom &g, int32_t *x,
                           int32_t *y, int32_t *t, uint32_t *keys[2], uint32_t *vals[2],
                           void *sort_temp, hipStream_t s);
// Stable LSD radix sort of (key, value) by the low key_bits bits.  With
// n_segs > 1 the n entries are n_segs segments of n / n_segs entries, already
// in segment order, segment g holding keys in [g*seg_stride, (g+1)*seg_stride):
// each segment is sorted by key - g*seg_stride, key_bits covering seg_stride.
struct SortSeg {
  uint32_t len, tiles, stride;
  uint32_t items;  // keys per thread of a tile (tile = 256 threads x items)
};
size_t radix_sort_temp_bytes(uint32_t n, uint32_t n_segs = 1);
hipError_t radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                      uint32_t n, int key_bits, void *temp, hipStream_t s, int *result_in_alt,
                      uint32_t n_segs = 1, uint32_t seg_stride = 0);
size_t scan_temp_bytes(uint32_t n);
hipError_t exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t n, void *temp,
                          hipStream_t s);
// From the sorted keys and values: the cell bounds cs[k] (first index whose key
// >= k, k in [0, n_keys]) and the sorted records {x, y, t, distance to the
// study area's boundary, clamped to s_max}
hipError_t launch_bounds_gather(const uint32_t *keys, const uint32_t *vals, uint32_t n,
                                uint32_t n_keys, uint32_t *cs, const int32_t *x, const int32_t *y,
                                const int32_t *t, const Geom &g, int32_t clamp_e, int4 *P,
                                uint32_t *prow, hipStream_t s);
// rho[r] = 1 / lambda[vals[r]] for the sorted records, and the largest rho
// as its bit pattern in *rho_max (zeroed before; positive doubles order as
// their bit patterns); a value that is not positive and finite sets bit 2 of
// *err
hipError_t launch_gather_rho(const uint32_t *vals, uint32_t n, const double *lambda, double *rho,
                             uint32_t *err, unsigned long long *rho_max, hipStream_t s);
// With split > 1 and tmp (room for every item before splitting) the items are
// written once into tmp and expanded into their `split` parts in parallel
// (at most max_slots slots); otherwise each item's walk writes all its parts.
hipError_t launch_items(const uint32_t *cs, uint32_t n_sets, const Geom &g, bool row_items,
                        bool blocked, uint32_t split, uint32_t n_rows, uint32_t *chunks,
                        uint32_t *offs, uint32_t *set_base, Item *items, uint32_t *n_items,
                        void *scan_temp, hipStream_t s, Item *tmp = nullptr,
                        uint32_t max_slots = 0);
// zeroes the ranges (p[r], n[r]) in one launch (a kernel, not memset nodes)
struct Zero3 {
  unsigned long long *p[3];
  size_t n[3];
};
hipError_t launch_zero3(const Zero3 &z, hipStream_t s);
hipError_t launch_pair(const PairArgs &a, int grid, hipStream_t s);
// The cost-ordered work list of a launch of at most max_groups groups: an
// estimate of each group's candidates (centres x neighbour-run lengths of its
// stencil rows), an 8-bit key of its logarithm, a stable radix sort (keys
// and values in kA/vA with kB/vB and temp as scratch, each of max_groups
// words, max_groups a multiple of kQueues) and the round-robin deal into
// whichever value buffer the sort left free (*perm).
hipError_t launch_order_groups(const PairArgs &a, uint32_t max_groups, uint32_t *kA,
                               uint32_t *vA, uint32_t *kB, uint32_t *vB, void *temp,
                               const uint32_t **perm, hipStream_t s);
// LDS bin layouts of the pair kernel.  Packed: one 64-bit word per bin holds
// the pair count (bits 34-63) and the interior-path weights in units of 2^23
// (bits 0-33), so a pair costs one LDS atomic; boundary weights go to a second
// word.  Split: a fixed-point weight word and a 32- or 64-bit count word.
// Packed needs fewer than 2^30 pending pairs per bin (sets below 2^21 points,
// flushes every 2^29 candidates); 32-bit counts need sets below 2^23 points.
// Wide (polygon weights, whose 1/omega has no fixed bound, and inhomogeneous
// K): a 64-bit count word and three words summing the 32-bit pieces of each
// side's fixed-point weight (below 2^96); the sums stay below 2^63 while
// fewer than 2^31 pairs are pending per bin: sets below 2^22 points (one
// group examines fewer than 256 n candidates), flushes every 2^29 candidates.
constexpr int kBinsPacked = 0, kBinsSplit32 = 1, kBinsSplit64 = 2, kBinsWide = 3;
constexpr int64_t kPackedPoints = 1 << 21;
constexpr int64_t kWidePoints = 1 << 22;
int pair_lds_bytes(int n_s, int n_t, int bins, bool inhom = false);
// the bin layout of polygon-weight and inhomogeneous launches
inline int pair_bins_for_var(int var, int bins) { return var ? kBinsWide : bins; }
// the pair kernel takes the polygon weight path (a polygon and spatial correction)
bool pair_poly(const Geom &g);
// kernel variant: 0 rectangle, 1 polygon, 2 inhomogeneous (rectangle)
hipError_t pair_occupancy(int n_s, int n_t, int bins, int symmetric, int mode, int var,
                          int *per_cu);
// 64-bit LDS pair counts are needed from this many points per set on
constexpr int64_t kWideCountPoints = 1 << 23;
// The weight sums have kFracBits fraction bits, or with rho_max (inhomogeneous
// K) wide_fbits(*rho_max, wbudget).  scal[0] receives the candidates summed
// over the work-queue partitions `queues`, scal[1] the in-range pairs over
// all sets.
hipError_t launch_finalize(unsigned long long *binC, unsigned long long *binW,
                           uint32_t n_sets, int n_s, int n_t, double s_max, double t_max,
                           double AD, double N, unsigned long long *C, double *W, double *K,
                           double *L, const unsigned long long *queues,
                           unsigned long long *scal, hipStream_t s,
                           const unsigned long long *rho_max = nullptr, int wbudget = 0);
hipError_t launch_envelope(const double *K, const double *L, uint32_t m, int n_bins,
                           const double *L_obs, double *env, hipStream_t s);
// Results of a call brought to the host in one copy: kScalWords words of
// scal, then each non-null row of nb 8-byte words at its slot (row r at
// kScalWords + r*nb).
constexpr int kScalWords = 4;
constexpr int kPackRows = 9;
struct PackRows {
  const unsigned long long *p[kPackRows];
};
hipError_t launch_pack(const unsigned long long *scal, const PackRows &rows, int nb,
                       unsigned long long *out, hipStream_t s);

}  // namespace ripk
