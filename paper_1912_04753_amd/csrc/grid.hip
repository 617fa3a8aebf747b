// Cell-grid construction on gfx950: cell keys, on-device Monte Carlo CSR points
// (Philox4x64-10), a stable LSD radix sort, cell bounds, the sorted point
// records and the work items of the pair kernel.
//
// The uniform space-time cell grid stands in for the paper's R-tree (Sec. 4.2):
// with cells at least s_max wide in x and y and t_max long in t, every neighbour
// of a centre within (s_max, t_max) lies in the 3x3x3 block of cells around it.
#include "poly.h"
#include "ripk_internal.h"

namespace ripk {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t cell_of(int32_t x, int32_t y, int32_t t, const Geom &g,
                                            bool *outside) {
  bool bad = x < g.x0 || x > g.x1 || y < g.y0 || y > g.y1 || t < g.t0 || t > g.t1;
  *outside = bad;
  // Clamp so that a bad point still maps to a valid cell; the call reports
  // the error and discards every result.
  uint32_t X = (uint32_t)(min(max(x, g.x0), g.x1) - g.x0);
  uint32_t Y = (uint32_t)(min(max(y, g.y0), g.y1) - g.y0);
  uint32_t T = (uint32_t)(min(max(t, g.t0), g.t1) - g.t0);
  // the last cell of an axis absorbs the remainder, so it is never narrower
  // than the cell edge
  uint32_t cx = min(X / (uint32_t)g.cell_s, (uint32_t)g.nx - 1u);
  uint32_t cy = min(Y / (uint32_t)g.cell_s, (uint32_t)g.ny - 1u);
  uint32_t ct = min(T / (uint32_t)g.cell_t, (uint32_t)g.nt - 1u);
  return (ct * (uint32_t)g.ny + cy) * (uint32_t)g.nx + cx;
}

// Sort key of a point: interleaved ((set * n_cells + cell) << 1) | halo, so
// that a cell's centres precede its halo points; blocked (two-type sets)
// (2 * set + type) * n_cells + cell, so that each type of a set is one
// cell-sorted block.
__device__ __forceinline__ uint32_t sort_key(uint32_t set, uint32_t cell, uint32_t halo,
                                             const Geom &g, bool blocked) {
  return blocked ? (2u * set + halo) * g.n_cells + cell : ((set * g.n_cells + cell) << 1) | halo;
}

// val = global point index
__global__ void k_keys(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                       const int32_t *__restrict__ t, uint32_t n, uint32_t n_centres,
                       uint32_t set_base, Geom g, int blocked, uint32_t *__restrict__ keys,
                       uint32_t *__restrict__ vals, uint32_t *__restrict__ err) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool bad;
  uint32_t c = cell_of(x[i], y[i], t[i], g, &bad);
  // a polygon study area holds its points strictly inside
  if (!bad && g.poly_n && !poly_inside(g, x[i] - g.x0, y[i] - g.y0)) bad = true;
  if (bad) atomicOr(err, 1u);
  keys[i] = sort_key(set_base, c, i >= n_centres ? 1u : 0u, g, blocked != 0);
  vals[i] = i;
}

// ---- Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) -----------------------
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0h = __umul64hi(M0, c.v[0]), p0l = M0 * c.v[0];
    uint64_t p1h = __umul64hi(M1, c.v[2]), p1l = M1 * c.v[2];
    U64x4 o;
    o.v[0] = p1h ^ c.v[1] ^ k0;
    o.v[1] = p1l;
    o.v[2] = p0h ^ c.v[3] ^ k1;
    o.v[3] = p0l;
    c = o;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Simulation s, point i: counter (i, s, 0, 0), key (seed, 0).  Coordinates on
// the half-open window by 64x64 multiply-high.  In a polygon, attempt a uses
// counter (i, s, a, 0) until the point lies strictly inside (the polygon covers
// at least 1/1024 of the window, so 2^16 attempts all failing has probability
// below e^-64; it sets bit 1 of *err).  Writes the SoA points and the (key,
// value) pairs for the sort, sets ordered simulation-major; simulation s is
// stored as set s + set_off (entries from set_off * n on), its draws unchanged.
constexpr uint32_t kMaxAttempts = 1u << 16;

__global__ void k_csr(uint32_t n, uint32_t n_centres, uint32_t m, uint64_t seed, Geom g,
                      int blocked, int32_t *__restrict__ x,
                      int32_t *__restrict__ y, int32_t *__restrict__ t,
                      uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                      uint32_t *__restrict__ err, uint32_t set_off) {
  uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (uint64_t)n * m) return;
  uint32_t s = (uint32_t)(gid / n), i = (uint32_t)(gid - (uint64_t)s * n);
  const uint64_t W = (uint64_t)(g.x1 - g.x0), H = (uint64_t)(g.y1 - g.y0),
                 D = (uint64_t)(g.t1 - g.t0);
  int32_t px, py, pt;
  for (uint32_t a = 0;; ++a) {
    U64x4 c;
    c.v[0] = i;
    c.v[1] = s;
    c.v[2] = a;
    c.v[3] = 0;
    const U64x4 r = philox4x64_10(c, seed, 0);
    px = g.x0 + (int32_t)__umul64hi(r.v[0], W);
    py = g.y0 + (int32_t)__umul64hi(r.v[1], H);
    pt = g.t0 + (int32_t)__umul64hi(r.v[2], D);
    if (!g.poly_n || poly_inside(g, px - g.x0, py - g.y0)) break;
    if (a + 1 == kMaxAttempts) {
      atomicOr(err, 2u);
      break;
    }
  }
  const uint64_t w = gid + (uint64_t)set_off * n;
  x[w] = px;
  y[w] = py;
  t[w] = pt;
  bool bad;
  uint32_t cell = cell_of(px, py, pt, g, &bad);
  keys[w] = sort_key(s + set_off, cell, i >= n_centres ? 1u : 0u, g, blocked != 0);
  vals[w] = (uint32_t)w;
}

// ---- simulations drawn from the observed points (Sec. 3) --------------------
// Random permutation keeps every location and exchanges time labels: set s
// gives point k the time of observed point order_s[k], where order_s lists the
// points by increasing high 32 bits of word 0 of Philox(counter (j, s, 0, 0),
// key (seed, 1)), equal values by index.  Bootstrap takes point k of set s
// from observed point floor(r0 * n / 2^64), r = Philox((k, s, 0, 0), (seed, 2));
// with two types (n_centres < n) each type draws from itself: point k <
// n_centres from floor(r0 * n_centres / 2^64), the others from n_centres +
// floor(r0 * (n - n_centres) / 2^64).

// permutation, stage 1: the random rank key of every (set, point); value = index
__global__ void k_perm_keys(uint32_t n, uint32_t m, uint64_t seed, uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ vals) {
  uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (uint64_t)n * m) return;
  uint32_t s = (uint32_t)(gid / n), i = (uint32_t)(gid - (uint64_t)s * n);
  U64x4 c;
  c.v[0] = i;
  c.v[1] = s;
  c.v[2] = 0;
  c.v[3] = 0;
  U64x4 r = philox4x64_10(c, seed, 1);
  keys[gid] = (uint32_t)(r.v[0] >> 32);
  vals[gid] = (uint32_t)gid;
}

// permutation, stage 2 key: the set of each entry (a stable sort by it keeps
// the rank order inside every set)
__global__ void k_set_of(const uint32_t *__restrict__ vals, uint64_t total, uint32_t n,
                         uint32_t *__restrict__ keys) {
  uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  keys[gid] = vals[gid] / n;
}

// Assembles the simulated sets (as k_csr does for CSR): points and cell keys.
// `order` (permutation only) may be the same array as `vals`: each thread reads
// its own entry before writing it.
__global__ void k_resample(uint32_t n, uint32_t n_centres, uint32_t m, uint64_t seed, int method,
                           const uint32_t *order, const int32_t *__restrict__ ox,
                           const int32_t *__restrict__ oy, const int32_t *__restrict__ ot, Geom g,
                           int blocked, int32_t *__restrict__ x, int32_t *__restrict__ y,
                           int32_t *__restrict__ t, uint32_t *__restrict__ keys, uint32_t *vals) {
  uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (uint64_t)n * m) return;
  uint32_t s = (uint32_t)(gid / n), k = (uint32_t)(gid - (uint64_t)s * n);
  int32_t px, py, pt;
  if (method == 1) {
    const uint32_t src = order[gid] - s * n;
    px = ox[k];
    py = oy[k];
    pt = ot[src];
  } else {
    U64x4 c;
    c.v[0] = k;
    c.v[1] = s;
    c.v[2] = 0;
    c.v[3] = 0;
    U64x4 r = philox4x64_10(c, seed, 2);
    const uint32_t j = k < n_centres
                           ? (uint32_t)__umul64hi(r.v[0], (uint64_t)n_centres)
                           : n_centres + (uint32_t)__umul64hi(r.v[0], (uint64_t)(n - n_centres));
    px = ox[j];
    py = oy[j];
    pt = ot[j];
  }
  x[gid] = px;
  y[gid] = py;
  t[gid] = pt;
  bool bad;
  uint32_t cell = cell_of(px, py, pt, g, &bad);
  keys[gid] = sort_key(s, cell, k >= n_centres ? 1u : 0u, g, blocked != 0);
  vals[gid] = (uint32_t)gid;
}

// ---- exclusive scan of uint32 ------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds,
                                                         uint32_t *total) {
  // lds: kThreads/64 + 1 words
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t nb = __shfl_up(incl, o, 64);
    if (lane >= o) incl += nb;
  }
  if (lane == 63) lds[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      uint32_t c = lds[i];
      lds[i] = run;
      run += c;
    }
    lds[blockDim.x >> 6] = run;
  }
  __syncthreads();
  uint32_t res = lds[w] + incl - v;
  *total = lds[blockDim.x >> 6];
  __syncthreads();
  return res;
}

__global__ void k_scan_reduce(const uint32_t *__restrict__ in, uint32_t n,
                              uint32_t *__restrict__ part) {
  __shared__ uint32_t lds[kThreads / 64 + 1];
  uint32_t base = blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t i = base + k * kThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block: exclusive scan of part[0..nb) in place, part[nb] = total
__global__ void k_scan_partials(uint32_t *part, uint32_t nb) {
  __shared__ uint32_t lds[kThreads / 64 + 1];
  uint32_t per = (nb + kThreads - 1) / kThreads;
  uint32_t b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (uint32_t k = 0; k < per; ++k)
    if (b0 + k < nb) s += part[b0 + k];
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, lds, &tot);
  for (uint32_t k = 0; k < per; ++k)
    if (b0 + k < nb) {
      uint32_t c = part[b0 + k];
      part[b0 + k] = run;
      run += c;
    }
  if (threadIdx.x == 0) part[nb] = tot;
}

// Down-sweep: each block first adds up the tile sums before it (a few hundred
// at most, read by all threads at once), so no separate pass scans them.
__global__ void k_scan_down(const uint32_t *__restrict__ in, uint32_t n,
                            const uint32_t *__restrict__ part, uint32_t *__restrict__ out) {
  __shared__ uint32_t lds[kThreads / 64 + 1];
  __shared__ uint32_t tile[kScanTile];
  __shared__ uint32_t before;
  uint32_t base = blockIdx.x * kScanTile;
  {
    uint32_t s = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kThreads) s += part[b];
    uint32_t tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) before = tot;
  }
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t i = base + k * kThreads + threadIdx.x;
    tile[k * kThreads + threadIdx.x] = i < n ? in[i] : 0u;
  }
  __syncthreads();
  uint32_t loc[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = tile[threadIdx.x * kScanItems + k];
    s += loc[k];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, lds, &tot) + before;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    tile[threadIdx.x * kScanItems + k] = run;
    run += loc[k];
  }
  __syncthreads();
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t i = base + k * kThreads + threadIdx.x;
    if (i < n) out[i] = tile[k * kThreads + threadIdx.x];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = before + tot;
}

// ---- stable LSD radix sort, 8-bit digits --------------------------------------
// Segmented: segment g holds entries [g*len, (g+1)*len), its keys lie in
// [g*stride, (g+1)*stride), and the segments are already in order, so only the
// offset within the segment (key - g*stride) is sorted, and tiles never
// straddle a segment.  Digit counts are laid out (segment, digit, tile), so
// their exclusive scan gives each tile's start for each digit.  One segment
// with stride 0 is a plain sort.
// Keys per thread of a tile: 16 (4,096 keys per workgroup); 2 for sorts of at
// most kSmallSort keys, which would otherwise run on too few workgroups (a
// 200k-key pass on 49 of them was latency-bound in its 16 serial rounds); 1
// for at most kTinySort keys (the work list's cost order).
constexpr uint32_t kSortItems = 16;
constexpr uint32_t kSortItemsSmall = 2;
constexpr uint32_t kSmallSort = 1u << 20;
constexpr uint32_t kSortItemsTiny = 1;
constexpr uint32_t kTinySort = 1u << 16;
__host__ __device__ inline uint32_t sort_items(uint32_t n) {
  return n <= kTinySort ? kSortItemsTiny : n <= kSmallSort ? kSortItemsSmall : kSortItems;
}

struct SortTile {
  uint32_t seg, t, base, end, key0;
};

// Workgroups go to the chip's 8 XCDs in turn (hardware block b to XCD b % 8).
// For a grid padded to a multiple of 8, the logical block (b % 8) * (grid / 8)
// + b / 8 hands each XCD one contiguous eighth of the logical blocks, so the
// sets one XCD gathers from stay in its own L2 (k_bounds_gather; the radix
// scatter measured slower with it).  A bijection of [0, grid): logical blocks
// past the real grid do nothing.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t grid) {
  return (b % kXcds) * (grid / kXcds) + b / kXcds;
}

__device__ __forceinline__ SortTile sort_tile(const SortSeg &sg, uint32_t b) {
  SortTile r;
  r.seg = b / sg.tiles;
  r.t = b - r.seg * sg.tiles;
  const uint32_t tile = (uint32_t)kThreads * sg.items;
  r.base = r.seg * sg.len + r.t * tile;
  r.end = min(r.base + tile, (r.seg + 1) * sg.len);
  r.key0 = r.seg * sg.stride;
  return r;
}

__device__ __forceinline__ uint32_t count_slot(const SortSeg &sg, const SortTile &tl, uint32_t d) {
  return (tl.seg * 256u + d) * sg.tiles + tl.t;
}

__global__ void k_sort_hist(const uint32_t *__restrict__ keys, SortSeg sg, int shift,
                            uint32_t mask, uint32_t *__restrict__ counts) {
  __shared__ uint32_t h[256];
  const SortTile tl = sort_tile(sg, blockIdx.x);
  h[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t k = 0; k < sg.items; ++k) {
    uint32_t i = tl.base + k * kThreads + threadIdx.x;
    if (i < tl.end) atomicAdd(&h[((keys[i] - tl.key0) >> shift) & mask], 1u);
  }
  __syncthreads();
  counts[count_slot(sg, tl, threadIdx.x)] = h[threadIdx.x];
}

// Tile order is round-major (round k holds items base + k*256 + tid), so a key's
// stable rank is: keys of its digit in earlier rounds + in earlier waves of the
// same round + in lower lanes of the same wave.
__global__ void k_sort_scatter(const uint32_t *__restrict__ keys,
                               const uint32_t *__restrict__ vals, SortSeg sg, int shift,
                               int nbits, const uint32_t *__restrict__ offs,
                               uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[kThreads / 64][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  const SortTile tl = sort_tile(sg, blockIdx.x);
  run[threadIdx.x] = offs[count_slot(sg, tl, threadIdx.x)];
  for (int q = 0; q < kThreads / 64; ++q) wc[q][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint32_t k = 0; k < sg.items; ++k) {
    uint32_t i = tl.base + k * kThreads + threadIdx.x;
    bool valid = i < tl.end;
    uint32_t key = valid ? keys[i] : 0u;
    uint32_t val = valid ? vals[i] : 0u;
    uint32_t d = ((key - tl.key0) >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int q = 0; q < w; ++q) pos += wc[q][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    {
      uint32_t add = 0;
      for (int q = 0; q < kThreads / 64; ++q) {
        add += wc[q][threadIdx.x];
        wc[q][threadIdx.x] = 0;
      }
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// One pass over the sorted keys: the cell bounds cs[k] = first index whose
// key >= k, for k in [0, n_keys], and the sorted point records: window-relative
// coordinates (all >= 0) and the distance to the nearest side clamped to s_max
// (a circle no larger than that is whole); with a polygon and spatial
// correction, each record's row of edge distance ranges (poly_row).
__global__ void k_bounds_gather(const uint32_t *__restrict__ keys,
                                const uint32_t *__restrict__ vals, uint32_t n, uint32_t n_keys,
                                uint32_t *__restrict__ cs, const int32_t *__restrict__ x,
                                const int32_t *__restrict__ y, const int32_t *__restrict__ t,
                                Geom g, int32_t clamp_e, int4 *__restrict__ P,
                                uint32_t *__restrict__ prow) {
  const uint32_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (r > n) return;
  const int64_t prev = (r == 0) ? -1 : (int64_t)keys[r - 1];
  const int64_t cur = (r == n) ? (int64_t)n_keys : (int64_t)keys[r];
  for (int64_t k = prev + 1; k <= cur; ++k) cs[k] = r;
  if (r == n) return;
  uint32_t i = vals[r];
  int32_t X = x[i] - g.x0, Y = y[i] - g.y0, T = t[i] - g.t0;
  int32_t e;
  if (g.poly_n) {
    e = poly_edist(g, X, Y, clamp_e);
    if (g.prow) poly_row(g, X, Y, prow + (size_t)r * kRowWords);
  } else {
    e = min(min(X, g.x1 - g.x0 - X), min(Y, g.y1 - g.y0 - Y));
    e = min(max(e, 0), clamp_e);
  }
  P[r] = make_int4(X, Y, T, e);
}

// 1/lambda of the sorted records (inhomogeneous K)
// (lambda must lie in [2^-400, 2^400], so that the fixed-point scale 2^F of
// the weight sums and every rho_i rho_j 2^F are normal doubles)
__global__ void k_gather_rho(const uint32_t *__restrict__ vals, uint32_t n,
                             const double *__restrict__ lambda, double *__restrict__ rho,
                             uint32_t *__restrict__ err, unsigned long long *__restrict__ rho_max) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (r < n) {
    const double l = lambda[vals[r]];
    const bool ok = l >= 0x1p-400 && l <= 0x1p400;
    if (!ok) atomicOr(err, 4u);
    v = ok ? 1.0 / l : 0.0;
    rho[r] = v;
  }
  // positive doubles order as their bit patterns: a wave maximum, then one
  // atomic per wave
  unsigned long long m = (unsigned long long)__double_as_longlong(v);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(m, o);
    m = y > m ? y : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax(rho_max, m);
}

// A unit is the run of cells whose centres a work item may mix: one cell, or a
// whole x-row of cells (unit = nx) when no halo entries lie between the cells
// (every point a centre, or the type-1 block of blocked keys).  Units cover cells [g*unit, (g+1)*unit) of the
// cell array of all sets.  Items are cut greedily: up to kChunk consecutive
// centres, all within 1 + kItemExtent consecutive cells of the unit (the
// candidate distance bound of the plan relies on it).  chunk_walk visits the
// items of unit g in order; emit(begin, count) is called for each.
// Centre entries of cell X (set-major index set * n_cells + cell) span
// [cs[k(X) * st], cs[k(X) * st + 1]): interleaved keys k(X) = X, st = 2;
// blocked keys k(X) = X + set * n_cells (the set's type-1 block), st = 1.
struct CentreIdx {
  uint32_t nc;
  bool blocked;
  __device__ __forceinline__ uint32_t at(uint32_t X) const {
    return blocked ? X + (X / nc) * nc : 2u * X;
  }
};

// One wave walks a unit (all lanes alike; the caller lets lane 0 store).  The
// unit's cell ends are read once, one per lane, when the unit has at most 64
// cells: the walk's many look-ups are then register reads, not a chain of
// dependent loads (a 3,000-centre row took about 50 us that way).
template <typename F>
__device__ __forceinline__ uint32_t chunk_walk(const uint32_t *__restrict__ cs, uint32_t g,
                                               uint32_t unit, CentreIdx ci, int lane, F emit) {
  const uint32_t c0 = g * unit;
  const bool in_regs = unit <= 64u;
  const uint32_t mine = (in_regs && (uint32_t)lane < unit) ? cs[ci.at(c0 + (uint32_t)lane) + 1] : 0u;
  auto end_of = [&](uint32_t c) -> uint32_t {
    return in_regs ? (uint32_t)__shfl((int)mine, (int)c) : cs[ci.at(c0 + c) + 1];
  };
  uint32_t pos = cs[ci.at(c0)];
  const uint32_t end = end_of(unit - 1);
  uint32_t c = 0, items = 0;
  while (pos < end) {
    while (end_of(c) <= pos) ++c;  // cell holding pos (row units: no halo entries)
    // while kChunk centres remain in this cell the greedy item is exactly
    // those kChunk: emit the whole run of them at once
    const uint32_t ce = end_of(c);
    if (ce - pos >= (uint32_t)kChunk) {
      const uint32_t k = (ce - pos) / (uint32_t)kChunk;
      for (uint32_t j = 0; j < k; ++j) emit(pos + j * (uint32_t)kChunk, (uint32_t)kChunk);
      items += k;
      pos += k * (uint32_t)kChunk;
      continue;
    }
    const uint32_t last = min(c + (uint32_t)kItemExtent, unit - 1);
    const uint32_t lim = min(min(pos + (uint32_t)kChunk, end), end_of(last));
    emit(pos, lim - pos);
    ++items;
    pos = lim;
  }
  return items;
}

// one wave per unit
__global__ void k_chunks(const uint32_t *__restrict__ cs, uint32_t nunit_total, uint32_t unit,
                         CentreIdx ci, uint32_t *__restrict__ chunks) {
  const uint32_t g = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = (int)(threadIdx.x & 63u);
  if (g >= nunit_total) return;
  const uint32_t items = chunk_walk(cs, g, unit, ci, lane, [](uint32_t, uint32_t) {});
  if (lane == 0) chunks[g] = items;
}

// Item bases per set (before splitting), each set padded to whole groups; the
// emitted array holds every item `split` times, once per part of its stencil
// rows.
__global__ void k_set_base(const uint32_t *__restrict__ offs, uint32_t n_sets,
                           uint32_t n_units, uint32_t split, uint32_t *__restrict__ set_base,
                           uint32_t *__restrict__ n_items) {
  // one block: each thread pads the item counts of a run of sets, then one
  // block-wide scan places the runs
  __shared__ uint32_t lds[kThreads / 64 + 1];
  const uint32_t per = (n_sets + kThreads - 1) / kThreads;
  const uint32_t s0 = threadIdx.x * per;
  auto padded = [&](uint32_t s) {
    const uint32_t tot = offs[(s + 1) * n_units] - offs[s * n_units];
    return (tot + kItemsPerGroup - 1) / kItemsPerGroup * kItemsPerGroup;
  };
  uint32_t sum = 0;
  for (uint32_t k = 0; k < per && s0 + k < n_sets; ++k) sum += padded(s0 + k);
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, lds, &total);
  for (uint32_t k = 0; k < per && s0 + k < n_sets; ++k) {
    set_base[s0 + k] = run;
    run += padded(s0 + k);
  }
  if (threadIdx.x == 0) {
    set_base[n_sets] = total;
    *n_items = total * split;
  }
}

// count word of part p of `split` parts of n_rows stencil rows (see Item)
__device__ __forceinline__ uint32_t item_count(uint32_t cnt, uint32_t p, uint32_t split,
                                               uint32_t n_rows) {
  if (split == 1) return cnt;
  if (split > n_rows) {  // split = n_rows * k: row p / k, fraction p % k of its run
    const uint32_t k = split / n_rows;
    return cnt | ((p / k) << 7) | ((p % k) << 19) | (k << 25) | 0x80000000u;
  }
  const uint32_t r0 = p * n_rows / split, r1 = (p + 1) * n_rows / split;
  return cnt | (r0 << 7) | (r1 << 19);
}

// Slot of part p of item o (o counts items over all sets, each set padded to
// whole groups starting at sb = set_base of its set).  A group holds part p of
// kItemsPerGroup consecutive items, not the parts of one item: the waves of a
// workgroup then take stencil parts of the same index, alike in cost (split
// items of clustered sets differ most between parts, rows near the centres'
// own time cell holding the clusters).
__device__ __forceinline__ uint32_t item_slot(uint32_t sb, uint32_t o, uint32_t p,
                                              uint32_t split) {
  const uint32_t q = o - sb;
  return sb * split + ((q / kItemsPerGroup) * split + p) * kItemsPerGroup + q % kItemsPerGroup;
}

// one wave per unit; lane p writes part p of each item (split <= 64)
__global__ void k_emit(const uint32_t *__restrict__ cs, const uint32_t *__restrict__ offs,
                       const uint32_t *__restrict__ set_base, uint32_t n_sets, uint32_t n_units,
                       uint32_t unit, uint32_t split, uint32_t n_rows, CentreIdx ci,
                       Item *__restrict__ items) {
  const uint32_t gidx = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (gidx >= n_sets * n_units) return;
  const uint32_t s = gidx / n_units, c = gidx - s * n_units;
  const uint32_t sb = set_base[s];
  uint32_t o = sb + offs[gidx] - offs[s * n_units];
  chunk_walk(cs, gidx, unit, ci, (int)lane, [&](uint32_t b, uint32_t cnt) {
    if (lane < split) {
      Item it;
      it.set = s;
      it.cell = c;
      it.begin = b;
      it.count = item_count(cnt, lane, split, n_rows);
      items[item_slot(sb, o, lane, split)] = it;
    }
    ++o;
  });
  if (c == n_units - 1 && lane < split) {
    const uint32_t end = sb + offs[(s + 1) * n_units] - offs[s * n_units];
    for (uint32_t q = end; q < set_base[s + 1]; ++q) {
      Item it;
      it.set = s;
      it.cell = 0;
      it.begin = 0;
      it.count = 0;
      items[item_slot(sb, q, lane, split)] = it;
    }
  }
}

// Part p of every item, one thread per slot (the serial walk of k_emit then
// writes each item once, not `split` times): the slot's set from set_base
// (binary search), its item o and part p by inverting item_slot.
__global__ void k_expand(const Item *__restrict__ base, const uint32_t *__restrict__ set_base,
                         uint32_t n_sets, uint32_t split, uint32_t n_rows,
                         const uint32_t *__restrict__ n_items, uint32_t max_slots,
                         Item *__restrict__ items) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_slots || s >= *n_items) return;
  uint32_t lo = 0, hi = n_sets;  // largest k with set_base[k] * split <= s
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (set_base[mid] * split <= s) lo = mid; else hi = mid;
  }
  const uint32_t sb = set_base[lo];
  const uint32_t r = s - sb * split, gp = r / kItemsPerGroup;
  const uint32_t q = (gp / split) * kItemsPerGroup + r % kItemsPerGroup, p = gp % split;
  Item it = base[sb + q];
  const uint32_t cnt = it.count & 0x7Fu;
  it.count = cnt ? item_count(cnt, p, split, n_rows) : 0u;
  items[s] = it;
}

// zeroes up to three ranges in one launch
__global__ void k_zero3(Zero3 z) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int r = 0; r < 3; ++r)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.n[r]; i += stride)
      z.p[r][i] = 0ull;
}

inline uint32_t blocks_for(uint64_t n, int per) { return (uint32_t)((n + per - 1) / per); }
// a grid of at least `blocks` workgroups, a multiple of the XCD count (see xcd_block)
inline uint32_t xcd_grid(uint32_t blocks) { return (blocks + kXcds - 1) / kXcds * kXcds; }

}  // namespace

hipError_t launch_keys(const int32_t *x, const int32_t *y, const int32_t *t, uint32_t n,
                       uint32_t n_centres, uint32_t set_base, uint32_t n_sets, const Geom &g,
                       int blocked, uint32_t *keys, uint32_t *vals, uint32_t *err,
                       hipStream_t s) {
  (void)n_sets;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, x, y, t, n,
                     n_centres, set_base, g, blocked, keys, vals, err);
  return hipGetLastError();
}

hipError_t launch_csr(uint32_t n, uint32_t n_centres, uint32_t m, uint64_t seed, const Geom &g,
                      int blocked, int32_t *x, int32_t *y, int32_t *t, uint32_t *keys,
                      uint32_t *vals, uint32_t *err, uint32_t set_off, hipStream_t s) {
  uint64_t tot = (uint64_t)n * m;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_csr, dim3(blocks_for(tot, kThreads)), dim3(kThreads), 0, s, n, n_centres,
                     m, seed, g, blocked, x, y, t, keys, vals, err, set_off);
  return hipGetLastError();
}

hipError_t launch_resample(int method, uint32_t n, uint32_t n_centres, uint32_t m, uint64_t seed,
                           int blocked, const int32_t *ox,
                           const int32_t *oy, const int32_t *ot, const Geom &g, int32_t *x,
                           int32_t *y, int32_t *t, uint32_t *keys[2], uint32_t *vals[2],
                           void *sort_temp, hipStream_t s) {
  const uint64_t tot = (uint64_t)n * m;
  if (tot == 0) return hipSuccess;
  const dim3 grid(blocks_for(tot, kThreads)), block(kThreads);
  const uint32_t *order = nullptr;
  if (method == 1) {
    hipLaunchKernelGGL(k_perm_keys, grid, block, 0, s, n, m, seed, keys[0], vals[0]);
    int alt = 0;
    hipError_t e = radix_sort(keys[0], vals[0], keys[1], vals[1], (uint32_t)tot, 32, sort_temp, s,
                              &alt);
    if (e != hipSuccess) return e;
    int a = alt;  // buffer holding the rank order
    if (m > 1) {
      int bits = 0;
      while ((1u << bits) < m) ++bits;
      hipLaunchKernelGGL(k_set_of, grid, block, 0, s, vals[a], tot, n, keys[a]);
      e = radix_sort(keys[a], vals[a], keys[1 - a], vals[1 - a], (uint32_t)tot, bits, sort_temp, s,
                     &alt);
      if (e != hipSuccess) return e;
      if (alt) a = 1 - a;
    }
    order = vals[a];
    // writing keys[0]/vals[0]: when a == 0 each thread reads order[gid] first
  }
  hipLaunchKernelGGL(k_resample, grid, block, 0, s, n, n_centres, m, seed, method, order, ox, oy,
                     ot, g, blocked, x, y, t, keys[0], vals[0]);
  return hipGetLastError();
}

size_t scan_temp_bytes(uint32_t n) {
  return sizeof(uint32_t) * ((size_t)blocks_for(n, kScanTile) + 1);
}

hipError_t exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t n, void *temp,
                          hipStream_t s) {
  uint32_t nb = blocks_for(n, kScanTile);
  uint32_t *part = (uint32_t *)temp;
  if (n == 0) {
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, s, out, 0u);
    return hipGetLastError();
  }
  // (one tile: the down-sweep alone, which reads no tile sums for block 0)
  if (nb > 1) hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, s, in, n, part);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kThreads), 0, s, in, n, part, out);
  return hipGetLastError();
}

size_t radix_sort_temp_bytes(uint32_t n, uint32_t n_segs) {
  // tiles: at most one partial tile per segment beyond the whole ones
  // (the tile is smaller for small sorts: the larger of the two block counts)
  const uint32_t m = n > 0 ? n : 1;
  size_t nb = std::max<size_t>({blocks_for(m, kThreads * kSortItems),
                                blocks_for(std::min(m, kSmallSort), kThreads * kSortItemsSmall),
                                blocks_for(std::min(m, kTinySort), kThreads * kSortItemsTiny)}) +
              n_segs;
  size_t cnt = 256 * nb;
  return sizeof(uint32_t) * (2 * cnt + 1) + scan_temp_bytes((uint32_t)cnt) + 256;
}

hipError_t radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                      uint32_t n, int key_bits, void *temp, hipStream_t s, int *result_in_alt,
                      uint32_t n_segs, uint32_t seg_stride) {
  *result_in_alt = 0;
  if (n <= 1 || key_bits <= 0) return hipSuccess;
  if (n_segs == 0 || n % n_segs != 0) return hipErrorInvalidValue;
  SortSeg sg;
  sg.len = n / n_segs;
  sg.items = sort_items(n);
  sg.tiles = blocks_for(sg.len, kThreads * sg.items);
  sg.stride = n_segs > 1 ? seg_stride : 0u;
  const uint32_t nb = n_segs * sg.tiles;
  size_t cnt = 256 * (size_t)nb;
  uint32_t *counts = (uint32_t *)temp;
  uint32_t *offs = counts + cnt;
  void *stemp = (void *)(((uintptr_t)(offs + cnt + 1) + 255) & ~(uintptr_t)255);
  uint32_t *ka = keys, *va = vals, *kb = keys_alt, *vb = vals_alt;
  int alt = 0;
  // as many passes as 8-bit digits need, with the bits spread evenly over
  // them: the first pass's scatter runs are then longer (13-bit keys: 7 + 6
  // bits, not 8 + 5)
  const int passes = (key_bits + 7) / 8, per = (key_bits + passes - 1) / passes;
  for (int shift = 0; shift < key_bits; shift += per) {
    int nbits = key_bits - shift < per ? key_bits - shift : per;
    uint32_t mask = (1u << nbits) - 1u;
    hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(kThreads), 0, s, ka, sg, shift, mask, counts);
    hipError_t e = exclusive_scan(counts, offs, (uint32_t)cnt, stemp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(kThreads), 0, s, ka, va, sg, shift, nbits,
                       offs, kb, vb);
    uint32_t *tk = ka, *tv = va;
    ka = kb; va = vb; kb = tk; vb = tv;
    alt ^= 1;
  }
  *result_in_alt = alt;
  return hipGetLastError();
}

hipError_t launch_bounds_gather(const uint32_t *keys, const uint32_t *vals, uint32_t n,
                                uint32_t n_keys, uint32_t *cs, const int32_t *x, const int32_t *y,
                                const int32_t *t, const Geom &g, int32_t clamp_e, int4 *P,
                                uint32_t *prow, hipStream_t s) {
  hipLaunchKernelGGL(k_bounds_gather, dim3(xcd_grid(blocks_for((uint64_t)n + 1, kThreads))),
                     dim3(kThreads), 0, s, keys, vals, n, n_keys, cs, x, y, t, g, clamp_e, P,
                     prow);
  return hipGetLastError();
}

hipError_t launch_gather_rho(const uint32_t *vals, uint32_t n, const double *lambda, double *rho,
                             uint32_t *err, unsigned long long *rho_max, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rho, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, vals, n,
                     lambda, rho, err, rho_max);
  return hipGetLastError();
}

hipError_t launch_items(const uint32_t *cs, uint32_t n_sets, const Geom &g, bool row_items,
                        bool blocked, uint32_t split, uint32_t n_rows, uint32_t *chunks,
                        uint32_t *offs, uint32_t *set_base, Item *items, uint32_t *n_items,
                        void *scan_temp, hipStream_t s, Item *tmp, uint32_t max_slots) {
  const uint32_t unit = row_items ? (uint32_t)g.nx : 1u;
  const uint32_t n_units = g.n_cells / unit;
  const uint32_t tot = n_sets * n_units;
  const CentreIdx ci{g.n_cells, blocked};
  const uint32_t wave_blocks = blocks_for((uint64_t)tot * 64u, kThreads);
  hipLaunchKernelGGL(k_chunks, dim3(wave_blocks), dim3(kThreads), 0, s, cs, tot, unit, ci, chunks);
  hipError_t e = exclusive_scan(chunks, offs, tot, scan_temp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(kThreads), 0, s, offs, n_sets, n_units, split,
                     set_base, n_items);
  if (split > 1 && tmp) {
    // each item once into tmp, then its parts in parallel
    hipLaunchKernelGGL(k_emit, dim3(wave_blocks), dim3(kThreads), 0, s, cs, offs, set_base, n_sets,
                       n_units, unit, 1u, n_rows, ci, tmp);
    hipLaunchKernelGGL(k_expand, dim3(blocks_for(max_slots, kThreads)), dim3(kThreads), 0, s, tmp,
                       set_base, n_sets, split, n_rows, n_items, max_slots, items);
  } else {
    hipLaunchKernelGGL(k_emit, dim3(wave_blocks), dim3(kThreads), 0, s, cs, offs, set_base, n_sets,
                       n_units, unit, split, n_rows, ci, items);
  }
  return hipGetLastError();
}

hipError_t launch_zero3(const Zero3 &z, hipStream_t s) {
  const size_t n = std::max(z.n[0], std::max(z.n[1], z.n[2]));
  if (n == 0) return hipSuccess;
  uint32_t nb = blocks_for(n, kThreads);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero3, dim3(nb), dim3(kThreads), 0, s, z);
  return hipGetLastError();
}

}  // namespace ripk
