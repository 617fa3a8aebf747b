// The pair range count on gfx950 -- the hot loop of the space-time K estimator.
//
// For every centre i and every neighbour j of i in the cell stencil, the kernel
// decides the indicator of Eq. 3 (d_ij <= s_max and u_ij <= t_max, exact
// integers), finds the smallest grid step (k, l) that contains the pair, and
// adds the count and the edge-corrected weight 1/(omega_ij v_ij) of Sec. 3 to
// an (s, t) histogram held in LDS.  Histograms are merged into the set's global
// fixed-point bins with 64-bit atomics when a workgroup moves on to another
// point set.
//
// Mapping
//   * workgroup = 4 wavefronts; a work item = up to 64 consecutive centres of
//     one x-row of cells (or of one cell when some points are not centres), one
//     lane per centre; a workgroup grabs 4 items of one set at a time from a
//     work queue in one partition per XCD (persistent launch, items padded per
//     set);
//   * neighbours are visited as contiguous runs of the sorted point array (the
//     x-cells within reach of the item's first to last centre, per (y, t) row
//     of the stencil), staged per wave in an LDS tile of 64 points (the next
//     tile is fetched into registers while the current one is scanned; pending
//     pairs are drained before the tile is refilled) and read back as
//     wave-uniform broadcasts, two neighbours per LDS round trip;
//   * symmetric mode visits each unordered pair once (forward half of the
//     stencil, j > i inside the home cell) and adds both weights, since
//     omega_ij / v_ij depend on the centre while the bin depends on d and u only;
//   * divergence is removed in two levels: in-range pairs are compacted into a
//     per-wave LDS queue (4-byte tags naming the centre and the tile entry) and
//     binned 64 at a time (integer bin search, temporal weight, interior fast
//     path for omega); the pairs whose circle crosses the study boundary are
//     compacted again into a second queue where the trigonometric weight runs
//     with full lanes.  Each queue has one drain site in the scan loop, so the
//     drains are inlined once rather than at every push.
//
// Candidate test (one neighbour against 64 centres), by distance mode:
//   PACKED: low 16 bits of x and y packed in one word; one packed 16-bit
//           subtract and one 2-way dot product give dx^2 + dy^2 exactly while
//           |dx|, |dy| < 2^15 (cells no wider than 2^15 / (reach + 1));
//   U32:    32-bit squares with the 24-bit multiplier (d^2 < 2^32);
//   WIDE:   64-bit squares and compare.
// The time test is |t_i - t_j| <= t_max  <=>  (t_i + t_max - t_j) <= 2 t_max as
// unsigned 32-bit values (t_max < 2^30).
//
// Weights are FP32: w = 1/omega * 1/v lies in [1, 8], so w * 2^23 is an exact
// integer and the fixed-point sums are exact and order independent.  Polygon
// weights (1/omega has no fixed bound there) and inhomogeneous weights are
// rounded per side to a fixed-point integer below 2^96 in FP64 and summed as
// three 32-bit pieces, equally exact and order independent.
#include "poly.h"
#include "ripk_internal.h"

namespace ripk {

namespace {

constexpr int kJT = 64;     // points per tile slot (two slots per wave)
constexpr int kGroup = 2;       // neighbours tested between two drain checks
// ring of queue A tags: at most 63 + 64 * kGroup are pending at any time
constexpr uint32_t kQA = 64 * kGroup + 64;
constexpr int kQB = 128;    // ring of queue B records: < 64 + 64 pending between drains
constexpr int kWaves = kPairThreads / 64;
// Bound on the candidates a workgroup evaluates between histogram flushes
// (checked before each group of items).  Counts hold pairs (not doubled in
// symmetric mode), and one group examines fewer than 256 n candidates.  Split
// bins: a 32-bit count stays below 2^31 + 2^31 when a set has fewer than 2^23
// points (larger sets use 64-bit count words).  Packed bins: a count stays
// below 2^29 + 2^29 = 2^30 when a set has fewer than 2^21 points, and the
// interior weight field (at most 4 units of 2^23 per pair) below 2^32.  Wide
// bins take the packed bound: with sets below 2^22 points fewer than 2^31
// pairs are pending per bin, each adding below 2^33 to a piece sum.
constexpr unsigned long long kFlushEvals = 1ull << 31;
constexpr unsigned long long kFlushEvalsPacked = 1ull << 29;
constexpr int kCountShift = 34;
constexpr unsigned long long kUnitMask = (1ull << kCountShift) - 1ull;
constexpr uint32_t kFarTime = 0xC0000000u;  // tile padding: fails every time test
constexpr uint32_t kClampE = 32767u;         // side distances stored in 15 bits (PACKED)

// LDS image of a point.  PACKED: {x|y<<16 (low 16 bits each), t, ex|ey<<16,
// min(ex,ey)^2}; U32 / WIDE: {x, y, t, min side distance}.  Coordinates are
// window relative; ex, ey are the distances to the nearer x and y side.
// Images are stored as structures of arrays (component c of entry e at
// f[c][e]): lanes that read different entries hit consecutive banks, and the
// scan reads one component of four consecutive neighbours in one access.
struct WaveLds {
  uint32_t tile[4][kJT];      // the tile of neighbour points being scanned
  uint32_t cen[4][64];        // the wave's centres
  uint32_t qa[kQA + 64];  // in-range pairs: byte offsets in this block, centre | neighbour << 16;
                          // the 64 extra entries take a push that crosses the ring's end
  uint4 qb[kQB];       // boundary weights, see drain_b
};

static_assert(sizeof(WaveLds) % 16 == 0, "the histogram after the wave blocks must stay 16-byte aligned");
constexpr uint32_t kTileStride = kJT * 4;  // bytes between components of a tile entry
constexpr uint32_t kCenStride = 64 * 4;        // bytes between components of a centre
constexpr uint32_t kTileOff = 0;               // byte offsets of tile and cen in WaveLds
constexpr uint32_t kCenOff = 4 * kJT * 4;
static_assert(offsetof(WaveLds, tile) == kTileOff && offsetof(WaveLds, cen) == kCenOff,
              "tag decoding assumes the WaveLds layout");

__device__ __forceinline__ int4 load_image(const unsigned char *base, uint32_t stride) {
  return make_int4(*(const int *)base, *(const int *)(base + stride),
                   *(const int *)(base + 2 * stride), *(const int *)(base + 3 * stride));
}

struct QState {
  uint32_t ha, ta;      // queue A head and tail positions in [0, kQA); the head is a
                        // multiple of 64 (full drains take 64 entries, and a partial
                        // drain empties the queue and restarts it at 0)
  uint32_t hb, nb;      // queue B head and length
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// dx^2 + dy^2 of two signed 16-bit halves (|dx|, |dy| < 2^15, so the sum fits
// in 31 bits).  The three-operand dot product takes its zero addend inline;
// the accumulating two-operand form would need a register cleared each time.
__device__ __forceinline__ uint32_t sq16x2(uint32_t d) {
  uint32_t r;
  asm("v_dot2_i32_i16 %0, %1, %1, 0" : "=v"(r) : "v"(d));
  return r;
}

// |a - b| of unsigned values in one instruction (sum of absolute differences)
__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// position of this lane among the set lanes of `mask`, plus `base`
__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask, uint32_t base) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, base));
}

// arctan(z) for z in [0, 1]: z * P(z^2), P of degree 8 in z^2 fitted (near-minimax,
// iteratively reweighted least squares) to arctan over [0, 1]; largest error of the
// fit 6e-9, about 1e-7 once evaluated in FP32 with fused multiply-adds.
__device__ __forceinline__ float atan01(float z) {
  const float w = z * z;
  float p = 0.002456706715747714f;
  p = fmaf(p, w, -0.014401290565729141f);
  p = fmaf(p, w, 0.0397811196744442f);
  p = fmaf(p, w, -0.07234849780797958f);
  p = fmaf(p, w, 0.1049894317984581f);
  p = fmaf(p, w, -0.14161229133605957f);
  p = fmaf(p, w, 0.19985906779766083f);
  p = fmaf(p, w, -0.33332598209381104f);
  p = fmaf(p, w, 0.9999998807907104f);
  return p * z;
}

// Isotropic correction on the rectangle in FP32 from the distances ex, ey to the
// nearer x side and the nearer y side (only these can cut a circle of radius
// <= min(W, H)/2).  With h_e = sqrt(max(d2 - e^2, 0)) (d2 - e^2 is an exact
// integer), the angle beta_e = atan2(e, h_e) between the radius to a side's
// crossing point and that side is pi/2 for an uncut side; the excluded
// half-arcs are pi/2 - beta_e and two cut sides overlap by
// max(0, pi/2 - beta_x - beta_y), so without branches
//   omega = S/pi + max(0, pi/2 - S)/(2 pi),   S = beta_x + beta_y:
// 1 with no cut, 1/2 + beta/pi with one, S/pi with two and the corner outside
// the circle, 1/4 + S/(2 pi) with it inside.  S is the argument of the
// product (h_x + i e_x)(h_y + i e_y) = (h_x h_y - e_x e_y) + i (e_x h_y + e_y h_x),
// a vector of length d2 in the upper half plane, so one arctangent gives it:
// S in [0, pi], the real part rounded with an absolute error near 1e-7 d2.
__device__ __forceinline__ float omega_hh(float ex, float ey, float hx, float hy) {
  const float im = fmaf(ex, hy, ey * hx);
  const float re = fmaf(hx, hy, -(ex * ey));
  const float are = fabsf(re);
  const float lo = fminf(im, are), hi = fmaxf(im, are);
  // quotient from the hardware reciprocal (about 1 ulp): the weight stays
  // within 3e-7 of the exact one (FP32 emulation against FP64 acos)
  float a = atan01(lo * __builtin_amdgcn_rcpf(hi));
  a = im > are ? 1.5707963267948966f - a : a;
  const float S = re < 0.0f ? 3.14159265358979323846f - a : a;
  // S/pi + max(0, pi/2 - S)/(2 pi) = max(S/pi, 1/4 + S/(2 pi)) (equal at S = pi/2)
  const float inv_pi = 0.318309886183790671538f;
  return fmaxf(S * inv_pi, fmaf(S, 0.5f * inv_pi, 0.25f));
}

// An uncut side (e^2 >= d2) enters with h = 0 and e replaced by 1: its angle
// is pi/2 whatever e is, and with e = 1 the products above are exact, so the
// result does not depend on how e was stored (clamped in PACKED images).
__device__ __forceinline__ float omega_f32(uint32_t ex, uint32_t ey, uint64_t d2) {
  const uint64_t ex2 = (uint64_t)ex * ex, ey2 = (uint64_t)ey * ey;
  const bool cx = ex2 < d2, cy = ey2 < d2;
  const float hx = __builtin_amdgcn_sqrtf((float)(cx ? d2 - ex2 : 0ull));
  const float hy = __builtin_amdgcn_sqrtf((float)(cy ? d2 - ey2 : 0ull));
  return omega_hh(cx ? (float)ex : 1.0f, cy ? (float)ey : 1.0f, hx, hy);
}

// the same with d2 < 2^31 and ex, ey < 2^15 (all squares exact in 32 bits)
__device__ __forceinline__ float omega_f32(uint32_t ex, uint32_t ey, uint32_t d2) {
  const uint32_t ex2 = __umul24(ex, ex), ey2 = __umul24(ey, ey);
  const bool cx = ex2 < d2, cy = ey2 < d2;
  const float hx = __builtin_amdgcn_sqrtf((float)(cx ? d2 - ex2 : 0u));
  const float hy = __builtin_amdgcn_sqrtf((float)(cy ? d2 - ey2 : 0u));
  return omega_hh(cx ? (float)ex : 1.0f, cy ? (float)ey : 1.0f, hx, hy);
}

// Queue B: boundary weights with full lanes.  Records:
//   PACKED: one per pair, {bin | half_i<<12 | half_j<<13 | slow_i<<14 | slow_j<<15,
//           d2, ex_i|ey_i<<16, ex_j|ey_j<<16}: both sides' weights in one pass;
//   U32 / WIDE: one per side, {bin | half<<12 | d2 hi<<13, d2 lo, ex, ey}.
// The weight goes to the bin's weight word hw[bin].
__device__ __forceinline__ uint32_t qweight(float om, uint32_t half) {
  // w = 1/omega >= 1 has at most 23 fraction bits: w * 2^23 is an exact integer;
  // the reciprocal is within an ulp, well inside the error budget
  const float w = fmaxf(__builtin_amdgcn_rcpf(om), 1.0f);
  return (uint32_t)(w * (float)(1u << kFracBits)) << half;
}

// Wide weights: x, a non-negative integer below 2^96 held exactly in a double,
// added to the sums p0, p1, p2 of its three 32-bit pieces (the differences
// below are exact, so is each piece).
struct Pieces {
  unsigned long long p0 = 0, p1 = 0, p2 = 0;
  __device__ __forceinline__ void add(double x) {
    const double hi = floor(x * 0x1p-64);
    const double r1 = fma(hi, -0x1p64, x);
    const double mid = floor(r1 * 0x1p-32);
    const double r0 = fma(mid, -0x1p32, r1);
    p0 += (uint32_t)r0;
    p1 += (uint32_t)mid;
    p2 += (uint32_t)hi;
  }
  // into the bin's three LDS words (pieces that are zero cost no atomic)
  __device__ __forceinline__ void commit(unsigned long long *w3) const {
    if (p0) atomicAdd(&w3[0], p0);
    if (p1) atomicAdd(&w3[1], p1);
    if (p2) atomicAdd(&w3[2], p2);
  }
};

// Polygon weight of one side: 1/omega (omega from FP64 angles) times 2^(23 +
// half), rounded to an integer.  A neighbour j lies strictly inside the polygon
// and on the circle, at least 1/|E| from every edge line on the integer
// lattice (|E| < 2^24.5), so omega >= 1/(pi |E| s_max) and the value stays
// below 2^75.
__device__ __forceinline__ double qweight_poly(double inv_om, uint32_t half) {
  return rint(inv_om * (double)(1u << (kFracBits + half)));
}

// Polygon records (every distance mode), one per boundary side: {bin |
// half<<12 | d2 hi<<16, d2 lo, c, 0} with c the sorted-record index of the
// side's centre; the weight goes to the bin's three wide words hw[3 bin ..]
// (see Pieces).
// INHOM records name both points, one per pair with a boundary side: {bin |
// half_i<<12 | half_j<<13 | slow_i<<14 | slow_j<<15 | d2 hi<<16, d2 lo, i, j};
// per side the rectangle's weight w times
// 1/(lambda_i lambda_j) = rho_i rho_j, scaled by 2^F (wscale) and 2^half and
// rounded: round(((w rho_i rho_j) 2^F) 2^half), which is the interior path's
// value when w = 1.
template <int MODE, bool POLY, bool INHOM>
__device__ __forceinline__ void drain_b(WaveLds &W, QState &q, uint32_t c, int lane,
                                        unsigned long long *hw, const Geom &g,
                                        const int4 *__restrict__ P,
                                        const double *__restrict__ rho, double wscale) {
  wave_sync();
  const uint4 r = W.qb[(q.hb + lane) & (kQB - 1)];
  wave_sync();
  const uint32_t bin = r.x & 0xFFFu;
  if (POLY) {
    // one side per record: {bin | half<<12 | d2 hi<<16, d2 lo, centre record, 0}
    const uint64_t d2 = (uint64_t)r.y | ((uint64_t)(r.x >> 16) << 32);
    if ((uint32_t)lane < c) {
      Pieces pc;
      const int4 p = P[r.z];
      pc.add(qweight_poly(poly_inv_omega(g, p.x, p.y, d2, r.z), (r.x >> 12) & 1u));
      pc.commit(hw + 3 * bin);
    }
    q.hb = (q.hb + c) & (kQB - 1);
    q.nb -= c;
    return;
  }
  if (INHOM) {
    const uint64_t d2 = (uint64_t)r.y | ((uint64_t)(r.x >> 16) << 32);
    if ((uint32_t)lane < c) {
      Pieces pc;
      const double rr = rho[r.z] * rho[r.w];
#pragma unroll 1
      for (uint32_t side = 0; side < 2; ++side) {
        if ((r.x >> (14 + side)) & 1u) {
          const int4 p = P[side ? r.w : r.z];
          const uint32_t half = (r.x >> (12 + side)) & 1u;
          const uint32_t ex = (uint32_t)min(p.x, g.x1 - g.x0 - p.x);
          const uint32_t ey = (uint32_t)min(p.y, g.y1 - g.y0 - p.y);
          const float w = fmaxf(__builtin_amdgcn_rcpf(omega_f32(ex, ey, d2)), 1.0f);
          pc.add(rint((((double)w * rr) * wscale) * (double)(1u << half)));
        }
      }
      pc.commit(hw + 3 * bin);
    }
    q.hb = (q.hb + c) & (kQB - 1);
    q.nb -= c;
    return;
  }
  // rectangle: queue A already added the interior value (1 + half) 2^23 of
  // every side, so a boundary side adds its excess over it (w >= 1)
  uint32_t qv;
  if (MODE == kModePacked) {
    // d2 < 2^31 and side distances < 2^15: 32-bit arithmetic throughout
    const float oi = omega_f32(r.z & 0xFFFFu, r.z >> 16, r.y);
    const float oj = omega_f32(r.w & 0xFFFFu, r.w >> 16, r.y);
    const uint32_t hi = (r.x >> 12) & 1u, hj = (r.x >> 13) & 1u;
    qv = (((r.x >> 14) & 1u) ? qweight(oi, hi) - ((1u + hi) << kFracBits) : 0u) +
         (((r.x >> 15) & 1u) ? qweight(oj, hj) - ((1u + hj) << kFracBits) : 0u);
  } else {
    const uint32_t h = (r.x >> 12) & 1u;
    qv = qweight(omega_f32(r.z, r.w, (uint64_t)r.y | ((uint64_t)(r.x >> 13) << 32)), h) -
         ((1u + h) << kFracBits);
  }
  if ((uint32_t)lane < c) atomicAdd(&hw[bin], (unsigned long long)qv);
  q.hb = (q.hb + c) & (kQB - 1);
  q.nb -= c;
}

// pending queue A entries (fewer than kQA, so head == tail means none)
__device__ __forceinline__ uint32_t na_of(const QState &q) {
  return q.ta >= q.ha ? q.ta - q.ha : q.ta + kQA - q.ha;
}

struct Side {
  uint32_t T, ex, ey;
  bool slow;  // the circle of radius d crosses the study boundary (never true
              // without spatial correction: the image's interior bound is then
              // out of reach)
};

template <int MODE>
__device__ __forceinline__ Side side_of(const int4 p, uint32_t d2lo, uint64_t d2, const Geom &g) {
  Side s;
  if (MODE == kModePacked) {
    s.T = (uint32_t)p.y;
    s.ex = (uint32_t)p.z & 0xFFFFu;
    s.ey = (uint32_t)p.z >> 16;
    s.slow = d2lo > (uint32_t)p.w;
  } else {
    s.T = (uint32_t)p.z;
    s.ex = (uint32_t)min(p.x, g.x1 - g.x0 - p.x);
    s.ey = (uint32_t)min(p.y, g.y1 - g.y0 - p.y);
    s.slow = d2 > (uint64_t)(uint32_t)p.w * (uint32_t)p.w;
  }
  return s;
}

// Queue A: the c oldest in-range pairs.  Distances are recomputed from the
// centre and neighbour images; the bin, the temporal weight and the interior
// fast path of omega are evaluated without branches on per-lane data (lanes
// past c compute on entry 0 and store nothing); boundary sides go to queue B.
// (POLY: `begin` is the first centre's record index, `tb` the tile's.)
template <bool SYM, int MODE, bool POLY, bool INHOM>
__device__ __forceinline__ void drain_a(WaveLds &W, QState &q,
                                        uint32_t c, int lane, const Geom &g,
                                        unsigned long long *hist, void *aux, int bins,
                                        const uint32_t *S2lo,
                                        const uint32_t *S2hi, const uint32_t *T,
                                        uint32_t begin, uint32_t tb, const int4 *P,
                                        const double *rho, const double *rho_c,
                                        const double *rho_t, double wscale) {
  // boundary weights: their own words with packed or wide bins, else the
  // weight words
  unsigned long long *hw =
      (POLY || INHOM || bins == kBinsPacked) ? (unsigned long long *)aux : hist;
  wave_sync();
  const uint32_t tag0 = W.qa[q.ha + (uint32_t)lane];  // q.ha + 63 < kQA: no wrap
  wave_sync();
  const bool v = (uint32_t)lane < c;
  const unsigned long long vmask = c >= 64 ? ~0ull : ((1ull << c) - 1ull);
  // a tag holds the byte offsets, within the wave's LDS block, of the centre
  // (low half) and of the neighbour (high half); lanes past c read offset 0
  // and store nothing
  const uint32_t tag = v ? tag0 : 0u;
  const unsigned char *wb = (const unsigned char *)&W;
  const int4 pi = load_image(wb + (tag & 0xFFFFu), kCenStride);
  const int4 pj = load_image(wb + (tag >> 16), kTileStride);
  uint32_t d2lo, d2hi = 0, u;
  if (MODE == kModePacked) {
    typedef short s2 __attribute__((ext_vector_type(2)));
    const s2 dd = __builtin_bit_cast(s2, pi.x) - __builtin_bit_cast(s2, pj.x);
    d2lo = sq16x2(__builtin_bit_cast(uint32_t, dd));
    u = absdiff((uint32_t)pi.y, (uint32_t)pj.y);
  } else if (MODE == kModeU32) {
    const int32_t dx = pi.x - pj.x, dy = pi.y - pj.y;
    d2lo = (uint32_t)__mul24(dx, dx) + (uint32_t)__mul24(dy, dy);
    u = absdiff((uint32_t)pi.z, (uint32_t)pj.z);
  } else {
    const int64_t dx = (int64_t)(pi.x - pj.x), dy = (int64_t)(pi.y - pj.y);
    const uint64_t dd = (uint64_t)(dx * dx + dy * dy);
    d2lo = (uint32_t)dd;
    d2hi = (uint32_t)(dd >> 32);
    u = absdiff((uint32_t)pi.z, (uint32_t)pj.z);
  }
  const uint64_t d2 = ((uint64_t)d2hi << 32) | d2lo;
  // The step k* = max(1, ceil(x)), x = sqrt(d2) n_s / s_max, is exact in the
  // tables (S2[k] = floor(s_k^2) and d2 is an integer).  inv_ds carries a
  // factor 1 - 2^-20, larger than the FP32 error of the quotient, so x' < x
  // whenever x > 0 and trunc(x') + 1 is k* or k* - 1: one comparison with the
  // table restores the exact step.  The time estimate u n_t / t_max is formed
  // the same way (inv_dt; u < 2^30 is rounded to FP32 within 2^-24) and
  // corrected with the T table.  kk, ll are the 0-based steps.
  const float d2f = MODE == kModeWide ? (float)d2 : (float)d2lo;
  const uint32_t k0 = (uint32_t)(__builtin_amdgcn_sqrtf(d2f) * g.inv_ds);
  const uint32_t l0 = (uint32_t)((float)u * g.inv_dt);
  const uint32_t sk = S2lo[k0], tl = T[l0];
  bool up_k;
  if (MODE == kModeWide)
    up_k = d2 > ((uint64_t)sk | ((uint64_t)S2hi[k0] << 32));
  else
    up_k = d2lo > sk;
  const uint32_t kk = k0 + (uint32_t)up_k, ll = l0 + (uint32_t)(u > tl);
  const uint32_t bin = __umul24(kk, (uint32_t)g.n_t) + ll;
  const uint32_t D = (uint32_t)(g.t1 - g.t0);
  const bool tp = (g.edge & 2u) != 0;
  // v = 1/2 when an end of [t-u, t+u] leaves the period: the weight doubles
  const Side si = side_of<MODE>(pi, d2lo, d2, g);
  const uint32_t hfi = (tp && u > min(si.T, D - si.T)) ? 1u : 0u;
  Side sj = si;
  sj.slow = false;
  uint32_t hfj = 0;
  if (SYM) {
    sj = side_of<MODE>(pj, d2lo, d2, g);
    hfj = (tp && u > min(sj.T, D - sj.T)) ? 1u : 0u;
  }
  // interior values in units of 2^23: the rectangle adds 1 + half for every
  // side (queue B adds a boundary side's excess); polygon launches only the
  // sides that take the interior path (queue B adds the others whole)
  uint32_t units;
  if (POLY || INHOM)
    units = (si.slow ? 0u : 1u + hfi) + ((SYM && !sj.slow) ? 1u + hfj : 0u);
  else
    units = 1u + hfi + (SYM ? 1u + hfj : 0u);
  const uint32_t qsum = units << kFracBits;
  // boundary-queue mask, taken next to the compares (separate ballots fold
  // into their masks; taken after the branch below they would be rebuilt)
  const unsigned long long mslow =
      (__builtin_amdgcn_ballot_w64(si.slow) | (SYM ? __builtin_amdgcn_ballot_w64(sj.slow) : 0ull)) & vmask;
  // packed bins: the count and the interior weights in one atomic; split
  // bins: weights hist[bin], counts in the aux array (32-bit words unless the
  // set is large); wide bins (POLY, INHOM): counts hist[bin], weights in the
  // three words aux[3 bin ..]
  if (POLY || INHOM) {
    if (v) {
      atomicAdd(&hist[bin], 1ull);
      unsigned long long *w3 = (unsigned long long *)aux + 3 * bin;
      if (INHOM) {
        // interior sides: round((rho_i rho_j 2^F) 2^half) each
        const uint32_t ci = ((tag & 0xFFFFu) - kCenOff) >> 2;
        const uint32_t tj = ((tag >> 16) - kTileOff) >> 2;
        const double r = (rho_c[ci] * rho_t[tj]) * wscale;
        Pieces pc;
        if (!si.slow) pc.add(rint(r * (double)(1u << hfi)));
        if (SYM && !sj.slow) pc.add(rint(r * (double)(1u << hfj)));
        pc.commit(w3);
      } else if (qsum) {
        atomicAdd(w3, (unsigned long long)qsum);
      }
    }
  } else if (v) {
    if (bins == kBinsPacked) {
      atomicAdd(&hist[bin], (1ull << kCountShift) | (unsigned long long)units);
    } else {
      atomicAdd(&hist[bin], (unsigned long long)qsum);
      if (bins == kBinsSplit64)
        atomicAdd((unsigned long long *)aux + bin, 1ull);
      else
        atomicAdd((uint32_t *)aux + bin, 1u);
    }
  }
  if (c == 64) {
    q.ha = q.ha + 64 == kQA ? 0u : q.ha + 64;
  } else {
    // a partial drain takes every pending entry
    q.ha = 0;
    q.ta = 0;
  }
  if (POLY) {
    // one record per boundary side, naming its centre's sorted record: the
    // costly weight then runs once per record with every lane busy
#pragma unroll 1
    for (int side = 0; side < (SYM ? 2 : 1); ++side) {
      const bool need = side ? sj.slow : si.slow;
      const unsigned long long m = __builtin_amdgcn_ballot_w64(need) & vmask;
      if (m) {
        const uint32_t pos = lane_rank(m, q.hb + q.nb) & (kQB - 1);
        q.nb += (uint32_t)__popcll(m);
        if (need && v)
          W.qb[pos] = make_uint4(bin | ((side ? hfj : hfi) << 12) | (d2hi << 16), d2lo,
                                 side ? tb + (((tag >> 16) - kTileOff) >> 2)
                                      : begin + (((tag & 0xFFFFu) - kCenOff) >> 2),
                                 0u);
        if (q.nb >= 64) drain_b<MODE, POLY, INHOM>(W, q, 64, lane, hw, g, P, rho, wscale);
      }
    }
  } else if (INHOM) {
    // one record per pair with a boundary side, naming both points
    const bool need = si.slow || sj.slow;
    const unsigned long long m = mslow;
    if (m) {
      const uint32_t pos = lane_rank(m, q.hb + q.nb) & (kQB - 1);
      q.nb += (uint32_t)__popcll(m);
      if (need && v)
        W.qb[pos] = make_uint4(bin | (hfi << 12) | (hfj << 13) | ((uint32_t)si.slow << 14) |
                                   ((uint32_t)(SYM && sj.slow) << 15) | (d2hi << 16),
                               d2lo, begin + (((tag & 0xFFFFu) - kCenOff) >> 2),
                               tb + (((tag >> 16) - kTileOff) >> 2));
      if (q.nb >= 64) drain_b<MODE, POLY, INHOM>(W, q, 64, lane, hw, g, P, rho, wscale);
    }
  } else if (MODE == kModePacked) {
    // one record per pair with a boundary side
    const bool need = si.slow || sj.slow;
    const unsigned long long m = mslow;
    if (m) {
      const uint32_t pos = lane_rank(m, q.hb + q.nb) & (kQB - 1);
      q.nb += (uint32_t)__popcll(m);
      if (need && v)
        W.qb[pos] = make_uint4(bin | (hfi << 12) | (hfj << 13) | ((uint32_t)si.slow << 14) |
                                   ((uint32_t)(SYM && sj.slow) << 15),
                               d2lo, (uint32_t)pi.z, (uint32_t)pj.z);
      if (q.nb >= 64) drain_b<MODE, POLY, INHOM>(W, q, 64, lane, hw, g, P, rho, wscale);
    }
  } else {
    // one record per boundary side, one side per pass through a single drain site
    const uint32_t w0 = bin | (d2hi << 13);
#pragma unroll 1
    for (int side = 0; side < (SYM ? 2 : 1); ++side) {
      const bool need = side ? sj.slow : si.slow;
      const unsigned long long m = __builtin_amdgcn_ballot_w64(need) & vmask;
      if (m) {
        const uint32_t pos = lane_rank(m, q.hb + q.nb) & (kQB - 1);
        q.nb += (uint32_t)__popcll(m);
        if (need && v)
          W.qb[pos] = make_uint4(w0 | ((side ? hfj : hfi) << 12), d2lo, side ? sj.ex : si.ex,
                                 side ? sj.ey : si.ey);
        if (q.nb >= 64) drain_b<MODE, POLY, INHOM>(W, q, 64, lane, hw, g, P, rho, wscale);
      }
    }
  }
}

// LDS image of a sorted point (see WaveLds).  Without spatial correction the
// interior bound (min(ex,ey)^2, or the side distance) is set to 2^32 - 1 so
// that no pair takes the boundary path.  (POLY: the interior bound is the
// record's distance to the polygon.)
template <int MODE, bool POLY>
__device__ __forceinline__ int4 image(const int4 p, const Geom &g) {
  const bool iso = (g.edge & 1u) != 0;
  if (MODE == kModePacked) {
    const uint32_t ex = min((uint32_t)min(p.x, g.x1 - g.x0 - p.x), kClampE);
    const uint32_t ey = min((uint32_t)min(p.y, g.y1 - g.y0 - p.y), kClampE);
    const uint32_t e = POLY ? (uint32_t)p.w : min(ex, ey);
    return make_int4((int)(((uint32_t)p.x & 0xFFFFu) | ((uint32_t)p.y << 16)), p.z,
                     (int)(ex | (ey << 16)), iso ? (int)(e * e) : -1);
  }
  return make_int4(p.x, p.y, p.z, iso ? p.w : -1);
}

template <int MODE>
__device__ __forceinline__ int4 far_image() {
  return MODE == kModePacked ? make_int4(0, (int)kFarTime, 0, 0)
                             : make_int4(0, 0, (int)kFarTime, 0);
}

// Candidate test of one neighbour against this lane's centre: cs = space test,
// ct = time test (kept apart so that each ballot folds to its compare mask).
// PACKED compares d2 (< 2^31) as a signed value with the lane's own bound:
// s2max for a centre, -1 for an empty lane, which then never passes.
template <int MODE>
__device__ __forceinline__ void cand(const int4 me, uint32_t tplus, int thr, const int4 pj,
                                     const Geom &g, bool &cs, bool &ct) {
  uint32_t dtp;
  if (MODE == kModePacked) {
    typedef short s2 __attribute__((ext_vector_type(2)));
    const s2 d = __builtin_bit_cast(s2, me.x) - __builtin_bit_cast(s2, pj.x);
    cs = (int)sq16x2(__builtin_bit_cast(uint32_t, d)) <= thr;
    dtp = tplus - (uint32_t)pj.y;
  } else if (MODE == kModeU32) {
    const int32_t dx = me.x - pj.x, dy = me.y - pj.y;
    cs = (uint32_t)__mul24(dx, dx) + (uint32_t)__mul24(dy, dy) <= (uint32_t)g.s2max;
    dtp = tplus - (uint32_t)pj.z;
  } else {
    const int64_t dx = (int64_t)(me.x - pj.x), dy = (int64_t)(me.y - pj.y);
    cs = (uint64_t)(dx * dx + dy * dy) <= g.s2max;
    dtp = tplus - (uint32_t)pj.z;
  }
  ct = dtp <= 2u * g.tmax;
}

template <bool SYM, int MODE, bool POLY, bool INHOM>
struct Ctx {
  WaveLds &W;
  QState &q;
  const Geom &g;
  unsigned long long *hist;  // packed count and weight, the weight, or the count per bin
  void *aux;                 // boundary weights (packed), pair counts (split) or the
                             // three piece sums of the weights (wide)
  int bins;                  // bin layout
  const uint32_t *S2lo, *S2hi, *T;
  int lane;
  uint32_t begin;  // record index of the item's first centre
  uint32_t tb;     // record index of the first entry of the tile in LDS
  const int4 *P;   // sorted records
  const double *rho;            // INHOM: 1/lambda per sorted record
  double *rho_c, *rho_t;        // INHOM: rho of the wave's centres and tile (LDS)
  double wscale;                // INHOM: 2^F of the fixed-point weights
};

template <bool SYM, int MODE, bool POLY, bool INHOM>
__device__ __forceinline__ void drain_oldest(Ctx<SYM, MODE, POLY, INHOM> &x, uint32_t c) {
  drain_a<SYM, MODE, POLY, INHOM>(x.W, x.q, c, x.lane, x.g, x.hist, x.aux, x.bins,
                                  x.S2lo, x.S2hi, x.T, x.begin, x.tb, x.P, x.rho, x.rho_c,
                                  x.rho_t, x.wscale);
}

// One run of consecutive sorted points [j0, j1) against the wave's centres.
// HOME: the run holds the centres' own cell (j > i in symmetric mode, j != i
// otherwise).
template <bool SYM, int MODE, bool POLY, bool INHOM, bool HOME>
__device__ __forceinline__ void scan_run(Ctx<SYM, MODE, POLY, INHOM> &x, uint32_t j0, uint32_t j1,
                                         const int4 me, uint32_t tplus, int thr, bool lv,
                                         unsigned long long valid, uint32_t mi,
                                         const int4 *__restrict__ P) {
  QState &q = x.q;
  WaveLds &W = x.W;
  const int lane = x.lane;
  if (j0 >= j1) return;
  // raw record of the next tile; converted to its LDS image only when stored,
  // so that the load stays in flight while the current tile is scanned
  int4 nxt = make_int4(0, 0, 0, 0);
  double nxt_rho = 0.0;
  bool nxt_ok = j0 + (uint32_t)lane < j1;
  if (nxt_ok) {
    nxt = P[j0 + lane];
    if (INHOM) nxt_rho = x.rho[j0 + lane];
  }
  for (uint32_t tb = j0; tb < j1; tb += kJT) {
    const uint32_t nt = uni(min((uint32_t)kJT, j1 - tb));
    // every pending entry refers to the tile about to be overwritten
    {
      const uint32_t na = na_of(q);
      if (na) drain_oldest(x, na);
    }
    x.tb = tb;
    wave_sync();
    {
      const int4 im = nxt_ok ? image<MODE, POLY>(nxt, x.g) : far_image<MODE>();
      W.tile[0][lane] = (uint32_t)im.x;
      W.tile[1][lane] = (uint32_t)im.y;
      W.tile[2][lane] = (uint32_t)im.z;
      W.tile[3][lane] = (uint32_t)im.w;
      if (INHOM) x.rho_t[lane] = nxt_ok ? nxt_rho : 0.0;
    }
    wave_sync();
    const uint32_t tn = tb + kJT;
    if (tn < j1) {
      nxt_ok = tn + (uint32_t)lane < j1;
      if (nxt_ok) {
        nxt = P[tn + lane];
        if (INHOM) nxt_rho = x.rho[tn + lane];
      }
    }
    // byte offsets, within the wave's LDS block, of this lane's centre and of
    // the tile's first entry
    const uint32_t lane_tag =
        (uint32_t)((const unsigned char *)&W.cen[0][lane] - (const unsigned char *)&W) |
        ((uint32_t)((const unsigned char *)&W.tile[0][0] - (const unsigned char *)&W) << 16);
    // four neighbours per LDS access, a drain check after every kGroup; a
    // partial last group reads padding entries, which fail every time test
    typedef uint32_t gvec __attribute__((ext_vector_type(4)));
    static_assert(kGroup == 2, "the scan takes two pushes per drain check");
    for (uint32_t jj = 0; jj < nt; jj += 4) {
      int4 pj[4];
      {
        // components the candidate test needs
        const gvec c0 = *(const gvec *)&W.tile[0][jj];
        const gvec c1 = *(const gvec *)&W.tile[1][jj];
        gvec c2 = c1;
        if (MODE != kModePacked) c2 = *(const gvec *)&W.tile[2][jj];
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = make_int4((int)c0[u], (int)c1[u], (int)c2[u], 0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bool cs, ct;
        cand<MODE>(me, tplus, thr, pj[u], x.g, cs, ct);
        const uint32_t j = tb + jj + u;
        const bool hc = HOME ? (SYM ? (j > mi) : (j != mi)) : true;
        // separate ballots fold into the compare masks; the per-lane predicate
        // only steers the store (PACKED: empty lanes already fail cs).  Almost
        // every neighbour has some centre in range, so there is no test for
        // an empty mask.
        unsigned long long mask = __builtin_amdgcn_ballot_w64(cs) & __builtin_amdgcn_ballot_w64(ct);
        if (MODE != kModePacked) mask &= valid;
        if (HOME) mask &= __builtin_amdgcn_ballot_w64(hc);
        const uint32_t base = q.ta;
        q.ta = base + (uint32_t)__popcll(mask);
        const bool pass = MODE == kModePacked ? (cs & ct & hc) : (cs & ct & lv & hc);
        if (pass) W.qa[base + lane_rank(mask, 0)] = lane_tag + ((jj + u) << 18);
        if (q.ta >= kQA) {
          // the push reached the ring's end: move what ran past it to the
          // start (those slots were drained: fewer than kQA are pending)
          const uint32_t over = q.ta - kQA;
          if (over) {
            wave_sync();
            if ((uint32_t)lane < over) W.qa[lane] = W.qa[kQA + lane];
            wave_sync();
          }
          q.ta = over;
        }
        if (u & 1)
          for (uint32_t na = na_of(q); na >= 64; na -= 64) drain_oldest(x, 64);
      }
    }
  }
}

// (the polygon variants are held to 128 VGPRs: 4 waves per SIMD)
template <bool SYM, int MODE, bool POLY, bool INHOM>
__global__ void __launch_bounds__(kPairThreads) __attribute__((amdgpu_waves_per_eu(POLY ? 4 : 1)))
k_pair(PairArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom &g = a.g;
  const int NB = g.n_s * g.n_t;
  // LDS: the waves' blocks first (fixed offsets), then the bin words, the aux
  // words (boundary weights or pair counts, see kBinsPacked), the threshold
  // tables (n_s, n_s and n_t words, each padded to 16 bytes) and two scalars
  // (layout in pair_lds_bytes)
  constexpr bool WIDE = POLY || INHOM;  // the host passes kBinsWide for these
  const int bins = WIDE ? kBinsWide : a.bins;
  const bool packed = bins == kBinsPacked;
  WaveLds *wl = (WaveLds *)smem;
  unsigned long long *hist = (unsigned long long *)(wl + kWaves);
  void *aux = (void *)(hist + NB);
  const int aux_words = WIDE ? 6 * NB
                             : bins == kBinsSplit32 ? ((NB + 3) & ~3) : 2 * NB;  // 32-bit words
  uint32_t *S2lo = (uint32_t *)aux + aux_words;
  uint32_t *S2hi = S2lo + ((g.n_s + 3) & ~3);
  uint32_t *T = S2hi + ((g.n_s + 3) & ~3);
  unsigned long long *evals_lds = (unsigned long long *)(T + ((g.n_t + 3) & ~3));
  uint32_t *grp_lds = (uint32_t *)(evals_lds + 1);
  // INHOM: rho of the centres and of the tile entries, per wave
  double *rho_lds = (double *)(evals_lds + 2);

  const int tid = threadIdx.x, lane = tid & 63, wv = (int)uni((uint32_t)tid >> 6);
  WaveLds &W = wl[wv];
  double *rho_c = rho_lds + wv * 64, *rho_t = rho_lds + (kWaves + wv) * 64;
  for (int b = tid; b < NB; b += kPairThreads) hist[b] = 0;
  for (int b = tid; b < aux_words; b += kPairThreads) ((uint32_t *)aux)[b] = 0;
  if (tid < g.n_s) {
    S2lo[tid] = (uint32_t)a.S2[tid];
    S2hi[tid] = (uint32_t)(a.S2[tid] >> 32);
  }
  if (tid < g.n_t) T[tid] = a.T[tid];
  if (tid == 0) *evals_lds = 0;
  // device sharing: the slots above share_grid stay free while other streams
  // have work (the word lives in host memory; one read per workgroup)
  if (a.share_word) {
    if (tid == 0)
      *grp_lds = (uint32_t)__hip_atomic_load(a.share_word, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
    const bool leave = uni(*grp_lds) > 1u && (int)blockIdx.x >= a.share_grid;
    __syncthreads();
    if (leave) {
      if (a.wg_times && tid == 0) {
        a.wg_times[2 * blockIdx.x] = 0ull;
        a.wg_times[2 * blockIdx.x + 1] = 0ull;
      }
      return;
    }
  }
  const unsigned long long t_start =
      (a.slice_ticks || a.wg_times) ? __builtin_amdgcn_s_memrealtime() : 0ull;
  const uint32_t n_items = *a.n_items;
  const unsigned long long flush_bound =
      a.flush_evals ? a.flush_evals : ((packed || WIDE) ? kFlushEvalsPacked : kFlushEvals);
  // 2^F of the inhomogeneous fixed-point weights (the same F in k_finalize)
  const double wscale = INHOM ? ldexp(1.0, wide_fbits(*a.rho_max, a.wbudget)) : 0.0;
  int cur_set = -1;
  unsigned long long evals_total = 0;

  // (no atomic here returns a value: each weight sum goes out as 32-bit
  // pieces, word k of the global bin summing the pieces of weight 2^(32 k))
  auto flush = [&](int set) {
    constexpr unsigned long long M = 0xFFFFFFFFull;
    for (int b = tid; b < NB; b += kPairThreads) {
      const unsigned long long hb = hist[b];
      unsigned long long c, w = 0;
      if (WIDE) {
        c = hb;
      } else if (packed) {
        // interior units of 2^23 plus the boundary weights: below 2^55 + 2^57
        c = hb >> kCountShift;
        w = ((hb & kUnitMask) << kFracBits) + ((unsigned long long *)aux)[b];
      } else {
        c = bins == kBinsSplit64 ? ((unsigned long long *)aux)[b]
                                 : (unsigned long long)((uint32_t *)aux)[b];
        w = hb;
      }
      c *= SYM ? 2ull : 1ull;
      if (c) {
        const size_t o = (size_t)set * NB + b;
        // word k of bin b at gw[k * NB]: a wave's flush atomics on one word
        // touch consecutive addresses
        unsigned long long *gw = a.binW + (size_t)set * NB * kBinWords + b;
        atomicAdd(&a.binC[o], c);
        hist[b] = 0;
        if (WIDE) {
          // three sums of 32-bit pieces (each below 2^64) -> four words
          unsigned long long *w3 = (unsigned long long *)aux + 3 * b;
          const unsigned long long A = w3[0], B = w3[1], C = w3[2];
          if (A & M) atomicAdd(&gw[0], A & M);
          if ((A >> 32) + (B & M)) atomicAdd(&gw[NB], (A >> 32) + (B & M));
          if ((B >> 32) + (C & M)) atomicAdd(&gw[2 * NB], (B >> 32) + (C & M));
          if (C >> 32) atomicAdd(&gw[3 * NB], C >> 32);
          w3[0] = 0;
          w3[1] = 0;
          w3[2] = 0;
        } else {
          atomicAdd(&gw[0], w & M);
          if (w >> 32) atomicAdd(&gw[NB], w >> 32);
          if (bins == kBinsSplit32)
            ((uint32_t *)aux)[b] = 0;
          else
            ((unsigned long long *)aux)[b] = 0;
        }
      }
    }
  };

  // Work queue: partition q of the groups is [q*G/kQueues, (q+1)*G/kQueues)
  // with its own counter.  A workgroup starts in partition blockIdx % kQueues
  // (its XCD under round-robin dispatch, so neighbouring groups share an L2)
  // and moves to the next partition when one runs dry; a plain read of the
  // counter first spares the atomic on a partition already handed out.
  // (a cost-ordered list deals its groups over the partitions: whole rounds)
  const uint32_t n_groups =
      a.perm ? ordered_slots(n_items / kItemsPerGroup) : n_items / kItemsPerGroup;
  const int home = (int)(blockIdx.x % kQueues);
  int qp = home, q_left = kQueues;
  for (;;) {
    __syncthreads();  // previous group finished by every wave
    if (tid == 0) {
      uint32_t got = 0xFFFFFFFFu;
      // a sliced launch stops taking groups at the end of its slice
      if (a.slice_ticks && __builtin_amdgcn_s_memrealtime() - t_start > a.slice_ticks) q_left = 0;
      while (q_left > 0) {
        const uint32_t lo = (uint32_t)((uint64_t)qp * n_groups / kQueues);
        const uint32_t hi = (uint32_t)((uint64_t)(qp + 1) * n_groups / kQueues);
        uint32_t *ctr = (uint32_t *)(a.queues + (size_t)qp * kQueueStride);
        if (lo + __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < hi) {
          const uint32_t gq = lo + atomicAdd(ctr, 1u);
          if (gq < hi) {
            got = a.perm ? a.perm[gq] : gq;
            break;
          }
        }
        qp = qp + 1 == kQueues ? 0 : qp + 1;
        --q_left;
      }
      *grp_lds = got;
    }
    __syncthreads();
    const uint32_t grp = uni(*grp_lds);
    if (grp == 0xFFFFFFFFu) break;
    if (grp == kEmptySlot) continue;
    const uint32_t base = grp * kItemsPerGroup;
    const int set = (int)uni(a.items[base].set);
    const unsigned long long pend = *evals_lds;
    if (set != cur_set || pend > flush_bound) {
      if (cur_set >= 0) flush(cur_set);
      cur_set = set;
      __syncthreads();
      if (tid == 0) *evals_lds = 0;
      __syncthreads();
    }
    const Item it = a.items[base + wv];
    const uint32_t cw = uni(it.count);
    const uint32_t cnt = cw & 0x7Fu;
    if (cnt == 0) continue;
    // the part of the stencil rows this item covers (all when not split), or
    // one row and a fraction fr of kf of its neighbour run
    const bool frm = (cw >> 31) != 0;
    const int r0 = (int)((cw >> 7) & 0xFFFu);
    const int r1 = frm ? r0 + 1 : ((cw >> 19) ? (int)(cw >> 19) : 0x7FFFFFFF);
    const uint32_t fr = frm ? ((cw >> 19) & 63u) : 0u, kf = frm ? ((cw >> 25) & 63u) : 1u;
    const uint32_t begin = uni(it.begin);
    const uint32_t cell = uni(it.cell);
    const bool valid = (uint32_t)lane < cnt;
    const unsigned long long vmask = __builtin_amdgcn_ballot_w64(valid);
    const uint32_t mi = begin + (uint32_t)lane;
    const int4 raw = valid ? a.P[mi] : make_int4(0, 0, 0, 0);
    const int4 me = image<MODE, POLY>(raw, g);
    const uint32_t tplus = (uint32_t)(MODE == kModePacked ? me.y : me.z) + g.tmax;
    const int thr = valid ? (int)g.s2max : -1;
    W.cen[0][lane] = (uint32_t)me.x;
    W.cen[1][lane] = (uint32_t)me.y;
    W.cen[2][lane] = (uint32_t)me.z;
    W.cen[3][lane] = (uint32_t)me.w;
    if (INHOM) rho_c[lane] = valid ? a.rho[mi] : 0.0;
    wave_sync();
    // the centres' row (t * ny + y) and the x-cells of the first and the last
    // centre (points are sorted by cell, x fastest)
    uint32_t rest;
    int cxa, cxb;
    if (a.row_items) {
      const uint32_t cxl = min((uint32_t)raw.x / (uint32_t)g.cell_s, (uint32_t)g.nx - 1u);
      cxa = (int)uni(cxl);
      cxb = (int)__builtin_amdgcn_readlane(cxl, (int)cnt - 1);
      rest = cell;
    } else {
      cxa = cxb = (int)(cell % (uint32_t)g.nx);
      rest = cell / (uint32_t)g.nx;
    }
    const int cy = (int)(rest % (uint32_t)g.ny);
    const int ct = (int)(rest / (uint32_t)g.ny);
    // cell starts of the neighbour rows: interleaved keys (stride 2, the set's
    // cells), or the set's type-2 block of blocked keys (stride 1)
    const bool blocked = a.blocked != 0;
    const uint32_t cst = blocked ? 1u : 2u;
    const uint32_t nb_off = blocked ? (2u * (uint32_t)set + 1u) * g.n_cells : (uint32_t)set * g.n_cells;
    QState q = {0u, 0u, 0u, 0u};
    Ctx<SYM, MODE, POLY, INHOM> x{W,    q,     g,   hist,  aux,   bins,  S2lo,  S2hi, T,
                                  lane, begin, 0u,  a.P,   a.rho, rho_c, rho_t, wscale};
    unsigned long long ev = 0;
    int ridx = 0;  // index of the stencil row in visiting order
    for (int dt = SYM ? 0 : -g.rt; dt <= g.rt; ++dt) {
      const int tt = ct + dt;
      for (int dy = -g.rs; dy <= g.rs; ++dy) {
        if (SYM && dt == 0 && dy < 0) continue;
        const int rid = ridx++;
        if (rid < r0 || rid >= r1) continue;
        if (tt < 0 || tt >= g.nt) continue;
        const int yy = cy + dy;
        if (yy < 0 || yy >= g.ny) continue;
        // (blocked: the neighbours are the other type's block, never the
        // centres' own cell)
        const bool home = (dt == 0 && dy == 0) && !blocked;
        const int xlo = (SYM && home) ? cxa : max(cxa - g.rs, 0);
        const int xhi = min(cxb + g.rs, g.nx - 1);
        const uint32_t row = nb_off + (uint32_t)(tt * g.ny + yy) * (uint32_t)g.nx;
        uint32_t j0 = uni(a.cs[cst * (row + (uint32_t)xlo)]);
        const uint32_t j1 = uni(a.cs[cst * (row + (uint32_t)xhi + 1u)]);
        if (kf > 1) {
          // fraction fr of the run (in the symmetric home row, of j > the
          // first centre); candidates counted exactly
          const uint32_t a0 = (home && SYM) ? begin + 1 : j0;
          const uint32_t len = j1 > a0 ? j1 - a0 : 0u;
          const uint32_t s0 = a0 + (uint32_t)((uint64_t)len * fr / kf);
          const uint32_t s1 = a0 + (uint32_t)((uint64_t)len * (fr + 1) / kf);
          if (home) {
            if (SYM) {
              // each j pairs with the centres below it: j - begin of them, at most cnt
              const uint32_t m = begin + cnt;
              const uint32_t ta = min(s1, m), tb = max(s0, m);
              if (ta > s0)
                ev += (unsigned long long)(ta - s0) *
                      ((unsigned long long)s0 + ta - 1 - 2ull * begin) / 2;
              if (s1 > tb) ev += (unsigned long long)cnt * (s1 - tb);
            } else {
              const uint32_t lo = max(s0, begin), hi = min(s1, begin + cnt);
              ev += (unsigned long long)cnt * (s1 - s0) - (hi > lo ? hi - lo : 0u);
            }
            scan_run<SYM, MODE, POLY, INHOM, true>(x, s0, s1, me, tplus, thr, valid, vmask, mi, a.P);
          } else {
            ev += (unsigned long long)cnt * (s1 - s0);
            scan_run<SYM, MODE, POLY, INHOM, false>(x, s0, s1, me, tplus, thr, valid, vmask, mi, a.P);
          }
          continue;
        }
        if (home) {
          if (SYM) {
            j0 = begin + 1;
            ev += (unsigned long long)cnt * (j1 - begin - 1) - (unsigned long long)cnt * (cnt - 1) / 2;
          } else {
            ev += (unsigned long long)cnt * (j1 - j0) - cnt;
          }
          scan_run<SYM, MODE, POLY, INHOM, true>(x, j0, j1, me, tplus, thr, valid, vmask, mi, a.P);
        } else {
          ev += (unsigned long long)cnt * (j1 - j0);
          scan_run<SYM, MODE, POLY, INHOM, false>(x, j0, j1, me, tplus, thr, valid, vmask, mi, a.P);
        }
      }
    }
    {
      const uint32_t na = na_of(q);
      if (na) drain_oldest(x, na);
    }
    if (q.nb)
      drain_b<MODE, POLY, INHOM>(W, q, q.nb, lane,
                                 (WIDE || packed) ? (unsigned long long *)aux : hist, g, a.P,
                                 a.rho, wscale);
    if (lane == 0) atomicAdd(evals_lds, ev);
    evals_total += ev;
  }
  if (cur_set >= 0) flush(cur_set);
  if (lane == 0 && evals_total) atomicAdd(a.queues + (size_t)home * kQueueStride + 1, evals_total);
  if (a.wg_times && tid == 0) {
    a.wg_times[2 * blockIdx.x] = t_start;
    a.wg_times[2 * blockIdx.x + 1] = __builtin_amdgcn_s_memrealtime();
  }
}

// Estimated candidates of each group of the work list (slots past the
// groups get the largest key and an empty value): per item, its centres times
// the length of every neighbour run its part of the stencil rows covers (a
// fraction of a run when rows are cut into fractions), as the pair kernel
// walks them; key = 255 - round(6 log2(1 + cost)) (a sixth of an octave per
// step, costs up to 2^42), so that an ascending sort, one radix pass, puts the
// costliest groups first.
__global__ void k_group_cost(PairArgs a, uint32_t max_groups, uint32_t *__restrict__ keys,
                             uint32_t *__restrict__ vals) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_groups) return;
  const Geom &g = a.g;
  const uint32_t G = *a.n_items / kItemsPerGroup;
  if (s >= G) {
    keys[s] = 0xFFu;
    vals[s] = kEmptySlot;
    return;
  }
  const bool sym = a.symmetric != 0, blocked = a.blocked != 0;
  double cost = 0.0;
  for (int w = 0; w < kItemsPerGroup; ++w) {
    const Item it = a.items[s * kItemsPerGroup + w];
    const uint32_t cnt = it.count & 0x7Fu;
    if (cnt == 0) continue;
    const bool frm = (it.count >> 31) != 0;
    const int r0 = (int)((it.count >> 7) & 0xFFFu);
    const int r1 = frm ? r0 + 1 : ((it.count >> 19) ? (int)(it.count >> 19) : 0x7FFFFFFF);
    const uint32_t kf = frm ? ((it.count >> 25) & 63u) : 1u;
    uint32_t rest;
    int cxa, cxb;
    if (a.row_items) {
      cxa = min(a.P[it.begin].x / g.cell_s, g.nx - 1);
      cxb = min(a.P[it.begin + cnt - 1].x / g.cell_s, g.nx - 1);
      rest = it.cell;
    } else {
      cxa = cxb = (int)(it.cell % (uint32_t)g.nx);
      rest = it.cell / (uint32_t)g.nx;
    }
    const int cy = (int)(rest % (uint32_t)g.ny), ct = (int)(rest / (uint32_t)g.ny);
    const uint32_t cst = blocked ? 1u : 2u;
    const uint32_t nb_off =
        blocked ? (2u * it.set + 1u) * g.n_cells : it.set * g.n_cells;
    int ridx = 0;
    for (int dt = sym ? 0 : -g.rt; dt <= g.rt; ++dt)
      for (int dy = -g.rs; dy <= g.rs; ++dy) {
        if (sym && dt == 0 && dy < 0) continue;
        const int rid = ridx++;
        if (rid < r0 || rid >= r1) continue;
        const int tt = ct + dt, yy = cy + dy;
        if (tt < 0 || tt >= g.nt || yy < 0 || yy >= g.ny) continue;
        const bool home = dt == 0 && dy == 0 && !blocked;
        const int xlo = (sym && home) ? cxa : max(cxa - g.rs, 0);
        const int xhi = min(cxb + g.rs, g.nx - 1);
        const uint32_t row = nb_off + (uint32_t)(tt * g.ny + yy) * (uint32_t)g.nx;
        const uint32_t j0 = a.cs[cst * (row + (uint32_t)xlo)];
        const uint32_t j1 = a.cs[cst * (row + (uint32_t)xhi + 1u)];
        cost += (double)cnt * (double)(j1 - j0) / (double)kf;
      }
  }
  keys[s] = 0xFFu - min(0xFFu, (uint32_t)rint(6.0 * log2(1.0 + cost)));
  vals[s] = s;
}

// Sorted rank r goes to partition r % kQueues, at offset r / kQueues.
__global__ void k_deal_groups(const uint32_t *__restrict__ n_items, uint32_t max_groups,
                              const uint32_t *__restrict__ sorted, uint32_t *__restrict__ perm) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t slots = ordered_slots(*n_items / kItemsPerGroup);
  if (r >= slots || r >= max_groups) return;
  const uint32_t per = slots / kQueues;
  perm[(r % kQueues) * per + r / kQueues] = sorted[r];
}

template <bool SYM, int MODE, bool POLY, bool INHOM>
hipError_t launch_t(const PairArgs &a, int grid, hipStream_t s) {
  const int lds = pair_lds_bytes(a.g.n_s, a.g.n_t, a.bins, INHOM);
  hipLaunchKernelGGL((k_pair<SYM, MODE, POLY, INHOM>), dim3(grid), dim3(kPairThreads), lds, s, a);
  return hipGetLastError();
}

template <bool SYM, int MODE, bool POLY, bool INHOM>
hipError_t occ_t(int lds, int *per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_pair<SYM, MODE, POLY, INHOM>,
                                                      kPairThreads, lds);
}

// variants: rectangle, polygon (POLY), inhomogeneous on the rectangle (INHOM)
template <bool SYM, bool POLY, bool INHOM>
hipError_t occ_mode(int mode, int lds, int *per_cu) {
  if (mode == kModePacked) return occ_t<SYM, kModePacked, POLY, INHOM>(lds, per_cu);
  if (mode == kModeU32) return occ_t<SYM, kModeU32, POLY, INHOM>(lds, per_cu);
  return occ_t<SYM, kModeWide, POLY, INHOM>(lds, per_cu);
}

template <bool SYM, bool POLY, bool INHOM>
hipError_t launch_mode(const PairArgs &a, int grid, hipStream_t s) {
  if (a.g.mode == kModePacked) return launch_t<SYM, kModePacked, POLY, INHOM>(a, grid, s);
  if (a.g.mode == kModeU32) return launch_t<SYM, kModeU32, POLY, INHOM>(a, grid, s);
  return launch_t<SYM, kModeWide, POLY, INHOM>(a, grid, s);
}

template <bool SYM>
hipError_t occ_var(int var, int mode, int lds, int *per_cu) {
  if (var == 1) return occ_mode<SYM, true, false>(mode, lds, per_cu);
  if (var == 2) return occ_mode<SYM, false, true>(mode, lds, per_cu);
  return occ_mode<SYM, false, false>(mode, lds, per_cu);
}

template <bool SYM>
hipError_t launch_var(int var, const PairArgs &a, int grid, hipStream_t s) {
  if (var == 1) return launch_mode<SYM, true, false>(a, grid, s);
  if (var == 2) return launch_mode<SYM, false, true>(a, grid, s);
  return launch_mode<SYM, false, false>(a, grid, s);
}

}  // namespace

int pair_lds_bytes(int n_s, int n_t, int bins, bool inhom) {
  const int n_bins = n_s * n_t;
  const int aux_words = bins == kBinsWide      ? 6 * n_bins
                        : bins == kBinsSplit32 ? ((n_bins + 3) & ~3)
                                               : 2 * n_bins;
  const int tables = 2 * ((n_s + 3) & ~3) + ((n_t + 3) & ~3);
  return (int)sizeof(WaveLds) * kWaves + 8 * n_bins + 4 * aux_words + 4 * tables + 16 +
         (inhom ? 2 * kWaves * 64 * 8 : 0);
}

bool pair_poly(const Geom &g) { return g.poly_n >= 3 && (g.edge & 1u); }

hipError_t pair_occupancy(int n_s, int n_t, int bins, int symmetric, int mode, int var,
                          int *per_cu) {
  const int lds = pair_lds_bytes(n_s, n_t, bins, var == 2);
  return symmetric ? occ_var<true>(var, mode, lds, per_cu) : occ_var<false>(var, mode, lds, per_cu);
}

hipError_t launch_order_groups(const PairArgs &a, uint32_t max_groups, uint32_t *kA,
                               uint32_t *vA, uint32_t *kB, uint32_t *vB, void *temp,
                               const uint32_t **perm, hipStream_t s) {
  const uint32_t blocks = (max_groups + 255) / 256;
  hipLaunchKernelGGL(k_group_cost, dim3(blocks), dim3(256), 0, s, a, max_groups, kA, vA);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int alt = 0;
  e = radix_sort(kA, vA, kB, vB, max_groups, 8, temp, s, &alt);
  if (e != hipSuccess) return e;
  uint32_t *out = alt ? vA : vB;
  hipLaunchKernelGGL(k_deal_groups, dim3(blocks), dim3(256), 0, s, a.n_items, max_groups,
                     alt ? vB : vA, out);
  *perm = out;
  return hipGetLastError();
}

hipError_t launch_pair(const PairArgs &a, int grid, hipStream_t s) {
  const int var = a.rho ? 2 : (pair_poly(a.g) ? 1 : 0);
  return a.symmetric ? launch_var<true>(var, a, grid, s) : launch_var<false>(var, a, grid, s);
}

}  // namespace ripk
