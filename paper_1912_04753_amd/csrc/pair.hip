// The pair range count on gfx950 -- the hot loop of the space-time K estimator.
//
// For every centre i and every neighbour j of i in the cell stencil, the kernel
// decides the indicator of Eq. 3 (d_ij <= s_max and u_ij <= t_max, exact
// integers), finds the smallest grid step (k, l) that contains the pair, and
// adds the count and the edge-corrected weight 1/(omega_ij v_ij) of Sec. 3 to
// an (s, t) histogram held in LDS.  Histograms are merged into 128-bit global
// bins with 64-bit atomics when a workgroup moves on to another point set.
//
// Mapping
//   * workgroup = 4 wavefronts; a work item = up to 64 centres of one cell (one
//     lane per centre); a workgroup grabs 4 items of one set at a time from a
//     global counter (persistent launch, items padded per set);
//   * neighbours are visited as contiguous runs of the sorted point array (a run
//     of consecutive x-cells per (y, t) row of the stencil), staged per wave in
//     LDS tiles with coalesced loads and read back as wave-uniform broadcasts;
//   * symmetric mode visits each unordered pair once (forward half of the
//     stencil, j > i inside the home cell) and adds both weights, since
//     omega_ij / v_ij depend on the centre while the bin depends on d and u only;
//   * the rare in-range pairs are compacted into a per-wave LDS queue and
//     binned / weighted 64 at a time so that the costly part runs with full
//     lanes rather than under a divergent branch.
//
// Weights are FP32: w = 1/omega * 1/v lies in [1, 8], so w * 2^23 is an exact
// integer and the fixed-point sums are exact and order independent.
#include "ripk_internal.h"

namespace ripk {

namespace {

constexpr int kJT = 128;   // tile points per wave
constexpr int kQ = 128;    // per-wave queue ring (power of two, >= 2*64)
constexpr int kWaves = kPairThreads / 64;
constexpr unsigned long long kFlushEvals = 1ull << 34;  // bound on candidates between flushes

struct WaveLds {
  int4 tile[kJT];
  int4 cen[64];
  uint4 q[kQ];  // {j sorted index, centre lane | d2 high bits << 6, d2 low, u}
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Isotropic correction on the rectangle in FP32, complementary-angle form:
// beta_e = atan2(e, sqrt(d2 - e^2)) for each cut side (d2 - e^2 is an exact
// integer).  Only the nearer x side and the nearer y side can cut a circle of
// radius <= min(W, H)/2.  One side cut: 1/2 + beta/pi; two sides with the
// corner outside (or on) the circle: (beta_x + beta_y)/pi; corner inside:
// 1/4 + (beta_x + beta_y)/(2 pi).  All terms are non-negative.
__device__ __forceinline__ float omega_f32(int32_t X, int32_t Y, uint64_t d2, const Geom &g) {
  const int32_t ex = min(X, g.x1 - g.x0 - X);
  const int32_t ey = min(Y, g.y1 - g.y0 - Y);
  const uint64_t ex2 = (uint64_t)ex * (uint64_t)ex, ey2 = (uint64_t)ey * (uint64_t)ey;
  const bool cx = ex2 < d2, cy = ey2 < d2;
  const float inv_pi = 0.318309886183790671538f;
  float bx = 0.0f, by = 0.0f;
  if (cx) bx = atan2f((float)ex, sqrtf((float)(d2 - ex2)));
  if (cy) by = atan2f((float)ey, sqrtf((float)(d2 - ey2)));
  if (cx && cy) {
    if (ex2 + ey2 < d2) return 0.25f + (bx + by) * (0.5f * inv_pi);
    return (bx + by) * inv_pi;
  }
  if (cx) return 0.5f + bx * inv_pi;
  if (cy) return 0.5f + by * inv_pi;
  return 1.0f;
}

// Fixed-point weight of one ordered pair with centre p: (1/omega)(1/v) * 2^23.
__device__ __forceinline__ uint32_t qweight(const int4 p, uint64_t d2, uint32_t u, const Geom &g) {
  uint32_t q = 1u << kFracBits;
  if (g.edge & 2u) {
    const uint32_t D = (uint32_t)(g.t1 - g.t0);
    const uint32_t T = (uint32_t)p.z;
    if (u > T || u > D - T) q <<= 1;  // an end of [t-u, t+u] leaves the period: v = 1/2
  }
  if (g.edge & 1u) {
    const uint64_t e = (uint64_t)(uint32_t)p.w;
    if (d2 > e * e) {
      const float om = omega_f32(p.x, p.y, d2, g);
      const float w = fmaxf(__frcp_rn(om), 1.0f);
      q = (uint32_t)(w * (float)q);  // exact: w >= 1 has at most 23 fraction bits
    }
  }
  return q;
}

__device__ __forceinline__ int kbin(uint64_t d2, const unsigned long long *S2, const Geom &g) {
  int k = (int)ceilf(sqrtf((float)d2) * g.inv_ds);
  k = min(max(k, 1), g.n_s);
  while (k > 1 && d2 <= S2[k - 2]) --k;
  while (d2 > S2[k - 1]) ++k;
  return k - 1;
}

__device__ __forceinline__ int lbin(uint32_t u, const uint32_t *T, const Geom &g) {
  int l = (int)ceilf((float)u * g.inv_dt);
  l = min(max(l, 1), g.n_t);
  while (l > 1 && u <= T[l - 2]) --l;
  while (u > T[l - 1]) ++l;
  return l - 1;
}

template <bool SYM>
__device__ __forceinline__ void drain(WaveLds &W, uint32_t head, uint32_t c, int lane,
                                      const PairArgs &a, unsigned long long *hc,
                                      unsigned long long *hw, const unsigned long long *S2,
                                      const uint32_t *T) {
  const Geom &g = a.g;
  wave_sync();
  const uint4 r = W.q[(head + lane) & (kQ - 1)];
  wave_sync();
  if ((uint32_t)lane < c) {
    const uint32_t il = r.y & 63u;
    const uint64_t d2 = (uint64_t)r.z | ((uint64_t)(r.y >> 6) << 32);
    const uint32_t u = r.w;
    const int bin = kbin(d2, S2, g) * g.n_t + lbin(u, T, g);
    const int4 pi = W.cen[il];
    uint32_t q = qweight(pi, d2, u, g);
    if (SYM) {
      const int4 pj = a.P[r.x];
      q += qweight(pj, d2, u, g);
    }
    atomicAdd(&hc[bin], SYM ? 2ull : 1ull);
    atomicAdd(&hw[bin], (unsigned long long)q);
  }
}

template <bool SYM, bool WIDE, bool HOME>
__device__ __forceinline__ void scan_run(uint32_t j0, uint32_t j1, const int4 me, bool valid,
                                         uint32_t mi, int lane, WaveLds &W, uint32_t &qhead,
                                         uint32_t &qn, const PairArgs &a, unsigned long long *hc,
                                         unsigned long long *hw, const unsigned long long *S2,
                                         const uint32_t *T) {
  const Geom &g = a.g;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint32_t tb = j0; tb < j1; tb += kJT) {
    const uint32_t nt = min((uint32_t)kJT, j1 - tb);
    wave_sync();
    for (uint32_t q = lane; q < nt; q += 64) W.tile[q] = a.P[tb + q];
    wave_sync();
    for (uint32_t jj = 0; jj < nt; ++jj) {
      const int4 pj = W.tile[jj];
      const uint32_t adx = __usad((uint32_t)me.x, (uint32_t)pj.x, 0u);
      const uint32_t ady = __usad((uint32_t)me.y, (uint32_t)pj.y, 0u);
      const uint32_t u = __usad((uint32_t)me.z, (uint32_t)pj.z, 0u);
      uint64_t d2;
      bool acc;
      if (WIDE) {
        d2 = (uint64_t)adx * adx + (uint64_t)ady * ady;
        acc = valid && d2 <= g.s2max && u <= g.tmax;
      } else {
        const uint32_t d2n = __umul24(adx, adx) + __umul24(ady, ady);
        d2 = d2n;
        acc = valid && d2n <= (uint32_t)g.s2max && u <= g.tmax;
      }
      const uint32_t j = tb + jj;
      if (HOME) acc = acc && (SYM ? (j > mi) : (j != mi));
      const unsigned long long mask = __ballot(acc);
      if (mask) {
        const uint32_t pos = (qhead + qn + (uint32_t)__popcll(mask & lt)) & (kQ - 1);
        if (acc) W.q[pos] = make_uint4(j, (uint32_t)lane | ((uint32_t)(d2 >> 32) << 6),
                                       (uint32_t)d2, u);
        qn += (uint32_t)__popcll(mask);
        if (qn >= 64) {
          drain<SYM>(W, qhead, 64, lane, a, hc, hw, S2, T);
          qhead = (qhead + 64) & (kQ - 1);
          qn -= 64;
        }
      }
    }
  }
}

template <bool SYM, bool WIDE>
__global__ void __launch_bounds__(kPairThreads) k_pair(PairArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom &g = a.g;
  const int NB = g.n_s * g.n_t;
  unsigned long long *hc = (unsigned long long *)smem;
  unsigned long long *hw = hc + NB;
  unsigned long long *S2 = hw + NB;
  uint32_t *T = (uint32_t *)(S2 + kMaxSteps);
  WaveLds *wl = (WaveLds *)(T + kMaxSteps);
  unsigned long long *evals_lds = (unsigned long long *)(wl + kWaves);
  uint32_t *grp_lds = (uint32_t *)(evals_lds + 1);

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  WaveLds &W = wl[wv];
  for (int b = tid; b < NB; b += kPairThreads) {
    hc[b] = 0;
    hw[b] = 0;
  }
  if (tid < g.n_s) S2[tid] = a.S2[tid];
  if (tid < g.n_t) T[tid] = a.T[tid];
  if (tid == 0) *evals_lds = 0;
  const uint32_t n_items = *a.n_items;
  int cur_set = -1;
  unsigned long long evals_total = 0;

  auto flush = [&](int set) {
    for (int b = tid; b < NB; b += kPairThreads) {
      const unsigned long long c = hc[b];
      if (c) {
        const unsigned long long w = hw[b];
        const size_t o = (size_t)set * NB + b;
        atomicAdd(&a.binC[o], c);
        const unsigned long long old = atomicAdd(&a.binW[2 * o], w);
        if (old + w < old) atomicAdd(&a.binW[2 * o + 1], 1ull);
        hc[b] = 0;
        hw[b] = 0;
      }
    }
  };

  for (;;) {
    __syncthreads();  // previous group finished by every wave
    if (tid == 0) *grp_lds = atomicAdd(a.item_ctr, 1u);
    __syncthreads();
    const uint32_t grp = __builtin_amdgcn_readfirstlane(*grp_lds);
    const uint32_t base = grp * kItemsPerGroup;
    if (base >= n_items) break;
    const int set = (int)__builtin_amdgcn_readfirstlane(a.items[base].set);
    const unsigned long long pend = *evals_lds;
    if (set != cur_set || pend > kFlushEvals) {
      if (cur_set >= 0) flush(cur_set);
      cur_set = set;
      __syncthreads();
      if (tid == 0) *evals_lds = 0;
      __syncthreads();
    }
    const Item it = a.items[base + wv];
    const uint32_t cnt = __builtin_amdgcn_readfirstlane(it.count);
    if (cnt == 0) continue;
    const uint32_t begin = __builtin_amdgcn_readfirstlane(it.begin);
    const uint32_t cell = __builtin_amdgcn_readfirstlane(it.cell);
    const bool valid = (uint32_t)lane < cnt;
    const uint32_t mi = begin + (uint32_t)lane;
    const int4 me = valid ? a.P[mi] : make_int4(0, 0, 0, 0);
    W.cen[lane] = me;
    wave_sync();
    const int cx = (int)(cell % (uint32_t)g.nx);
    const uint32_t rest = cell / (uint32_t)g.nx;
    const int cy = (int)(rest % (uint32_t)g.ny);
    const int ct = (int)(rest / (uint32_t)g.ny);
    const uint32_t set_off = (uint32_t)set * g.n_cells;
    uint32_t qhead = 0, qn = 0;
    unsigned long long ev = 0;
    for (int dt = SYM ? 0 : -g.rt; dt <= g.rt; ++dt) {
      const int tt = ct + dt;
      if (tt < 0 || tt >= g.nt) continue;
      for (int dy = -g.rs; dy <= g.rs; ++dy) {
        if (SYM && dt == 0 && dy < 0) continue;
        const int yy = cy + dy;
        if (yy < 0 || yy >= g.ny) continue;
        const bool home = (dt == 0 && dy == 0);
        const int xlo = (SYM && home) ? cx : max(cx - g.rs, 0);
        const int xhi = min(cx + g.rs, g.nx - 1);
        const uint32_t row = set_off + (uint32_t)(tt * g.ny + yy) * (uint32_t)g.nx;
        uint32_t j0 = a.cs[2 * (row + (uint32_t)xlo)];
        const uint32_t j1 = a.cs[2 * (row + (uint32_t)xhi) + 2];
        if (home) {
          if (SYM) {
            j0 = begin + 1;
            ev += (unsigned long long)cnt * (j1 - begin - 1) - (unsigned long long)cnt * (cnt - 1) / 2;
          } else {
            ev += (unsigned long long)cnt * (j1 - j0) - cnt;
          }
          scan_run<SYM, WIDE, true>(j0, j1, me, valid, mi, lane, W, qhead, qn, a, hc, hw, S2, T);
        } else {
          ev += (unsigned long long)cnt * (j1 - j0);
          scan_run<SYM, WIDE, false>(j0, j1, me, valid, mi, lane, W, qhead, qn, a, hc, hw, S2, T);
        }
      }
    }
    if (qn) drain<SYM>(W, qhead, qn, lane, a, hc, hw, S2, T);
    if (lane == 0) atomicAdd(evals_lds, ev);
    evals_total += ev;
  }
  if (cur_set >= 0) flush(cur_set);
  if (lane == 0 && evals_total) atomicAdd(a.n_eval, evals_total);
}

template <bool SYM, bool WIDE>
hipError_t launch_t(const PairArgs &a, int grid, hipStream_t s) {
  const int lds = pair_lds_bytes(a.g.n_s * a.g.n_t);
  hipLaunchKernelGGL((k_pair<SYM, WIDE>), dim3(grid), dim3(kPairThreads), lds, s, a);
  return hipGetLastError();
}

template <bool SYM, bool WIDE>
hipError_t occ_t(int lds, int *per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_pair<SYM, WIDE>, kPairThreads,
                                                      lds);
}

}  // namespace

int pair_lds_bytes(int n_bins) {
  return 16 * n_bins + 8 * kMaxSteps + 4 * kMaxSteps + (int)sizeof(WaveLds) * kWaves + 16;
}

hipError_t pair_occupancy(int n_bins, int symmetric, int wide, int *per_cu) {
  const int lds = pair_lds_bytes(n_bins);
  if (symmetric) return wide ? occ_t<true, true>(lds, per_cu) : occ_t<true, false>(lds, per_cu);
  return wide ? occ_t<false, true>(lds, per_cu) : occ_t<false, false>(lds, per_cu);
}

hipError_t launch_pair(const PairArgs &a, int grid, hipStream_t s) {
  if (a.symmetric) return a.g.wide ? launch_t<true, true>(a, grid, s) : launch_t<true, false>(a, grid, s);
  return a.g.wide ? launch_t<false, true>(a, grid, s) : launch_t<false, false>(a, grid, s);
}

}  // namespace ripk
