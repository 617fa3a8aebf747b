// Cumulation, normalisation and envelopes on gfx950.
//
// The pair kernel leaves, per set, a histogram over the smallest grid step
// (k, l) containing each pair.  Because the indicator of Eq. 3 is monotone in
// s and t and the weights do not depend on the threshold, the sums of Eq. 2 at
// every grid point are the 2-D inclusive prefix sums of that histogram.  This
// file forms them (exact integers: counts in u64, weights in 128-bit fixed point
// with 23 fraction bits, or the launch's scale for inhomogeneous K, assembled
// from the pair kernel's four sums of 32-bit pieces), then K = A*D*W/N (Eq. 2)
// and L = sqrt(K/(2 pi t)) - s
// (Eq. 4) in FP64, and the pointwise min/max envelopes over simulations (Sec. 3).
#include "ripk_internal.h"

namespace ripk {

namespace {

__device__ __forceinline__ void add128(unsigned long long &lo, unsigned long long &hi,
                                       unsigned long long blo, unsigned long long bhi) {
  unsigned long long r = lo + blo;
  hi += bhi + (r < lo ? 1ull : 0ull);
  lo = r;
}

// One workgroup per set.  The set's bins are read once into LDS (the counts,
// and each weight assembled as a 128-bit value from its four sums of 32-bit
// pieces, sum_k w_k 2^(32 k) mod 2^128), cumulated there along t and then
// along s, and the results written once: the prefix loops then wait on LDS,
// not on a chain of global loads.  LDS: 24 bytes per bin.
__global__ void k_finalize(const unsigned long long *__restrict__ binC,
                           const unsigned long long *__restrict__ binW, int n_s, int n_t,
                           double s_max, double t_max, double AD, double N,
                           unsigned long long *__restrict__ C, double *__restrict__ W,
                           double *__restrict__ K, double *__restrict__ L,
                           const unsigned long long *__restrict__ queues,
                           unsigned long long *__restrict__ scal,
                           const unsigned long long *__restrict__ rho_max, int wbudget) {
  extern __shared__ unsigned long long fin_lds[];
  const int set = blockIdx.x;
  const int nb = n_s * n_t;
  const unsigned long long *c = binC + (size_t)set * nb;
  const unsigned long long *w = binW + (size_t)set * nb * kBinWords;
  unsigned long long *lc = fin_lds, *llo = fin_lds + nb, *lhi = fin_lds + 2 * nb;
  const int fbits = rho_max ? wide_fbits(*rho_max, wbudget) : kFracBits;
  if (set == 0 && threadIdx.x == 0) {
    unsigned long long ev = 0;
    for (int q = 0; q < kQueues; ++q) ev += queues[q * kQueueStride + 1];
    scal[0] = ev;
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const unsigned long long s0 = w[b], s1 = w[nb + b], s2 = w[2 * nb + b], s3 = w[3 * nb + b];
    unsigned long long lo = 0, hi = 0;
    add128(lo, hi, s0, 0ull);
    add128(lo, hi, s1 << 32, s1 >> 32);
    add128(lo, hi, 0ull, s2);
    add128(lo, hi, 0ull, s3 << 32);
    lc[b] = c[b];
    llo[b] = lo;
    lhi[b] = hi;
  }
  __syncthreads();
  // prefix along t within each s row
  for (int k = threadIdx.x; k < n_s; k += blockDim.x) {
    unsigned long long rc = 0, rlo = 0, rhi = 0;
    for (int l = 0; l < n_t; ++l) {
      const int b = k * n_t + l;
      rc += lc[b];
      lc[b] = rc;
      add128(rlo, rhi, llo[b], lhi[b]);
      llo[b] = rlo;
      lhi[b] = rhi;
    }
  }
  __syncthreads();
  // prefix along s within each t column
  for (int l = threadIdx.x; l < n_t; l += blockDim.x) {
    unsigned long long rc = 0, rlo = 0, rhi = 0;
    for (int k = 0; k < n_s; ++k) {
      const int b = k * n_t + l;
      rc += lc[b];
      lc[b] = rc;
      add128(rlo, rhi, llo[b], lhi[b]);
      llo[b] = rlo;
      lhi[b] = rhi;
    }
  }
  __syncthreads();
  const double two_pi = 6.283185307179586476925286766559;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    int k = b / n_t, l = b - k * n_t;
    // fixed point: W = (hi * 2^64 + lo) * 2^-F
    double wv = ldexp((double)lhi[b], 64 - fbits) + ldexp((double)llo[b], -fbits);
    double Kv = AD * wv / N;
    double sk = (double)(k + 1) * s_max / (double)n_s;
    double tl = (double)(l + 1) * t_max / (double)n_t;
    size_t o = (size_t)set * nb + b;
    C[o] = lc[b];
    W[o] = wv;
    K[o] = Kv;
    L[o] = sqrt(Kv / (two_pi * tl)) - sk;
  }
  if (threadIdx.x == 0) atomicAdd(scal + 1, lc[nb - 1]);
}

// env rows: K_lo, K_hi, L_lo, L_hi, dL_hi
__global__ void k_envelope(const double *__restrict__ K, const double *__restrict__ L,
                           uint32_t m, int nb, const double *__restrict__ L_obs,
                           double *__restrict__ env) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double klo = K[b], khi = K[b], llo = L[b], lhi = L[b];
  for (uint32_t s = 1; s < m; ++s) {
    double kv = K[(size_t)s * nb + b], lv = L[(size_t)s * nb + b];
    klo = fmin(klo, kv);
    khi = fmax(khi, kv);
    llo = fmin(llo, lv);
    lhi = fmax(lhi, lv);
  }
  env[b] = klo;
  env[nb + b] = khi;
  env[2 * nb + b] = llo;
  env[3 * nb + b] = lhi;
  env[4 * nb + b] = L_obs ? L_obs[b] - lhi : 0.0;
}

// The call's scalars and up to kPackRows output rows of nb words, one after
// another, so that one copy brings them to the host.
__global__ void k_pack(const unsigned long long *__restrict__ scal, PackRows rows, int nb,
                       unsigned long long *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kScalWords) out[i] = scal[i];
  for (int r = 0; r < kPackRows; ++r)
    if (rows.p[r] && i < nb) out[kScalWords + r * nb + i] = rows.p[r][i];
}

}  // namespace

hipError_t launch_pack(const unsigned long long *scal, const PackRows &rows, int nb,
                       unsigned long long *out, hipStream_t s) {
  const int n = nb > kScalWords ? nb : kScalWords;
  hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, scal, rows, nb, out);
  return hipGetLastError();
}

hipError_t launch_finalize(unsigned long long *binC, unsigned long long *binW, uint32_t n_sets,
                           int n_s, int n_t, double s_max, double t_max, double AD, double N,
                           unsigned long long *C, double *W, double *K, double *L,
                           const unsigned long long *queues, unsigned long long *scal,
                           hipStream_t s, const unsigned long long *rho_max, int wbudget) {
  hipLaunchKernelGGL(k_finalize, dim3(n_sets), dim3(256), 24 * n_s * n_t, s, binC, binW, n_s,
                     n_t, s_max,
                     t_max, AD, N, C, W, K, L, queues, scal, rho_max, wbudget);
  return hipGetLastError();
}

hipError_t launch_envelope(const double *K, const double *L, uint32_t m, int n_bins,
                           const double *L_obs, double *env, hipStream_t s) {
  hipLaunchKernelGGL(k_envelope, dim3((n_bins + 255) / 256), dim3(256), 0, s, K, L, m, n_bins,
                     L_obs, env);
  return hipGetLastError();
}

}  // namespace ripk
