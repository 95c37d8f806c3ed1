// Spherical k-means++ seeding (Section 6 of the paper, "Spherical
// k-means++"): the first centre is a uniformly drawn row, every further one
// is drawn with probability proportional to alpha - max_c <x(i), c> over the
// centres chosen so far.  The maximum is cached per row and refreshed once
// per new centre, so the whole seeding costs one pass over the rows per
// centre (n k similarities in total).  The random draws are inputs: u[t] in
// [0, 1) selects centre t by inverse transform sampling.
//
//  k_kpp_select   one block: centre t = row floor(u[0] n) for t = 0, else the
//                 first row whose running weight sum exceeds u[t] W, found
//                 through the per-block weight sums of the previous update
//                 (a fixed summation order, so the choice is deterministic);
//                 rows already chosen have weight 0; W = 0 takes the lowest
//                 unchosen row
//  k_kpp_densify  writes chosen row t into the dense FP32 centre matrix
//  (the FP64 unit centre comes from k_init_centres, exactly as a fit
//   rescales its initial centres)
//  k_kpp_update   per row: <x(i), c_t> in the canonical FP64 order, running
//                 top-2 (strictly greater replaces, so ties keep the lower
//                 centre index), the row's weight, and per-block weight sums
#include <float.h>
#include <limits.h>

#include "skm_device.h"
#include "skm_internal.h"

namespace skm {
namespace {
using namespace dev;

__global__ __launch_bounds__(kBlock) void k_kpp_update(
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const float* __restrict__ v,
    int64_t n, const double* __restrict__ c, int32_t t, double alpha,
    const uint8_t* __restrict__ taken, int32_t* __restrict__ a, double* __restrict__ best,
    double* __restrict__ second, double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sw[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double wi = 0.0;
  if (i < n) {
    const double s = dot64_serial(ci, v, rp[i], rp[i + 1], c);
    double b = best[i], s2 = second[i];
    if (s > b) {
      s2 = b;
      b = s;
      a[i] = t;
    } else if (s > s2) {
      s2 = s;
    }
    best[i] = b;
    second[i] = s2;
    wi = taken[i] ? 0.0 : alpha - b;
    if (!(wi > 0.0)) wi = 0.0;
    w[i] = wi;
  }
  sw[threadIdx.x] = wi;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int q = 0; q < kBlock; ++q) sum += sw[q];
    part[blockIdx.x] = sum;
  }
}

__global__ __launch_bounds__(kBlock) void k_kpp_select(const double* __restrict__ part,
                                                       int64_t nb, const double* __restrict__ w,
                                                       int64_t n, const double* __restrict__ u,
                                                       int32_t t, uint8_t* __restrict__ taken,
                                                       int32_t* __restrict__ chosen) {
  __shared__ double range_sum[kBlock];
  __shared__ int64_t first_free[kBlock];
  __shared__ int64_t pick;
  const int r = threadIdx.x;
  if (t == 0) {
    if (r == 0) {
      int64_t p = (int64_t)floor(u[0] * (double)n);
      if (p > n - 1) p = n - 1;
      if (p < 0) p = 0;
      chosen[0] = (int32_t)p;
      taken[p] = 1;
    }
    return;
  }
  // thread r owns weight blocks [r * per, (r + 1) * per)
  const int64_t per = (nb + kBlock - 1) / kBlock;
  const int64_t b0 = (int64_t)r * per, b1 = (b0 + per < nb) ? b0 + per : nb;
  double rs = 0.0;
  for (int64_t b = b0; b < b1; ++b) rs += part[b];
  range_sum[r] = rs;
  if (r == 0) pick = -1;
  __syncthreads();
  if (r == 0) {
    double W = 0.0;
    for (int q = 0; q < kBlock; ++q) W += range_sum[q];
    if (W > 0.0) {
      const double target = u[t] * W;
      double run = 0.0;
      int q = 0, q_last = -1;
      for (; q < kBlock; ++q) {
        if (range_sum[q] > 0.0) q_last = q;
        if (run + range_sum[q] > target) break;
        run += range_sum[q];
      }
      bool crossed = q < kBlock;
      if (!crossed) q = q_last;  // rounding left the target unreached
      const int64_t qb0 = (int64_t)q * per, qb1 = (qb0 + per < nb) ? qb0 + per : nb;
      int64_t bsel = -1, b_last = -1;
      for (int64_t b = qb0; b < qb1; ++b) {
        if (part[b] > 0.0) b_last = b;
        if (crossed && run + part[b] > target) {
          bsel = b;
          break;
        }
        run += part[b];
      }
      crossed = crossed && bsel >= 0;
      if (bsel < 0) bsel = b_last;
      const int64_t i0 = bsel * kBlock, i1 = (i0 + kBlock < n) ? i0 + kBlock : n;
      int64_t p = -1, p_last = -1;
      for (int64_t i = i0; i < i1; ++i) {
        if (w[i] > 0.0) p_last = i;
        if (crossed && run + w[i] > target) {
          p = i;
          break;
        }
        run += w[i];
      }
      pick = p >= 0 ? p : p_last;
    }
  }
  __syncthreads();
  if (pick < 0) {  // W = 0: the lowest-index row not chosen yet
    int64_t f = INT64_MAX;
    for (int64_t i = r; i < n; i += kBlock)
      if (!taken[i]) {
        f = i;
        break;
      }
    first_free[r] = f;
    __syncthreads();
    if (r == 0) {
      int64_t m = INT64_MAX;
      for (int q = 0; q < kBlock; ++q) m = first_free[q] < m ? first_free[q] : m;
      pick = m;
    }
    __syncthreads();
  }
  if (r == 0) {
    chosen[t] = (int32_t)pick;
    taken[pick] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_kpp_densify(const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const float* __restrict__ v, int64_t d,
                                                        const int32_t* __restrict__ chosen,
                                                        int32_t t, float* __restrict__ centres) {
  const int64_t p = chosen[t];
  float* c = centres + (size_t)t * d;
  for (int64_t e = rp[p] + threadIdx.x; e < rp[p + 1]; e += kBlock) c[ci[e]] = v[e];
}

}  // namespace

hipError_t launch_kpp_step(const int64_t* rp, const int32_t* ci, const float* v, int64_t n,
                           int64_t d, int32_t t, double alpha, const double* u_dev,
                           uint8_t* taken, int32_t* chosen, float* centres, double* c64,
                           int32_t* a, double* best, double* second, double* w, double* part,
                           hipStream_t s) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_kpp_select, dim3(1), dim3(kBlock), 0, s, part, nb, w, n, u_dev, t, taken,
                     chosen);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kpp_densify, dim3(1), dim3(kBlock), 0, s, rp, ci, v, d, chosen, t,
                     centres);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_init_centres(centres + (size_t)t * d, 1, d, 1, c64, nullptr, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_kpp_update, dim3((unsigned)nb), dim3(kBlock), 0, s, rp, ci, v, n, c64, t,
                     alpha, taken, a, best, second, w, part);
  return hipGetLastError();
}

}  // namespace skm
