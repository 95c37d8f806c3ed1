// Spherical k-means++ seeding (Section 5.6 of the paper, "Spherical
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

// The canonical FP64 similarity (dot64_serial / dot64_group) of a dense row:
// a dense row is a CSR row that stores every column, entry t being column
// t, so the partial sums, chains and pairwise tree are the same.
__device__ __forceinline__ double dot64_serial_dense(const float* __restrict__ x, int64_t d,
                                                     const double* __restrict__ c) {
  double st[7];
#pragma unroll
  for (int p = 0; p < 64; ++p) {
    double s = 0.0;
    for (int64_t t = p; t < d; t += 64) s = fma((double)x[t], c[t], s);
    int lev = 0;
#pragma unroll
    for (int q = p; q & 1; q >>= 1) s = st[lev++] + s;
    st[lev] = s;
  }
  return st[6];
}

// One lane per partial sum (G = 64 lanes), then the same pairwise tree.
__device__ __forceinline__ double dot64_wave_dense(const float* __restrict__ x, int64_t d,
                                                   const double* __restrict__ c, int lane) {
  double s = 0.0;
  for (int64_t t = lane; t < d; t += 64) s = fma((double)x[t], c[t], s);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// Rows of either layout: CSR (rp, ci, v) or dense (x non-null, ld, d).
struct SeedRows {
  const int64_t* rp;
  const int32_t* ci;
  const float* v;
  const float* x;
  int64_t ld;
};

__device__ __forceinline__ double row_dot64(const SeedRows& R, int64_t i, int64_t d,
                                            const double* __restrict__ c) {
  if (R.x) return dot64_serial_dense(R.x + (size_t)i * R.ld, d, c);
  return dot64_serial(R.ci, R.v, R.rp[i], R.rp[i + 1], c);
}

__global__ __launch_bounds__(kBlock) void k_kpp_update(
    SeedRows R, int64_t n, int64_t d, const double* __restrict__ c, int32_t t, double alpha,
    const uint8_t* __restrict__ taken, int32_t* __restrict__ a, double* __restrict__ best,
    double* __restrict__ second, double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sw[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double wi = 0.0;
  if (i < n) {
    const double s = row_dot64(R, i, d, c);
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

__global__ __launch_bounds__(kBlock) void k_kpp_densify(SeedRows R, int64_t d,
                                                        const int32_t* __restrict__ chosen,
                                                        int32_t t, float* __restrict__ centres) {
  const int64_t p = chosen[t];
  float* c = centres + (size_t)t * d;
  if (R.x) {
    for (int64_t q = threadIdx.x; q < d; q += kBlock) c[q] = R.x[(size_t)p * R.ld + q];
  } else {
    for (int64_t e = R.rp[p] + threadIdx.x; e < R.rp[p + 1]; e += kBlock) c[R.ci[e]] = R.v[e];
  }
}

}  // namespace

hipError_t launch_kpp_step(const int64_t* rp, const int32_t* ci, const float* v, const float* x,
                           int64_t ld, int64_t n, int64_t d, int32_t t, double alpha,
                           const double* u_dev,
                           uint8_t* taken, int32_t* chosen, float* centres, double* c64,
                           int32_t* a, double* best, double* second, double* w, double* part,
                           hipStream_t s) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  const SeedRows R{rp, ci, v, x, ld};
  hipLaunchKernelGGL(k_kpp_select, dim3(1), dim3(kBlock), 0, s, part, nb, w, n, u_dev, t, taken,
                     chosen);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kpp_densify, dim3(1), dim3(kBlock), 0, s, R, d, chosen, t, centres);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_init_centres(centres + (size_t)t * d, 1, d, 1, c64, nullptr, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_kpp_update, dim3((unsigned)nb), dim3(kBlock), 0, s, R, n, d, c64, t,
                     alpha, taken, a, best, second, w, part);
  return hipGetLastError();
}

}  // namespace skm

// ------------------------------------------------------------------------
// AFK-MC2 seeding (the Markov-chain alternative to k-means++ that Section 5.6
// cites, with the dissimilarity alpha - <x, c>).  Centre 0 fixes the
// proposal distribution q; every further centre runs a chain of m proposals
// drawn from q.  The proposals do not depend on the chain's state, so their
// dissimilarities to the centres chosen so far are computed together (one
// block per proposal); only the accept/reject walk is sequential.
// ------------------------------------------------------------------------
namespace skm {
namespace {
using namespace dev;

// w(x) = max(0, alpha - <x, c0>) in the canonical FP64 order.
__global__ __launch_bounds__(kBlock) void k_afk_weights(SeedRows R, int64_t n, int64_t d,
                                                        const double* __restrict__ c0,
                                                        double alpha, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double x = alpha - row_dot64(R, i, d, c0);
  w[i] = x > 0.0 ? x : 0.0;
}

// One thread: W = sum w in row order, then the running sums of
// q(x) = w(x) / (2W) + 1 / (2n) (1/n when W = 0), in row order, so every
// value is the same sequence of FP64 operations a plain loop performs.
__global__ void k_afk_prefix(const double* __restrict__ w, int64_t n, double* __restrict__ W_out,
                             double* __restrict__ prefix) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double W = 0.0;
  for (int64_t i = 0; i < n; ++i) W += w[i];
  double run = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double q = W > 0.0 ? 0.5 * w[i] / W + 0.5 / (double)n : 1.0 / (double)n;
    run += q;
    prefix[i] = run;
  }
  *W_out = W;
}

// Proposal j of the chain: the first row whose running q sum exceeds u[j]
// (binary search on the non-decreasing prefix), the last row if none does.
__global__ void k_afk_propose(const double* __restrict__ prefix, int64_t n,
                              const double* __restrict__ u, int32_t m,
                              int32_t* __restrict__ cand) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= m) return;
  const double target = u[j];
  int64_t lo = 0, hi = n;  // first index with prefix > target lies in [lo, hi]
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (prefix[mid] > target) hi = mid;
    else lo = mid + 1;
  }
  cand[j] = (int32_t)(lo < n ? lo : n - 1);
}

// d(y_j) = max(0, alpha - max_{c < t} <y_j, c>): one block per proposal,
// each wave takes every fourth centre.
__global__ __launch_bounds__(kBlock) void k_afk_dissim(
    SeedRows R, int64_t d, const double* __restrict__ C64, int32_t t, double alpha,
    const int32_t* __restrict__ cand, double* __restrict__ dcand) {
  __shared__ double wmax[kBlock / 64];
  const int j = blockIdx.x;
  const int64_t y = cand[j];
  const int64_t beg = R.x ? 0 : R.rp[y], end = R.x ? 0 : R.rp[y + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double best = -INFINITY;
  for (int c = wave; c < t; c += kBlock / 64) {
    const double s =
        R.x ? dot64_wave_dense(R.x + (size_t)y * R.ld, d, C64 + (size_t)c * d, lane)
            : dot64_group<64>(R.ci, R.v, beg, end, C64 + (size_t)c * d, lane);
    best = s > best ? s : best;
  }
  if (lane == 0) wmax[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = wmax[0];
    for (int q = 1; q < kBlock / 64; ++q) b = wmax[q] > b ? wmax[q] : b;
    const double x = alpha - b;
    dcand[j] = x > 0.0 ? x : 0.0;
  }
}

// The chain: start at y_1, move to y_j when d(y_j) q(x) > u d(x) q(y_j).
__global__ void k_afk_chain(const int32_t* __restrict__ cand, const double* __restrict__ dcand,
                            const double* __restrict__ w, const double* __restrict__ Wp,
                            int64_t n, const double* __restrict__ uacc, int32_t m, int32_t t,
                            int32_t* __restrict__ chosen) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double W = *Wp;
  auto q = [&](int64_t i) {
    return W > 0.0 ? 0.5 * w[i] / W + 0.5 / (double)n : 1.0 / (double)n;
  };
  int64_t x = cand[0];
  double dx = dcand[0];
  for (int j = 1; j < m; ++j) {
    const int64_t y = cand[j];
    const double dy = dcand[j];
    if (dy * q(x) > uacc[j - 1] * dx * q(y)) {
      x = y;
      dx = dy;
    }
  }
  chosen[t] = (int32_t)x;
}

__global__ void k_afk_first(const double* __restrict__ u, int64_t n, int32_t* __restrict__ chosen) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t p = (int64_t)floor(u[0] * (double)n);
  if (p > n - 1) p = n - 1;
  if (p < 0) p = 0;
  chosen[0] = (int32_t)p;
}

}  // namespace

hipError_t launch_afkmc2(const int64_t* rp, const int32_t* ci, const float* v, const float* x,
                         int64_t ld, int64_t n, int64_t d, int32_t k, int32_t m, double alpha,
                         const double* u_dev,
                         int32_t* chosen, float* centres, double* C64, double* w, double* W,
                         double* prefix, int32_t* cand, double* dcand, hipStream_t s) {
  hipError_t e;
  const unsigned nblk = (unsigned)((n + kBlock - 1) / kBlock);
  const SeedRows R{rp, ci, v, x, ld};
  hipLaunchKernelGGL(k_afk_first, dim3(1), dim3(64), 0, s, u_dev, n, chosen);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_kpp_densify, dim3(1), dim3(kBlock), 0, s, R, d, chosen, 0, centres);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_init_centres(centres, 1, d, 1, C64, nullptr, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_afk_weights, dim3(nblk), dim3(kBlock), 0, s, R, n, d, C64, alpha, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_afk_prefix, dim3(1), dim3(64), 0, s, w, n, W, prefix);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int32_t t = 1; t < k; ++t) {
    const double* ut = u_dev + 1 + (size_t)(t - 1) * (2 * m - 1);
    hipLaunchKernelGGL(k_afk_propose, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, prefix, n, ut, m, cand);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_afk_dissim, dim3((unsigned)m), dim3(kBlock), 0, s, R, d, C64, t, alpha,
                       cand, dcand);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_afk_chain, dim3(1), dim3(64), 0, s, cand, dcand, w, W, n, ut + m, m, t,
                       chosen);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_kpp_densify, dim3(1), dim3(kBlock), 0, s, R, d, chosen, t, centres);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_init_centres(centres + (size_t)t * d, 1, d, 1, C64 + (size_t)t * d, nullptr,
                                 s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

}  // namespace skm
