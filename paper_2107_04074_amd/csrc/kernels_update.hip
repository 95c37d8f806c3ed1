// Centre-step, movement, centre-centre and Hamerly kernels for gfx950.
//
//  k_row_eta           per-row bound on | |x(i)| - 1 | (rows are unit only
//                      to float rounding; every bound accounts for it)
//  k_init_centres      FP64 master centres from the initial rows, rescaled to
//                      unit length
//  k_transpose         FP64 k x d masters -> FP32 d x kp centre-minor copy
//                      read by the similarity kernels (LDS-tiled transpose)
//  k_update_scan       S(old) -= x(i), S(new) += x(i) for every row whose
//                      assignment changed (Section 5, baseline optimisation
//                      (iii): keep the unnormalised sums and update them on
//                      reassignment) in 64-bit fixed point, so the sums do
//                      not depend on the order of the atomics
//  k_sumsq_partial     |S(j)|^2 over column chunks for every touched cluster
//  k_normalize_move    c(j) = S(j)/|S(j)| and |c(j) - c'(j)|^2 partials
//  k_centre_finalize   movement p(j) = <c(j), c'(j)> (Section 4) as the
//                      cosine/sine of an upper bound of the movement angle,
//                      the two largest movements (p' of Section 5.3) and the
//                      objective sum_j |S(j)|
//  k_gram_*            <c(j), c(j')> for the centre-centre tests of Sections
//                      5.2 and 5.4 (split-K tiles, deterministic reduction)
#include <float.h>
#include <limits.h>

#include <algorithm>

#include <hip/hip_fp16.h>

#include "skm_device.h"
#include "skm_internal.h"

namespace skm {
namespace {
using namespace dev;

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
#pragma unroll
  for (int s = kBlock / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void row_eta_body(const int64_t* __restrict__ rp,
                                             const float* __restrict__ v, int64_t n,
                                             float* __restrict__ eta,
                                             float* __restrict__ max_eta, int64_t bx) {
  const int64_t i = bx * kBlock + threadIdx.x;
  float e32 = 0.f;
  if (i < n) {
    const int64_t beg = rp[i], end = rp[i + 1];
    double ss = 0.0;
    for (int64_t e = beg; e < end; ++e) ss = fma((double)v[e], (double)v[e], ss);
    const double dev = fabs(sqrt(ss) - 1.0) + (double)(end - beg + 4) * kU64 * 2.0 + 1e-300;
    e32 = __double2float_ru(dev);
    eta[i] = e32;
  }
  if (max_eta) {
    // non-negative floats order like their bit patterns; one atomic per
    // block, spread over kCounterSlots words
    __shared__ float wmax[kBlock / 64];
    for (int off = 32; off >= 1; off >>= 1) e32 = fmaxf(e32, __shfl_xor(e32, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = e32;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = 0.f;
      for (int w = 0; w < kBlock / 64; ++w) m = fmaxf(m, wmax[w]);
      if (m > 0.f) atomicMax(reinterpret_cast<int*>(max_eta) + (int)(bx % kCounterSlots),
                             __float_as_int(m));
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_row_eta(const int64_t* __restrict__ rp,
                                                    const float* __restrict__ v, int64_t n,
                                                    float* __restrict__ eta,
                                                    float* __restrict__ max_eta) {
  row_eta_body(rp, v, n, eta, max_eta, blockIdx.x);
}

__device__ __forceinline__ void init_centres_body(const float* __restrict__ init, int64_t d,
                                                  int normalize, double* __restrict__ C64,
                                                  double* __restrict__ init_norm, int j) {
  __shared__ double sh[kBlock];
  const float* x = init + (size_t)j * d;
  double ss = 0.0;
  for (int64_t t = threadIdx.x; t < d; t += kBlock) ss = fma((double)x[t], (double)x[t], ss);
  const double nrm = sqrt(block_sum(ss, sh));
  if (threadIdx.x == 0 && init_norm) init_norm[j] = nrm;
  const bool scale = normalize && nrm > 0.0;
  double* c = C64 + (size_t)j * d;
  for (int64_t t = threadIdx.x; t < d; t += kBlock) c[t] = scale ? (double)x[t] / nrm : (double)x[t];
}

__global__ __launch_bounds__(kBlock) void k_init_centres(const float* __restrict__ init,
                                                         int64_t d, int normalize,
                                                         double* __restrict__ C64,
                                                         double* __restrict__ init_norm) {
  init_centres_body(init, d, normalize, C64, init_norm, blockIdx.x);
}

// 64 x 64 tile transpose with float conversion.  Tiles whose 64 centres are
// all clean are skipped (their FP32 copy is already current).
__device__ __forceinline__ void transpose_body(const double* __restrict__ C64, int32_t k,
                                               int64_t d, int32_t kp,
                                               const int32_t* __restrict__ dirty,
                                               float* __restrict__ CT, __half* __restrict__ CT16,
                                               int64_t bx, int by) {
  __shared__ float tile[64][65];
  __shared__ int any;
  const int64_t t0 = bx * 64;
  const int j0 = by * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (dirty) {
    if (threadIdx.x < 64 && j0 + (int)threadIdx.x < k && dirty[j0 + threadIdx.x]) any = 1;
    __syncthreads();
    if (!any) return;
  }
  for (int jj = ty; jj < 64; jj += 4) {
    const int j = j0 + jj;
    const int64_t t = t0 + tx;
    tile[jj][tx] = (j < k && t < d) ? (float)C64[(size_t)j * d + t] : 0.f;
  }
  __syncthreads();
  for (int tt = ty; tt < 64; tt += 4) {
    const int64_t t = t0 + tt;
    const int j = j0 + tx;
    if (t < d && j < k) {
      CT[(size_t)t * kp + j] = tile[tx][tt];
      if (CT16) CT16[(size_t)t * kp + j] = __float2half(tile[tx][tt]);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_transpose(const double* __restrict__ C64, int32_t k,
                                                      int64_t d, int32_t kp,
                                                      const int32_t* __restrict__ dirty,
                                                      float* __restrict__ CT,
                                                      __half* __restrict__ CT16) {
  transpose_body(C64, k, d, kp, dirty, CT, CT16, blockIdx.x, blockIdx.y);
}

// Sets *flag when a stored value or an initial-centre value is negative
// (plain stores of 1: every writer writes the same value).
__global__ void k_neg_scan(const float* __restrict__ v, int64_t nnz,
                           const float* __restrict__ init, int64_t ninit,
                           int32_t* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  bool neg = false;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz + ninit; e += stride)
    neg |= (e < nnz ? v[e] : init[e - nnz]) < 0.f;
  if (neg) *flag = 1;
}

// Input checks of validate = 2 (the matrix layout of Section 2: sparse rows
// as (index, value) pairs with ascending indices; finite values).  A
// violation is recorded as row * 8 + kind in *bad by an atomic minimum, so
// the host reports the first offending row.  The CSR checks run in two
// launches: k_check_rowptr reads row_ptr by flat index only, and
// k_check_entries runs only after the host has seen it pass, so every row
// range it walks lies inside [0, nnz).
__global__ void k_check_rowptr(const int64_t* __restrict__ rp, int64_t n, int64_t nnz,
                               unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i > n) return;
  const int64_t r = rp[i];
  bool ok = true;
  if (i == 0) ok = r == 0;
  if (i == n) ok = ok && r == nnz;
  if (i < n) ok = ok && rp[i + 1] >= r;
  if (!ok) atomicMin(bad, (unsigned long long)i * 8ull + kBadRowPtr);
}

__global__ void k_check_entries(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const float* __restrict__ v, int64_t n, int64_t d,
                                unsigned long long* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const int64_t beg = rp[i], end = rp[i + 1];
    int kind = 0;
    int64_t prev = -1;
    for (int64_t e = beg; e < end && kind == 0; ++e) {
      const int64_t c = ci[e];
      if (c < 0 || c >= d) kind = kBadColumn;
      else if (c <= prev) kind = kBadOrder;
      else if (!isfinite(v[e])) kind = kBadValue;
      prev = c;
    }
    if (kind) atomicMin(bad, (unsigned long long)i * 8ull + (unsigned long long)kind);
  }
}

__global__ void k_check_dense(const float* __restrict__ x, int64_t ld, int64_t n, int64_t d,
                              unsigned long long* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * d; e += stride) {
    const int64_t i = e / d, t = e - i * d;
    if (!isfinite(x[i * ld + t])) atomicMin(bad, (unsigned long long)i * 8ull + kBadValue);
  }
}

// Scans the assignment for rows that moved since the last centre step and
// applies S(old) -= x(i), S(new) += x(i) for each of them; a_old starts at -1
// so the first step adds every row.  A wave tests 64 rows, then the stored
// entries of its moved rows are laid end to end (a prefix sum of their
// lengths across the lanes) and the lanes take them 64 at a time, each lane
// finding its entry's row by a binary search over the prefix; a batch of
// entries is loaded before its atomics, so no lane waits for one row at a
// time.  Fixed-point sums make the order of the atomics irrelevant.
// Rows [row0, row_end) of one block, in steps of `stride` rows.
__device__ __forceinline__ void update_scan_body(
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const float* __restrict__ v,
    const int32_t* __restrict__ a, int32_t* __restrict__ a_old, int64_t row0, int64_t row_end,
    int64_t stride, int64_t d, double fx, long long* __restrict__ S,
    int32_t* __restrict__ dirty) {
  constexpr int kB = 4;  // entries per lane loaded before their atomics
  const int lane = threadIdx.x & 63;
  const int64_t n = row_end;
  const int64_t wave0 = row0 + (threadIdx.x & ~63);
  for (int64_t base = wave0; base < n; base += stride) {
    const int64_t i = base + lane;
    int32_t nw = -1, old = -1;
    if (i < n) {
      nw = a[i];
      old = a_old[i];
    }
    const bool mv = i < n && nw != old;
    if (__ballot(mv) == 0ull) continue;
    int64_t rb = 0;
    int len = 0;
    if (mv) {
      rb = rp[i];
      len = (int)(rp[i + 1] - rb);
      dirty[nw] = 1;
      if (old >= 0) dirty[old] = 1;
      a_old[i] = nw;
    }
    // inclusive prefix of the moved rows' lengths over the lanes
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    for (int e0 = 0; e0 < total; e0 += 64 * kB) {
      int32_t col[kB], rn[kB], ro[kB];
      long long q[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + 64 * u + lane;
        // source lane: the number of lanes whose prefix ends at or before e
        int r = 0;
#pragma unroll
        for (int b = 32; b >= 1; b >>= 1)
          if (__shfl(incl, r + b - 1, 64) <= e) r += b;
        const int rs = r < 63 ? r : 63;
        const int64_t rbr = __shfl(rb, rs, 64);
        const int exr = __shfl(incl, rs, 64) - __shfl(len, rs, 64);
        rn[u] = __shfl(nw, rs, 64);
        ro[u] = __shfl(old, rs, 64);
        col[u] = -1;
        q[u] = 0;
        if (e < total) {
          const int64_t idx = rbr + (e - exr);
          col[u] = ci[idx];
          q[u] = __double2ll_rn((double)v[idx] * fx);
        }
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        if (col[u] >= 0) {
          atomicAdd(reinterpret_cast<unsigned long long*>(S + (size_t)rn[u] * d + col[u]),
                    (unsigned long long)q[u]);
          if (ro[u] >= 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(S + (size_t)ro[u] * d + col[u]),
                      (unsigned long long)(-q[u]));
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_update_scan(
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const float* __restrict__ v,
    const int32_t* __restrict__ a, int32_t* __restrict__ a_old, int64_t n, int64_t d,
    double fx, long long* __restrict__ S, int32_t* __restrict__ dirty) {
  update_scan_body(rp, ci, v, a, a_old, (int64_t)blockIdx.x * kBlock, n,
                   (int64_t)gridDim.x * kBlock, d, fx, S, dirty);
}

constexpr int kMoveChunk = 4096;

// Partial sums of squares of S(j) over column chunks (dirty clusters only).
__device__ __forceinline__ void sumsq_partial_body(const long long* __restrict__ S, int64_t d,
                                                   double fx_inv,
                                                   const int32_t* __restrict__ dirty,
                                                   double* __restrict__ part_sq, int nchunk,
                                                   int ch, int j) {
  __shared__ double sh[kBlock];
  if (!dirty[j]) return;
  const int64_t t0 = (int64_t)ch * kMoveChunk;
  const int64_t t1 = (t0 + kMoveChunk < d) ? t0 + kMoveChunk : d;
  const long long* s = S + (size_t)j * d;
  double ss = 0.0;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += kBlock) {
    const double x = (double)s[t] * fx_inv;
    ss = fma(x, x, ss);
  }
  const double tot = block_sum(ss, sh);
  if (threadIdx.x == 0) part_sq[(size_t)j * nchunk + ch] = tot;
}

__global__ __launch_bounds__(kBlock) void k_sumsq_partial(const long long* __restrict__ S,
                                                          int64_t d, double fx_inv,
                                                          const int32_t* __restrict__ dirty,
                                                          double* __restrict__ part_sq,
                                                          int nchunk) {
  sumsq_partial_body(S, d, fx_inv, dirty, part_sq, nchunk, blockIdx.x, blockIdx.y);
}

__device__ __forceinline__ double chunk_norm(const double* __restrict__ part_sq, int j,
                                             int nchunk) {
  double ss = 0.0;
  for (int q = 0; q < nchunk; ++q) ss += part_sq[(size_t)j * nchunk + q];
  return sqrt(ss);
}

__device__ __forceinline__ void normalize_move_body(
    const long long* __restrict__ S, int64_t d, double fx_inv, const int32_t* __restrict__ dirty,
    const double* __restrict__ part_sq, double* __restrict__ C64, double* __restrict__ part,
    int nchunk, int ch, int j) {
  __shared__ double sh[kBlock];
  if (!dirty[j]) return;
  const double nrm = chunk_norm(part_sq, j, nchunk);
  const int64_t t0 = (int64_t)ch * kMoveChunk;
  const int64_t t1 = (t0 + kMoveChunk < d) ? t0 + kMoveChunk : d;
  double acc = 0.0;
  if (nrm > 0.0) {
    const long long* s = S + (size_t)j * d;
    double* c = C64 + (size_t)j * d;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kBlock) {
      const double nv = ((double)s[t] * fx_inv) / nrm;
      const double dd = nv - c[t];
      acc = fma(dd, dd, acc);
      c[t] = nv;
    }
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)j * nchunk + ch] = tot;
}

__global__ __launch_bounds__(kBlock) void k_normalize_move(
    const long long* __restrict__ S, int64_t d, double fx_inv, const int32_t* __restrict__ dirty,
    const double* __restrict__ part_sq, double* __restrict__ C64, double* __restrict__ part,
    int nchunk) {
  normalize_move_body(S, d, fx_inv, dirty, part_sq, C64, part, nchunk, blockIdx.x, blockIdx.y);
}

struct MinPair {
  double v;
  int j;
};

__device__ __forceinline__ MinPair min_pair(MinPair a, MinPair b) {
  if (b.v < a.v || (b.v == a.v && b.j < a.j)) return b;
  return a;
}

// Single block.
__device__ __forceinline__ void centre_finalize_body(
    int32_t k, int64_t d, const int32_t* __restrict__ dirty, double* __restrict__ norm64,
    const double* __restrict__ part_sq, const double* __restrict__ part, int nchunk,
    double delta_c, double* __restrict__ pc, double* __restrict__ ps, MoveMin* __restrict__ mm,
    Persist* __restrict__ per) {
  __shared__ double shd[kBlock];
  __shared__ double shv[kBlock];
  __shared__ int shj[kBlock];
  double obj = 0.0;
  MinPair best = {INFINITY, INT_MAX};
  const double grow = 1.0 + (double)(d + 4) * kU64;
  for (int j = threadIdx.x; j < k; j += kBlock) {
    double c = 1.0, s = 0.0;
    if (dirty[j]) norm64[j] = chunk_norm(part_sq, j, nchunk);
    if (dirty[j] && norm64[j] > 0.0) {
      double c2 = 0.0;
      for (int q = 0; q < nchunk; ++q) c2 += part[(size_t)j * nchunk + q];
      // chord |c - c'| between the stored FP64 vectors, widened for their
      // norms deviating from 1; the angle 2 asin(h/2) bounds the movement
      double h = sqrt(c2) * grow + 2.0 * delta_c + 1e-300;
      if (h > 2.0) h = 2.0;
      c = 1.0 - 0.5 * h * h;
      s = h * sqrt(fmax(0.0, 1.0 - 0.25 * h * h));
    }
    pc[j] = c;
    ps[j] = s;
    obj += norm64[j];
    best = min_pair(best, MinPair{c, j});
  }
  const double total = block_sum(obj, shd);
  // smallest movement cosine
  shv[threadIdx.x] = best.v;
  shj[threadIdx.x] = best.j;
  __syncthreads();
  for (int st = kBlock / 2; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) {
      MinPair r = min_pair(MinPair{shv[threadIdx.x], shj[threadIdx.x]},
                           MinPair{shv[threadIdx.x + st], shj[threadIdx.x + st]});
      shv[threadIdx.x] = r.v;
      shj[threadIdx.x] = r.j;
    }
    __syncthreads();
  }
  const int j1 = shj[0];
  __syncthreads();
  MinPair second = {INFINITY, INT_MAX};
  for (int j = threadIdx.x; j < k; j += kBlock)
    if (j != j1) second = min_pair(second, MinPair{pc[j], j});
  shv[threadIdx.x] = second.v;
  shj[threadIdx.x] = second.j;
  __syncthreads();
  for (int st = kBlock / 2; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) {
      MinPair r = min_pair(MinPair{shv[threadIdx.x], shj[threadIdx.x]},
                           MinPair{shv[threadIdx.x + st], shj[threadIdx.x + st]});
      shv[threadIdx.x] = r.v;
      shj[threadIdx.x] = r.j;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int j2 = shj[0];
    MoveMin r;
    r.idx1 = j1;
    r.pc1 = pc[j1];
    r.ps1 = ps[j1];
    r.pc2 = (j2 < k) ? pc[j2] : 1.0;
    r.ps2 = (j2 < k) ? ps[j2] : 0.0;
    r.pad = 0;
    *mm = r;
    per->objective = total;
  }
}

__global__ __launch_bounds__(kBlock) void k_centre_finalize(
    int32_t k, int64_t d, const int32_t* __restrict__ dirty, double* __restrict__ norm64,
    const double* __restrict__ part_sq, const double* __restrict__ part, int nchunk,
    double delta_c, double* __restrict__ pc, double* __restrict__ ps, MoveMin* __restrict__ mm,
    Persist* __restrict__ per) {
  centre_finalize_body(k, d, dirty, norm64, part_sq, part, nchunk, delta_c, pc, ps, mm, per);
}

__global__ void k_clear_dirty(int32_t* dirty, int32_t k) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < k) dirty[j] = 0;
}

// Gram matrix of the FP64 centres on the FP64 matrix cores: 64 x 64 output
// tiles (upper triangle of tiles), split over d into slices so that the
// launch fills the chip; partials persist so that tiles of clean centres
// need not be recomputed.  Each of the four waves owns a 32 x 32 quarter as
// 2 x 2 MFMA 16x16x4 tiles; centre panels of kGramK columns are staged in LDS
// with the next panel's loads in flight during the current panel's MFMAs.
// MFMA f64 16x16x4 lane layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element e of lane l is D[4 e + l / 16][l % 16].
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;
constexpr int kGramT = 64;
constexpr int kGramK = 32;
constexpr int kGramLoads = kGramT * kGramK / kBlock;  // per panel and thread

__device__ __forceinline__ void gram_partial_body(const double* __restrict__ C64, int32_t k,
                                                  int64_t d, const int32_t* __restrict__ dirty,
                                                  int force_all, double* __restrict__ part,
                                                  int64_t slice_len, Persist* __restrict__ per,
                                                  const StepCtl* __restrict__ ctl, int pair,
                                                  int s) {
  __shared__ double As[kGramT][kGramK + 1];
  __shared__ double Bs[kGramT][kGramK + 1];
  __shared__ int any;
  if (ctl) {
    if (ctl->gram_mode != 1) return;
    force_all = ctl->gram_force;
  }
  const int nt = (k + kGramT - 1) / kGramT;
  int idx = pair, ta = 0;
  while (idx >= nt - ta) {
    idx -= nt - ta;
    ++ta;
  }
  const int tb = ta + idx;
  const int a0 = ta * kGramT, b0 = tb * kGramT;
  if (!force_all) {
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (threadIdx.x < kGramT) {
      const int ja = a0 + threadIdx.x, jb = b0 + threadIdx.x;
      if ((ja < k && dirty[ja]) || (jb < k && dirty[jb])) any = 1;
    }
    __syncthreads();
    if (!any) return;
  }
  const int64_t ts = (int64_t)s * slice_len;
  const int64_t te = (ts + slice_len < d) ? ts + slice_len : d;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // staging: element q of this thread is row (tid + q*256) / kGramK, column
  // (tid + q*256) % kGramK of the panel (consecutive lanes, consecutive t)
  double ra[kGramLoads], rb[kGramLoads];
  auto load = [&](int64_t t0) {
#pragma unroll
    for (int q = 0; q < kGramLoads; ++q) {
      const int e = threadIdx.x + q * kBlock;
      const int r = e / kGramK, c = e % kGramK;
      const int64_t t = t0 + c;
      ra[q] = (a0 + r < k && t < te) ? C64[(size_t)(a0 + r) * d + t] : 0.0;
      rb[q] = (b0 + r < k && t < te) ? C64[(size_t)(b0 + r) * d + t] : 0.0;
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  load(ts);
  for (int64_t t0 = ts; t0 < te; t0 += kGramK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGramLoads; ++q) {
      const int e = threadIdx.x + q * kBlock;
      As[e / kGramK][e % kGramK] = ra[q];
      Bs[e / kGramK][e % kGramK] = rb[q];
    }
    __syncthreads();
    if (t0 + kGramK < te) load(t0 + kGramK);
#pragma unroll
    for (int kk = 0; kk < kGramK / 4; ++kk) {
      const int c = kk * 4 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = As[wr + i * 16 + (lane & 15)][c];
        bf[i] = Bs[wc + i * 16 + (lane & 15)][c];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  double* P = part + (size_t)s * k * k;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ja = a0 + wr + i * 16 + 4 * e + (lane >> 4);
        const int jb = b0 + wc + j * 16 + (lane & 15);
        if (ja < k && jb < k) P[(size_t)ja * k + jb] = acc[i][j][e];
      }
  if (s == 0 && threadIdx.x == 0) {
    unsigned long long pairs = 0;
    for (int i = 0; i < kGramT; ++i) {
      const int ja = a0 + i;
      if (ja >= k) break;
      const int lo = (ta == tb) ? ja + 1 : b0;
      const int hi = (b0 + kGramT < k) ? b0 + kGramT : k;
      if (hi > lo) pairs += (unsigned long long)(hi - lo);
    }
    atomicAdd(&per->ccsims, pairs);
  }
}

__global__ __launch_bounds__(kBlock) void k_gram_partial(const double* __restrict__ C64,
                                                         int32_t k, int64_t d,
                                                         const int32_t* __restrict__ dirty,
                                                         int force_all, double* __restrict__ part,
                                                         int64_t slice_len,
                                                         Persist* __restrict__ per,
                                                         const StepCtl* __restrict__ ctl) {
  gram_partial_body(C64, k, d, dirty, force_all, part, slice_len, per, ctl, blockIdx.x,
                    blockIdx.y);
}

// Row a of G (slices summed in slice order) and gmax[a] = the largest
// off-diagonal entry of the row widened by delta_g (capped at 1), or -3
// (no centre-centre pruning) for k = 1.  One block per row.
__device__ __forceinline__ void gram_finalize_body(const double* __restrict__ part, int32_t k,
                                                   int nslice, double delta_g,
                                                   double* __restrict__ G,
                                                   double* __restrict__ gmax,
                                                   const StepCtl* __restrict__ ctl, int a) {
  __shared__ double sh[kBlock / 64];
  if (ctl && ctl->gram_mode != 1) return;
  const int64_t kk = (int64_t)k * k;
  double m = -INFINITY;
  for (int b = threadIdx.x; b < k; b += kBlock) {
    const int64_t src = ((a / kGramT) <= (b / kGramT)) ? (int64_t)a * k + b : (int64_t)b * k + a;
    const double* p = part + src;
    double g = 0.0;
    int s = 0;
    for (; s + 16 <= nslice; s += 16) {  // 16 loads in flight, added in slice order
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = p[(size_t)(s + q) * kk];
#pragma unroll
      for (int q = 0; q < 16; ++q) g += v[q];
    }
    for (; s < nslice; ++s) g += p[(size_t)s * kk];
    G[(size_t)a * k + b] = g;
    if (b != a) m = fmax(m, g);
  }
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) mm = fmax(mm, sh[w]);
    gmax[a] = (k > 1) ? fmin(1.0, mm + delta_g) : -3.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_gram_finalize(const double* __restrict__ part,
                                                          int32_t k, int nslice, double delta_g,
                                                          double* __restrict__ G,
                                                          double* __restrict__ gmax,
                                                          const StepCtl* __restrict__ ctl) {
  gram_finalize_body(part, k, nslice, delta_g, G, gmax, ctl, blockIdx.x);
}

// Carries the centre-centre bounds across a centre step without the d-long
// products: centres a and b moved by at most the angles whose cosines and
// sines are (pc, ps), so their angle shrank by at most theta_a + theta_b and
// the guarded Eq. (7) with that combined movement keeps G(a, b) an upper
// bound of <c_a, c_b> (1 once theta_a + theta_b reaches pi or the old angle).
// Every update adds 4e-15 for its own FP64 rounding.  One block per row;
// (a, b) and (b, a) get bitwise equal values.
__device__ __forceinline__ void gram_carry_body(double* __restrict__ G, int32_t k,
                                                const double* __restrict__ pc,
                                                const double* __restrict__ ps, double delta_g,
                                                double* __restrict__ gmax,
                                                const StepCtl* __restrict__ ctl, int a) {
  __shared__ double sh[kBlock / 64];
  if (ctl && ctl->gram_mode != 2) return;
  const double pa = pc[a], sa = ps[a];
  double m = -INFINITY;
  for (int b = threadIdx.x; b < k; b += kBlock) {
    if (b == a) continue;
    const double pb = pc[b], sb = ps[b];
    double g = G[(size_t)a * k + b];
    if (pa + pb <= 0.0) {
      g = 1.0;
    } else {
      const double cm = pa * pb - sa * sb;  // cos(theta_a + theta_b)
      const double sm = sa * pb + pa * sb;  // sin(theta_a + theta_b) >= 0
      g = fmin(1.0, dev::upper_upd(g, cm, sm) + 4e-15);
    }
    G[(size_t)a * k + b] = g;
    m = fmax(m, g);
  }
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) mm = fmax(mm, sh[w]);
    gmax[a] = (k > 1) ? fmin(1.0, mm + delta_g) : -3.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_gram_carry(double* __restrict__ G, int32_t k,
                                                       const double* __restrict__ pc,
                                                       const double* __restrict__ ps,
                                                       double delta_g,
                                                       double* __restrict__ gmax,
                                                       const StepCtl* __restrict__ ctl) {
  gram_carry_body(G, k, pc, ps, delta_g, gmax, ctl, blockIdx.x);
}

__global__ void k_c64_to_f32(const double* __restrict__ in, int64_t count, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < count) out[e] = (float)in[e];
}

__global__ void k_fill_f64(double* p, int64_t count, double value) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < count) p[e] = value;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < count) p[e] = value;
}

__global__ void k_step_init(StepCtl* ctl, int gram_on, int warm, double test_min,
                            double tight_min) {
  StepCtl c{};
  c.gram_on = gram_on;
  if (warm && gram_on) {  // the warm start's centre update: exact, every tile
    c.gram_mode = 1;
    c.gram_force = 1;
    c.gram_updates = 1;
  }
  c.tests = 1;
  c.test_gap = 2;
  c.test_min = test_min;
  c.tighten = 1;
  c.tight_gap = 4;
  c.tight_rate = 1.0;
  c.tight_min = tight_min;
  *ctl = c;
}

// One wave.  Sums the step's counter slots into its record; a step that
// changed no assignment stops the fit (the kernels of later queued steps
// then do nothing or find nothing to do).  Otherwise it decides, for step
// t + 1 and the centre update in between:
//  - the bound tests: on while the last step that ran them pruned at least
//    test_min of the rows; after one that pruned fewer, the next probe comes
//    test_gap steps later and the gap doubles (at most 64);
//  - the centre-centre products, needed only before a step with tests:
//    exact for the first two updates, after three carried ones, when more
//    than 5% of the rows moved, or when an update was skipped since the
//    last one (then every tile); carried otherwise;
//  - tightening: always at the first three steps and while the last
//    measured pruning rate of tightening reaches tight_min, else probed
//    with the same doubling gap.
__device__ __forceinline__ void step_end_body(const Counters* __restrict__ cnt,
                                              StepCtl* __restrict__ ctl,
                                              StepRec* __restrict__ rec,
                                              const Persist* __restrict__ per, int32_t t,
                                              int64_t n, int32_t* __restrict__ dirty, int32_t k,
                                              int gram_queued) {
  const int i = threadIdx.x;
  // the previous centre update's dirty flags have been read by now
  for (int j = i; j < k; j += 64) dirty[j] = 0;
  if (ctl->stop) {
    if (i == 0) rec->valid = 0;
    return;
  }
  unsigned long long v[7];
  {
    const Counters& c = cnt[i];
    v[0] = c.changed;
    v[1] = c.sims;
    v[2] = c.rechecks;
    v[3] = c.tightened;
    v[4] = c.tight_saved;
    v[5] = c.rows_done;
    v[6] = c.nnz_done;
  }
#pragma unroll
  for (int q = 0; q < 7; ++q)
    for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  if (i != 0) return;
  StepRec r{};
  r.changed = v[0];
  r.sims = v[1];
  r.rechecks = v[2];
  r.tightened = v[3];
  r.tight_saved = v[4];
  r.rows_done = v[5];
  r.nnz_done = v[6];
  r.objective = per->objective;
  r.valid = 1;
  *rec = r;
  StepCtl c = *ctl;
  if (r.changed == 0) {
    c.stop = 1;
    c.gram_mode = 0;
    *ctl = c;
    return;
  }
  // bound tests of step t + 1 (step 0 walks every row and runs none)
  const bool tested = t > 0 && c.tests != 0;
  if (tested) {
    // share of the point-centre similarities the tests saved (whole rows,
    // or groups of a row for Yin-Yang)
    const double pruned =
        1.0 - (double)(r.sims - r.tightened) / ((double)n * (double)k);
    if (pruned >= c.test_min) {
      c.tests = 1;
      c.test_gap = 2;
    } else {
      c.test_next = t + c.test_gap;
      c.test_gap = c.test_gap < 32 ? 2 * c.test_gap : 64;
      c.tests = (t + 1 >= c.test_next) ? 1 : 0;
    }
  } else {
    c.tests = (t + 1 >= c.test_next) ? 1 : 0;
  }
  // tests that need the centre-centre products wait for a step whose centre
  // update has the Gram kernels queued (the host leaves them out only where
  // it knows the tests are off)
  if (c.gram_on && !gram_queued) c.tests = 0;
  // centre-centre products for the coming centre update
  if (c.gram_on) {
    if (!c.tests) {
      c.gram_mode = 0;
      c.gram_stale = 1;
    } else {
      const bool exact = c.gram_stale ||
                         gram_exact_step(c.gram_updates, c.gram_since_exact,
                                         (int64_t)r.changed, n);
      c.gram_mode = exact ? 1 : 2;
      // after carried or skipped updates every tile's partial products are stale
      c.gram_force =
          (c.gram_updates == 0 || c.gram_since_exact > 0 || c.gram_stale) ? 1 : 0;
      c.gram_since_exact = exact ? 0 : c.gram_since_exact + 1;
      c.gram_updates += 1;
      c.gram_stale = 0;
    }
  }
  // tightening (it only matters in a step with tests)
  if (tested) {
    const bool was_on = c.tighten != 0;
    if (r.tightened > 0) c.tight_rate = (double)r.tight_saved / (double)r.tightened;
    if (t + 1 <= 2 || c.tight_rate >= c.tight_min) {
      c.tighten = 1;
      c.tight_gap = 4;
    } else {
      if (was_on) {
        c.tight_next = t + c.tight_gap;
        c.tight_gap = c.tight_gap < 32 ? 2 * c.tight_gap : 64;
      }
      c.tighten = (t + 1 >= c.tight_next) ? 1 : 0;
    }
  }
  *ctl = c;
}

__global__ void k_step_end(const Counters* __restrict__ cnt, StepCtl* __restrict__ ctl,
                           StepRec* __restrict__ rec, const Persist* __restrict__ per, int32_t t,
                           int64_t n, int32_t* __restrict__ dirty, int32_t k, int gram_queued) {
  step_end_body(cnt, ctl, rec, per, t, n, dirty, k, gram_queued);
}

// ------------------------------------------------------------------------
// Batched fits: the kernels above with their arguments taken from the
// problem's FitView; every block serves one work item (.x = problem).  The
// bodies are the single-problem ones, so every problem computes exactly
// what its own fit computes.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_b_row_eta(const FitView* __restrict__ V,
                                                      const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  row_eta_body(f.rp, f.v, f.n, f.eta, f.maxeta, (int64_t)w.y / kBlock);
}

__global__ __launch_bounds__(kBlock) void k_b_init_centres(const FitView* __restrict__ V,
                                                           const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  init_centres_body(f.init, f.d, 1, f.C64, f.initnorm, w.y);
}

__global__ __launch_bounds__(kBlock) void k_b_transpose(const FitView* __restrict__ V,
                                                        const int4* __restrict__ items,
                                                        int use_dirty) {
  const int4 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  const int64_t ntt = (f.d + 63) / 64;
  const int64_t end = ((int64_t)w.z + kTransposeGroup < ntt) ? w.z + kTransposeGroup : ntt;
  for (int64_t tt = w.z; tt < end; ++tt) {
    transpose_body(f.C64, f.k, f.d, f.kp, use_dirty ? f.dirty : nullptr, f.CT, nullptr, tt, w.y);
    __syncthreads();  // the next tile reuses the LDS tile
  }
}

__global__ void k_b_step_init(const FitView* __restrict__ V, int nprob) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= nprob) return;
  const FitView& f = V[p];
  StepCtl c{};
  c.gram_on = f.gram;
  c.tests = 1;
  c.test_gap = 2;
  c.test_min = f.test_min;
  c.tighten = 1;
  c.tight_gap = 4;
  c.tight_rate = 1.0;
  c.tight_min = f.tight_min;
  c.max_iter = f.max_iter;
  *f.ctl = c;
}

// One wave per problem: step_end_body with the step index the problem keeps
// in its StepCtl; a problem that reaches its max_iter stops with stop = 2
// (the centre update of that last step still runs, as in a single fit).
__global__ void k_b_step_end(const FitView* __restrict__ V, int slot) {
  const FitView& f = V[blockIdx.x];
  StepCtl* ctl = f.ctl;
  const int32_t t = ctl->step;
  const int32_t was_stopped = ctl->stop;
  step_end_body(f.cnt + (size_t)slot * kCounterSlots, ctl, f.rec + slot, f.per, t, f.n,
                f.dirty, f.k, 1);
  if (threadIdx.x == 0 && !was_stopped) {
    ctl->step = t + 1;
    if (t + 1 >= ctl->max_iter && ctl->stop == 0) {
      ctl->stop = 2;
      ctl->gram_mode = 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_b_update_scan(const FitView* __restrict__ V,
                                                          const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  const int64_t end = ((int64_t)w.y + kBlock < f.n) ? (int64_t)w.y + kBlock : f.n;
  update_scan_body(f.rp, f.ci, f.v, f.a, f.a_old, w.y, end, kBlock, f.d, f.fx, f.S, f.dirty);
}

__global__ __launch_bounds__(kBlock) void k_b_sumsq(const FitView* __restrict__ V,
                                                    const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  for (int ch = 0; ch < f.nchunk; ++ch)
    sumsq_partial_body(f.S, f.d, f.fx_inv, f.dirty, f.part_sq, f.nchunk, ch, w.y);
}

__global__ __launch_bounds__(kBlock) void k_b_normalize(const FitView* __restrict__ V,
                                                        const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  for (int ch = 0; ch < f.nchunk; ++ch)
    normalize_move_body(f.S, f.d, f.fx_inv, f.dirty, f.part_sq, f.C64, f.part, f.nchunk, ch,
                        w.y);
}

__global__ __launch_bounds__(kBlock) void k_b_finalize(const FitView* __restrict__ V) {
  const FitView& f = V[blockIdx.x];
  centre_finalize_body(f.k, f.d, f.dirty, f.norm64, f.part_sq, f.part, f.nchunk, f.delta_c, f.pc,
                       f.ps, f.mm, f.per);
}

__global__ __launch_bounds__(kBlock) void k_b_gram_partial(const FitView* __restrict__ V,
                                                           const int4* __restrict__ items) {
  const int4 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  gram_partial_body(f.C64, f.k, f.d, f.dirty, 0, f.gpart, f.slice_len, f.per, f.ctl, w.y, w.z);
}

__global__ __launch_bounds__(kBlock) void k_b_gram_finalize(const FitView* __restrict__ V,
                                                            const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  gram_finalize_body(f.gpart, f.k, f.nslice, f.delta_g, f.G, f.gmax, f.ctl, w.y);
}

__global__ __launch_bounds__(kBlock) void k_b_gram_carry(const FitView* __restrict__ V,
                                                         const int2* __restrict__ items) {
  const int2 w = items[blockIdx.x];
  const FitView& f = V[w.x];
  gram_carry_body(f.G, f.k, f.pc, f.ps, f.delta_g, f.gmax, f.ctl, w.y);
}

unsigned blocks_for(int64_t count) {
  int64_t b = (count + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_row_eta(const int64_t* rp, const float* v, int64_t n, float* eta,
                          float* max_eta, hipStream_t s) {
  hipLaunchKernelGGL(k_row_eta, dim3(blocks_for(n)), dim3(kBlock), 0, s, rp, v, n, eta, max_eta);
  return hipGetLastError();
}

hipError_t launch_init_centres(const float* init, int32_t k, int64_t d, int normalize,
                               double* C64, double* init_norm, hipStream_t s) {
  hipLaunchKernelGGL(k_init_centres, dim3(k), dim3(kBlock), 0, s, init, d, normalize, C64,
                     init_norm);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* C64, int32_t k, int64_t d, int32_t kp,
                            const int32_t* dirty, float* CT, hipStream_t s, void* CT16) {
  const dim3 grid((unsigned)((d + 63) / 64), (unsigned)((k + 63) / 64));
  hipLaunchKernelGGL(k_transpose, grid, dim3(kBlock), 0, s, C64, k, d, kp, dirty, CT,
                     static_cast<__half*>(CT16));
  return hipGetLastError();
}

hipError_t launch_neg_scan(const float* v, int64_t nnz, const float* init, int64_t ninit,
                           int32_t* flag, hipStream_t s) {
  int64_t blocks = (nnz + ninit + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_neg_scan, dim3((unsigned)blocks), dim3(kBlock), 0, s, v, nnz, init, ninit,
                     flag);
  return hipGetLastError();
}

hipError_t launch_check_rowptr(const int64_t* rp, int64_t n, int64_t nnz,
                               unsigned long long* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_check_rowptr, dim3(blocks_for(n + 1)), dim3(kBlock), 0, s, rp, n, nnz,
                     bad);
  return hipGetLastError();
}

hipError_t launch_check_entries(const int64_t* rp, const int32_t* ci, const float* v, int64_t n,
                                int64_t d, unsigned long long* bad, hipStream_t s) {
  const unsigned blocks = std::min(blocks_for(n), 4096u);
  hipLaunchKernelGGL(k_check_entries, dim3(blocks), dim3(kBlock), 0, s, rp, ci, v, n, d, bad);
  return hipGetLastError();
}

hipError_t launch_check_dense(const float* x, int64_t ld, int64_t n, int64_t d,
                              unsigned long long* bad, hipStream_t s) {
  const unsigned blocks = std::min(blocks_for(n * d), 4096u);
  hipLaunchKernelGGL(k_check_dense, dim3(blocks), dim3(kBlock), 0, s, x, ld, n, d, bad);
  return hipGetLastError();
}

hipError_t launch_update_scan(const int64_t* rp, const int32_t* ci, const float* v,
                              const int32_t* a, int32_t* a_old, int64_t n, int64_t d,
                              double fx_scale, long long* S, int32_t* dirty, hipStream_t s) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > kMaxGridBlocks) blocks = kMaxGridBlocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_update_scan, dim3((unsigned)blocks), dim3(kBlock), 0, s, rp, ci, v, a,
                     a_old, n, d, fx_scale, S, dirty);
  return hipGetLastError();
}

hipError_t launch_sumsq_partial(const long long* S, int32_t k, int64_t d, double fx_inv,
                               const int32_t* dirty, double* part_sq, int nchunk, hipStream_t s) {
  const dim3 grid((unsigned)nchunk, (unsigned)k);
  hipLaunchKernelGGL(k_sumsq_partial, grid, dim3(kBlock), 0, s, S, d, fx_inv, dirty, part_sq,
                     nchunk);
  return hipGetLastError();
}

hipError_t launch_normalize_move(const long long* S, int32_t k, int64_t d, double fx_inv,
                                 const int32_t* dirty, const double* part_sq, double* C64,
                                 double* part, int nchunk, hipStream_t s) {
  const dim3 grid((unsigned)nchunk, (unsigned)k);
  hipLaunchKernelGGL(k_normalize_move, grid, dim3(kBlock), 0, s, S, d, fx_inv, dirty, part_sq,
                     C64, part, nchunk);
  return hipGetLastError();
}

hipError_t launch_centre_finalize(int32_t k, int64_t d, const int32_t* dirty, double* norm64,
                                  const double* part_sq, const double* part, int nchunk,
                                  double delta_c, double* pc, double* ps, MoveMin* mm,
                                  Persist* per, hipStream_t s) {
  hipLaunchKernelGGL(k_centre_finalize, dim3(1), dim3(kBlock), 0, s, k, d, dirty, norm64,
                     part_sq, part, nchunk, delta_c, pc, ps, mm, per);
  return hipGetLastError();
}

hipError_t launch_clear_dirty(int32_t* dirty, int32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_dirty, dim3(blocks_for(k)), dim3(kBlock), 0, s, dirty, k);
  return hipGetLastError();
}

void gram_slicing(int32_t k, int64_t d, int* nslice, int64_t* slice_len) {
  // about 1024 blocks (four per CU), slices of at least 256 columns
  const int nt = (k + kGramT - 1) / kGramT;
  const int tiles = nt * (nt + 1) / 2;
  int ns = (1024 + tiles - 1) / tiles;
  const int64_t max_ns = d / 256 > 1 ? d / 256 : 1;
  if (ns > max_ns) ns = (int)max_ns;
  if (ns < 1) ns = 1;
  int64_t len = (d + ns - 1) / ns;
  len = (len + kGramK - 1) / kGramK * kGramK;
  *slice_len = len;
  *nslice = (int)((d + len - 1) / len);
}

hipError_t launch_gram(const double* C64, int32_t k, int64_t d, const int32_t* dirty,
                       int force_all, double* part, int nslice, int64_t slice_len, double* G,
                       double* gmax, double delta_g, Persist* per, hipStream_t s,
                       const StepCtl* ctl) {
  const int nt = (k + kGramT - 1) / kGramT;
  const dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)nslice);
  hipLaunchKernelGGL(k_gram_partial, grid, dim3(kBlock), 0, s, C64, k, d, dirty, force_all, part,
                     slice_len, per, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_finalize, dim3((unsigned)k), dim3(kBlock), 0, s, part, k, nslice,
                     delta_g, G, gmax, ctl);
  return hipGetLastError();
}

hipError_t launch_gram_carry(double* G, int32_t k, const double* pc, const double* ps,
                             double delta_g, double* gmax, hipStream_t s, const StepCtl* ctl) {
  hipLaunchKernelGGL(k_gram_carry, dim3((unsigned)k), dim3(kBlock), 0, s, G, k, pc, ps, delta_g,
                     gmax, ctl);
  return hipGetLastError();
}

hipError_t launch_step_init(StepCtl* ctl, int gram_on, int warm, double test_min,
                            double tight_min, hipStream_t s) {
  hipLaunchKernelGGL(k_step_init, dim3(1), dim3(1), 0, s, ctl, gram_on, warm, test_min,
                     tight_min);
  return hipGetLastError();
}

hipError_t launch_step_end(const Counters* cnt, StepCtl* ctl, StepRec* rec, const Persist* per,
                           int32_t t, int64_t n, int32_t* dirty, int32_t k, int gram_queued,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, s, cnt, ctl, rec, per, t, n, dirty, k,
                     gram_queued);
  return hipGetLastError();
}

hipError_t launch_c64_to_f32(const double* C64, int64_t count, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_c64_to_f32, dim3(blocks_for(count)), dim3(kBlock), 0, s, C64, count, out);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t count, double value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_b_row_eta(const FitView* V, const int2* items, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_row_eta, dim3((unsigned)n_items), dim3(kBlock), 0, s, V, items);
  return hipGetLastError();
}

hipError_t launch_b_init_centres(const FitView* V, const int2* items, int n_items,
                                 hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_init_centres, dim3((unsigned)n_items), dim3(kBlock), 0, s, V, items);
  return hipGetLastError();
}

hipError_t launch_b_transpose(const FitView* V, const int4* items, int n_items, int use_dirty,
                              hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_transpose, dim3((unsigned)n_items), dim3(kBlock), 0, s, V, items,
                     use_dirty);
  return hipGetLastError();
}

hipError_t launch_b_step_init(const FitView* V, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_b_step_init, dim3(blocks_for(nprob)), dim3(kBlock), 0, s, V, nprob);
  return hipGetLastError();
}

hipError_t launch_b_step_end(const FitView* V, int nprob, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_b_step_end, dim3((unsigned)nprob), dim3(64), 0, s, V, slot);
  return hipGetLastError();
}

hipError_t launch_b_update_scan(const FitView* V, const int2* items, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_update_scan, dim3((unsigned)n_items), dim3(kBlock), 0, s, V, items);
  return hipGetLastError();
}

hipError_t launch_b_sumsq(const FitView* V, const int2* items, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_sumsq, dim3((unsigned)n_items), dim3(kBlock), 0, s, V, items);
  return hipGetLastError();
}

hipError_t launch_b_normalize(const FitView* V, const int2* items, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_normalize, dim3((unsigned)n_items), dim3(kBlock), 0, s, V, items);
  return hipGetLastError();
}

hipError_t launch_b_finalize(const FitView* V, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_b_finalize, dim3((unsigned)nprob), dim3(kBlock), 0, s, V);
  return hipGetLastError();
}

hipError_t launch_b_gram(const FitView* V, const int4* pair_items, int n_pair_items,
                         const int2* centre_items, int n_centre_items, hipStream_t s) {
  if (n_pair_items <= 0 || n_centre_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_gram_partial, dim3((unsigned)n_pair_items), dim3(kBlock), 0, s, V,
                     pair_items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_gram_finalize, dim3((unsigned)n_centre_items), dim3(kBlock), 0, s, V,
                     centre_items);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_gram_carry, dim3((unsigned)n_centre_items), dim3(kBlock), 0, s, V,
                     centre_items);
  return hipGetLastError();
}

}  // namespace skm
