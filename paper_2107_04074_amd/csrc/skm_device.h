// Device helpers shared by every kernel file of libskm: the tie order of
// the argmax, the canonical FP64 similarity used for every re-decision,
// and the guarded bound updates of Section 4 (Eq. (6), (7)) and the
// centre-centre threshold of Section 5.2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace skm {
namespace dev {

// Strict order used for every argmax: larger value first; on equal values
// the previous assignment first; then the lower index.
__device__ __forceinline__ bool better32(float s, int j, float t, int tj, int prev) {
  if (s != t) return s > t;
  const bool pj = (j == prev), pt = (tj == prev);
  if (pj != pt) return pj;
  return j < tj;
}

__device__ __forceinline__ bool better64(double s, int j, double t, int tj, int prev) {
  if (s != t) return s > t;
  const bool pj = (j == prev), pt = (tj == prev);
  if (pj != pt) return pj;
  return j < tj;
}

// Canonical FP64 similarity of a CSR row with one FP64 centre.  Entry e of
// the row (position p = e - beg) goes into partial sum p mod 64; every
// partial is a sequential FMA chain in storage order and the 64 partials
// are added by a balanced pairwise tree (pairs (2i, 2i+1), then pairs of
// pairs, ...).  Every FP64 re-decision uses exactly this value, computed
// either by a group of G lanes together (dot64_group: lane gl holds the
// partials gl + G r) or by one lane (dot64_serial: a pairwise stack), and
// both give bit-identical results (each tree node is one FP64 addition of
// the same two operands; addition is commutative).
template <int G>
__device__ __forceinline__ double dot64_group(const int32_t* __restrict__ ci,
                                              const float* __restrict__ v, int64_t beg,
                                              int64_t end, const double* __restrict__ c, int gl) {
  constexpr int P = 64 / G;
  double part[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    double s = 0.0;
    for (int64_t e = beg + gl + G * r; e < end; e += 64) s = fma((double)v[e], c[ci[e]], s);
    part[r] = s;
  }
#pragma unroll
  for (int r = 0; r < P; ++r)
#pragma unroll
    for (int off = 1; off < G; off <<= 1) part[r] += __shfl_xor(part[r], off, G);
#pragma unroll
  for (int w = 1; w < P; w <<= 1)
#pragma unroll
    for (int r = 0; r < P; r += 2 * w) part[r] += part[r + w];
  return part[0];
}

// The same canonical value computed by one lane for a row of at most 8
// stored entries: partials 8 ... 63 are zero, so the tree reduces to the
// pairwise sum of the first eight partials plus the zero subtrees (+0.0).
__device__ __forceinline__ double dot64_short(const int32_t* __restrict__ ci,
                                              const float* __restrict__ v, int64_t beg,
                                              int64_t end, const double* __restrict__ c) {
  double p[8];
#pragma unroll
  for (int q = 0; q < 8; ++q)
    p[q] = (beg + q < end) ? fma((double)v[beg + q], c[ci[beg + q]], 0.0) : 0.0;
  return (((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]))) + 0.0;
}

__device__ __forceinline__ double dot64_serial(const int32_t* __restrict__ ci,
                                               const float* __restrict__ v, int64_t beg,
                                               int64_t end, const double* __restrict__ c) {
  double st[7];
#pragma unroll
  for (int p = 0; p < 64; ++p) {
    double s = 0.0;
    for (int64_t e = beg + p; e < end; e += 64) s = fma((double)v[e], c[ci[e]], s);
    int lev = 0;
#pragma unroll
    for (int q = p; q & 1; q >>= 1) s = st[lev++] + s;
    st[lev] = s;
  }
  return st[6];
}

// Guarded Eq. (6): cos(theta_l + theta_p), or -1 once the sum reaches pi.
__device__ __forceinline__ double lower_upd(double l, double pc, double ps) {
  l = fmin(1.0, fmax(-1.0, l));
  if (l <= -pc) return -1.0;
  return l * pc - sqrt((1.0 - l) * (1.0 + l)) * ps;
}

// Guarded Eq. (7): cos(theta_u - theta_p), or 1 once theta_p >= theta_u.
__device__ __forceinline__ double upper_upd(double u, double pc, double ps) {
  u = fmin(1.0, fmax(-1.0, u));
  if (u >= pc) return 1.0;
  return u * pc + sqrt((1.0 - u) * (1.0 + u)) * ps;
}

// cos(theta_l + theta_M) for l, M in (0, 1]: the largest centre-centre
// cosine that still proves every point of the cap is at most M.
__device__ __forceinline__ double cc_threshold(double l, double M) {
  return l * M - sqrt((1.0 - l) * (1.0 + l) * (1.0 - M) * (1.0 + M));
}

template <int G>
__device__ __forceinline__ void group_top2(float& b, int& bj, float& s2, int prev) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    const float ob = __shfl_xor(b, off, G);
    const int oj = __shfl_xor(bj, off, G);
    const float o2 = __shfl_xor(s2, off, G);
    const float m2 = fmaxf(s2, o2);
    if (better32(ob, oj, b, bj, prev)) {
      s2 = fmaxf(m2, b);
      b = ob;
      bj = oj;
    } else {
      s2 = fmaxf(m2, ob);
    }
  }
}

template <int G>
__device__ __forceinline__ void group_best64(double& b, int& bj, int prev) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(b, off, G);
    const int oj = __shfl_xor(bj, off, G);
    if (better64(ob, oj, b, bj, prev)) {
      b = ob;
      bj = oj;
    }
  }
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, G);
  return x;
}

template <int G>
__device__ __forceinline__ unsigned group_or(unsigned x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) x |= (unsigned)__shfl_xor((int)x, off, G);
  return x;
}

// FP32 similarity of row [beg, end) with centre j read as one column of the
// centre-minor FP32 copy CT (d x kp): the group's lanes take every G-th
// entry and the partial sums are combined by the group.  Used where only a
// few centres of a row are needed (tightening, surviving Elkan pairs); the
// summation order differs from the full row walk, which the FP32 error
// bound (m + 3) 2^-24 |x| covers for any order.
template <int G>
__device__ __forceinline__ float group_col_dot32(const int32_t* __restrict__ ci,
                                                 const float* __restrict__ v, int64_t beg,
                                                 int64_t end, const float* __restrict__ CT,
                                                 int kp, int j, int gl) {
  float p0 = 0.f, p1 = 0.f;
  int64_t e = beg + gl;
  for (; e + G < end; e += 2 * G) {
    const int32_t c0 = ci[e], c1 = ci[e + G];
    const float x0 = v[e], x1 = v[e + G];
    p0 = fmaf(x0, CT[(uint32_t)c0 * (uint32_t)kp + (uint32_t)j], p0);
    p1 = fmaf(x1, CT[(uint32_t)c1 * (uint32_t)kp + (uint32_t)j], p1);
  }
  if (e < end) p0 = fmaf(v[e], CT[(uint32_t)ci[e] * (uint32_t)kp + (uint32_t)j], p0);
  return group_sum<G>(p0 + p1);
}

// Appends `item` to list[] for every lane with `push` set, with one atomic
// per wave: the wave reserves a contiguous range and each pushing lane
// writes at its rank.  Must be reached by all active lanes of the wave.
__device__ __forceinline__ void wave_append(bool push, int32_t item,
                                            unsigned long long* counter,
                                            int32_t* list, int32_t item2,
                                            int32_t* list2) {
  const unsigned long long mask = __ballot(push);
  if (mask == 0ull) return;
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0ull;
  if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (push) {
    const unsigned long long rank = __popcll(mask & ((1ull << lane) - 1ull));
    list[base + rank] = item;
    if (list2) list2[base + rank] = item2;
  }
}

}  // namespace dev
}  // namespace skm
