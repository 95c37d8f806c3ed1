// Assignment-step kernels for gfx950 (wave64).
//
//  k_assign_csr  similarities of CSR rows against all k centres (Section 5,
//                assignment equation; sparse-dense products as in Section 2),
//                group top-2 reduction, FP64 re-decision of near ties, and in
//                fit mode the bounds of Section 4; in Hamerly mode each row
//                first runs the bound update and tests of Section 5.3 and is
//                walked only when they fail.
//                In Elkan mode the row first runs Eq. (6) for l(i), the
//                guarded Eq. (7) for every pair bound u(i,j), the point test
//                on s(a(i)) and the pair tests u(i,j) <= l(i), cc(a(i),j) <=
//                l(i) (Sections 5.1, 5.2); in Yin-Yang mode one bound per
//                group of 32 centres (Section 5.5).  Rows with a surviving
//                candidate are walked in full and get exact bounds.
//
// Row mapping: for k <= 64 a group of G = 4, 8 or 16 lanes owns one row and
// lane g owns the float4 chunk g of each centre-minor CT row (row_sims);
// for larger k one wave owns a row (row_walk: S sub-waves interleave the
// row's entries, every lane owns R 16-byte chunks of VEC centres, read from
// the FP32 copy or, with precision 2, from the FP16 copy).  Similarities are
// FP32 FMA chains over stored entries in storage order; near ties are
// re-decided in FP64 (dot64_group, the canonical order).
#include <float.h>
#include <limits.h>

#include <hip/hip_fp16.h>

#include "skm_device.h"
#include "skm_internal.h"

namespace skm {

Geometry pick_geometry(int k) {
  if (k <= 16) return {4, 1, 16};
  if (k <= 32) return {8, 1, 32};
  if (k <= 64) return {16, 1, 64};
  if (k <= 128) return {32, 1, 128};
  if (k <= 256) return {64, 1, 256};
  if (k <= 512) return {64, 2, 512};
  if (k <= 1024) return {64, 4, 1024};
  if (k <= 2048) return {64, 8, 2048};
  if (k <= 4096) return {64, 16, 4096};
  return {0, 0, 0};
}

namespace {
using namespace dev;

__device__ __forceinline__ float f4get(const float4& f, int q) {
  return q == 0 ? f.x : (q == 1 ? f.y : (q == 2 ? f.z : f.w));
}

__device__ __forceinline__ void f4set(float4& f, int q, float x) {
  if (q == 0) f.x = x;
  else if (q == 1) f.y = x;
  else if (q == 2) f.z = x;
  else f.w = x;
}

// Gathers in flight per lane and batch: enough independent float4 loads
// to cover L2/MALL latency without exhausting registers.
template <int G, int R>
struct Batch {
  static constexpr int raw = (R >= 8) ? 1 : (R >= 4 ? 2 : (R >= 2 ? 4 : 8));
  static constexpr int U = raw < G ? raw : G;
};

// Accumulates the FP32 similarities of the row [beg, end) for the chunks
// selected by `need` (bit r = chunk r).  Entries are handled G at a time
// (one per lane, broadcast by shuffles) in batches of U: the U gathers of a
// batch are issued before any of its FMAs, and the next G entries are
// fetched while the current ones are consumed.  Entries past the end of the
// row are padded with x = 0, which leaves every FMA chain unchanged, so
// each similarity is still the sequential chain over the stored entries.
// Returns the row's squared norm summed over the group (float).
template <int G, int R, bool MASKED>
__device__ __forceinline__ float row_sims(const int32_t* __restrict__ ci,
                                          const float* __restrict__ v, int64_t beg,
                                          int64_t end, const float4* __restrict__ CT4,
                                          int kp4, int gl, unsigned need, float4 (&acc)[R]) {
  constexpr int U = Batch<G, R>::U;
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = make_float4(0.f, 0.f, 0.f, 0.f);
  float nrm2 = 0.f;
  int c = 0;
  float x = 0.f;
  if (beg + gl < end) {
    c = ci[beg + gl];
    x = v[beg + gl];
  }
  for (int64_t base = beg; base < end; base += G) {
    const int cnt = (int)((end - base) < G ? (end - base) : G);
    // prefetch the next G entries
    int cn = 0;
    float xn = 0.f;
    const int64_t en = base + G + gl;
    if (en < end) {
      cn = ci[en];
      xn = v[en];
    }
    nrm2 = fmaf(x, x, nrm2);
    for (int q0 = 0; q0 < cnt; q0 += U) {
      int cq[U];
      float xq[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cq[u] = __shfl(c, q0 + u, G);
        xq[u] = __shfl(x, q0 + u, G);
      }
      float4 f[U][R];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float4* p = CT4 + (uint32_t)((uint32_t)cq[u] * (uint32_t)kp4) + gl;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!MASKED || ((need >> r) & 1u)) f[u][r] = p[r * G];
          else f[u][r] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc[r].x = fmaf(xq[u], f[u][r].x, acc[r].x);
          acc[r].y = fmaf(xq[u], f[u][r].y, acc[r].y);
          acc[r].z = fmaf(xq[u], f[u][r].z, acc[r].z);
          acc[r].w = fmaf(xq[u], f[u][r].w, acc[r].w);
        }
    }
    c = cn;
    x = xn;
  }
  return group_sum<G>(nrm2);
}

// One row per wave.  The 64 lanes form S = 64 / L sub-waves of L lanes;
// sub-wave s takes the entries s, s + S, s + 2S, ... of the row, and lane
// gl of a sub-wave owns chunks gl + L r (r < R) of every centre row: VEC
// consecutive centres, stored as FP32 (VEC = 4) or FP16 (VEC = 8), 16 bytes
// either way, so one gather instruction fetches S entries' rows.  Column
// ids and values of 64 consecutive entries sit one per lane and are handed
// to the sub-waves by readlane (S = 1) or a lane shuffle; gathers are double
// buffered in batches of U entries per sub-wave, the next batch in flight
// while the current one is consumed, also across 64-entry windows.  Lanes
// past the row end hold column 0 and value 0: their gathers read centre row
// 0 and add exactly nothing, so no bounds branch sits between the loads.
// Each sub-wave's sums are a sequential FMA chain; the S partial chains are
// added by a fixed xor tree at the end, so all sub-waves hold the same sums
// (the order is covered by the error bound of the re-decision).
template <int R>
struct WalkBatch {
  static constexpr int U = (R >= 4) ? 1 : 4 / R;
};

__device__ __forceinline__ int lane_int(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_float(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <int S>
__device__ __forceinline__ int entry_int(int w, int idx_uniform, int sub) {
  if constexpr (S == 1) return lane_int(w, idx_uniform);
  else return __shfl(w, idx_uniform + sub, 64);
}
template <int S>
__device__ __forceinline__ float entry_float(float w, int idx_uniform, int sub) {
  if constexpr (S == 1) return lane_float(w, idx_uniform);
  else return __shfl(w, idx_uniform + sub, 64);
}

template <int L, int R, bool MASKED>
__device__ __forceinline__ void walk_issue(uint4 (&dst)[WalkBatch<R>::U][R], int cw, int first,
                                           int sub, const uint4* __restrict__ C16B, int kp16,
                                           int gl, unsigned need) {
  constexpr int S = 64 / L;
  constexpr int U = WalkBatch<R>::U;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int cu = entry_int<S>(cw, S * (first + u), sub);
    const uint4* p = C16B + (uint32_t)((uint32_t)cu * (uint32_t)kp16) + gl;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!MASKED || ((need >> r) & 1u)) dst[u][r] = p[L * r];
      else dst[u][r] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

template <int L, int R, int VEC>
__device__ __forceinline__ void walk_consume(const uint4 (&src)[WalkBatch<R>::U][R], float xw,
                                             int first, int sub,
                                             float4 (&acc)[R * VEC / 4]) {
  constexpr int S = 64 / L;
  constexpr int U = WalkBatch<R>::U;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const float xu = entry_float<S>(xw, S * (first + u), sub);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (VEC == 4) {
        float4& a = acc[r];
        a.x = fmaf(xu, __uint_as_float(src[u][r].x), a.x);
        a.y = fmaf(xu, __uint_as_float(src[u][r].y), a.y);
        a.z = fmaf(xu, __uint_as_float(src[u][r].z), a.z);
        a.w = fmaf(xu, __uint_as_float(src[u][r].w), a.w);
      } else {
        const uint32_t wv[4] = {src[u][r].x, src[u][r].y, src[u][r].z, src[u][r].w};
        float4& a = acc[2 * r];
        float4& b = acc[2 * r + 1];
        a.x = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[0] & 0xffffu))), a.x);
        a.y = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[0] >> 16))), a.y);
        a.z = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[1] & 0xffffu))), a.z);
        a.w = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[1] >> 16))), a.w);
        b.x = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[2] & 0xffffu))), b.x);
        b.y = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[2] >> 16))), b.y);
        b.z = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[3] & 0xffffu))), b.z);
        b.w = fmaf(xu, __half2float(__ushort_as_half((unsigned short)(wv[3] >> 16))), b.w);
      }
    }
  }
}

// col16 >= 0: the lane reads 16-byte unit col16 of each centre row instead
// of unit lane % L (a packed subset of the row's units).
template <int L, int R, int VEC, bool MASKED = false>
__device__ __forceinline__ float row_walk(const int32_t* __restrict__ ci,
                                          const float* __restrict__ v, int64_t beg, int64_t end,
                                          int c0, float x0, const void* __restrict__ CTB, int kp,
                                          int lane, float4 (&acc)[R * VEC / 4],
                                          unsigned need = ~0u, int col16 = -1) {
  constexpr int S = 64 / L;
  constexpr int U = WalkBatch<R>::U;
  constexpr int PER_WIN = 64 / (S * U);  // batches per 64-entry window (even)
  static_assert(PER_WIN % 2 == 0, "double buffering needs an even batch count");
  const int sub = lane / L, gl = col16 >= 0 ? col16 : lane % L;
  const uint4* C16B = reinterpret_cast<const uint4*>(CTB);
  const int kp16 = kp / VEC;  // 16-byte chunks per centre row
#pragma unroll
  for (int q = 0; q < R * VEC / 4; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  float nrm2 = 0.f;
  uint4 buf0[U][R], buf1[U][R];
  int c = c0;  // entries beg .. beg + 63, loaded by the caller (0 past the end)
  float x = x0;
  walk_issue<L, R, MASKED>(buf0, c, 0, sub, C16B, kp16, gl, need);
  for (int64_t w0 = beg; w0 < end; w0 += 64) {
    int cn = 0;
    float xn = 0.f;
    if (w0 + 64 + lane < end) {
      cn = ci[w0 + 64 + lane];
      xn = v[w0 + 64 + lane];
    }
    nrm2 = fmaf(x, x, nrm2);
    // unrolled: straight-line code lets the compiler count the loads in
    // flight exactly and wait only for the buffer being consumed
#pragma unroll
    for (int b = 0; b < PER_WIN; b += 2) {
      const int64_t eb = w0 + (int64_t)(S * U) * b;
      if (eb >= end) break;
      walk_issue<L, R, MASKED>(buf1, c, (b + 1) * U, sub, C16B, kp16, gl, need);
      __builtin_amdgcn_sched_barrier(0);  // keep these loads ahead of the FMAs below
      walk_consume<L, R, VEC>(buf0, x, b * U, sub, acc);
      if (eb + S * U >= end) break;
      if (b + 2 < PER_WIN)
        walk_issue<L, R, MASKED>(buf0, c, (b + 2) * U, sub, C16B, kp16, gl, need);
      else
        walk_issue<L, R, MASKED>(buf0, cn, 0, sub, C16B, kp16, gl, need);
      __builtin_amdgcn_sched_barrier(0);
      walk_consume<L, R, VEC>(buf1, x, (b + 1) * U, sub, acc);
    }
    c = cn;
    x = xn;
  }
#pragma unroll
  for (int off = L; off < 64; off <<= 1)
#pragma unroll
    for (int q = 0; q < R * VEC / 4; ++q) {
      acc[q].x += __shfl_xor(acc[q].x, off, 64);
      acc[q].y += __shfl_xor(acc[q].y, off, 64);
      acc[q].z += __shfl_xor(acc[q].z, off, 64);
      acc[q].w += __shfl_xor(acc[q].w, off, 64);
    }
  return group_sum<64>(nrm2);
}

// ------------------------------------------------------------------------
// k_assign_csr
// ------------------------------------------------------------------------
// Per-row inputs of the bound tests: previous assignment, l(i), u(i) and the
// row's norm deviation (loaded one row ahead in the one-row-per-wave layout).
struct RowIn {
  int prev;
  float l, u, eta;
  int run;  // chunked walks after the first chunk: the row is walked this step
  uint64_t surv0, surv1;  // chunked Yin-Yang walks: the groups left to walk
};

// Hamerly mode prologue (Sections 5.3 / 5.4): Eq. (6) for l(i), the guarded
// Eq. (7) with p'(a) = min_{j != a} p(j) (or Eq. (9)) for u(i), the tests
// l >= u and l >= s(a), and the tightening of l(i).  Returns true when the
// row needs no similarity walk; the bounds are then already stored.
template <int G>
__device__ __forceinline__ bool hamerly_prologue(const AssignArgs& A, int64_t row, const RowIn& ri,
                                                 int64_t beg, int64_t end, int gl, bool leader,
                                                 int tighten, unsigned long long& tight,
                                                 unsigned long long& saved) {
  const int prev = ri.prev;
  const int m = (int)(end - beg);
  const double eta = (double)ri.eta;
  const double slack = 1.01 * (eta + A.delta_c);
  const double rho32 = (double)(m + 3) * kU32 * (1.0 + eta) * 1.01 + slack + 1e-12;
  // prune margin: keeps the FP64 re-decision of every pruned pair on the
  // side the bounds prove
  const double mu = 4.0 * (double)(m + 2) * kU64 * (1.0 + eta) + 4.0 * A.delta_c + 1e-15;
  const MoveMin mm = *A.mm;
  double ld = lower_upd((double)ri.l, A.pc[prev], A.ps[prev]) - 4e-15;
  const double pcx = (prev == mm.idx1) ? mm.pc2 : mm.pc1;
  const double psx = (prev == mm.idx1) ? mm.ps2 : mm.ps1;
  const double u0 = fmin(1.0, fmax(-1.0, (double)ri.u));
  double ud;
  if (A.bound_form == 1 && u0 >= 0.0 && pcx >= 0.0)
    ud = u0 + sqrt((1.0 - u0) * (1.0 + u0)) * psx;  // Eq. (9)
  else
    ud = upper_upd(u0, pcx, psx);
  ud = fmin(1.0, ud + 4e-15);
  const double smax = A.simplified ? 2.0 : A.gmax[prev];
  auto pruned = [&](double lcur) -> bool {
    if (lcur - ud >= mu) return true;
    const double M = lcur - mu;
    return !A.simplified && lcur > 0.0 && M > 0.0 && smax <= cc_threshold(lcur, M) - 4e-15;
  };
  bool skip = pruned(ld);
  if (!skip && tighten) {
    const float s32 = group_col_dot32<G>(A.ci, A.v, beg, end, A.CT, A.kp, prev, gl);
    ld = fmax(ld, (double)s32 - rho32);
    if (leader) tight += 1;
    skip = pruned(ld);
    if (skip && leader) saved += 1;
  }
  if (skip && leader) {
    A.l[row] = __double2float_rd(fmax(ld, -1.0));
    A.u[row] = __double2float_ru(ud);
  }
  return skip;
}

// Yin-Yang prologue (Section 5.5 with the bounds of Section 4): Eq. (6) for
// l(i), the guarded Eq. (7) for every group bound u(i, f) with the group's
// largest movement, and the global filter l(i) >= max_f u(i, f), first
// as is, then with l(i) tightened.  Lanes share the groups.  Returns true
// when the row needs no walk; the bounds are then stored.  PARTIAL (one row
// per wave): when the row is walked, the group filter u(i, f) <= l(i) marks
// the groups that cannot hold a better centre; their updated bounds are
// stored here, they are left out of the walk, and surv0/surv1 (bit f) get
// the groups that must be walked.
template <int G, bool PARTIAL>
__device__ __forceinline__ bool yinyang_prologue(const AssignArgs& A, int64_t row, const RowIn& ri,
                                                 int64_t beg, int64_t end, int gl, bool leader,
                                                 int tighten, unsigned long long& tight,
                                                 unsigned long long& saved, uint64_t& surv0,
                                                 uint64_t& surv1) {
  const int prev = ri.prev;
  const int m = (int)(end - beg);
  const double eta = (double)ri.eta;
  const double slack = 1.01 * (eta + A.delta_c);
  const double rho32 = (double)(m + 3) * kU32 * (1.0 + eta) * 1.01 + slack + 1e-12;
  const double mu = 4.0 * (double)(m + 2) * kU64 * (1.0 + eta) + 4.0 * A.delta_c + 1e-15;
  double ld = lower_upd((double)ri.l, A.pc[prev], A.ps[prev]) - 4e-15;
  float* uyr = A.uy + (size_t)row * A.ng;
  double umax = -INFINITY;
  for (int f = gl; f < A.ng; f += G) {
    const double uf = fmin(1.0, upper_upd((double)uyr[f], A.gpc[f], A.gps[f]) + 4e-15);
    umax = fmax(umax, uf);
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) umax = fmax(umax, __shfl_xor(umax, off, G));
  bool skip = ld - umax >= mu;
  if (!skip && tighten) {
    const float s32 = group_col_dot32<G>(A.ci, A.v, beg, end, A.CT, A.kp, prev, gl);
    ld = fmax(ld, (double)s32 - rho32);
    if (leader) tight += 1;
    skip = ld - umax >= mu;
    if (skip && leader) saved += 1;
  }
  if (skip) {
    if (leader) A.l[row] = __double2float_rd(fmax(ld, -1.0));
    for (int f = gl; f < A.ng; f += G)
      uyr[f] = __double2float_ru(fmin(1.0, upper_upd((double)uyr[f], A.gpc[f], A.gps[f]) + 4e-15));
  } else if constexpr (PARTIAL) {
    uint64_t m0 = 0ull, m1 = 0ull;
    for (int i = 0; G * i < A.ng; ++i) {  // wave-uniform trip count
      const int f = gl + G * i;
      bool alive = false;
      if (f < A.ng) {
        const double uf = fmin(1.0, upper_upd((double)uyr[f], A.gpc[f], A.gps[f]) + 4e-15);
        // the assigned centre's group is always walked (its exact similarity
        // gives the new l(i))
        alive = !(ld - uf >= mu) || f == prev / kYYGroup;
        if (!alive) uyr[f] = __double2float_ru(uf);
      }
      uint64_t bits = __ballot(alive);
      if constexpr (G < 64) bits &= (1ull << G) - 1ull;  // sub-wave 0 holds groups f = gl + G i
      const int sh = G * i;
      if (sh < 64) m0 |= bits << sh;
      else m1 |= bits << (sh - 64);
    }
    surv0 = m0;
    surv1 = m1;
  }
  return skip;
}

// Elkan prologue (Sections 5.1 and 5.2): Eq. (6) for l(i), the guarded
// Eq. (7) for every pair bound u(i, j), the point test s(a) <= l(i) and the
// pair tests u(i, j) <= l(i), cc(a, j) <= l(i) (the latter two dropped by the
// simplified variant), first as is, then with l(i) tightened.  A row
// without a surviving pair keeps its updated bounds and is not walked; a
// walked row gets every similarity and hence every pair bound exactly.
// The lanes hold the pair bounds in the walk's layout.  Returns true when
// the row needs no walk.
template <int G, int R, int VEC>
__device__ __forceinline__ bool elkan_prologue(const AssignArgs& A, int64_t row, const RowIn& ri,
                                               int64_t beg, int64_t end, int gl, bool leader,
                                               int tighten, bool writer, unsigned long long& tight,
                                               unsigned long long& saved) {
  constexpr int NACC = R * VEC / 4;
  const int k = A.k;
  const int prev = ri.prev;
  const int m = (int)(end - beg);
  const double eta = (double)ri.eta;
  const double slack = 1.01 * (eta + A.delta_c);
  const double rho32 = (double)(m + 3) * kU32 * (1.0 + eta) * 1.01 + slack + 1e-12;
  const double mu = 4.0 * (double)(m + 2) * kU64 * (1.0 + eta) + 4.0 * A.delta_c + 1e-15;
  double ld = lower_upd((double)ri.l, A.pc[prev], A.ps[prev]) - 4e-15;
  float4* uer4 = reinterpret_cast<float4*>(A.ue + (size_t)row * A.kp);
  float4 uv[NACC];
#pragma unroll
  for (int q4 = 0; q4 < NACC; ++q4) {
    const int r = (4 * q4) / VEC, q0 = (4 * q4) % VEC;
    const int jb = VEC * (gl + G * r) + q0;
    uv[q4] = uer4[jb / 4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = jb + q;
      if (j < k) {
        const double nu = upper_upd((double)f4get(uv[q4], q), A.pc[j], A.ps[j]) + 4e-15;
        f4set(uv[q4], q, __double2float_ru(fmin(nu, 1.0)));
      }
    }
  }
  const double* Grow = A.Gm ? A.Gm + (size_t)prev * k : nullptr;
  // cmask: bit r set when chunk r of this lane holds a centre that survives
  unsigned cmask = 0u;
  auto any_alive = [&](double lcur) -> bool {
    cmask = 0u;
    const double M = lcur - mu;
    const bool cc_ok = !A.simplified && Grow != nullptr && lcur > 0.0 && M > 0.0;
    const double T = cc_ok ? cc_threshold(lcur, M) - 4e-15 : -3.0;
    if (cc_ok && A.gmax[prev] <= T) return false;  // point test: no other centre can win
#pragma unroll
    for (int q4 = 0; q4 < NACC; ++q4) {
      const int r = (4 * q4) / VEC, q0 = (4 * q4) % VEC;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = VEC * (gl + G * r) + q0 + q;
        if (j < k && j != prev) {
          const bool by_u = (lcur - (double)f4get(uv[q4], q)) >= mu;  // u(i, j) <= l(i)
          const bool by_cc = cc_ok && (Grow[j] + A.delta_g <= T);     // cc(a, j) <= l(i)
          cmask |= (!by_u && !by_cc) ? (1u << r) : 0u;
        }
      }
    }
    return group_or<G>(cmask) != 0u;
  };
  bool alive = any_alive(ld);
  if (alive && tighten) {
    const float s32 = group_col_dot32<G>(A.ci, A.v, beg, end, A.CT, A.kp, prev, gl);
    ld = fmax(ld, (double)s32 - rho32);
    if (leader) tight += 1;
    alive = any_alive(ld);
    if (!alive && leader) saved += 1;
  }
  if (!alive) {
    if (leader) A.l[row] = __double2float_rd(fmax(ld, -1.0));
    if (writer) {
#pragma unroll
      for (int q4 = 0; q4 < NACC; ++q4) {
        const int r = (4 * q4) / VEC, q0 = (4 * q4) % VEC;
        uer4[(VEC * (gl + G * r) + q0) / 4] = uv[q4];
      }
    }
  }
  return !alive;
}

// Elkan prologue of a chunked walk (first launch of a step, one row per
// wave): the same tests as elkan_prologue over all kp / (64 VEC) slices of
// the row's pair bounds.  Every pair bound is updated with its centre's
// movement (guarded Eq. (7)) and stored; a walked row then gets exact bounds
// for the centres it walks.  The survivors go to A.umask (bit q of word t:
// unit 64 t + q, i.e. centres 64 VEC t + VEC q ... + VEC - 1, holds a centre
// whose tests failed; the assigned centre's unit is always set); word 0 is
// also returned in w0.  Returns true when the row needs no walk (l(i)
// stored).
template <int VEC>
__device__ __forceinline__ bool elkan_chunk_prologue(const AssignArgs& A, int64_t row,
                                                     const RowIn& ri, int64_t beg, int64_t end,
                                                     int gl, bool leader, int tighten,
                                                     unsigned long long& tight,
                                                     unsigned long long& saved, uint64_t& w0) {
  constexpr int SL = 64 * VEC;  // centres per slice (one launch of the walk)
  const int k = A.k;
  const int prev = ri.prev;
  const int m = (int)(end - beg);
  const double eta = (double)ri.eta;
  const double slack = 1.01 * (eta + A.delta_c);
  const double rho32 = (double)(m + 3) * kU32 * (1.0 + eta) * 1.01 + slack + 1e-12;
  const double mu = 4.0 * (double)(m + 2) * kU64 * (1.0 + eta) + 4.0 * A.delta_c + 1e-15;
  double ld = lower_upd((double)ri.l, A.pc[prev], A.ps[prev]) - 4e-15;
  float4* uer4 = reinterpret_cast<float4*>(A.ue + (size_t)row * A.kp);
  const int nw = A.kp / SL;
  uint64_t* um = A.umask + (size_t)row * nw;
  // every pair bound updated with its centre's movement, kept in place
  for (int t = 0; t < nw; ++t) {
#pragma unroll
    for (int h = 0; h < VEC / 4; ++h) {
      const int jb = SL * t + VEC * gl + 4 * h;
      float4 uv = uer4[jb / 4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jb + q;
        if (j < k) {
          const double nu = upper_upd((double)f4get(uv, q), A.pc[j], A.ps[j]) + 4e-15;
          f4set(uv, q, __double2float_ru(fmin(nu, 1.0)));
        }
      }
      uer4[jb / 4] = uv;
    }
  }
  const double* Grow = A.Gm ? A.Gm + (size_t)prev * k : nullptr;
  // the point test, then the pair tests of every unit (bounds read back
  // from where this lane stored them); the leader stores the words
  auto tests = [&](double lcur) -> bool {
    const double M = lcur - mu;
    const bool cc_ok = !A.simplified && Grow != nullptr && lcur > 0.0 && M > 0.0;
    const double T = cc_ok ? cc_threshold(lcur, M) - 4e-15 : -3.0;
    if (cc_ok && A.gmax[prev] <= T) return false;  // no other centre can win
    bool any = false;
    for (int t = 0; t < nw; ++t) {
      bool alive = false;
#pragma unroll
      for (int h = 0; h < VEC / 4; ++h) {
        const int jb = SL * t + VEC * gl + 4 * h;
        const float4 uv = uer4[jb / 4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = jb + q;
          if (j < k && j != prev) {
            const bool by_u = (lcur - (double)f4get(uv, q)) >= mu;  // u(i, j) <= l(i)
            const bool by_cc = cc_ok && (Grow[j] + A.delta_g <= T);  // cc(a, j) <= l(i)
            alive = alive || (!by_u && !by_cc);
          }
        }
      }
      uint64_t w = __ballot(alive);
      any = any || w != 0ull;
      if (t == prev / SL) w |= 1ull << ((prev % SL) / VEC);
      if (t == 0) w0 = w;
      if (leader) um[t] = w;
    }
    return any;
  };
  bool alive = tests(ld);
  if (alive && tighten) {
    const float s32 = group_col_dot32<64>(A.ci, A.v, beg, end, A.CT, A.kp, prev, gl);
    ld = fmax(ld, (double)s32 - rho32);
    if (leader) tight += 1;
    alive = tests(ld);
    if (!alive && leader) saved += 1;
  }
  if (!alive && leader) A.l[row] = __double2float_rd(fmax(ld, -1.0));
  return !alive;
}

// After a walk: every walked Yin-Yang group's bound becomes the largest
// computed similarity of the group's centres other than `abest` (plus the
// error band, rounded up); -1 for a group with no other centre.  A group of
// kYYGroup centres is kYYGroup / VEC consecutive lanes of one chunk; need
// has bit r set when chunk r was walked.  The lanes hold centres cbase ...
// cbase + kc - 1 (a chunked walk's slice; cbase a multiple of kYYGroup).
template <int G, int R, int VEC>
__device__ __forceinline__ void write_group_bounds(const AssignArgs& A, int64_t row,
                                                   const float4 (&acc)[R * VEC / 4], int gl,
                                                   int abest, double rho32, bool writer,
                                                   unsigned need, int cbase = 0, int kc = -1) {
  constexpr int SEG = (kYYGroup / VEC < G) ? kYYGroup / VEC : G;  // lanes per group
  if (kc < 0) kc = A.k;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    float m = -INFINITY;
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      const int j = VEC * (gl + G * r) + q;
      if (j < kc && cbase + j != abest) m = fmaxf(m, f4get(acc[(r * VEC + q) >> 2], q & 3));
    }
#pragma unroll
    for (int off = SEG / 2; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, SEG));
    const int j0 = VEC * (gl + G * r);
    if (writer && (gl % SEG) == 0 && j0 < kc && ((need >> r) & 1u)) {
      const int f = (cbase + j0) / kYYGroup;
      const float val = (m == -INFINITY) ? -1.0f
                                         : __double2float_ru(fmin((double)m + rho32, 1.0));
      A.uy[(size_t)row * A.ng + f] = val;
    }
  }
}

// FP64 re-decision among a group's candidates: lane gl's candidates are the
// set bits of cm (bit VEC r + q = centre VEC (gl + G r) + q).  Candidates are
// taken one at a time, lowest lane and bit first, and the whole group
// computes each one's canonical FP64 similarity; every lane returns the same
// winner under the tie order.  Rows of at most 8 stored entries (where whole
// sets of centres tie exactly: those holding none of the row's terms) let
// every lane evaluate its own candidates with the one-lane form of the same
// value, and the group keeps the best under the tie order.
template <int G, int VEC>
__device__ __forceinline__ void group_redecide(unsigned long long cm, const int32_t* ci,
                                               const float* v, int64_t beg, int64_t end,
                                               const double* C64, int64_t d, int gl, int prev,
                                               double& cb, int& cj, int j0 = 0) {
  cb = -INFINITY;
  cj = INT_MAX;
  if (end - beg <= 8) {
    for (unsigned long long c = cm; c != 0ull; c &= c - 1ull) {
      const int bit = __builtin_ctzll(c);
      const int j = j0 + VEC * (gl + G * (bit / VEC)) + bit % VEC;
      const double sv = dot64_short(ci, v, beg, end, C64 + (size_t)j * d);
      if (better64(sv, j, cb, cj, prev)) {
        cb = sv;
        cj = j;
      }
    }
    group_best64<G>(cb, cj, prev);
    return;
  }
  const int base = (int)(threadIdx.x & 63) - gl;  // first lane of the group
  for (;;) {
    const unsigned long long wave = __ballot(cm != 0ull);
    unsigned long long mine = wave;
    if constexpr (G < 64) mine = (wave >> base) & ((1ull << G) - 1ull);
    if (!mine) break;
    const int src = __builtin_ctzll(mine);
    const int lo = __shfl((int)(unsigned)cm, src, G);
    const int hi = __shfl((int)(unsigned)(cm >> 32), src, G);
    const unsigned long long sm = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    const int bit = __builtin_ctzll(sm);
    if (gl == src) cm &= cm - 1ull;
    const int j = j0 + VEC * (src + G * (bit / VEC)) + bit % VEC;
    const double sv = dot64_group<G>(ci, v, beg, end, C64 + (size_t)j * d, gl);
    if (better64(sv, j, cb, cj, prev)) {
      cb = sv;
      cj = j;
    }
  }
}

// Bound on |fl32 sim - <x, c>| when the centre copy is FP16: every centre
// value is rounded twice (FP64 -> FP32 -> FP16), relative error at most
// 2^-11 + 2^-23 in the normal range and absolute 2^-25 (times 1.01) below
// it; the FP32 FMA chain adds (m+1) 2^-24 of the sum of |x_t c_t|.  With
// non-negative rows and centres that sum is the similarity itself, so the
// bound is relative to the computed best value b (solved for the true
// value); otherwise it is taken at |x| |c|.
__device__ __forceinline__ double fp16_eps(double b, int m, double nx, double delta_c,
                                           bool nonneg) {
  const double chain = (double)(m + 1) * kU32 * 1.01;
  const double B = (0x1p-11 + 0x1p-23) * (1.0 + chain) + chain;
  const double A = 0x1p-25 * 1.01 * sqrt((double)m) * nx * (1.0 + chain);
  if (nonneg) {
    const double s = (fmax(b, 0.0) + A) / (1.0 - B);
    return (B * s + A) * 1.01 + 1e-30;
  }
  return (B * nx * (1.0 + delta_c) * 1.01 + A) * 1.01 + 1e-30;
}

// G lanes share the centres of a row: lane gl owns chunks gl + G r (r < R)
// of VEC centres.  WAVE_ROW: one row per wave, walked by row_walk (VEC = 4
// reads the FP32 centre copy, VEC = 8 the FP16 one); otherwise several rows
// per wave (G <= 16, FP32), walked by row_sims.
// One row per wave with one chunk per lane (k <= 256 FP32, k <= 512 FP16):
// the walk is latency-bound, so at least three waves per SIMD are kept.
template <int R, bool WAVE_ROW>
constexpr int assign_min_waves() {
  return (WAVE_ROW && R == 1) ? 3 : 1;
}

// Rows row_base + (row group of this thread), then every rstride rows, below
// row_end; per-step counts go to counter slot `slot`.
template <int G, int R, int VEC, int MODE, bool WAVE_ROW, bool CHUNK = false>
__device__ __forceinline__ void assign_rows(const AssignArgs& A, int64_t row_base,
                                            int64_t row_end, int64_t rstride, int slot) {
  static_assert(!CHUNK || (WAVE_ROW && G == 64 && R == 1 &&
                           (VEC == 4 || MODE == kModeYinYang || MODE == kModeElkan) &&
                           (MODE == kModeFit || MODE == kModeHamerly || MODE == kModeYinYang ||
                            MODE == kModeElkan || MODE == kModeFitElkanInit)),
                "chunked walks: one chunk of 64 x VEC centres per lane row (FP16: Yin-Yang)");
  // chunked Yin-Yang: the first chunk's prologue leaves a set of groups to
  // walk (kept in the row's running record); every chunk walks its own
  constexpr bool kChunkYY = CHUNK && MODE == kModeYinYang;
  // chunked walks that may carry Yin-Yang group bounds (the Yin-Yang step
  // and the fit's plain walk)
  constexpr bool kChunkGroups = CHUNK && (MODE == kModeYinYang || MODE == kModeFit);
  // chunked Elkan: the first launch's prologue stores which 4-centre units
  // of each 256-centre slice hold a surviving centre; every launch packs its
  // slice's surviving units onto the first lanes of a sub-wave
  constexpr bool kChunkEl = CHUNK && MODE == kModeElkan;
  // chunked walks that store exact Elkan pair bounds for what they walk
  constexpr bool kChunkPairs = CHUNK && (MODE == kModeElkan || MODE == kModeFitElkanInit);
  constexpr bool kPacked = kChunkYY || kChunkEl;
  static_assert(VEC == 4 || (VEC == 8 && WAVE_ROW), "FP16 centres need the wave layout");
  constexpr int NACC = R * VEC / 4;
  const int gl = threadIdx.x & (G - 1);
  const int gib = WAVE_ROW ? (int)(threadIdx.x >> 6) : (int)(threadIdx.x / G);
  // the lane that writes per-row results and counts (one row per wave: every
  // sub-wave holds the same values; lane 0 writes)
  const bool leader = WAVE_ROW ? (threadIdx.x & 63) == 0 : gl == 0;
  const bool lead_sub = WAVE_ROW ? (int)(threadIdx.x & 63) < G : true;
  // a fit that has stopped leaves the steps queued after it without work;
  // of the two kernels queued for a step with or without bound tests only
  // the one that matches runs
  if (A.ctl) {
    const StepCtl* c = A.ctl;
    if (c->stop || (A.gate == 1 && !c->tests) || (A.gate == 2 && c->tests)) return;
  }
  const int tighten = A.ctl ? A.ctl->tighten : A.try_tighten;
  __shared__ unsigned long long sh[7];
  if (threadIdx.x < 7) sh[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long my_rows = 0, my_rechecks = 0, my_nnz = 0, my_changed = 0, my_tight = 0,
                     my_saved = 0, my_sims = 0;
  const float4* CT4 = reinterpret_cast<const float4*>(A.CT);
  const int kp4 = A.kp >> 2;
  // a chunked launch walks centres j0 ... j0 + k - 1 (k counts them)
  const int j0 = CHUNK ? A.j0 : 0;
  const int k = CHUNK ? min(A.k - j0, R * G * VEC) : A.k;

  // one row per wave: the bounds and the first 64 entries of the wave's next
  // row are loaded while the current row is processed, so a row's walk
  // starts without waiting for them
  const int wl = threadIdx.x & 63;
  constexpr bool kBounded = MODE == kModeHamerly || MODE == kModeYinYang || MODE == kModeElkan;
  // row pointers of the next row as loaded (made wave-uniform only when
  // needed, so that nothing waits for them at the top of a row)
  int64_t nbr = 0, ner = 0;
  int64_t nbeg = 0, nend = 0;
  int wc = 0;
  float wx = 0.f;
  auto uniform64 = [](int64_t x) -> int64_t {
    return ((int64_t)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
  };
  auto next_window = [&]() {
    nbeg = uniform64(nbr);
    nend = uniform64(ner);
    wc = 0;
    wx = 0.f;
    if (nbeg + wl < nend) {
      wc = A.ci[nbeg + wl];
      wx = A.v[nbeg + wl];
    }
  };
  auto load_in = [&](int64_t r) -> RowIn {
    RowIn x{-1, 0.f, 0.f, 0.f, 1, ~0ull, ~0ull};
    if (A.read_prev) x.prev = A.a[r];
    if constexpr (kBounded) x.l = A.l[r];
    if constexpr (MODE == kModeHamerly) x.u = A.u[r];
    if constexpr (MODE != kModeAssign) x.eta = A.eta[r];
    if constexpr (CHUNK) x.run = j0 > 0 ? (A.rs[r].flags & 1) : 1;
    if constexpr (kChunkYY)
      if (j0 > 0) {
        x.surv0 = A.rs[r].surv0;
        x.surv1 = A.rs[r].surv1;
      }
    return x;
  };
  RowIn nin{-1, 0.f, 0.f, 0.f, 1, ~0ull, ~0ull};
  if constexpr (WAVE_ROW) {
    const int64_t r0 = row_base + gib;
    if (r0 < row_end) {
      nbr = A.rp[r0];
      ner = A.rp[r0 + 1];
      nin = load_in(r0);
      next_window();
    }
  }

  for (int64_t row = row_base + gib; row < row_end; row += rstride) {
    int64_t beg, end;
    int c0 = 0;
    float x0 = 0.f;
    RowIn ri;
    if constexpr (WAVE_ROW) {
      beg = nbeg;
      end = nend;
      c0 = wc;
      x0 = wx;
      ri = nin;
      nbr = ner = 0;
      if (row + rstride < row_end) {
        nbr = A.rp[row + rstride];
        ner = A.rp[row + rstride + 1];
        nin = load_in(row + rstride);
      }
    } else {
      beg = A.rp[row];
      end = A.rp[row + 1];
      ri = load_in(row);
    }
    const int m = (int)(end - beg);
    const int prev = ri.prev;
    // lanes whose centres the walk computes (bit r: chunk r of the lane);
    // only the packed chunked walks leave lanes out
    unsigned need = ~0u;
    if constexpr (CHUNK) {
      // later chunks walk only the rows the first chunk's tests left
      if (j0 > 0 && !ri.run) {
        next_window();
        continue;
      }
    }
    // groups (bit f) a Yin-Yang walk visits this step
    uint64_t surv0 = ri.surv0, surv1 = ri.surv1;
    // chunked Elkan: surviving units of the first slice (first launch)
    uint64_t ew0 = 0ull;
    if constexpr (kBounded) if (!CHUNK || j0 == 0) {
      bool skip;
      if constexpr (MODE == kModeHamerly)
        skip = hamerly_prologue<G>(A, row, ri, beg, end, gl, leader, tighten, my_tight,
                                   my_saved);
      else if constexpr (MODE == kModeYinYang)
        skip = yinyang_prologue<G, kChunkYY>(A, row, ri, beg, end, gl, leader, tighten,
                                             my_tight, my_saved, surv0, surv1);
      else if constexpr (kChunkEl)
        skip = elkan_chunk_prologue<VEC>(A, row, ri, beg, end, gl, leader, tighten, my_tight,
                                         my_saved, ew0);
      else
        skip = elkan_prologue<G, R, VEC>(A, row, ri, beg, end, gl, leader, tighten, lead_sub,
                                         my_tight, my_saved);
      if (skip) {
        if constexpr (CHUNK) {
          if (leader) A.rs[row].flags = 0;  // pruned: the later chunks skip the row
        }
        if constexpr (WAVE_ROW) next_window();
        continue;
      }
    }
    // Chunked Yin-Yang: the chunk's groups that the filters left (the
    // assigned centre's group among them), na of its 64 / GL, packed onto
    // the lanes: the GL lanes of packed segment t (a group is GL 16-byte
    // units of a centre row: 8 with the FP32 copy, 4 with FP16) read the
    // t-th surviving group, and a sub-wave of L = GL na lanes (rounded up to
    // 8, 16, 32 or 64) walks the row, so one gather instruction serves
    // 64 / L entries.  Lane wl holds centres VEC cw_col ... VEC cw_col +
    // VEC - 1 of the chunk when live (need = 1: wl < L and its segment < na).
    constexpr int GL = kYYGroup / VEC;
    int cw_L = 64, cw_col = 0;
    unsigned cw_walk = 1u;  // the lane fetches (every sub-wave)
    if constexpr (kChunkYY) {
      const int gb = j0 / kYYGroup;  // a multiple of 64 / GL: one mask word holds the chunk
      const int ngc = (k + kYYGroup - 1) / kYYGroup;
      const uint64_t sv = gb < 64 ? (surv0 >> gb) : (surv1 >> (gb - 64));
      const unsigned am = (unsigned)(sv & ((1ull << ngc) - 1ull));
      const int na = __popc(am);
      const int lanes = GL * na;
      cw_L = lanes <= 8 ? 8 : lanes <= 16 ? 16 : lanes <= 32 ? 32 : 64;
      const int seg = (wl % cw_L) / GL;
      unsigned rest = am;
      for (int i = 0; i < seg && rest != 0u; ++i) rest &= rest - 1u;
      const int grp = rest != 0u ? __builtin_ctz(rest) : 0;
      cw_col = grp * GL + (wl % GL);
      cw_walk = seg < na ? 1u : 0u;
      need = (seg < na && wl < cw_L) ? 1u : 0u;
    }
    if constexpr (kChunkEl) {
      // the slice's surviving 4-centre units (ns of 64) onto lanes 0 ... ns-1
      // in unit order: lane wl's unit goes to slot (units set below it) when
      // set, else to ns + (units clear below it) -- a permutation of the
      // lanes; a sub-wave of L = 8, 16, 32 or 64 lanes walks them
      const uint64_t w =
          j0 == 0 ? ew0 : A.umask[(size_t)row * (A.kp / (64 * VEC)) + j0 / (64 * VEC)];
      const int ns = __popcll(w);
      cw_L = ns <= 8 ? 8 : ns <= 16 ? 16 : ns <= 32 ? 32 : 64;
      const bool mine = ((w >> wl) & 1ull) != 0ull;
      const int below = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(w >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)w, 0u));
      const int slot = mine ? below : ns + (wl - below);
      const int unit = __builtin_amdgcn_ds_permute(slot * 4, wl);
      const int pos = wl % cw_L;
      cw_col = __shfl(unit, pos, 64) & 63;
      cw_walk = pos < ns ? 1u : 0u;
      need = wl < ns ? 1u : 0u;
    }

    float4 acc[NACC];
    float nrm2 = 0.f;
    // false: no group of this chunk is walked (chunked Yin-Yang); the row's
    // running result is carried on unchanged
    bool walked = true;
    if constexpr (kPacked) walked = group_or<G>(need) != 0u;
    if constexpr (WAVE_ROW) {
      const char* ctb = VEC == 8 ? static_cast<const char*>(A.CT16)
                                 : reinterpret_cast<const char*>(A.CT);
      if constexpr (CHUNK) ctb += (size_t)j0 * (VEC == 8 ? 2 : 4);
      if (!walked) {
      } else if constexpr (kPacked) {
        if (cw_L == 8)
          nrm2 = row_walk<8, 1, VEC, true>(A.ci, A.v, beg, end, c0, x0, ctb, A.kp, wl, acc,
                                         cw_walk, cw_col);
        else if (cw_L == 16)
          nrm2 = row_walk<16, 1, VEC, true>(A.ci, A.v, beg, end, c0, x0, ctb, A.kp, wl, acc,
                                          cw_walk, cw_col);
        else if (cw_L == 32)
          nrm2 = row_walk<32, 1, VEC, true>(A.ci, A.v, beg, end, c0, x0, ctb, A.kp, wl, acc,
                                          cw_walk, cw_col);
        else
          nrm2 = row_walk<64, 1, VEC, true>(A.ci, A.v, beg, end, c0, x0, ctb, A.kp, wl, acc,
                                          cw_walk, cw_col);
      } else {
        nrm2 = row_walk<G, R, VEC>(A.ci, A.v, beg, end, c0, x0, ctb, A.kp, wl, acc);
      }
      if (!walked) {
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      next_window();
    } else {
      nrm2 = row_sims<G, R, false>(A.ci, A.v, beg, end, CT4, kp4, gl, ~0u, acc);
    }
    // similarities computed for this row (wave-uniform)
    unsigned long long row_sims_done = (unsigned long long)k;
    if constexpr (kPacked) {
      const int left = k - VEC * cw_col;
      const int mine = need ? (left < VEC ? (left > 0 ? left : 0) : VEC) : 0;
      row_sims_done = (unsigned long long)group_sum<G>(mine);
    }

    float b = -INFINITY, s2 = -INFINITY;
    int bj = INT_MAX;
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const int j = VEC * (kPacked ? cw_col : gl + G * r) + q;
        if (j < k && ((need >> r) & 1u)) {
          const float sv = f4get(acc[(r * VEC + q) >> 2], q & 3);
          if (better32(sv, j0 + j, b, bj, prev)) {
            s2 = fmaxf(s2, b);
            b = sv;
            bj = j0 + j;
          } else {
            s2 = fmaxf(s2, sv);
          }
        }
      }
    }
    group_top2<G>(b, bj, s2, prev);

    // rigorous bound on |fl32 sim - <x, c>| for any summation order: (m+1)
    // roundings of the FMA chain plus the rounding of the centre copy,
    // scaled by |x| |c| (|x| <= 1 + eta where the walk measured no norm)
    const double nx = walked ? sqrt((double)nrm2) * 1.01 + 1e-30
                             : (1.0 + (double)ri.eta) * 1.01 + 1e-30;
    const double eps = VEC == 8 ? fp16_eps((double)b, m, nx, A.delta_c, *A.negflag == 0)
                                : (double)(m + 3) * kU32 * nx;

    bool rechecked = false;
    double best64 = 0.0;
    int abest = bj;
    // (chunked walks defer this decision: see the merge below)
    if (!CHUNK && k > 1 && (double)b - (double)s2 <= 2.0 * eps) {
      // 1e-12 below the band: the FP64 winner is a candidate whichever FP32
      // summation order produced b
      const double thr = (double)b - 2.0 * eps - 1e-12;
      unsigned long long cm = 0ull;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          const int j = VEC * (gl + G * r) + q;
          if (j < k && ((need >> r) & 1u) &&
              (double)f4get(acc[(r * VEC + q) >> 2], q & 3) >= thr)
            cm |= 1ull << (VEC * r + q);
        }
      double cb;
      int cj;
      group_redecide<G, VEC>(cm, A.ci, A.v, beg, end, A.C64, A.d, gl, prev, cb, cj, j0);
      abest = cj;
      best64 = cb;
      rechecked = true;
    }

    if constexpr (CHUNK) {
      // Merge this chunk into the row's running result.  A winner is kept as
      // its FP32 value (error bound ew) until an FP64 decision is needed: a
      // chunk whose FP32 top two lie within their error bounds is marked
      // ambiguous (its FP32 winner may not be its FP64 winner) and resolved
      // only if it can still win -- if its value overlaps another winner's,
      // or if it is the winner after the last chunk -- by re-evaluating every
      // centre of that chunk in the canonical FP64 order.  Overlapping
      // winners are compared by their canonical FP64 values.  `sec` bounds
      // every other centre's similarity (FP32 values, error <= emax).
      constexpr int CW = R * G * VEC;  // centres per chunk
      auto resolve = [&](int jsel, int flags, double& v, int& j, double& sec_io) {
        if (flags & 8) {  // ambiguous chunk: its exact winner among all its centres
          const int c0 = (jsel / CW) * CW;
          const int kc = min(A.k - c0, CW);
          const int lo = VEC * gl;
          const unsigned long long cm =
              kc - lo >= VEC ? ((1ull << VEC) - 1ull)
                             : (kc - lo > 0 ? (1ull << (kc - lo)) - 1ull : 0ull);
          sec_io = fmax(sec_io, v);  // the FP32 best may be another centre's
          double cb;
          int cj;
          group_redecide<G, VEC>(cm, A.ci, A.v, beg, end, A.C64, A.d, gl, prev, cb, cj, c0);
          v = cb;
          j = cj;
        } else if (!(flags & 2)) {
          v = dot64_group<G>(A.ci, A.v, beg, end, A.C64 + (size_t)j * A.d, gl);
        }
      };
      double vw = (double)b, ew = eps, sec = (double)s2, emax = eps;
      int jw = bj;
      int fw = (k > 1 && (double)b - (double)s2 <= 2.0 * eps) ? 8 : 0;
      bool any = false;
      // this chunk's winner is the row's running winner after the merge
      bool cand_running = true;
      // Yin-Yang group bounds (the fit's plain walk too): every group bound
      // must cover each of its centres other than the final assignment.  A
      // chunk's groups leave out the chunk's winner only while it is the
      // running winner and exactly decided; a running winner that later
      // loses is added to its group's bound here.
      const double eta_r = (double)ri.eta;
      const double slack_r = 1.01 * (eta_r + A.delta_c);
      auto raise_group = [&](int j, double v, double e) {
        if (kChunkGroups && A.uy != nullptr && leader && j >= 0 && j < A.k) {
          float* p = A.uy + (size_t)row * A.ng + j / kYYGroup;
          const double hi = v + e + (double)(m + 2) * kU64 * nx + slack_r + 1e-12;
          *p = fmaxf(*p, __double2float_ru(fmin(hi, 1.0)));
        }
      };
      if (j0 > 0) {
        const RowRun rr = A.rs[row];
        double vc = rr.best, ec = rr.err;
        int jc = rr.bj, fc = rr.flags;
        any = (fc & 4) != 0;
        emax = fmax(emax, rr.errmax);
        sec = fmax(sec, rr.second);
        // A chunk that walked no centre (chunked Yin-Yang: every group of
        // the chunk filtered out) has no candidate (index INT_MAX), and the
        // running result has none until some chunk walked: an empty side
        // never takes part in a comparison.
        bool win;
        if (!walked) {
          win = false;
        } else if (jc == INT_MAX) {
          win = true;
        } else if (vw - ew > vc + ec + 1e-12) {
          win = true;
        } else if (vc - ec > vw + ew + 1e-12) {
          win = false;
        } else {
          resolve(jw, fw, vw, jw, sec);
          resolve(jc, fc, vc, jc, sec);
          fw = fc = 2;
          ew = ec = 0.0;
          any = true;
          win = better64(vw, jw, vc, jc, prev);
        }
        if (win) {
          sec = fmax(sec, vc);
          raise_group(jc, vc, ec);
        } else {
          sec = fmax(sec, vw);
          vw = vc;
          ew = ec;
          jw = jc;
          fw = fc;
          cand_running = false;
        }
      }
      if (A.chunk_last && (fw & 8)) {
        resolve(jw, fw, vw, jw, sec);
        fw = 2;
        ew = 0.0;
        any = true;
      }
      if constexpr (kChunkPairs) {
        // exact pair bounds of the centres this launch walked (padding: 1)
        if (walked && need) {
          const int jl = VEC * (kChunkEl ? cw_col : gl);
          const double rb = eps + slack_r + 1e-12;
#pragma unroll
          for (int h = 0; h < VEC / 4; ++h) {
            float4 o;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int j = jl + 4 * h + q;
              f4set(o, q,
                    j < k ? __double2float_ru(fmin((double)f4get(acc[h], q) + rb, 1.0)) : 1.0f);
            }
            reinterpret_cast<float4*>(A.ue + (size_t)row * A.kp + j0)[jl / 4 + h] = o;
          }
        }
      }
      if (kChunkGroups && A.uy != nullptr && walked) {
        const int excl = (cand_running && !(fw & 8)) ? jw : -1;
        const double rb = eps + slack_r + 1e-12;
        if constexpr (kChunkYY) {
          // packed lanes: segment-aligned groups of GL lanes
          float mv = -INFINITY;
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            const int j = VEC * cw_col + q;
            if (need && j < k && j0 + j != excl) mv = fmaxf(mv, f4get(acc[q >> 2], q & 3));
          }
#pragma unroll
          for (int off = GL / 2; off >= 1; off >>= 1) mv = fmaxf(mv, __shfl_xor(mv, off, GL));
          if (need && (wl % GL) == 0) {
            const float val =
                (mv == -INFINITY) ? -1.0f : __double2float_ru(fmin((double)mv + rb, 1.0));
            A.uy[(size_t)row * A.ng + (j0 + VEC * cw_col) / kYYGroup] = val;
          }
        } else {
          write_group_bounds<G, R, VEC>(A, row, acc, gl, excl, rb, lead_sub, need, j0, k);
        }
      }
      if (!A.chunk_last) {
        if (leader) {
          RowRun o;
          o.best = vw;
          o.second = sec;
          o.err = ew;
          o.errmax = emax;
          o.bj = jw;
          o.flags = 1 | (fw & 10) | (any ? 4 : 0);
          o.surv0 = surv0;
          o.surv1 = surv1;
          A.rs[row] = o;
        }
      } else if (leader) {
        const bool xw = (fw & 2) != 0;
        const double eta = (double)ri.eta;
        const double slack = 1.01 * (eta + A.delta_c);
        const double rho32 = emax + slack + 1e-12;
        const double rho64 = (double)(m + 2) * kU64 * nx + slack + 1e-15;
        // jw is a centre: the chunk holding the previous assignment's group
        // is always walked (the guard only keeps the store in range)
        jw = (jw >= 0 && jw < A.k) ? jw : (prev >= 0 ? prev : 0);
        A.a[row] = jw;
        my_changed += (jw != prev) ? 1ull : 0ull;
        if (A.l) A.l[row] = __double2float_rd(fmax(xw ? vw - rho64 : vw - rho32, -1.0));
        if (A.u) {
          const double hi = (A.k == 1) ? -1.0 : sec + rho32;
          A.u[row] = __double2float_ru(fmin(hi, 1.0));
        }
        my_rows += 1;
        my_nnz += (unsigned long long)m;
        my_rechecks += any ? 1 : 0;
      }
      if (leader) my_sims += row_sims_done;
      continue;
    }

    if (MODE == kModeAssign) {
      if (leader) {
        A.a[row] = abest;
        if (A.best_out) A.best_out[row] = rechecked ? (float)best64 : b;
        if (A.second_out) A.second_out[row] = (rechecked && abest != bj) ? b : s2;
      }
    } else {
      // bounds on true cosines (Section 4): l(i) <= cos(x, c_a),
      // u(i) >= max_{j != a} cos(x, c_j)
      const double eta = (double)ri.eta;
      const double slack = 1.01 * (eta + A.delta_c);
      const double rho32 = eps + slack + 1e-12;
      if (leader) {
        const double rho64 = (double)(m + 2) * kU64 * nx + slack + 1e-15;
        A.a[row] = abest;
        my_changed += (abest != prev) ? 1ull : 0ull;
        if (A.l) {
          const double lo = rechecked ? best64 - rho64 : (double)b - rho32;
          A.l[row] = __double2float_rd(fmax(lo, -1.0));
        }
        if (A.u) {
          const double hi = (k == 1) ? -1.0 : (rechecked ? (double)b : (double)s2) + rho32;
          A.u[row] = __double2float_ru(fmin(hi, 1.0));
        }
      }
      if (A.uy) write_group_bounds<G, R, VEC>(A, row, acc, gl, abest, rho32, lead_sub, need);
      if ((MODE == kModeFitElkanInit || MODE == kModeElkan) && lead_sub) {
        float4* uer4 = reinterpret_cast<float4*>(A.ue + (size_t)row * A.kp);
#pragma unroll
        for (int q4 = 0; q4 < NACC; ++q4) {
          const int r = (4 * q4) / VEC, q0 = (4 * q4) % VEC;
          float4 o;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = VEC * (gl + G * r) + q0 + q;
            const float val =
                (j < k) ? __double2float_ru(fmin((double)f4get(acc[q4], q) + rho32, 1.0)) : 1.0f;
            f4set(o, q, val);
          }
          uer4[(VEC * (gl + G * r) + q0) / 4] = o;
        }
      }
    }
    if (leader) {
      my_rows += 1;
      my_nnz += (unsigned long long)m;
      my_rechecks += rechecked ? 1 : 0;
      my_sims += row_sims_done;
    }
  }

  if (A.cnt == nullptr) return;
  if (my_rows) atomicAdd(&sh[0], my_rows);
  if (my_nnz) atomicAdd(&sh[1], my_nnz);
  if (my_rechecks) atomicAdd(&sh[2], my_rechecks);
  if (my_changed) atomicAdd(&sh[3], my_changed);
  if (my_tight) atomicAdd(&sh[4], my_tight);
  if (my_saved) atomicAdd(&sh[5], my_saved);
  if (my_sims) atomicAdd(&sh[6], my_sims);
  __syncthreads();
  if (threadIdx.x == 0) {
    Counters* c = A.cnt + slot;
    // similarities: those of the walked rows (all k, or the walked groups)
    // plus one per tightened row
    if (sh[6] + sh[4]) atomicAdd(&c->sims, sh[6] + sh[4]);
    if (sh[0]) {
      atomicAdd(&c->rows_done, sh[0]);
      atomicAdd(&c->nnz_done, sh[1]);
    }
    if (sh[2]) atomicAdd(&c->rechecks, sh[2]);
    if (sh[3]) atomicAdd(&c->changed, sh[3]);
    if (sh[4]) atomicAdd(&c->tightened, sh[4]);
    if (sh[5]) atomicAdd(&c->tight_saved, sh[5]);
  }
}

template <int G, int R, int VEC, int MODE, bool WAVE_ROW, bool CHUNK = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    assign_min_waves<R, WAVE_ROW>()))) void k_assign_csr(AssignArgs A) {
  constexpr int GPB = WAVE_ROW ? kBlock / 64 : kBlock / G;
  assign_rows<G, R, VEC, MODE, WAVE_ROW, CHUNK>(A, (int64_t)blockIdx.x * GPB, A.n_rows,
                                                (int64_t)gridDim.x * GPB,
                                                (int)(blockIdx.x % kCounterSlots));
}

// Batched fits: a persistent grid takes (problem, first row) items from the
// atomic counter *queue and walks the item's tile of rows with the
// problem's own arguments (the same body as k_assign_csr, so each problem's
// rows get exactly its single-fit results).
template <int G, int R, int VEC, int MODE, bool WAVE_ROW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    assign_min_waves<R, WAVE_ROW>()))) void k_assign_batched(const AssignArgs* __restrict__ args,
                                                             int arg_stride, int arg_off,
                                                             const int2* __restrict__ items,
                                                             int n_items, int tile_rows,
                                                             unsigned int* __restrict__ queue) {
  constexpr int GPB = WAVE_ROW ? kBlock / 64 : kBlock / G;
  __shared__ int sh_item;
  for (;;) {
    if (threadIdx.x == 0) sh_item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int it = sh_item;
    __syncthreads();  // read by every thread before thread 0 takes the next item
    if (it >= n_items) break;
    const int2 w = items[it];
    const int p = __builtin_amdgcn_readfirstlane(w.x);
    const AssignArgs& A = args[(size_t)p * arg_stride + arg_off];
    const int64_t r0 = w.y;
    const int64_t r1 = (r0 + tile_rows < A.n_rows) ? r0 + tile_rows : A.n_rows;
    assign_rows<G, R, VEC, MODE, WAVE_ROW>(A, r0, r1, GPB, it % kCounterSlots);
  }
}

// First assignment step taken from a given assignment and its FP64 top-2
// (canonical order, e.g. cached by the k-means++ seeding): the assignment is
// copied and the bounds are those of an exhaustive step whose decision was
// taken in FP64 -- l <= cos(x, c_a), u and every Elkan u(i, j) >= the
// second-best cosine (u(i, a) >= the best), rounded outward to float.
__global__ __launch_bounds__(kBlock) void k_warm_start(
    const int64_t* __restrict__ rp, int64_t n, int32_t k, int32_t kp,
    const int32_t* __restrict__ wa, const double* __restrict__ wb,
    const double* __restrict__ ws2, const float* __restrict__ eta, double delta_c,
    int32_t* __restrict__ a, float* __restrict__ l, float* __restrict__ u,
    float* __restrict__ ue, float* __restrict__ uy, int32_t ng, int64_t dense_d) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t m = rp ? rp[i + 1] - rp[i] : dense_d;  // terms of the FP64 chain
  const double e = (double)eta[i];
  const double nx = (1.0 + e) * 1.01 + 1e-30;
  const double rho64 = (double)(m + 2) * kU64 * nx + 1.01 * (e + delta_c) + 1e-15;
  const int32_t ai = wa[i];
  a[i] = ai;
  const double lo = wb[i] - rho64;
  const double hi = (k == 1) ? -1.0 : ws2[i] + rho64;
  if (l) l[i] = __double2float_rd(fmax(lo, -1.0));
  if (u) u[i] = __double2float_ru(fmin(hi, 1.0));
  if (ue) {
    const float top = __double2float_ru(fmin(wb[i] + rho64, 1.0));
    const float other = __double2float_ru(fmin(hi, 1.0));
    float* row = ue + (size_t)i * kp;
    for (int j = 0; j < kp; ++j) row[j] = (j >= k) ? 1.0f : (j == ai ? top : other);
  }
  if (uy) {  // every centre other than a(i) is at most the second best
    const float other = __double2float_ru(fmin(hi, 1.0));
    for (int f = 0; f < ng; ++f) uy[(size_t)i * ng + f] = other;
  }
}

// Cosine and sine of every Yin-Yang group's largest movement (the member
// with the smallest movement cosine).
__global__ void k_group_move(const double* __restrict__ pc, const double* __restrict__ ps,
                             int32_t k, int32_t ng, double* __restrict__ gpc,
                             double* __restrict__ gps) {
  const int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= ng) return;
  double c = 2.0, sn = 0.0;
  for (int j = f * kYYGroup; j < k && j < (f + 1) * kYYGroup; ++j)
    if (pc[j] < c) {
      c = pc[j];
      sn = ps[j];
    }
  gpc[f] = c;
  gps[f] = sn;
}

template <int MODE>
hipError_t launch_assign_mode(const AssignArgs& A, hipStream_t s) {
  const Geometry g = pick_geometry(A.k);
  if (g.G == 0 || g.kp != A.kp) return hipErrorInvalidValue;
  const bool half = A.CT16 != nullptr && A.kp >= 128;
  // the alternative layout of the measured table (FP32 copy, k in (16, 512],
  // plain and Hamerly walks): one row per wave at k <= 64, four rows per
  // wave (groups of 16 lanes) above
  constexpr bool kLayouts = MODE == kModeFit || MODE == kModeHamerly;
  const bool alt = kLayouts && !half && A.layout == 1 && A.kp >= 32 && A.kp <= 512;
  const int gpb = alt ? (A.kp <= 64 ? kBlock / 64 : kBlock / 16)
                      : ((half || g.G >= 32) ? kBlock / 64 : kBlock / g.G);  // rows per block
  int64_t blocks = (A.n_rows + gpb - 1) / gpb;
  if (blocks > kMaxGridBlocks) blocks = kMaxGridBlocks;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(kBlock);
#define SKM_CASE(KP, GG, RR, VV, WW)                                                  \
  case KP:                                                                            \
    hipLaunchKernelGGL((k_assign_csr<GG, RR, VV, MODE, WW>), grid, block, 0, s, A); \
    break;
  if (half) {
    // FP16 centre copy, 8 centres per 16-byte chunk: 16, 32 or 64 lanes cover
    // a centre row, so 4, 2 or 1 entries per gather instruction
    switch (A.kp) {
      SKM_CASE(128, 16, 1, 8, true)
      SKM_CASE(256, 32, 1, 8, true)
      SKM_CASE(512, 64, 1, 8, true)
      SKM_CASE(1024, 64, 2, 8, true)
      SKM_CASE(2048, 64, 4, 8, true)
      SKM_CASE(4096, 64, 8, 8, true)
      default:
        return hipErrorInvalidValue;
    }
  } else {
    if constexpr (kLayouts) {
      if (alt) {
        // k <= 64: one row per wave in sub-waves of 8 / 16 lanes; above:
        // a group of 16 lanes per row, each lane k_p / 64 16-byte units
        switch (A.kp) {
          SKM_CASE(32, 8, 1, 4, true)
          SKM_CASE(64, 16, 1, 4, true)
          SKM_CASE(128, 16, 2, 4, false)
          SKM_CASE(256, 16, 4, 4, false)
          SKM_CASE(512, 16, 8, 4, false)
          default:
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
      }
    }
    // k <= 64: several rows per wave (groups of 4..16 lanes); k in (64, 128]:
    // one row per wave, half-waves on alternating entries; larger k: one row
    // per wave, R float4 chunks per lane
    switch (A.kp) {
      SKM_CASE(16, 4, 1, 4, false)
      SKM_CASE(32, 8, 1, 4, false)
      SKM_CASE(64, 16, 1, 4, false)
      SKM_CASE(128, 32, 1, 4, true)
      SKM_CASE(256, 64, 1, 4, true)
      SKM_CASE(512, 64, 2, 4, true)
      SKM_CASE(1024, 64, 4, 4, true)
      SKM_CASE(2048, 64, 8, 4, true)
      SKM_CASE(4096, 64, 16, 4, true)
      default:
        return hipErrorInvalidValue;
    }
  }
#undef SKM_CASE
  return hipGetLastError();
}

}  // namespace

hipError_t launch_warm_start(const int64_t* rp, int64_t n, int32_t k, int32_t kp,
                             const int32_t* wa, const double* wb, const double* ws2,
                             const float* eta, double delta_c, int32_t* a, float* l, float* u,
                             float* ue, float* uy, int32_t ng, hipStream_t s, int64_t dense_d) {
  const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_warm_start, dim3(blocks), dim3(kBlock), 0, s, rp, n, k, kp, wa, wb, ws2,
                     eta, delta_c, a, l, u, ue, uy, ng, dense_d);
  return hipGetLastError();
}

hipError_t launch_group_move(const double* pc, const double* ps, int32_t k, int32_t ng,
                             double* gpc, double* gps, hipStream_t s) {
  hipLaunchKernelGGL(k_group_move, dim3((unsigned)((ng + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, pc, ps, k, ng, gpc, gps);
  return hipGetLastError();
}

namespace {
template <int MODE>
hipError_t launch_assign_batched_mode(const AssignArgs* args, int arg_stride, int arg_off,
                                      const int2* items, int n_items, int tile_rows, int kp,
                                      unsigned int* queue, hipStream_t s) {
  int blocks = n_items < kMaxGridBlocks ? n_items : kMaxGridBlocks;
  if (blocks < 1) return hipSuccess;
  const dim3 grid((unsigned)blocks), block(kBlock);
#define SKM_BCASE(KP, GG, RR, WW)                                                          \
  case KP:                                                                                  \
    hipLaunchKernelGGL((k_assign_batched<GG, RR, 4, MODE, WW>), grid, block, 0, s, args,    \
                       arg_stride, arg_off, items, n_items, tile_rows, queue);              \
    break;
  switch (kp) {
    SKM_BCASE(16, 4, 1, false)
    SKM_BCASE(32, 8, 1, false)
    SKM_BCASE(64, 16, 1, false)
    SKM_BCASE(128, 32, 1, true)
    SKM_BCASE(256, 64, 1, true)
    SKM_BCASE(512, 64, 2, true)
    SKM_BCASE(1024, 64, 4, true)
    SKM_BCASE(2048, 64, 8, true)
    SKM_BCASE(4096, 64, 16, true)
    default:
      return hipErrorInvalidValue;
  }
#undef SKM_BCASE
  return hipGetLastError();
}

}  // namespace

hipError_t launch_assign_batched(const AssignArgs* args, int arg_stride, int arg_off,
                                 const int2* items, int n_items, int tile_rows, int kp,
                                 int mode, unsigned int* queue, hipStream_t s) {
  if (mode == kModeFit)
    return launch_assign_batched_mode<kModeFit>(args, arg_stride, arg_off, items, n_items,
                                                tile_rows, kp, queue, s);
  if (mode == kModeHamerly)
    return launch_assign_batched_mode<kModeHamerly>(args, arg_stride, arg_off, items, n_items,
                                                    tile_rows, kp, queue, s);
  return hipErrorInvalidValue;
}

hipError_t launch_assign_chunk(const AssignArgs& A, int mode, hipStream_t s) {
  // FP16 centre copy: Yin-Yang and Elkan steps only (chunks of 512 centres)
  if (A.CT16 != nullptr && mode != kModeYinYang && mode != kModeElkan)
    return hipErrorInvalidValue;
  // one row per wave; twice the usual persistent grid: the rows of a wave
  // vary in length, and more, shorter row sets end closer together (C3:
  // 3% faster per launch than 2048 blocks, 1024 blocks 2% slower)
  int64_t blocks = (A.n_rows + 3) / 4;
  if (blocks > 2 * kMaxGridBlocks) blocks = 2 * kMaxGridBlocks;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(kBlock);
  if (mode == kModeFit)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 4, kModeFit, true, true>), grid, block, 0, s, A);
  else if (mode == kModeHamerly)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 4, kModeHamerly, true, true>), grid, block, 0, s, A);
  else if (mode == kModeYinYang && A.CT16 != nullptr)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 8, kModeYinYang, true, true>), grid, block, 0, s, A);
  else if (mode == kModeYinYang)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 4, kModeYinYang, true, true>), grid, block, 0, s, A);
  else if (mode == kModeElkan && A.CT16 != nullptr)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 8, kModeElkan, true, true>), grid, block, 0, s, A);
  else if (mode == kModeElkan)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 4, kModeElkan, true, true>), grid, block, 0, s, A);
  else if (mode == kModeFitElkanInit)
    hipLaunchKernelGGL((k_assign_csr<64, 1, 4, kModeFitElkanInit, true, true>), grid, block, 0,
                       s, A);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_assign(const AssignArgs& A, int mode, hipStream_t s) {
  if (mode == kModeAssign) return launch_assign_mode<kModeAssign>(A, s);
  if (mode == kModeFit) return launch_assign_mode<kModeFit>(A, s);
  if (mode == kModeHamerly) return launch_assign_mode<kModeHamerly>(A, s);
  if (mode == kModeYinYang) return launch_assign_mode<kModeYinYang>(A, s);
  if (mode == kModeElkan) return launch_assign_mode<kModeElkan>(A, s);
  return launch_assign_mode<kModeFitElkanInit>(A, s);
}


}  // namespace skm
