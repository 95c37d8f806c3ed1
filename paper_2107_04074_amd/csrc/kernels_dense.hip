// Dense-row kernels for gfx950: the similarity contraction of the assignment
// step (Section 5) on MFMA matrix cores, in BF16 (FP32 accumulate) or FP32.
//
//  k_dense_prep     one pass over the rows: the bound on | |x(i)| - 1 | per
//                   row and, for BF16, the padded BF16 copy of the rows.
//  k_dense_sim      rows x centres on MFMA.  Centres are streamed through LDS
//                   in chunks shared by the block's waves (BF16: loaded into
//                   two buffers directly, one chunk ahead); every wave keeps
//                   its rows' operand fragments in registers for the whole
//                   centre loop.  Epilogue: running top-2 per row (assignment,
//                   bounds; BF16 folds a tile while the next one multiplies)
//                   or, in candidate mode, every centre within the error band
//                   of the row's best value.
//  k_dense_exact    FP64 re-decision of the rows whose best and second best
//                   lie within the rigorous error band: one canonical FP64
//                   chain per candidate against the FP64 master centre.
//  k_dense_hamerly  Eq. (6), guarded Eq. (7) / Eq. (9) and the tests of
//                   Sections 5.3 / 5.4 per row, tightening l(i) with an FP64
//                   dot product; rows that fail are flagged for recompute.
//  k_cluster_sums   S(j) recomputed from scratch per cluster (rows sorted by
//                   cluster), 64-bit fixed point as in the sparse path.
//  compaction       flags -> dense row list via per-block counts, a scan and
//                   a scatter (no contended atomics).
//
// MFMA lane layouts (checked on the device): 32x32x16 bf16 takes
// A[m = l%32][k = 8(l/32)+e] and B[k = 8(l/32)+e][n = l%32] (e < 8);
// 32x32x2 f32 takes A[l%32][l/32] and B[l/32][l%32]; both return element i of
// lane l as C[8(i/4) + 4(l/32) + i%4][l%32].  Here A holds 32 centres and B
// holds 32 rows, so every lane ends with 16 centres of one row.
#include <float.h>
#include <limits.h>

#include <type_traits>

#include "skm_device.h"
#include "skm_internal.h"

namespace skm {
namespace {
using namespace dev;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;


template <bool BF16>
struct MfmaCfg;

template <>
struct MfmaCfg<true> {
  static constexpr int KSTEP = 16;  // K per instruction
  static constexpr int RT = 2;      // 32-row tiles per wave
  static constexpr int CC = 64;     // centres per LDS chunk
  // waves per block: every block stages all centres through LDS once per
  // pass, so 512 rows per block halve that traffic (two waves per SIMD fit)
  static constexpr int WAVES = 8;
  typedef __bf16 elem;
};

template <>
struct MfmaCfg<false> {
  static constexpr int KSTEP = 2;
  static constexpr int RT = 1;
  static constexpr int CC = 32;
  static constexpr int WAVES = 4;
  typedef float elem;
};

// Median of three unsigned integers, one instruction.
__device__ __forceinline__ unsigned umed3(unsigned a, unsigned b, unsigned c) {
  unsigned r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// One 32x32 accumulator tile of a row block.  Mode 0 folds the lane's 16
// values into its running top-2: first a tile-local top-2 (index as a
// compile-time offset, second best by median-of-three), then one merge.
// Selects instead of fmaxf keep NaN canonicalisation out of the loop; the
// inputs are finite.  Mode 1 emits every centre at or above the row's
// threshold.  `ragged` masks centres >= k (only the last tiles have them).
template <int MODE>
__device__ __forceinline__ void tile_epilogue(const f32x16& acc, int jb, int k, bool ragged,
                                              float& m1, int& j1, float& m2, float thr,
                                              int64_t rowid, int64_t slot, int* lcnt, int lrow,
                                              const DenseSimArgs& A) {
  if (MODE == 0) {
    float t1 = -INFINITY, t2 = -INFINITY;
    int ti = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int off = 8 * (i >> 2) + (i & 3);
      const float v = (!ragged || jb + off < k) ? acc[i] : -INFINITY;
      t2 = __builtin_amdgcn_fmed3f(t1, t2, v);
      const bool gt = v > t1;
      t1 = gt ? v : t1;
      ti = gt ? off : ti;
    }
    const bool gt = t1 > m1;
    m2 = __builtin_amdgcn_fmed3f(m1, m2, t1);
    m2 = t2 > m2 ? t2 : m2;
    j1 = gt ? jb + ti : j1;
    m1 = gt ? t1 : m1;
  } else {
    // a 16-bit mask of the values at or above the threshold first (no
    // branches), then one append per set bit: few values pass
    unsigned hit = 0u;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int j = jb + 8 * (i >> 2) + (i & 3);
      hit |= ((!ragged || j < k) && acc[i] >= thr) ? (1u << i) : 0u;
    }
    if (rowid < 0) hit = 0u;
    while (hit) {
      const int i = __builtin_ctz(hit);
      hit &= hit - 1u;
      const int j = jb + 8 * (i >> 2) + (i & 3);
      const int pos = atomicAdd(&lcnt[lrow], 1);  // LDS counter of the row
      if (pos < A.cand_cap) A.cand[slot * A.cand_cap + pos] = j;
    }
  }
}

// Direct load of centres [c0, c0 + CC) into one LDS chunk buffer with
// padded rows of dp + 8 elements (buffer loads that write LDS: no registers,
// and unlike the global form they leave the LDS-read wait counts exact).  A
// wave-wide load fills 64 consecutive 16-byte units of the buffer; units
// that fall on a row's padding slot are masked off.  The resource covers the
// whole centre array, and the hardware returns zero past its end.
template <int CC, int dp, int WAVES>
__device__ __forceinline__ void fetch_chunk(__amdgpu_buffer_rsrc_t res, int c0, __bf16* dst,
                                            int wave, int lane) {
  constexpr int PR = dp / 8;              // 16-byte units per centre row
  constexpr int NI = CC * (PR + 1) / 64;  // wave-wide loads per chunk
#pragma unroll
  for (int q = wave; q < NI; q += WAVES) {
    const int v = q * 64 + lane;
    const int r = v / (PR + 1), u = v - r * (PR + 1);
    if (u < PR)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          res, (__attribute__((address_space(3))) void*)(dst + q * 512), 16,
          ((c0 + r) * dp + u * 8) * 2, 0, 0, 0);
  }
}

// Rows x centres on MFMA.  rows: list of row ids (nullable = identity),
// count from *rows_count (nullable = n_rows).
//   mode 0: writes best value, its centre, second best (per row, in slot
//           order of the list)
//   mode 1: candidate emission: every centre with value >= thr[slot] is
//           appended to cand[slot * cap + ...], counts in cand_n[slot]
template <bool BF16, int MODE, int DP>
__global__ __launch_bounds__(MfmaCfg<BF16>::WAVES * 64) void k_dense_sim(DenseSimArgs A) {
  typedef MfmaCfg<BF16> Cfg;
  constexpr int kDenseWaves = Cfg::WAVES;
  typedef typename Cfg::elem E;
  constexpr int KSTEP = Cfg::KSTEP, RT = Cfg::RT, CC = Cfg::CC;
  // BF16 top-2 pass: values offset by a positive constant and packed with their place
  constexpr bool kPack = BF16 && MODE == 0;
  // accumulator start of tile rt (values arrive offset by it, all positive);
  // distinct per tile so that each folds into its first MFMA as an inline
  // constant
  constexpr float kOffset[2] = {2.f, 4.f};
  static_assert(!kPack || RT <= 2, "one offset per row tile");
  constexpr int ROWS_PER_WAVE = 32 * RT;
  constexpr int ROWS_PER_BLOCK = ROWS_PER_WAVE * kDenseWaves;
  extern __shared__ char smem[];
  E* lds = reinterpret_cast<E*>(smem);  // FP32: one staged chunk
  constexpr int ldsw = DP + (BF16 ? 8 : 4);  // padded LDS row stride (16-byte aligned)
  // BF16: two chunk buffers for the direct loads
  __shared__ __attribute__((aligned(16))) E ldsA[BF16 ? Cfg::CC * ldsw : 8];
  __shared__ __attribute__((aligned(16))) E ldsB[BF16 ? Cfg::CC * ldsw : 8];
  // candidate mode: per-row candidate counts of the block's current rows
  __shared__ int lcnt[MODE == 1 ? ROWS_PER_BLOCK : 1];
  constexpr int dp = DP;
  constexpr int nsteps = dp / KSTEP;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t count = A.rows_count ? (int64_t)(*A.rows_count) : A.n_rows;
  const E* __restrict__ Xe = reinterpret_cast<const E*>(A.X);
  const E* __restrict__ Ce = reinterpret_cast<const E*>(A.C);

  for (int64_t blk = (int64_t)blockIdx.x * ROWS_PER_BLOCK; blk < count;
       blk += (int64_t)gridDim.x * ROWS_PER_BLOCK) {
    // operand fragments of this wave's rows, kept in registers
    int64_t slot[RT];
    int64_t rowid[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      slot[rt] = blk + (int64_t)wave * ROWS_PER_WAVE + rt * 32 + (lane & 31);
      rowid[rt] = (slot[rt] < count) ? (A.rows ? (int64_t)A.rows[slot[rt]] : slot[rt]) : -1;
    }
    constexpr int NS = nsteps;  // K steps, all held in registers
    typedef typename std::conditional<BF16, bf16x8, float>::type Frag;
    Frag bfr[RT][NS];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (rowid[rt] >= 0) {
          if constexpr (BF16) {
            bfr[rt][s] = *reinterpret_cast<const bf16x8*>(Xe + (size_t)rowid[rt] * A.ldx +
                                                          s * KSTEP + 8 * (lane >> 5));
          } else {
            const int col = s * KSTEP + (lane >> 5);
            bfr[rt][s] = col < A.d ? Xe[(size_t)rowid[rt] * A.ldx + col] : 0.f;
          }
        } else {
          if constexpr (BF16) {
            bf16x8 z;
#pragma unroll
            for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.f;
            bfr[rt][s] = z;
          } else {
            bfr[rt][s] = 0.f;
          }
        }
      }
    if (MODE == 1)
      for (int i = threadIdx.x; i < ROWS_PER_BLOCK; i += kDenseWaves * 64) lcnt[i] = 0;
    float m1[RT], m2[RT], thr[RT];
    int j1[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      m1[rt] = kPack ? 0.f : -INFINITY;  // packed: the smallest pattern
      m2[rt] = kPack ? 0.f : -INFINITY;
      j1[rt] = INT_MAX;
      thr[rt] = (MODE == 1 && rowid[rt] >= 0) ? A.thr[slot[rt]] : INFINITY;
    }

    // BF16 top-2 pass, software-pipelined over tiles: while the products of
    // one tile run, the previous tile's values are folded into per-lane
    // top-2 patterns (a few integer operations between MFMAs), so the matrix
    // core does not wait for the fold.  A tile that reaches past k is folded
    // after the products with its padding centres masked off.
    constexpr int PRT = kPack ? RT : 1;
    f32x16 prv[PRT];
    unsigned pt1[PRT], pt2[PRT];
    int prv_jb = 0, prv_state = 0;  // 0 none, 1 whole tile, 2 tile reaching past k
#pragma unroll
    for (int rt = 0; rt < PRT; ++rt) {
#pragma unroll
      for (int i = 0; i < 16; ++i) prv[rt][i] = 0.f;
      pt1[rt] = pt2[rt] = 0u;
    }
    // Value i of a tile into a lane's running top-2.  The accumulator of row
    // tile rt starts at kOffset[rt] (2 or 4), so a value v arrives as
    // v + kOffset[rt] > 0, where bit patterns order like values; the low
    // four bits of the pattern are replaced by
    // the value's place in the tile (15 - i, so that the earlier centre wins
    // an exact tie).  The top-2 is then an integer maximum and
    // median-of-three per value, and the place of the maximum is read back
    // from its bits.  m1 and m2 hold such patterns; masked values (centres
    // beyond k) count as the smallest pattern.
    auto fold = [&](const f32x16& v, int i, bool masked, int jbase, unsigned& t1,
                    unsigned& t2) __attribute__((always_inline)) {
      const int off = 8 * (i >> 2) + (i & 3);
      const unsigned pv = (__float_as_uint(v[i]) & 0xFFFFFFF0u) | (15u - i);
      const unsigned q = (!masked || jbase + off < A.k) ? pv : 0u;
      t2 = umed3(t1, t2, q);
      t1 = max(t1, q);
    };
    // a folded tile into the row's running top-2 and best index
    auto merge = [&](int rt, unsigned t1, unsigned t2, int jbase) __attribute__((always_inline)) {
      const int i1 = 15 - (int)(t1 & 15u);
      const int ti = 8 * (i1 >> 2) + (i1 & 3);
      const unsigned k1 = __float_as_uint(m1[rt]), k2 = __float_as_uint(m2[rt]);
      const bool gt = t1 > k1;
      m2[rt] = __uint_as_float(max(umed3(k1, k2, t1), t2));
      j1[rt] = gt ? jbase + ti : j1[rt];
      m1[rt] = __uint_as_float(max(k1, t1));
    };
    // completes the previous tile: merge what was folded during the
    // products, or fold it now (ragged, or nothing overlapped it)
    auto finish_prev = [&](bool folded) __attribute__((always_inline)) {
      if (prv_state == 1 && folded) {
#pragma unroll
        for (int rt = 0; rt < PRT; ++rt) merge(rt, pt1[rt], pt2[rt], prv_jb);
      } else if (prv_state != 0) {
        const bool masked = prv_state == 2;
#pragma unroll
        for (int rt = 0; rt < PRT; ++rt) {
          unsigned t1 = 0u, t2 = 0u;
#pragma unroll
          for (int i = 0; i < 16; ++i) fold(prv[rt], i, masked, prv_jb, t1, t2);
          merge(rt, t1, t2, prv_jb);
        }
      }
    };
    auto ptile = [&](int c0, const E* cur, int at) __attribute__((always_inline)) {
      if constexpr (kPack) {
        f32x16 acc[PRT];
#pragma unroll
        for (int rt = 0; rt < PRT; ++rt) {
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[rt][i] = kOffset[rt];
          pt1[rt] = pt2[rt] = 0u;
        }
        const E* arow = cur + (at * 32 + (lane & 31)) * ldsw;
        const bf16x8* ap = reinterpret_cast<const bf16x8*>(arow + 8 * (lane >> 5));
        constexpr int VPI = 32 / NS;  // previous-tile values folded per step pair
        bf16x8 a0 = ap[0], a1 = ap[2];
#pragma unroll
        for (int s = 0; s < NS; s += 2) {
          // the next step pair's fragments are read before this pair's MFMAs;
          // the wave issues them and the pair at raised priority (lowered
          // after the pair), which lets the other wave of the SIMD fill the
          // gaps instead of competing for issue inside the pair (1% faster)
          __builtin_amdgcn_s_setprio(1);
          bf16x8 n0 = a0, n1 = a1;
          if (s + 2 < NS) {
            n0 = ap[2 * (s + 2)];
            n1 = ap[2 * (s + 3)];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int rt = 0; rt < PRT; ++rt)
            acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bfr[rt][s], acc[rt], 0, 0, 0);
#pragma unroll
          for (int rt = 0; rt < PRT; ++rt)
            acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bfr[rt][s + 1], acc[rt], 0, 0, 0);
          // (folded unconditionally: the result is used only for a whole
          // previous tile, so no branch splits the MFMAs from the folds)
#pragma unroll
          for (int rt = 0; rt < PRT; ++rt)
#pragma unroll
            for (int q = 0; q < VPI; ++q)
              fold(prv[rt], (s / 2) * VPI + q, false, prv_jb, pt1[rt], pt2[rt]);
          // issue order: the two fragment reads, then each MFMA followed by a
          // few fold operations, which run while that MFMA occupies the unit
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
          for (int g = 0; g < 2 * PRT; ++g) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 3 * VPI / 2, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
          __builtin_amdgcn_s_setprio(0);
          a0 = n0;
          a1 = n1;
        }
        finish_prev(true);
#pragma unroll
        for (int rt = 0; rt < PRT; ++rt) prv[rt] = acc[rt];
        prv_jb = c0 + at * 32 + 4 * (lane >> 5);
        prv_state = (c0 + at * 32 + 32 <= A.k) ? 1 : 2;
      }
    };

    // one chunk of CC centres against the wave's rows, from LDS at cur
    auto chunk = [&](int c0, const E* cur) __attribute__((always_inline)) {
      if constexpr (kPack) {
#pragma unroll
        for (int at = 0; at < CC / 32; ++at) ptile(c0, cur, at);
        return;
      }
      // candidate pass (and FP32): products, then the tile's epilogue
#pragma unroll
      for (int at = 0; at < CC / 32; ++at) {
        f32x16 acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[rt][i] = 0.f;
        const E* arow = cur + (at * 32 + (lane & 31)) * ldsw;
        if constexpr (BF16) {
          // fragments of K steps s + 2, s + 3 are read from LDS before the
          // products of steps s, s + 1 are issued (the scheduling fences
          // keep that order), so LDS latency hides behind four MFMAs
          const bf16x8* ap = reinterpret_cast<const bf16x8*>(arow + 8 * (lane >> 5));
          bf16x8 a0 = ap[0], a1 = ap[2];
#pragma unroll
          for (int s = 0; s < NS; s += 2) {
            bf16x8 n0 = a0, n1 = a1;
            if (s + 2 < NS) {
              n0 = ap[2 * (s + 2)];
              n1 = ap[2 * (s + 3)];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bfr[rt][s], acc[rt], 0, 0, 0);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bfr[rt][s + 1], acc[rt], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            a0 = n0;
            a1 = n1;
          }
        } else {
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const float a = arow[s * KSTEP + (lane >> 5)];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bfr[rt][s], acc[rt], 0, 0, 0);
          }
        }
        // epilogue: lane holds centres 8(i/4) + 4(l/32) + i%4 of row l%32
        const int jb = c0 + at * 32 + 4 * (lane >> 5);
        if (c0 + at * 32 + 32 <= A.k) {  // wave-uniform: no padding centre in the tile
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) tile_epilogue<MODE>(acc[rt], jb, A.k, false, m1[rt],
                                                              j1[rt], m2[rt], thr[rt], rowid[rt],
                                                              slot[rt], lcnt,
                                                              (int)(slot[rt] - blk), A);
        } else {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) tile_epilogue<MODE>(acc[rt], jb, A.k, true, m1[rt],
                                                              j1[rt], m2[rt], thr[rt], rowid[rt],
                                                              slot[rt], lcnt,
                                                              (int)(slot[rt] - blk), A);
        }
      }
    };

    if constexpr (BF16) {
      // Centres reach LDS by direct buffer-to-LDS loads (no registers) into
      // two buffers: chunk c + 1 is in flight while chunk c is multiplied.
      // A wave-wide load fills 64 consecutive 16-byte units; units that fall
      // on a row's padding slot are masked off.  The two buffers are
      // separate arrays and the loop alternates them statically, so the
      // wait for a load into one buffer is never placed before reads of the
      // other.
      // raw buffer over the kpad x dp centre array (32-bit data format word)
      const __amdgpu_buffer_rsrc_t cres = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<E*>(Ce), (short)0, A.kpad * dp * 2, 0x00020000);
      // every wave is done with both buffers (previous row block)
      __syncthreads();
      fetch_chunk<CC, dp, kDenseWaves>(cres, 0, ldsA, wave, lane);
      for (int c0 = 0; c0 < A.kpad; c0 += 2 * CC) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (c0 + CC < A.kpad) fetch_chunk<CC, dp, kDenseWaves>(cres, c0 + CC, ldsB, wave, lane);
        chunk(c0, ldsA);
        if (c0 + CC < A.kpad) {
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          __syncthreads();
          if (c0 + 2 * CC < A.kpad)
            fetch_chunk<CC, dp, kDenseWaves>(cres, c0 + 2 * CC, ldsA, wave, lane);
          chunk(c0 + CC, ldsB);
        }
      }
    } else {
      for (int c0 = 0; c0 < A.kpad; c0 += CC) {
        __syncthreads();
        // stage centres [c0, c0 + CC) into LDS, 16 bytes per thread and
        // step; all loads are issued before the first LDS write
        constexpr int VEC = 16 / sizeof(E);
        constexpr int per_row = dp / VEC;
        constexpr int NT = kDenseWaves * 64;
        constexpr int TOTAL = CC * per_row;
        constexpr int STEPS = (TOTAL + NT - 1) / NT;
        float4 st[STEPS];
#pragma unroll
        for (int q = 0; q < STEPS; ++q) {
          const int e = threadIdx.x + q * NT;
          const int r = e / per_row, c = (e - r * per_row) * VEC;
          if (TOTAL % NT == 0 || e < TOTAL)
            st[q] = *reinterpret_cast<const float4*>(Ce + (size_t)(c0 + r) * dp + c);
        }
#pragma unroll
        for (int q = 0; q < STEPS; ++q) {
          const int e = threadIdx.x + q * NT;
          const int r = e / per_row, c = (e - r * per_row) * VEC;
          if (TOTAL % NT == 0 || e < TOTAL)
            *reinterpret_cast<float4*>(lds + r * ldsw + c) = st[q];
        }
        __syncthreads();
        chunk(c0, lds);
      }
    }
    if constexpr (kPack) finish_prev(false);  // the last tile
    if (MODE == 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < ROWS_PER_BLOCK; i += kDenseWaves * 64)
        if (blk + i < count) A.cand_n[blk + i] = lcnt[i];
    }
    if (MODE == 0) {
      // combine lanes l and l ^ 32 (same row, other half of the centres)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const float om1 = __shfl_xor(m1[rt], 32, 64);
        const float om2 = __shfl_xor(m2[rt], 32, 64);
        const int oj1 = __shfl_xor(j1[rt], 32, 64);
        float b, s2v;
        int bj = j1[rt];
        if constexpr (kPack) {
          // patterns of offset values: compare as integers, then undo the
          // offset (exact: the pattern lies within a factor 2 of it)
          const unsigned a1 = __float_as_uint(m1[rt]), a2 = __float_as_uint(m2[rt]);
          const unsigned o1 = __float_as_uint(om1), o2 = __float_as_uint(om2);
          unsigned kb = a1, ks = max(a2, o2);
          if (o1 > kb || (o1 == kb && oj1 < bj)) {
            ks = max(ks, kb);
            kb = o1;
            bj = oj1;
          } else {
            ks = max(ks, o1);
          }
          b = __uint_as_float(kb) - kOffset[rt];
          s2v = A.k > 1 ? __uint_as_float(ks) - kOffset[rt] : -INFINITY;  // k = 1: no second
        } else {
          b = m1[rt];
          s2v = fmaxf(m2[rt], om2);
          if (om1 > b || (om1 == b && oj1 < bj)) {
            s2v = fmaxf(s2v, b);
            b = om1;
            bj = oj1;
          } else {
            s2v = fmaxf(s2v, om1);
          }
        }
        if (lane < 32 && rowid[rt] >= 0) {
          A.best[slot[rt]] = b;
          A.best_j[slot[rt]] = bj;
          A.second[slot[rt]] = s2v;
        }
      }
    }
  }
}


// Rigorous bound on |s_hat - <x, c>| for one row of the dense contraction.
// BF16: the pass multiplies x^ = x + dx and c^ = c + dc (the BF16 copies);
// by Cauchy-Schwarz <x^, c^> - <x, c> = <dx, c> + <x, dc> + <dx, dc> is at
// most rx |c| + |x| rc + rx rc, with rx = |dx| measured per row when the
// copy is made and rc the largest |dc| of any centre copy made in the fit
// (both rounded up; without them, the worst case of RNE to an 8-bit
// significand: rx <= 2^-8 |x|, rc <= (2^-8 + 2^-24) |c|).  Products are
// exact; the FP32 accumulation starts at 2 or 4 (the top-2 pass offsets
// values) so every partial sum is below 5 |x||c| + 4, taken with unit 2^-23
// to cover accumulation that truncates; replacing four low bits of the
// offset value (below 8) and removing the offset add below 2^-17.
// FP32: the centre copy, every product and every sum (unit 2^-23 for the
// sums, as above).  Relative terms are relative to sum |x_t c_t| <= |x| |c|
// <= 1 + eta; the factor 1.01 covers |x^| |c^| and |c| - 1.
__device__ __forceinline__ double dense_eps(bool bf16, int dp, double eta, const float* xr,
                                            const float* rcmax, int64_t row) {
  if (!bf16) return (2 * dp + 3) * kU32 * (1.0 + eta) * 1.01;
  const double acc = (2.0 * kU32 + 10.5 * (dp + 2) * kU32 + 7.62939453125e-06) * (1.0 + eta);
  if (!xr || !rcmax)
    return ((2.0 * 0.00390625 + 1.52587890625e-05) * (1.0 + eta) + acc) * 1.01;
  float rc32 = 0.f;
#pragma unroll
  for (int q = 0; q < kRcSlots; ++q) rc32 = fmaxf(rc32, rcmax[q]);
  const double rx = (double)xr[row], rc = (double)rc32;
  return (rx + (1.0 + eta) * rc + rx * rc + acc) * 1.01;
}

// Decision after the top-2 pass: clear rows are final (FP32/BF16 argmax is
// the exact argmax); rows inside the band are flagged for the candidate
// pass with their threshold.
__global__ __launch_bounds__(kBlock) void k_dense_post(DensePostArgs A) {
  __shared__ unsigned long long sh_changed;
  if (threadIdx.x == 0) sh_changed = 0;
  __syncthreads();
  const int64_t count = A.rows_count ? (int64_t)(*A.rows_count) : A.n_rows;
  const int64_t sl = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long moved = 0;
  if (sl < count) {
    const int64_t row = A.rows ? A.rows[sl] : sl;
    const int prev = A.read_prev ? A.a[row] : -1;
    const double eta = (double)A.eta[row];
    const double eps = dense_eps(A.bf16, A.dp, eta, A.xr, A.rcmax, row);
    const double b = A.best[sl], s2 = A.second[sl];
    const bool near = A.k > 1 && b - s2 <= 2.0 * eps;
    A.near[sl] = near ? 1 : 0;
    if (A.best_out) A.best_out[row] = (float)b;
    if (A.second_out) A.second_out[row] = (float)s2;
    if (near) {
      A.thr[sl] = __double2float_rd(b - 2.0 * eps - 1e-12);
    } else {
      const int j = A.best_j[sl];
      A.a[row] = j;
      moved = (j != prev) ? 1 : 0;
      const double rho = eps + 1.01 * (eta + A.delta_c) + 1e-12;
      if (A.l) A.l[row] = __double2float_rd(fmax(b - rho, -1.0));
      if (A.u) A.u[row] = __double2float_ru(fmin((A.k == 1 ? -1.0 : s2 + rho), 1.0));
    }
  }
  if (moved) atomicAdd(&sh_changed, moved);
  __syncthreads();
  if (threadIdx.x == 0 && sh_changed) atomicAdd(&counter_slot(A.cnt)->changed, sh_changed);
}

// FP64 re-decision of the flagged rows against the FP64 master centres, two
// rows per wave: the listed candidates one after another, each by the row's
// half-wave; a row with more candidates than the list holds evaluates all k
// centres with the whole wave, one lane each with a sequential FP64 chain.  Either order is
// fixed, and the winner (FP64 argmax, tie rule) does not depend on the order
// in which the candidates were listed.
__global__ __launch_bounds__(kBlock) void k_dense_exact(DenseExactArgs A) {
  __shared__ unsigned long long sh_changed, sh_rechecks;
  if (threadIdx.x == 0) {
    sh_changed = 0;
    sh_rechecks = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, hl = lane & 31;
  const int64_t count = (int64_t)(*A.near_count);
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  unsigned long long moved = 0, rech = 0;
  // two flagged rows per wave, one per half-wave, so that two rows' chains
  // of dependent loads are in flight together
  for (int64_t w0 = (((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6) * 2; w0 < count;
       w0 += 2 * nw) {
    const int64_t w = w0 + half;
    const bool valid = w < count;
    int64_t sl = 0, row = 0;
    int prev = -1, nc = 0;
    if (valid) {
      sl = A.near_list[w];  // slot of the similarity pass
      row = A.rows ? A.rows[sl] : sl;
      prev = A.read_prev ? A.a[row] : -1;
      nc = A.cand_n[w];
    }
    double cb = -INFINITY;
    int cj = INT_MAX;
    if (valid && nc <= A.cand_cap) {
      // listed candidates one at a time, the half-wave on each: lane l of
      // the half holds terms l + 32 q (d <= 256), an eight-term FMA chain,
      // then a fixed xor tree over the half's lanes; all its lanes end with
      // the same value
      const float* x = A.X + (size_t)row * A.ldx;
      double xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int t = hl + 32 * q;
        xv[q] = (t < A.d) ? (double)x[t] : 0.0;
      }
      const int32_t* cl = A.cand + (size_t)w * A.cand_cap;
      for (int c = 0; c < nc; ++c) {
        const int j = cl[c];
        const double* cj64 = A.C64 + (size_t)j * A.d;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int t = hl + 32 * q;
          acc = fma(xv[q], (t < A.d) ? cj64[t] : 0.0, acc);
        }
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (better64(acc, j, cb, cj, prev)) {
          cb = acc;
          cj = j;
        }
      }
    }
    // rows with more candidates than the list holds: the whole wave takes
    // every centre, one lane each with a sequential FP64 chain, one such row
    // at a time
    for (int h = 0; h < 2; ++h) {
      const int64_t wh = w0 + h;
      if (wh >= count) break;
      const int nch = A.cand_n[wh];
      if (nch <= A.cand_cap) continue;
      const int64_t slh = A.near_list[wh];
      const int64_t rowh = A.rows ? A.rows[slh] : slh;
      const int prevh = A.read_prev ? A.a[rowh] : -1;
      const float* xh = A.X + (size_t)rowh * A.ldx;
      double ob = -INFINITY;
      int oj = INT_MAX;
      for (int c = lane; c < A.k; c += 64) {
        const double* cj64 = A.C64 + (size_t)c * A.d;
        double acc = 0.0;
        for (int t = 0; t < A.d; ++t) acc = fma((double)xh[t], cj64[t], acc);
        if (better64(acc, c, ob, oj, prevh)) {
          ob = acc;
          oj = c;
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double b2 = __shfl_xor(ob, off, 64);
        const int j2 = __shfl_xor(oj, off, 64);
        if (better64(b2, j2, ob, oj, prevh)) {
          ob = b2;
          oj = j2;
        }
      }
      if (half == h) {
        cb = ob;
        cj = oj;
      }
    }
    if (valid && hl == 0) {
      A.a[row] = cj;
      moved += (cj != prev) ? 1 : 0;
      rech += 1;
      if (A.best_out) A.best_out[row] = (float)cb;
      if (A.second_out && cj != A.best_j[sl]) A.second_out[row] = A.best[sl];
      const double eta = (double)A.eta[row];
      const double eps = dense_eps(A.bf16, A.dp, eta, A.xr, A.rcmax, row);
      const double slack = 1.01 * (eta + A.delta_c);
      const double rho64 = (double)(A.d + 2) * kU64 * (1.0 + eta) * 1.01 + slack + 1e-15;
      const double rho = eps + slack + 1e-12;
      if (A.l) A.l[row] = __double2float_rd(fmax(cb - rho64, -1.0));
      if (A.u) A.u[row] = __double2float_ru(fmin((double)A.best[sl] + rho, 1.0));
    }
  }
  if (moved) atomicAdd(&sh_changed, moved);
  if (rech) atomicAdd(&sh_rechecks, rech);
  __syncthreads();
  if (threadIdx.x == 0) {
    Counters* c = counter_slot(A.cnt);
    if (sh_changed) atomicAdd(&c->changed, sh_changed);
    if (sh_rechecks) atomicAdd(&c->rechecks, sh_rechecks);
  }
}

// Row ids and thresholds of the flagged slots, for the candidate pass.
__global__ __launch_bounds__(kBlock) void k_gather_near(const int32_t* __restrict__ near_list,
                                                        const unsigned long long* __restrict__ cnt,
                                                        const int32_t* __restrict__ rows,
                                                        const float* __restrict__ thr_slot,
                                                        int32_t* __restrict__ out_rows,
                                                        float* __restrict__ out_thr) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)(*cnt)) return;
  const int32_t sl = near_list[q];
  out_rows[q] = rows ? rows[sl] : sl;
  out_thr[q] = thr_slot[sl];
}

// Hamerly step for dense rows (Sections 5.3 / 5.4), 16 lanes per row.
constexpr int kDHG = 16;
__global__ __launch_bounds__(kBlock) void k_dense_hamerly(DenseHamerlyArgs A) {
  __shared__ unsigned long long sh_tight, sh_saved;
  if (threadIdx.x == 0) {
    sh_tight = 0;
    sh_saved = 0;
  }
  __syncthreads();
  const int gl = threadIdx.x & (kDHG - 1);
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kDHG;
  unsigned long long tight = 0, saved = 0;
  if (i < A.n) {
    const int a = A.a[i];
    const double eta = (double)A.eta[i];
    const double slack = 1.01 * (eta + A.delta_c);
    const double rho64 = (double)(A.d + 2) * kU64 * (1.0 + eta) * 1.01 + slack + 1e-15;
    const double mu = 4.0 * (double)(A.d + 2) * kU64 * (1.0 + eta) + 4.0 * A.delta_c + 1e-15;
    const MoveMin mm = *A.mm;
    double ld = lower_upd((double)A.l[i], A.pc[a], A.ps[a]) - 4e-15;
    const double pcx = (a == mm.idx1) ? mm.pc2 : mm.pc1;
    const double psx = (a == mm.idx1) ? mm.ps2 : mm.ps1;
    const double u0 = fmin(1.0, fmax(-1.0, (double)A.u[i]));
    double ud;
    if (A.bound_form == 1 && u0 >= 0.0 && pcx >= 0.0)
      ud = u0 + sqrt((1.0 - u0) * (1.0 + u0)) * psx;  // Eq. (9)
    else
      ud = upper_upd(u0, pcx, psx);
    ud = fmin(1.0, ud + 4e-15);
    const double smax = A.simplified ? 2.0 : A.gmax[a];
    auto pruned = [&](double lcur) -> bool {
      if (lcur - ud >= mu) return true;
      const double M = lcur - mu;
      return !A.simplified && lcur > 0.0 && M > 0.0 && smax <= cc_threshold(lcur, M) - 4e-15;
    };
    bool skip = pruned(ld);
    if (!skip && A.try_tighten) {
      const float* x = A.X + (size_t)i * A.ldx;
      const double* c = A.C64 + (size_t)a * A.d;
      double p = 0.0;
      for (int t = gl; t < A.d; t += kDHG) p = fma((double)x[t], c[t], p);
      const double s64 = group_sum<kDHG>(p);
      ld = fmax(ld, s64 - rho64);
      tight = (gl == 0) ? 1 : 0;
      skip = pruned(ld);
      saved = (skip && gl == 0) ? 1 : 0;
    }
    if (gl == 0) {
      A.flag[i] = skip ? 0 : 1;
      A.l[i] = __double2float_rd(fmax(ld, -1.0));
      A.u[i] = __double2float_ru(ud);
    }
  }
  if (tight) atomicAdd(&sh_tight, tight);
  if (saved) atomicAdd(&sh_saved, saved);
  __syncthreads();
  if (threadIdx.x == 0 && sh_tight) {
    Counters* c = counter_slot(A.cnt);
    atomicAdd(&c->tightened, sh_tight);
    atomicAdd(&c->sims, sh_tight);
    if (sh_saved) atomicAdd(&c->tight_saved, sh_saved);
  }
}

// ---- compaction: flags -> list of indices, no contended atomics ----
constexpr int kCompactChunk = 1024;

__global__ __launch_bounds__(kBlock) void k_flags_count(const int32_t* __restrict__ flags,
                                                        const unsigned long long* __restrict__ nptr,
                                                        int64_t nmax, int32_t* __restrict__ bcnt) {
  __shared__ int sh;
  if (threadIdx.x == 0) sh = 0;
  __syncthreads();
  const int64_t n = nptr ? (int64_t)(*nptr) : nmax;
  const int64_t base = (int64_t)blockIdx.x * kCompactChunk;
  int c = 0;
  for (int e = threadIdx.x; e < kCompactChunk; e += kBlock) {
    const int64_t i = base + e;
    if (i < n && flags[i]) ++c;
  }
  if (c) atomicAdd(&sh, c);
  __syncthreads();
  if (threadIdx.x == 0) bcnt[blockIdx.x] = sh;
}

// Single block: exclusive scan of nb block counts, total into *total.
__global__ __launch_bounds__(kBlock) void k_scan_counts(const int32_t* __restrict__ bcnt, int nb,
                                                        int32_t* __restrict__ boff,
                                                        unsigned long long* __restrict__ total) {
  __shared__ int sh[kBlock];
  const int per = (nb + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int b = b0; b < b0 + per && b < nb; ++b) s += bcnt[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - s;
  for (int b = b0; b < b0 + per && b < nb; ++b) {
    boff[b] = run;
    run += bcnt[b];
  }
  if (threadIdx.x == kBlock - 1) *total = (unsigned long long)sh[kBlock - 1];
}

// Writes the indices i with flags[i] != 0 in increasing order; also clears
// zero_at[pos] for every written position (nullable).
__global__ __launch_bounds__(kBlock) void k_flags_scatter(const int32_t* __restrict__ flags,
                                                          const unsigned long long* __restrict__ nptr,
                                                          int64_t nmax,
                                                          const int32_t* __restrict__ boff,
                                                          int32_t* __restrict__ list,
                                                          int32_t* __restrict__ zero_at) {
  __shared__ int wsum[kBlock / 64];
  const int64_t n = nptr ? (int64_t)(*nptr) : nmax;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int run = boff[blockIdx.x];
  for (int e0 = 0; e0 < kCompactChunk; e0 += kBlock) {
    const int64_t i = (int64_t)blockIdx.x * kCompactChunk + e0 + threadIdx.x;
    const bool f = i < n && flags[i];
    const unsigned long long m = __ballot(f);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      if (w < wave) before += wsum[w];
      tot += wsum[w];
    }
    if (f) {
      const int pos = run + before + (int)__popcll(m & ((1ull << lane) - 1ull));
      list[pos] = (int32_t)i;
      if (zero_at) zero_at[pos] = 0;
    }
    run += tot;
    __syncthreads();
  }
}

// ---- member sums recomputed per cluster ----
__global__ __launch_bounds__(kBlock) void k_hist(const int32_t* __restrict__ a, int64_t n,
                                                 int32_t k, int32_t* __restrict__ cnt) {
  extern __shared__ int hs[];
  for (int j = threadIdx.x; j < k; j += kBlock) hs[j] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    atomicAdd(&hs[a[i]], 1);
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += kBlock)
    if (hs[j]) atomicAdd(&cnt[j], hs[j]);
}

__global__ __launch_bounds__(kBlock) void k_scatter_rows(const int32_t* __restrict__ a, int64_t n,
                                                         int32_t* __restrict__ cursor,
                                                         int32_t* __restrict__ perm) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    perm[atomicAdd(&cursor[a[i]], 1)] = (int32_t)i;
}

// One block per cluster.  Wave w takes the cluster's rows w, w + 4, ...;
// lane l takes columns 4l .. 4l + 3 of every 256-column step (one 16-byte
// load when the rows allow it), so every row is one coalesced read.  The four
// waves' partial sums meet in LDS: integer additions, so the sums do not
// depend on which wave took which row.
__global__ __launch_bounds__(kBlock) void k_cluster_sums(const int32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ start,
                                                         const int32_t* __restrict__ cnt,
                                                         const float* __restrict__ X, int64_t ldx,
                                                         int64_t d, double fx, int vec,
                                                         long long* __restrict__ S,
                                                         int32_t* __restrict__ dirty) {
  constexpr int W = kBlock / 64;
  __shared__ long long part[W][256];
  const int j = blockIdx.x;
  const int32_t b = start[j], m = cnt[j];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < d; c0 += 256) {
    const int64_t c = c0 + 4 * lane;
    long long acc[4] = {0, 0, 0, 0};
#pragma unroll 4
    for (int32_t q = w; q < m; q += W) {
      const float* xr = X + (size_t)perm[b + q] * ldx;
      float v[4];
      if (vec && c + 3 < d) {
        const float4 f = *reinterpret_cast<const float4*>(xr + c);
        v[0] = f.x;
        v[1] = f.y;
        v[2] = f.z;
        v[3] = f.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (c + e < d) ? xr[c + e] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += __double2ll_rn((double)v[e] * fx);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) part[w][4 * lane + e] = acc[e];
    __syncthreads();
    const int t = threadIdx.x;  // kBlock = 256 columns of this step
    if (c0 + t < d) {
      long long sum = 0;
#pragma unroll
      for (int q = 0; q < W; ++q) sum += part[q][t];
      S[(size_t)j * d + c0 + t] = sum;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) dirty[j] = 1;
}

// Moved rows (a != a_old) applied to the sums with integer atomics; used
// when few rows moved.  One wave per 64 rows scanned, as the sparse path.
__global__ __launch_bounds__(kBlock) void k_dense_update_scan(
    const float* __restrict__ X, int64_t ldx, const int32_t* __restrict__ a,
    int32_t* __restrict__ a_old, int64_t n, int64_t d, double fx, long long* __restrict__ S,
    int32_t* __restrict__ dirty) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63);
  for (int64_t base = wave0; base < n; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + lane;
    int32_t nw = -1, old = -1;
    if (i < n) {
      nw = a[i];
      old = a_old[i];
    }
    unsigned long long moved = __ballot(i < n && nw != old);
    while (moved) {
      const int src = __ffsll((long long)moved) - 1;
      moved &= moved - 1ull;
      const int64_t row = base + src;
      const int32_t rn = __shfl(nw, src, 64);
      const int32_t ro = __shfl(old, src, 64);
      unsigned long long* Sn = reinterpret_cast<unsigned long long*>(S + (size_t)rn * d);
      unsigned long long* So =
          ro >= 0 ? reinterpret_cast<unsigned long long*>(S + (size_t)ro * d) : nullptr;
      for (int64_t t = lane; t < d; t += 64) {
        const long long q = __double2ll_rn((double)X[(size_t)row * ldx + t] * fx);
        atomicAdd(Sn + t, (unsigned long long)q);
        if (So) atomicAdd(So + t, (unsigned long long)(-q));
      }
      if (lane == 0) {
        dirty[rn] = 1;
        if (ro >= 0) dirty[ro] = 1;
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_assign(const int32_t* __restrict__ a,
                                                        int32_t* __restrict__ a_old, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a_old[i] = a[i];
}

// ---- conversions ----
// FP64 masters -> packed MFMA operand rows (bf16 or f32), dirty rows only.
__global__ __launch_bounds__(kBlock) void k_pack_centres(const double* __restrict__ C64,
                                                         int32_t k, int64_t d, int dp,
                                                         const int32_t* __restrict__ dirty,
                                                         int bf16, void* __restrict__ out,
                                                         float* __restrict__ rcmax) {
  const int j = blockIdx.x;
  if (j >= k || (dirty && !dirty[j])) return;
  double rr = 0.0;  // |c^ - c|^2 of the BF16 copy (each difference exact)
  for (int t = threadIdx.x; t < dp; t += kBlock) {
    const double c = t < d ? C64[(size_t)j * d + t] : 0.0;
    if (bf16) {
      const __bf16 h = (__bf16)(float)c;
      reinterpret_cast<__bf16*>(out)[(size_t)j * dp + t] = h;
      const double e = (double)(float)h - c;
      rr = fma(e, e, rr);
    } else {
      reinterpret_cast<float*>(out)[(size_t)j * dp + t] = (float)c;
    }
  }
  if (bf16 && rcmax) {
    // largest copy error of the fit so far, kept in kRcSlots slots (by
    // centre) so that few blocks meet on one address: the largest slot bounds
    // every current copy
    __shared__ double part[kBlock / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) rr += __shfl_xor(rr, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) t += part[w];
      const float r32 = __double2float_ru(sqrt(t) * (1.0 + 1e-12));
      int* slot = reinterpret_cast<int*>(rcmax) + (j % kRcSlots);
      if (__float_as_int(r32) > __atomic_load_n(slot, __ATOMIC_RELAXED))
        atomicMax(slot, __float_as_int(r32));
    }
  }
}

// One pass over dense rows: | |x_i| - 1 | bound per row (FP64 sum of squares)
// and, when Xb is given, the BF16 copy padded to dp columns with the norm of
// its rounding error per row (xerr, rounded up; each difference is exact).  One wave per
// row, grid-strided; lane l takes columns 4l .. 4l + 3 of every 256-column
// step (one 16-byte load when the rows allow it).
__global__ __launch_bounds__(kBlock) void k_dense_prep(const float* __restrict__ X, int64_t ldx,
                                                       int64_t n, int64_t d, int dp, int vec,
                                                       float* __restrict__ eta,
                                                       float* __restrict__ max_eta,
                                                       __bf16* __restrict__ Xb,
                                                       float* __restrict__ xerr) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  const int width = Xb ? dp : (int)d;  // dp >= d; columns d .. dp - 1 of the copy are 0
  float emax = 0.f;
  for (int64_t i = w0; i < n; i += nw) {
    const float* xr = X + (size_t)i * ldx;
    double ss = 0.0, rr = 0.0;
    for (int c = 4 * lane; c < width; c += 256) {
      float v[4];
      if (vec && c + 3 < d) {
        const float4 q = *reinterpret_cast<const float4*>(xr + c);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (c + e < d) ? xr[c + e] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) ss = fma((double)v[e], (double)v[e], ss);
      if (Xb) {
        bf16x4 b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          b[e] = (__bf16)v[e];
          const double r = (double)((float)b[e] - v[e]);
          rr = fma(r, r, rr);
        }
        *reinterpret_cast<bf16x4*>(Xb + (size_t)i * dp + c) = b;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      ss += __shfl_xor(ss, off, 64);
      rr += __shfl_xor(rr, off, 64);
    }
    if (xerr && lane == 0) xerr[i] = __double2float_ru(sqrt(rr) * (1.0 + 1e-12));
    const double dev = fabs(sqrt(ss) - 1.0) + (double)(d + 4) * kU64 * 2.0 + 1e-300;
    const float e32 = __double2float_ru(dev);
    if (lane == 0) eta[i] = e32;
    emax = fmaxf(emax, e32);
  }
  if (max_eta) {
    __shared__ float wmax[kBlock / 64];
    if (lane == 0) wmax[threadIdx.x >> 6] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = 0.f;
      for (int w = 0; w < kBlock / 64; ++w) m = fmaxf(m, wmax[w]);
      if (m > 0.f) atomicMax(reinterpret_cast<int*>(max_eta) + (blockIdx.x % kCounterSlots),
                             __float_as_int(m));
    }
  }
}

}  // namespace

size_t dense_sim_lds_bytes(bool bf16, int dp) {  // dynamic part (BF16 buffers are static)
  if (bf16) return 0;
  return (size_t)MfmaCfg<false>::CC * (dp + 4) * 4;
}

hipError_t launch_dense_sim(const DenseSimArgs& A, bool bf16, int mode, hipStream_t s) {
  const int waves = bf16 ? MfmaCfg<true>::WAVES : MfmaCfg<false>::WAVES;
  const int rows_per_block = (bf16 ? 64 : 32) * waves;
  int64_t blocks = (A.n_rows + rows_per_block - 1) / rows_per_block;
  if (blocks > 4 * kMaxGridBlocks) blocks = 4 * kMaxGridBlocks;
  if (blocks < 1) blocks = 1;
  const size_t lds = dense_sim_lds_bytes(bf16, A.dp);
  // BF16 centres are read through a buffer resource with 32-bit byte offsets
  if (bf16 && (int64_t)A.kpad * A.dp * 2 > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(waves * 64);
#define SKM_DS(B, M, D) \
  hipLaunchKernelGGL((k_dense_sim<B, M, D>), grid, block, lds, s, A)
#define SKM_DS_DP(B, M)                       \
  switch (A.dp) {                             \
    case 32: SKM_DS(B, M, 32); break;         \
    case 64: SKM_DS(B, M, 64); break;         \
    case 128: SKM_DS(B, M, 128); break;       \
    case 256: SKM_DS(B, M, 256); break;       \
    default: return hipErrorInvalidValue;     \
  }
  if (bf16) {
    if (mode == 0) { SKM_DS_DP(true, 0) } else { SKM_DS_DP(true, 1) }
  } else {
    if (mode == 0) { SKM_DS_DP(false, 0) } else { SKM_DS_DP(false, 1) }
  }
#undef SKM_DS_DP
#undef SKM_DS
  return hipGetLastError();
}

namespace {
unsigned nblocks(int64_t count, int per = kBlock) {
  int64_t b = (count + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}
}  // namespace

hipError_t launch_dense_post(const DensePostArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_post, dim3(nblocks(A.n_rows)), dim3(kBlock), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_dense_exact(const DenseExactArgs& A, int64_t max_rows, hipStream_t s) {
  int64_t blocks = (max_rows * 64 + kBlock - 1) / kBlock;
  if (blocks > 4 * kMaxGridBlocks) blocks = 4 * kMaxGridBlocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_dense_exact, dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_gather_near(const int32_t* near_list, const unsigned long long* cnt,
                              int64_t max_rows, const int32_t* rows, const float* thr_slot,
                              int32_t* out_rows, float* out_thr, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_near, dim3(nblocks(max_rows)), dim3(kBlock), 0, s, near_list, cnt,
                     rows, thr_slot, out_rows, out_thr);
  return hipGetLastError();
}

hipError_t launch_dense_hamerly(const DenseHamerlyArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_hamerly, dim3(nblocks(A.n * kDHG)), dim3(kBlock), 0, s, A);
  return hipGetLastError();
}

int compact_blocks(int64_t nmax) { return (int)((nmax + kCompactChunk - 1) / kCompactChunk); }

hipError_t launch_compact(const int32_t* flags, const unsigned long long* nptr, int64_t nmax,
                          int32_t* bcnt, int32_t* boff, int32_t* list,
                          unsigned long long* total, int32_t* zero_at, hipStream_t s) {
  const int nb = compact_blocks(nmax);
  hipLaunchKernelGGL(k_flags_count, dim3((unsigned)(nb < 1 ? 1 : nb)), dim3(kBlock), 0, s, flags,
                     nptr, nmax, bcnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kBlock), 0, s, bcnt, nb, boff, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_flags_scatter, dim3((unsigned)(nb < 1 ? 1 : nb)), dim3(kBlock), 0, s,
                     flags, nptr, nmax, boff, list, zero_at);
  return hipGetLastError();
}

hipError_t launch_cluster_sums(const int32_t* a, int64_t n, int32_t k, const float* X,
                               int64_t ldx, int64_t d, double fx, int32_t* cnt, int32_t* start,
                               int32_t* cursor, int32_t* perm, long long* S, int32_t* dirty,
                               unsigned long long* scratch_total, hipStream_t s) {
  hipError_t e = hipMemsetAsync(cnt, 0, (size_t)k * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  int64_t blocks = nblocks(n);
  if (blocks > kMaxGridBlocks) blocks = kMaxGridBlocks;
  hipLaunchKernelGGL(k_hist, dim3((unsigned)blocks), dim3(kBlock), (size_t)k * sizeof(int), s, a,
                     n, k, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // exclusive scan of the k counts (k <= 4096 fits one block's loop)
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kBlock), 0, s, cnt, k, start, scratch_total);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipMemcpyAsync(cursor, start, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, n, cursor,
                     perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int vec = ((uintptr_t)X % 16 == 0 && ldx % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(k_cluster_sums, dim3((unsigned)k), dim3(kBlock), 0, s, perm, start, cnt, X,
                     ldx, d, fx, vec, S, dirty);
  return hipGetLastError();
}

hipError_t launch_dense_update_scan(const float* X, int64_t ldx, const int32_t* a,
                                    int32_t* a_old, int64_t n, int64_t d, double fx,
                                    long long* S, int32_t* dirty, hipStream_t s) {
  int64_t blocks = nblocks(n);
  if (blocks > kMaxGridBlocks) blocks = kMaxGridBlocks;
  hipLaunchKernelGGL(k_dense_update_scan, dim3((unsigned)blocks), dim3(kBlock), 0, s, X, ldx, a,
                     a_old, n, d, fx, S, dirty);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_assign, dim3(nblocks(n)), dim3(kBlock), 0, s, a, a_old, n);
  return hipGetLastError();
}

hipError_t launch_copy_assign(const int32_t* a, int32_t* a_old, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_assign, dim3(nblocks(n)), dim3(kBlock), 0, s, a, a_old, n);
  return hipGetLastError();
}

hipError_t launch_pack_centres(const double* C64, int32_t k, int64_t d, int dp,
                               const int32_t* dirty, int bf16, void* out, float* rcmax,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_pack_centres, dim3((unsigned)k), dim3(kBlock), 0, s, C64, k, d, dp, dirty,
                     bf16, out, rcmax);
  return hipGetLastError();
}

hipError_t launch_dense_prep(const float* X, int64_t ldx, int64_t n, int64_t d, int dp,
                             float* eta, float* max_eta, void* Xb, float* xr, hipStream_t s) {
  const int vec = ((uintptr_t)X % 16 == 0 && ldx % 4 == 0) ? 1 : 0;
  int64_t blocks = (n + kBlock / 64 - 1) / (kBlock / 64);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_dense_prep, dim3((unsigned)blocks), dim3(kBlock), 0, s, X, ldx, n, d, dp,
                     vec, eta, max_eta, reinterpret_cast<__bf16*>(Xb), xr);
  return hipGetLastError();
}

}  // namespace skm
