// Host side of libskm: argument validation, workspace planning and the
// iteration driver behind the C ABI declared in include/skm.h.
//
// One fit runs, per assignment step (Section 5 outline of the paper):
//   step 1          exhaustive similarities for every row -> a, l, u (or the
//                   warm-start arrays of a seeding)
//   later steps     Lloyd: exhaustive again; Hamerly, Yin-Yang, Elkan: the
//                   bound update and tests of the variant per row, then the
//                   full similarity walk of the rows that failed them
//   sync            read the changed count; stop when it is zero
//   centre step     fixed-point sums of the changed rows, renormalisation,
//                   movement p(j), FP32 (and FP16) transpose, centre-centre
//                   products (full Elkan and Hamerly only)
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/skm.h"
#include "batch_tuning.h"
#include "skm_internal.h"
#include "walk_tuning.h"

// Device buffer of skm_assign_noalloc: every GPU that loads this library
// holds one copy until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (on the host it only names the symbol): its
// address on a device comes from hipGetSymbolAddress (scratch_address).
static __device__ __align__(256) unsigned char scratch[SKM_NOALLOC_SCRATCH_BYTES];

namespace skm {
namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

#define SKM_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) {                                                            \
      rc = fail(SKM_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),    \
                __FILE__, __LINE__);                                                   \
      goto done;                                                                       \
    }                                                                                  \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Plan {
  int64_t n = 0, d = 0, nnz = 0;
  int32_t k = 0, kp = 0;
  int variant = 0;
  bool bounds = false, elkan = false, gram = false;
  int nchunk = 1, nslice = 1;
  int64_t slice_len = 0;
  // byte offsets into the workspace
  bool half = false;  // FP16 centre copy for the row walk
  bool yy = false;    // Yin-Yang group bounds
  int32_t ng = 0;     // Yin-Yang groups
  int chunk = 0;      // centres per launch of a chunked row walk (0: one launch)
  int chunk16 = 0, nq16 = 0;  // Yin-Yang / Elkan steps, FP16 copy: chunk width, launches
  int nq = 1;         // launches per walk
  // FP32 copy, whole rows chosen, Yin-Yang at kp >= 256 and Elkan at kp >=
  // 512: the steps with tests may switch to packed 256-centre slices during
  // the fit; Lloyd and Hamerly with a copy of 64 MB or more (pack_all): every
  // walk may switch to slices
  bool pack_adapt = false, pack_all = false;
  size_t uy = 0, gpc = 0, gps = 0;
  size_t CT = 0, CT16 = 0, negflag = 0, C64 = 0, S = 0, l = 0, u = 0, ue = 0, eta = 0,
         a_old = 0, norm64 = 0, part = 0, part_sq = 0, pc = 0, ps = 0, dirty = 0, mm = 0, G = 0,
         gmax = 0, gpart = 0, cnt = 0, per = 0, ctl = 0, rec = 0, maxeta = 0, initnorm = 0,
         vbad = 0, rs = 0, umask = 0, total = 0;
};

int check_matrix(const skm_matrix* X) {
  if (!X) return fail(SKM_ERR_INVALID_ARG, "X is NULL");
  if (X->n < 1 || X->d < 1) return fail(SKM_ERR_INVALID_ARG, "need n >= 1 and d >= 1");
  if (X->n > INT32_MAX) return fail(SKM_ERR_INVALID_ARG, "n must fit in int32");
  if (X->d > INT32_MAX) return fail(SKM_ERR_INVALID_ARG, "d must fit in int32");
  if (X->fmt == SKM_CSR_F32) {
    if (!X->row_ptr || (!X->col_idx && X->nnz > 0) || (!X->val && X->nnz > 0))
      return fail(SKM_ERR_INVALID_ARG, "CSR arrays must not be NULL");
    if (X->nnz < 0) return fail(SKM_ERR_INVALID_ARG, "nnz must be >= 0");
    return SKM_OK;
  }
  if (X->fmt == SKM_DENSE_F32) {
    if (!X->dense) return fail(SKM_ERR_INVALID_ARG, "dense pointer must not be NULL");
    if (X->ld < X->d) return fail(SKM_ERR_INVALID_ARG, "need ld >= d");
    if (X->d > 256)
      return fail(SKM_ERR_UNSUPPORTED, "dense input supports d <= 256 (MFMA operand tiles "
                  "are held in registers), got %lld", (long long)X->d);
    return SKM_OK;
  }
  return fail(SKM_ERR_INVALID_ARG, "unknown matrix format %d", (int)X->fmt);
}

// The row kernels address the centre-minor copy with 32-bit element offsets
// (column * kp + centre), which keeps their address arithmetic to one
// multiply-add per gather.
int check_ct_size(int64_t d, int32_t kp) {
  if ((uint64_t)d * (uint64_t)kp > (uint64_t)UINT32_MAX)
    return fail(SKM_ERR_UNSUPPORTED, "d * k_padded = %lld * %d exceeds 2^32 - 1 (the row kernels "
                "use 32-bit offsets into the centre copy)", (long long)d, (int)kp);
  return SKM_OK;
}

// validate = 2: the layout of the input rows (Section 2: sparse vectors as
// ascending (index, value) pairs) and finite values, checked before any
// kernel walks the rows.  row_ptr is checked first, by flat index; only
// when it is valid are the rows it delimits scanned.  `bad` is one device
// word of scratch.  Returns SKM_ERR_INVALID_ARG naming the first bad row.
int validate_input(const skm_matrix* X, unsigned long long* bad, hipStream_t s) {
  unsigned long long h = ~0ull;
  auto run = [&](int stage) -> hipError_t {
    hipError_t e = hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    if (X->fmt == SKM_DENSE_F32) e = launch_check_dense(X->dense, X->ld, X->n, X->d, bad, s);
    else if (stage == 0) e = launch_check_rowptr(X->row_ptr, X->n, X->nnz, bad, s);
    else e = launch_check_entries(X->row_ptr, X->col_idx, X->val, X->n, X->d, bad, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  };
  for (int stage = (X->fmt == SKM_DENSE_F32 ? 1 : 0); stage < 2; ++stage) {
    const hipError_t e = run(stage);
    if (e != hipSuccess) return fail(SKM_ERR_HIP, "input check: %s", hipGetErrorString(e));
    if (h == ~0ull) continue;
    const long long row = (long long)(h >> 3);
    switch ((int)(h & 7ull)) {
      case kBadRowPtr:
        return fail(SKM_ERR_INVALID_ARG, "row_ptr invalid at index %lld (need row_ptr[0] = 0, "
                    "non-decreasing, row_ptr[n] = nnz)", row);
      case kBadColumn:
        return fail(SKM_ERR_INVALID_ARG, "row %lld has a column id outside [0, d)", row);
      case kBadOrder:
        return fail(SKM_ERR_INVALID_ARG, "row %lld: column ids are not strictly ascending", row);
      default:
        return fail(SKM_ERR_INVALID_ARG, "row %lld holds a NaN or infinite value", row);
    }
  }
  return SKM_OK;
}

// validate >= 1: every initial centre has unit norm within tol (norms as
// computed by k_init_centres into `initnorm`).
int check_init_norms(const double* initnorm, int32_t k, double tol, hipStream_t s) {
  std::vector<double> hn((size_t)k);
  hipError_t e = hipMemcpyAsync(hn.data(), initnorm, (size_t)k * sizeof(double),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(SKM_ERR_HIP, "validation copy: %s", hipGetErrorString(e));
  for (int j = 0; j < k; ++j)
    if (!(std::fabs(hn[(size_t)j] - 1.0) <= tol))
      return fail(SKM_ERR_NOT_NORMALIZED, "initial centre %d has norm %.9g", j, hn[(size_t)j]);
  return SKM_OK;
}

// An FP32 centre copy above this size does not fit the 256 MB last-level
// cache; a 256-centre slice of it does (measured: 1.38 times faster than
// whole rows at a 410 MB copy, 10^6 rows of ~150 entries, k = 1000).
constexpr double kChunkAlwaysBytes = 256.0 * 1024.0 * 1024.0;
// Lloyd and Hamerly fits whose copy is at least this size (and below the one
// above) time slices against the table's whole rows in their first steps:
// the table was measured on 10,000-column copies (20 MB at 512 centres),
// and a 97 MB copy (47,236 columns, 512 centres) walked 1.02-1.10 times
// faster in slices, the more so on topic-structured rows.
constexpr double kTimedSliceBytes = 64.0 * 1024.0 * 1024.0;

// Row-length class of the tuning tables: the first class whose bound on the
// mean stored entries per row exceeds this matrix's mean, else the last.
int row_class(int64_t n, int64_t nnz) {
  int rc = 0;
  while (rc < kWalkTuneRowClasses - 1 && (double)nnz >= (double)kWalkTuneRowBound[rc] * (double)n)
    ++rc;
  return rc;
}

// Whether a fit's FP32 row walk takes 256 centres per launch (chunk_walk 1)
// or whole rows (2); 0: always sliced when the copy exceeds the last-level
// cache, else the measured table's entry for the variant's family (0 Lloyd
// and Hamerly, 1 Elkan, 2 Yin-Yang), the row-length class and the width.
bool chunk_fp32(int32_t chunk_walk, int family, int64_t n, int64_t d, int64_t nnz, int kp) {
  if (kp < kChunkF32) return false;
  // one slice of 256: Elkan and Yin-Yang on request, so that the walk visits
  // only the centres whose bounds fail (a whole-row walk visits all of a row's
  // centres once any pair survives); faster where the bounds prune most pairs
  if (kp == kChunkF32) return family != 0 && chunk_walk == 1;
  if (chunk_walk == 1) return true;
  if (chunk_walk == 2) return false;
  if ((double)d * (double)kp * 4.0 > kChunkAlwaysBytes) return true;
  int c = 0;
  while ((512 << c) < kp) ++c;
  return kChunkTune[family][row_class(n, nnz)][c < kChunkTuneWidths ? c : kChunkTuneWidths - 1] !=
         0;
}

int make_plan(const skm_matrix* X, int32_t k, int32_t variant, int32_t precision, Plan* P,
              int32_t chunk_walk = 0) {
  int rc = check_matrix(X);
  if (rc != SKM_OK) return rc;
  if (precision != 0 && precision != 2)
    return fail(SKM_ERR_UNSUPPORTED, "CSR input supports precision 0 (FP32) or 2 (FP16 centre "
                "copy), got %d", (int)precision);
  if (k < 1 || (int64_t)k > X->n) return fail(SKM_ERR_INVALID_ARG, "need 1 <= k <= n");
  if (variant < SKM_LLOYD || variant > SKM_YINYANG)
    return fail(SKM_ERR_INVALID_ARG, "unknown variant %d", (int)variant);
  const Geometry g = pick_geometry(k);
  if (g.G == 0) return fail(SKM_ERR_UNSUPPORTED, "k = %d exceeds the supported 4096", (int)k);
  rc = check_ct_size(X->d, g.kp);
  if (rc != SKM_OK) return rc;
  P->n = X->n;
  P->d = X->d;
  P->nnz = X->nnz;
  P->k = k;
  P->kp = g.kp;
  P->variant = variant;
  P->elkan = variant == SKM_ELKAN || variant == SKM_SIMP_ELKAN;
  P->yy = variant == SKM_YINYANG;
  P->ng = (k + kYYGroup - 1) / kYYGroup;
  P->bounds = variant != SKM_LLOYD;
  P->gram = variant == SKM_ELKAN || variant == SKM_HAMERLY;
  P->nchunk = (int)((X->d + 4095) / 4096);
  gram_slicing(k, X->d, &P->nslice, &P->slice_len);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += align256(bytes);
    return o;
  };
  const size_t n = (size_t)X->n, d = (size_t)X->d, kk = (size_t)k;
  P->CT = take(d * (size_t)g.kp * sizeof(float));
  // the FP16 copy pays where the row walk is gather-bound (kp >= 128)
  P->half = precision == 2 && g.kp >= 128;
  if (P->half) P->CT16 = take(d * (size_t)g.kp * 2);
  P->negflag = take(sizeof(int32_t));
  P->C64 = take(kk * d * sizeof(double));
  P->S = take(kk * d * sizeof(long long));
  P->eta = take(n * sizeof(float));
  P->a_old = take(n * sizeof(int32_t));
  if (P->bounds) {
    P->l = take(n * sizeof(float));
    if (!P->elkan && !P->yy) P->u = take(n * sizeof(float));
  }
  if (P->elkan) P->ue = take(n * (size_t)g.kp * sizeof(float));
  if (P->yy) {
    P->uy = take(n * (size_t)P->ng * sizeof(float));
    P->gpc = take((size_t)P->ng * sizeof(double));
    P->gps = take((size_t)P->ng * sizeof(double));
  }
  P->norm64 = take(kk * sizeof(double));
  P->part = take(kk * (size_t)P->nchunk * sizeof(double));
  P->part_sq = take(kk * (size_t)P->nchunk * sizeof(double));
  P->pc = take(kk * sizeof(double));
  P->ps = take(kk * sizeof(double));
  P->dirty = take(kk * sizeof(int32_t));
  P->mm = take(sizeof(MoveMin));
  if (P->gram) {
    P->G = take(kk * kk * sizeof(double));
    P->gmax = take(kk * sizeof(double));
    P->gpart = take((size_t)P->nslice * kk * kk * sizeof(double));
  }
  // counter slots of a chunk of steps; the persistent block, the step
  // control and the step records follow each other, so one copy per chunk
  // brings them to the host
  P->cnt = take((size_t)kStepChunk * kCounterSlots * sizeof(Counters));
  P->per = take(sizeof(Persist) + sizeof(StepCtl) + kStepChunk * sizeof(StepRec));
  P->ctl = P->per + sizeof(Persist);
  P->rec = P->ctl + sizeof(StepCtl);
  P->maxeta = take(kCounterSlots * sizeof(float));
  P->initnorm = take(kk * sizeof(double));
  P->vbad = take(sizeof(unsigned long long));
  // A wide FP32 centre copy is walked a chunk of 1 KB per centre row at a
  // time where that pays (chunk_fp32): the walk streams those fastest, a
  // chunk's slice of the copy is at most a quarter of it (k <= 1024), which
  // the last-level cache holds where the whole copy does not, and Elkan and
  // Yin-Yang pack each slice's surviving centres; short rows and
  // cache-resident copies can favour one launch over whole rows instead
  // (the measured table).  Elkan keeps one survival word per row and
  // 256-centre slice.
  if (!P->half && chunk_fp32(chunk_walk, P->elkan ? 1 : P->yy ? 2 : 0, P->n, P->d, P->nnz,
                             g.kp)) {
    P->chunk = kChunkF32;
    P->nq = (k + kChunkF32 - 1) / kChunkF32;
    P->rs = take(n * sizeof(RowRun));
    if (P->elkan) P->umask = take(n * (size_t)(g.kp / kChunkF32) * sizeof(uint64_t));
  } else if (!P->half && chunk_walk == 0 && row_class(P->n, P->nnz) > 0 &&
             ((P->yy && g.kp >= kChunkF32) || (P->elkan && g.kp > kChunkF32) ||
              (!P->yy && !P->elkan && g.kp > kChunkF32 &&
               (double)P->d * (double)g.kp * 4.0 >= kTimedSliceBytes))) {
    // whole rows: a row walk covers every centre of a row with a surviving
    // pair or group, so where the tests leave few per row, packed slices
    // walk far fewer centres (Lloyd and Hamerly: a slice of a large copy
    // stays cached); the fit measures which is faster.  Not for Elkan's one
    // slice at kp = 256 (it gained at most 6% on topical rows and lost up to
    // 7% to its timing steps on plain ones), nor for rows under 20 stored
    // entries (a slice's per-row work outweighs what it saves, and the two
    // timing steps alone cost Yin-Yang 7-13% of a fit).
    P->pack_adapt = true;
    P->pack_all = !P->yy && !P->elkan;
    P->nq = (k + kChunkF32 - 1) / kChunkF32;
    P->rs = take(n * sizeof(RowRun));
    if (P->elkan) P->umask = take(n * (size_t)(g.kp / kChunkF32) * sizeof(uint64_t));
  }
  // Yin-Yang and Elkan with the FP16 copy at k > 512: the steps with tests
  // walk 1 KB of every FP16 centre row per launch, packing each row's
  // surviving groups / units (the plain steps, and Lloyd and Hamerly with
  // the FP16 copy, walk whole rows in one launch: that copy fits the
  // last-level cache)
  if ((P->yy || P->elkan) && P->half && g.kp > kChunkF16) {
    P->chunk16 = kChunkF16;
    P->nq16 = (k + kChunkF16 - 1) / kChunkF16;
    P->rs = take(n * sizeof(RowRun));
    if (P->elkan) P->umask = take(n * (size_t)(g.kp / kChunkF16) * sizeof(uint64_t));
  }
  P->total = cur;
  return SKM_OK;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// Pinned host mirror of the counter slots and the persistent block, one
// per host thread.
struct HostMirror {
  Counters slots[kCounterSlots];
  Persist per;
  StepCtl ctl;
  StepRec rec[kStepChunk];
};
static_assert(offsetof(HostMirror, per) == kCounterSlots * sizeof(Counters) &&
                  offsetof(HostMirror, ctl) == offsetof(HostMirror, per) + sizeof(Persist) &&
                  offsetof(HostMirror, rec) == offsetof(HostMirror, ctl) + sizeof(StepCtl),
              "host mirror must match the device layout");

thread_local HostMirror* t_mirror = nullptr;

HostMirror* host_mirror() {
  if (!t_mirror) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(HostMirror), hipHostMallocDefault) != hipSuccess) return nullptr;
    t_mirror = static_cast<HostMirror*>(p);
  }
  return t_mirror;
}

// Frees this thread's mirror (worker threads call it before they exit).
void release_host_mirror() {
  if (t_mirror) (void)hipHostFree(t_mirror);
  t_mirror = nullptr;
}

// Worker threads of a batched call: the requested count, or min(nprob, 4)
// (four hardware queues per process by default), never more than nprob.
int batch_workers(int32_t workers, int32_t nprob) {
  int w = workers > 0 ? workers : 4;
  if (w > nprob) w = nprob;
  if (w > 64) w = 64;
  return w < 1 ? 1 : w;
}

Counters sum_slots(const HostMirror* h) {
  Counters t{};
  for (int i = 0; i < kCounterSlots; ++i) {
    const Counters& c = h->slots[i];
    t.changed += c.changed;
    t.sims += c.sims;
    t.rechecks += c.rechecks;
    t.tightened += c.tightened;
    t.tight_saved += c.tight_saved;
    t.rows_done += c.rows_done;
    t.nnz_done += c.nnz_done;
  }
  return t;
}

// Fixed-point scale for the member sums: |x_t| <= 1 (unit rows), so
// |S_jt| <= n and n * 2^F stays below 2^61.
double fixed_point_scale(int64_t n) {
  int bits = 0;
  while ((int64_t(1) << bits) <= n) ++bits;
  return std::ldexp(1.0, 61 - bits);
}


// ------------------------------------------------------------------------
// dense rows (MFMA path)
// ------------------------------------------------------------------------
struct DensePlan {
  int64_t n = 0, d = 0;
  int32_t k = 0, kpad = 0, dp = 0;
  bool bf16 = false, bounds = false, gram = false;
  int nchunk = 1, nslice = 1, nb = 1;
  int64_t slice_len = 0;
  int32_t cap = 64;  // candidate slots per flagged row
  size_t Xb = 0, Cp = 0, C64 = 0, S = 0, eta = 0, a_old = 0, l = 0, u = 0, best = 0, best_j = 0,
         second = 0, thr = 0, near = 0, rflag = 0, rows = 0, nlist = 0, nrows = 0, nthr = 0,
         bcnt = 0, boff = 0, cand = 0, cand_n = 0, ccnt = 0, cstart = 0, ccur = 0, perm = 0,
         norm64 = 0, part = 0, part_sq = 0, pc = 0, ps = 0, dirty = 0, mm = 0, G = 0, gmax = 0,
         gpart = 0, cnt = 0, per = 0, maxeta = 0, initnorm = 0, xr = 0, rcmax = 0, vbad = 0,
         total = 0;
};

int make_dense_plan(const skm_matrix* X, int32_t k, int32_t variant, int32_t precision,
                    DensePlan* P) {
  int rc = check_matrix(X);
  if (rc != SKM_OK) return rc;
  if (k < 1 || (int64_t)k > X->n) return fail(SKM_ERR_INVALID_ARG, "need 1 <= k <= n");
  if (variant < SKM_LLOYD || variant > SKM_YINYANG)
    return fail(SKM_ERR_INVALID_ARG, "unknown variant %d", (int)variant);
  if (variant == SKM_ELKAN || variant == SKM_SIMP_ELKAN || variant == SKM_YINYANG)
    return fail(SKM_ERR_UNSUPPORTED, "Elkan and Yin-Yang variants are implemented for CSR "
                "input only");
  if (precision != 0 && precision != 1)
    return fail(SKM_ERR_INVALID_ARG, "precision must be 0 (fp32) or 1 (bf16)");
  P->n = X->n;
  P->d = X->d;
  P->k = k;
  P->kpad = (k + 63) / 64 * 64;
  P->dp = 32;  // MFMA K padded to 32, 64, 128 or 256
  while (P->dp < X->d) P->dp *= 2;
  P->bf16 = precision == 1;
  P->bounds = variant != SKM_LLOYD;
  P->gram = variant == SKM_HAMERLY;
  P->nchunk = (int)((X->d + 4095) / 4096);
  P->nb = compact_blocks(X->n);
  gram_slicing(k, X->d, &P->nslice, &P->slice_len);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += align256(bytes);
    return o;
  };
  const size_t n = (size_t)X->n, d = (size_t)X->d, kk = (size_t)k;
  const size_t es = P->bf16 ? 2 : 4;
  if (P->bf16) {
    P->Xb = take(n * (size_t)P->dp * 2);
    P->xr = take(n * 4);
    P->rcmax = take(kRcSlots * 4);
  }
  P->Cp = take((size_t)P->kpad * P->dp * es);
  P->C64 = take(kk * d * sizeof(double));
  P->S = take(kk * d * sizeof(long long));
  P->eta = take(n * 4);
  P->a_old = take(n * 4);
  if (P->bounds) {
    P->l = take(n * 4);
    P->u = take(n * 4);
    P->rflag = take(n * 4);
    P->rows = take(n * 4);
  }
  P->best = take(n * 4);
  P->best_j = take(n * 4);
  P->second = take(n * 4);
  P->thr = take(n * 4);
  P->near = take(n * 4);
  P->nlist = take(n * 4);
  P->nrows = take(n * 4);
  P->nthr = take(n * 4);
  P->bcnt = take((size_t)P->nb * 4);
  P->boff = take((size_t)P->nb * 4);
  P->cand = take(n * (size_t)P->cap * 4);
  P->cand_n = take(n * 4);
  P->ccnt = take(kk * 4);
  P->cstart = take(kk * 4);
  P->ccur = take(kk * 4);
  P->perm = take(n * 4);
  P->norm64 = take(kk * 8);
  P->part = take(kk * (size_t)P->nchunk * 8);
  P->part_sq = take(kk * (size_t)P->nchunk * 8);
  P->pc = take(kk * 8);
  P->ps = take(kk * 8);
  P->dirty = take(kk * 4);
  P->mm = take(sizeof(MoveMin));
  if (P->gram) {
    P->G = take(kk * kk * 8);
    P->gmax = take(kk * 8);
    P->gpart = take((size_t)P->nslice * kk * kk * 8);
  }
  P->cnt = take(kCounterSlots * sizeof(Counters) + sizeof(Persist));
  P->per = P->cnt + kCounterSlots * sizeof(Counters);
  P->maxeta = take(kCounterSlots * 4);
  P->initnorm = take(kk * 8);
  P->vbad = take(8);
  P->total = cur;
  return SKM_OK;
}

struct DenseRun {
  const DensePlan& P;
  const skm_matrix* X;
  void* ws;
  hipStream_t s;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // bracket the first similarity pass
  template <typename T>
  T* ptr(size_t off) const {
    return at<T>(ws, off);
  }
};

// One assignment step over dense rows: similarity pass on MFMA (all rows, or
// the compacted rows that failed the Hamerly tests), decision, candidate pass
// for the rows inside the error band, FP64 re-decision.
hipError_t dense_step(const DenseRun& R, int32_t* a, int read_prev, const int32_t* rows,
                      const unsigned long long* rows_count, float* best_out, float* second_out,
                      Counters* cnt) {
  const DensePlan& P = R.P;
  const skm_matrix* X = R.X;
  Persist* per = R.ptr<Persist>(P.per);
  hipError_t e;
  DenseSimArgs S1{};
  S1.X = P.bf16 ? (const void*)R.ptr<char>(P.Xb) : (const void*)X->dense;
  S1.ldx = P.bf16 ? P.dp : X->ld;
  S1.C = R.ptr<char>(P.Cp);
  S1.k = P.k;
  S1.kpad = P.kpad;
  S1.dp = P.dp;
  S1.d = (int32_t)P.d;
  S1.rows = rows;
  S1.rows_count = rows_count;
  S1.n_rows = P.n;
  S1.best = R.ptr<float>(P.best);
  S1.best_j = R.ptr<int32_t>(P.best_j);
  S1.second = R.ptr<float>(P.second);
  if (R.ev0 && (e = hipEventRecord(R.ev0, R.s)) != hipSuccess) return e;
  if ((e = launch_dense_sim(S1, P.bf16, 0, R.s)) != hipSuccess) return e;
  if (R.ev1 && (e = hipEventRecord(R.ev1, R.s)) != hipSuccess) return e;
  DensePostArgs Q{};
  Q.rows = rows;
  Q.rows_count = rows_count;
  Q.n_rows = P.n;
  Q.k = P.k;
  Q.dp = P.dp;
  Q.bf16 = P.bf16;
  Q.read_prev = read_prev;
  Q.best = S1.best;
  Q.best_j = S1.best_j;
  Q.second = S1.second;
  Q.eta = R.ptr<float>(P.eta);
  Q.xr = P.bf16 ? R.ptr<float>(P.xr) : nullptr;
  Q.rcmax = P.bf16 ? R.ptr<float>(P.rcmax) : nullptr;
  Q.delta_c = (double)(P.d + 8) * kU64 * 1.01 + 1e-300;
  Q.a = a;
  Q.l = P.bounds ? R.ptr<float>(P.l) : nullptr;
  Q.u = P.bounds ? R.ptr<float>(P.u) : nullptr;
  Q.near = R.ptr<int32_t>(P.near);
  Q.thr = R.ptr<float>(P.thr);
  Q.best_out = best_out;
  Q.second_out = second_out;
  Q.cnt = cnt;
  if ((e = launch_dense_post(Q, R.s)) != hipSuccess) return e;
  // flagged slots -> list (clears their candidate counters)
  if ((e = launch_compact(Q.near, rows_count, P.n, R.ptr<int32_t>(P.bcnt),
                          R.ptr<int32_t>(P.boff), R.ptr<int32_t>(P.nlist), &per->near_total,
                          R.ptr<int32_t>(P.cand_n), R.s)) != hipSuccess)
    return e;
  if ((e = launch_gather_near(R.ptr<int32_t>(P.nlist), &per->near_total, P.n, rows, Q.thr,
                              R.ptr<int32_t>(P.nrows), R.ptr<float>(P.nthr), R.s)) != hipSuccess)
    return e;
  DenseSimArgs S2 = S1;
  S2.rows = R.ptr<int32_t>(P.nrows);
  S2.rows_count = &per->near_total;
  S2.thr = R.ptr<float>(P.nthr);
  S2.cand = R.ptr<int32_t>(P.cand);
  S2.cand_n = R.ptr<int32_t>(P.cand_n);
  S2.cand_cap = P.cap;
  if ((e = launch_dense_sim(S2, P.bf16, 1, R.s)) != hipSuccess) return e;
  DenseExactArgs E{};
  E.X = X->dense;
  E.ldx = X->ld;
  E.C64 = R.ptr<double>(P.C64);
  E.k = P.k;
  E.d = (int32_t)P.d;
  E.dp = P.dp;
  E.bf16 = P.bf16;
  E.read_prev = read_prev;
  E.rows = rows;
  E.near_list = R.ptr<int32_t>(P.nlist);
  E.near_count = &per->near_total;
  E.cand = S2.cand;
  E.cand_n = S2.cand_n;
  E.cand_cap = P.cap;
  E.best = S1.best;
  E.best_j = S1.best_j;
  E.eta = Q.eta;
  E.xr = Q.xr;
  E.rcmax = Q.rcmax;
  E.delta_c = Q.delta_c;
  E.a = a;
  E.l = Q.l;
  E.u = Q.u;
  E.best_out = best_out;
  E.second_out = second_out;
  E.cnt = cnt;
  return launch_dense_exact(E, P.n, R.s);
}

int fit_dense(const skm_matrix* X, int32_t k, const float* init_centers, int32_t variant,
              int32_t max_iter, const skm_options& o, void* workspace, size_t workspace_bytes,
              int32_t* assign_out, float* centers_out, double* centers64_out, skm_stats* stats,
              hipStream_t s) {
  DensePlan P;
  int rc = make_dense_plan(X, k, variant, o.precision, &P);
  if (rc != SKM_OK) return rc;
  const bool warm = o.warm_assign != nullptr;  // the three warm arrays go together
  if (workspace && workspace_bytes < P.total)
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                P.total);
  HostMirror* hm = host_mirror();
  if (!hm) return fail(SKM_ERR_HIP, "could not allocate pinned host memory");
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, P.total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", P.total);
    owned = true;
  }
  DenseRun R{P, X, ws, s};
  const int64_t n = P.n, d = P.d;
  const double delta_c = (double)(d + 8) * kU64 * 1.01 + 1e-300;
  // Gram entries on FP64 matrix cores: unit 2^-52 also covers accumulation
  // that truncates
  const double delta_g = (double)(d + 2) * 2.0 * kU64 * 1.01 + 2.0 * delta_c + 1e-15;
  const double fx = fixed_point_scale(n);
  const double fx_inv = 1.0 / fx;
  double* C64 = R.ptr<double>(P.C64);
  long long* S = R.ptr<long long>(P.S);
  int32_t* a_old = R.ptr<int32_t>(P.a_old);
  int32_t* dirty = R.ptr<int32_t>(P.dirty);
  Counters* cnt = R.ptr<Counters>(P.cnt);
  Persist* per = R.ptr<Persist>(P.per);
  double* part = R.ptr<double>(P.part);
  double* part_sq = R.ptr<double>(P.part_sq);
  double* norm64 = R.ptr<double>(P.norm64);
  double* pc = R.ptr<double>(P.pc);
  double* ps = R.ptr<double>(P.ps);
  MoveMin* mm = R.ptr<MoveMin>(P.mm);
  double* G = P.gram ? R.ptr<double>(P.G) : nullptr;
  double* gmax = P.gram ? R.ptr<double>(P.gmax) : nullptr;
  double* gpart = P.gram ? R.ptr<double>(P.gpart) : nullptr;
  void* Cp = R.ptr<char>(P.Cp);
  int32_t iterations = 0, converged = 0;
  int64_t tot_sims = 0, tot_rechecks = 0, sk_launches = 0, sk_rows = 0;
  double objective = 0.0, sk_ms = 0.0, tight_rate = 1.0;
  bool first_gram = true, gram_stale = false;
  int gram_updates = 0, gram_since_exact = 0;
  // The bound tests switch off while they do not pay; results are the same
  // either way, since a step without tests is an exhaustive step that sets l
  // and u afresh.  After a tested step that prunes fewer than
  // kDenseTestMin of the rows, the next off_gap steps run exhaustively, the
  // gap doubling from 2 up to 64 while tests keep failing (schedule = 1:
  // tests at every step, as the paper runs them).
  constexpr double kDenseTestMin = 0.15;
  int32_t off_until = 0, off_gap = 2;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  {
    if (o.validate >= 2) {
      rc = validate_input(X, R.ptr<unsigned long long>(P.vbad), s);
      if (rc != SKM_OK) goto done;
    }
    if (o.profile) {
      SKM_HIP(hipEventCreate(&ev0));
      SKM_HIP(hipEventCreate(&ev1));
    }
    SKM_HIP(hipMemsetAsync(Cp, 0, (size_t)P.kpad * P.dp * (P.bf16 ? 2 : 4), s));
    SKM_HIP(hipMemsetAsync(per, 0, sizeof(Persist), s));
    SKM_HIP(hipMemsetAsync(dirty, 0, (size_t)k * 4, s));
    SKM_HIP(hipMemsetAsync(norm64, 0, (size_t)k * 8, s));
    SKM_HIP(hipMemsetAsync(R.ptr<float>(P.maxeta), 0, kCounterSlots * 4, s));
    SKM_HIP(launch_fill_i32(a_old, n, -1, s));
    float* rcmax = P.bf16 ? R.ptr<float>(P.rcmax) : nullptr;
    if (rcmax) SKM_HIP(hipMemsetAsync(rcmax, 0, kRcSlots * 4, s));
    SKM_HIP(launch_dense_prep(X->dense, X->ld, n, d, P.dp, R.ptr<float>(P.eta),
                              R.ptr<float>(P.maxeta), P.bf16 ? R.ptr<char>(P.Xb) : nullptr,
                              P.bf16 ? R.ptr<float>(P.xr) : nullptr, s));
    SKM_HIP(launch_init_centres(init_centers, k, d, 1, C64, R.ptr<double>(P.initnorm), s));
    SKM_HIP(launch_pack_centres(C64, k, d, P.dp, nullptr, P.bf16, Cp, rcmax, s));
    if (o.validate >= 1) {
      rc = check_init_norms(R.ptr<double>(P.initnorm), k, o.norm_tol, s);
      if (rc != SKM_OK) goto done;
      float hslots[kCounterSlots];
      float hmax = 0.f;
      SKM_HIP(hipMemcpyAsync(hslots, R.ptr<float>(P.maxeta), sizeof(hslots),
                             hipMemcpyDeviceToHost, s));
      SKM_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < kCounterSlots; ++q) hmax = std::max(hmax, hslots[q]);
      if (o.validate >= 2 && !((double)hmax <= o.norm_tol)) {
        rc = fail(SKM_ERR_NOT_NORMALIZED, "a data row deviates from unit norm by %.3g", hmax);
        goto done;
      }
    }
    // centre step after assignment step t (changed rows moved): recompute all
    // sums when many rows moved, else apply the moved rows (both give the
    // same fixed-point sums); movement, packed copy, Gram, clear dirty flags
    auto centre_step = [&](int32_t t, int64_t changed) -> hipError_t {
      hipError_t e;
      if (t == 0 || changed * 32 > n) {
        if ((e = launch_cluster_sums(assign_out, n, k, X->dense, X->ld, d, fx,
                                     R.ptr<int32_t>(P.ccnt), R.ptr<int32_t>(P.cstart),
                                     R.ptr<int32_t>(P.ccur), R.ptr<int32_t>(P.perm), S, dirty,
                                     &per->scan_dummy, s)) != hipSuccess)
          return e;
        if ((e = launch_copy_assign(assign_out, a_old, n, s)) != hipSuccess) return e;
      } else {
        if ((e = launch_dense_update_scan(X->dense, X->ld, assign_out, a_old, n, d, fx, S, dirty,
                                          s)) != hipSuccess)
          return e;
      }
      if ((e = launch_sumsq_partial(S, k, d, fx_inv, dirty, part_sq, P.nchunk, s)) != hipSuccess)
        return e;
      if ((e = launch_normalize_move(S, k, d, fx_inv, dirty, part_sq, C64, part, P.nchunk, s)) !=
          hipSuccess)
        return e;
      if ((e = launch_centre_finalize(k, d, dirty, norm64, part_sq, part, P.nchunk, delta_c, pc,
                                      ps, mm, per, s)) != hipSuccess)
        return e;
      if ((e = launch_pack_centres(C64, k, d, P.dp, dirty, P.bf16, Cp,
                                   P.bf16 ? R.ptr<float>(P.rcmax) : nullptr, s)) != hipSuccess)
        return e;
      if (P.gram) {
        if (t + 1 < off_until) {
          gram_stale = true;  // no tests next step: the Gram waits for one that has them
        } else if (gram_stale || gram_exact_step(gram_updates, gram_since_exact, changed, n)) {
          // after carried or skipped steps every tile's partials are stale
          if ((e = launch_gram(C64, k, d, dirty,
                               (first_gram || gram_since_exact > 0 || gram_stale) ? 1 : 0, gpart,
                               P.nslice, P.slice_len, G, gmax, delta_g, per, s)) != hipSuccess)
            return e;
          first_gram = false;
          gram_stale = false;
          gram_since_exact = 0;
          ++gram_updates;
        } else {
          if ((e = launch_gram_carry(G, k, pc, ps, delta_g, gmax, s)) != hipSuccess) return e;
          ++gram_since_exact;
          ++gram_updates;
        }
      }
      return launch_clear_dirty(dirty, k, s);
    };
    int32_t t_first = 0;
    if (warm) {
      // the first step's assignment and FP64 top-2 are given (a seeding's
      // cache): bounds only, then the centre step
      SKM_HIP(launch_warm_start(nullptr, n, k, 0, o.warm_assign, o.warm_best, o.warm_second,
                                R.ptr<float>(P.eta), delta_c, assign_out,
                                P.bounds ? R.ptr<float>(P.l) : nullptr,
                                P.bounds ? R.ptr<float>(P.u) : nullptr, nullptr, nullptr, 0, s,
                                d));
      if (stats && stats->changed_per_iter && stats->per_iter_len > 0)
        stats->changed_per_iter[0] = n;
      if (stats && stats->sims_per_iter && stats->per_iter_len > 0) stats->sims_per_iter[0] = 0;
      iterations = 1;
      SKM_HIP(centre_step(0, n));
      t_first = 1;
    }
    for (int32_t t = t_first; t < max_iter; ++t) {
      SKM_HIP(hipMemsetAsync(cnt, 0, kCounterSlots * sizeof(Counters), s));
      const bool exhaustive = t == 0 || variant == SKM_LLOYD || t < off_until;
      const int32_t* rows = nullptr;
      const unsigned long long* rows_count = nullptr;
      if (!exhaustive) {
        DenseHamerlyArgs H{};
        H.X = X->dense;
        H.ldx = X->ld;
        H.C64 = C64;
        H.k = k;
        H.d = (int32_t)d;
        H.n = n;
        H.a = assign_out;
        H.l = R.ptr<float>(P.l);
        H.u = R.ptr<float>(P.u);
        H.eta = R.ptr<float>(P.eta);
        H.pc = pc;
        H.ps = ps;
        H.mm = mm;
        H.gmax = gmax;
        H.delta_c = delta_c;
        H.simplified = variant == SKM_SIMP_HAMERLY;
        H.bound_form = o.bound_form;
        H.try_tighten = (t <= 2 || tight_rate >= 0.2 || t % 4 == 0) ? 1 : 0;
        H.flag = R.ptr<int32_t>(P.rflag);
        H.cnt = cnt;
        SKM_HIP(launch_dense_hamerly(H, s));
        SKM_HIP(launch_compact(H.flag, nullptr, n, R.ptr<int32_t>(P.bcnt), R.ptr<int32_t>(P.boff),
                               R.ptr<int32_t>(P.rows), &per->list_total, nullptr, s));
        rows = R.ptr<int32_t>(P.rows);
        rows_count = &per->list_total;
      }
      R.ev0 = ev0;
      R.ev1 = ev1;
      SKM_HIP(dense_step(R, assign_out, t > 0 ? 1 : 0, rows, rows_count, nullptr, nullptr, cnt));
      R.ev0 = R.ev1 = nullptr;
      SKM_HIP(hipMemcpyAsync(hm, cnt, offsetof(HostMirror, ctl), hipMemcpyDeviceToHost, s));
      SKM_HIP(hipStreamSynchronize(s));
      const Counters tc = sum_slots(hm);
      const int64_t changed = (int64_t)tc.changed;
      const int64_t walked = exhaustive ? n : (int64_t)hm->per.list_total;
      if (!exhaustive && o.schedule == 0) {
        if ((double)(n - walked) < kDenseTestMin * (double)n) {
          off_until = t + 1 + off_gap;
          off_gap = std::min(off_gap * 2, 64);
        } else {
          off_gap = 2;
        }
      }
      if (ev0) {
        float ms = 0.f;
        SKM_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        sk_ms += ms;
      }
      if (tc.tightened > 0) tight_rate = (double)tc.tight_saved / (double)tc.tightened;
      const int64_t step_sims = walked * (int64_t)k + (int64_t)tc.sims;
      sk_launches += 1;
      sk_rows += walked;
      tot_sims += step_sims;
      tot_rechecks += (int64_t)tc.rechecks;
      if (t > 0) objective = hm->per.objective;
      if (stats && t < stats->per_iter_len) {
        if (stats->changed_per_iter) stats->changed_per_iter[t] = changed;
        if (stats->sims_per_iter) stats->sims_per_iter[t] = step_sims;
        if (stats->objective_per_iter && t > 0 && t - 1 < stats->per_iter_len)
          stats->objective_per_iter[t - 1] = hm->per.objective;
      }
      iterations = t + 1;
      if (changed == 0) {
        converged = 1;
        break;
      }
      SKM_HIP(centre_step(t, changed));
      SKM_HIP(launch_clear_dirty(dirty, k, s));
    }
    SKM_HIP(hipMemcpyAsync(&hm->per, per, sizeof(Persist), hipMemcpyDeviceToHost, s));
    if (centers_out) SKM_HIP(launch_c64_to_f32(C64, (int64_t)k * d, centers_out, s));
    if (centers64_out)
      SKM_HIP(hipMemcpyAsync(centers64_out, C64, (size_t)k * d * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    SKM_HIP(hipStreamSynchronize(s));
    objective = hm->per.objective;
    if (stats) {
      stats->iterations = iterations;
      stats->converged = converged;
      stats->objective = objective;
      stats->sims_point_center = tot_sims;
      stats->sims_center_center = (int64_t)hm->per.ccsims;
      stats->rechecks = tot_rechecks;
      if (stats->objective_per_iter && iterations - 1 < stats->per_iter_len)
        stats->objective_per_iter[iterations - 1] = objective;
      stats->sim_kernel_launches = sk_launches;
      stats->sim_kernel_rows = sk_rows;
      stats->sim_kernel_nnz = sk_rows * d;
      stats->sim_kernel_ms = sk_ms;
    }
  }
done:
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (owned) {
    (void)hipFreeAsync(ws, s);
    if (rc == SKM_OK) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = fail(SKM_ERR_HIP, "final synchronise: %s", hipGetErrorString(e));
    }
  }
  return rc;
}


int assign_dense(const skm_matrix* X, int32_t k, const float* centers, int32_t* assign_out,
                 float* best_out, float* second_out, void* workspace, size_t workspace_bytes,
                 hipStream_t s) {
  DensePlan P;
  int rc = make_dense_plan(X, k, SKM_LLOYD, 0, &P);
  if (rc != SKM_OK) return rc;
  if (workspace && workspace_bytes < P.total)
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                P.total);
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, P.total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", P.total);
    owned = true;
  }
  DenseRun R{P, X, ws, s};
  {
    void* Cp = R.ptr<char>(P.Cp);
    double* C64 = R.ptr<double>(P.C64);
    SKM_HIP(hipMemsetAsync(Cp, 0, (size_t)P.kpad * P.dp * 4, s));
    SKM_HIP(hipMemsetAsync(R.ptr<Persist>(P.per), 0, sizeof(Persist), s));
    SKM_HIP(hipMemsetAsync(R.ptr<Counters>(P.cnt), 0, kCounterSlots * sizeof(Counters), s));
    SKM_HIP(launch_dense_prep(X->dense, X->ld, P.n, P.d, P.dp, R.ptr<float>(P.eta), nullptr,
                              nullptr, nullptr, s));
    SKM_HIP(launch_init_centres(centers, k, P.d, 0, C64, nullptr, s));
    SKM_HIP(launch_pack_centres(C64, k, P.d, P.dp, nullptr, 0, Cp, nullptr, s));
    SKM_HIP(dense_step(R, assign_out, 0, nullptr, nullptr, best_out, second_out,
                       R.ptr<Counters>(P.cnt)));
  }
done:
  if (owned) (void)hipFreeAsync(ws, s);
  return rc;
}

// Device address of `scratch` on the device of `stream` (the current device
// for the null stream), looked up once per device with that device current
// and kept for later calls.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

int scratch_address(hipStream_t stream, void** out) {
  int cur = 0, dev = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess) {
    dev = cur;
    if (stream) e = hipStreamGetDevice(stream, &dev);
  }
  if (e != hipSuccess) return fail(SKM_ERR_HIP, "device of the stream: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SKM_ERR_UNSUPPORTED, "device %d beyond the %d this library tracks", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess)
      return fail(SKM_ERR_HIP, "hipSetDevice(%d): %s", dev, hipGetErrorString(e));
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(SKM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return SKM_OK;
}

// Assignment step of CSR rows against fixed centres, in the workspace `ws`
// (centre-minor FP32 copy, then the FP64 centres).  Only kernels are
// enqueued (the copy is cleared by a fill kernel), so the same path serves
// callers that capture the stream into a graph.
int assign_csr(const skm_matrix* X, int32_t k, int32_t kp, const float* centers,
               int32_t* assign_out, float* best_sim_out, float* second_sim_out, void* ws,
               hipStream_t s) {
  int rc = SKM_OK;
  float* CT = at<float>(ws, 0);
  double* C64 = at<double>(ws, align256((size_t)X->d * kp * sizeof(float)));
  {
    SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(CT), X->d * (int64_t)kp, 0, s));
    SKM_HIP(launch_init_centres(centers, k, X->d, 0, C64, nullptr, s));
    SKM_HIP(launch_transpose(C64, k, X->d, kp, nullptr, CT, s));
    AssignArgs A{};
    A.rp = X->row_ptr;
    A.ci = X->col_idx;
    A.v = X->val;
    A.CT = CT;
    A.C64 = C64;
    A.d = X->d;
    A.k = k;
    A.kp = kp;
    A.n_rows = X->n;
    A.a = assign_out;
    A.read_prev = 0;
    A.best_out = best_sim_out;
    A.second_out = second_sim_out;
    SKM_HIP(launch_assign(A, kModeAssign, s));
  }
done:
  return rc;
}

// ------------------------------------------------------------------------
// Batched fits in lockstep: every problem of the batch advances one
// assignment step at a time and each kernel of a step serves all problems
// (work items name the problem): the row walk runs as one persistent launch
// per centre-copy width over a queue of (problem, row tile) items, the centre
// step as one launch per kernel.  Steps after the first are queued eight at
// a time from one captured HIP graph (kernels only: counters and queues are
// cleared by fill kernels), replayed until every problem has stopped.  The
// kernels are the single-problem ones, so every problem's result and
// statistics equal those of its own skm_fit.
// ------------------------------------------------------------------------
constexpr int kArgSlots = 1 + 2 * kStepChunk;  // step 0, then (tested, plain) per slot
constexpr int kWidthClasses = 9;              // kp = 16 ... 4096
constexpr int kCtlBytes = 1024;               // Persist + StepCtl + kStepChunk StepRec
static_assert(sizeof(Persist) + sizeof(StepCtl) + kStepChunk * sizeof(StepRec) <= kCtlBytes,
              "control block");

// Row-walk layout of a fit's FP32 plain and Hamerly walks: forced by
// walk_layout (1 default, 2 alternative), else the measured table's entry
// for the padded width and the mean row length.
int32_t walk_layout_for(const skm_options& o, int32_t kp, int64_t n, int64_t nnz) {
  if (o.walk_layout != 0) return o.walk_layout - 1;
  int c = 0;
  while ((16 << c) < kp) ++c;
  if (c >= kWalkTuneWidths) return 0;
  return kWalkTune[row_class(n, nnz)][c];
}

int width_class(int kp) {
  int c = 0;
  while ((16 << c) < kp) ++c;
  return c;
}

// The lockstep path is switched off: its first GPU test did not finish
// (killed after 180 s without progress) and the cause has not been found
// yet, so every batched call takes the host-thread path.
constexpr bool kLockstepEnabled = false;

bool lockstep_eligible(int32_t nprob, const skm_matrix* Xs, int32_t variant,
                       const skm_options& o) {
  if (!kLockstepEnabled) return false;
  if (variant != SKM_LLOYD && variant != SKM_HAMERLY && variant != SKM_SIMP_HAMERLY)
    return false;
  if (o.precision != 0 || o.validate != 0 || o.profile != 0 || o.warm_assign) return false;
  for (int32_t b = 0; b < nprob; ++b)
    if (Xs[b].fmt != SKM_CSR_F32) return false;
  return true;
}

struct Lockstep {
  std::vector<Plan> plans;
  std::vector<size_t> base;     // start of each problem's region
  size_t views = 0, args = 0, ctl = 0, cnt = 0, queues = 0, items = 0, total = 0;
  size_t cnt_bytes = 0, queue_count = 0;
  // items (host copies, laid out back to back at `items`)
  std::vector<int2> rows256, centres, walk[kWidthClasses];
  std::vector<int4> tiles, pairs;
  size_t off_rows256 = 0, off_centres = 0, off_walk[kWidthClasses] = {}, off_tiles = 0,
         off_pairs = 0, items_bytes = 0;
  int tile_rows[kWidthClasses] = {};
};

int plan_lockstep(int32_t nprob, const skm_matrix* Xs, const int32_t* ks, int32_t variant,
                  const skm_options& o, Lockstep* L) {
  L->plans.resize((size_t)nprob);
  L->base.resize((size_t)nprob);
  size_t cur = 0;
  for (int32_t b = 0; b < nprob; ++b) {
    const int rc = make_plan(&Xs[b], ks[b], variant, 0, &L->plans[(size_t)b]);
    if (rc != SKM_OK) {
      const std::string m = g_last_error;
      return fail(rc, "problem %d: %s", (int)b, m.c_str());
    }
    L->base[(size_t)b] = cur;
    cur += align256(L->plans[(size_t)b].total);
  }
  const size_t np = (size_t)nprob;
  L->views = cur;
  cur += align256(np * sizeof(FitView));
  L->args = cur;
  cur += align256(np * kArgSlots * sizeof(AssignArgs));
  L->ctl = cur;
  cur += align256(np * kCtlBytes);
  L->cnt = cur;
  L->cnt_bytes = np * kStepChunk * kCounterSlots * sizeof(Counters);
  cur += align256(L->cnt_bytes);
  // queue counters, per width and gate: step 0, then every chunk slot
  L->queue_count = (size_t)(1 + kStepChunk) * kWidthClasses * 2;
  L->queues = cur;
  cur += align256(L->queue_count * sizeof(unsigned int));
  // work items, most expensive problems first within every list
  std::vector<int32_t> order((size_t)nprob);
  for (int32_t b = 0; b < nprob; ++b) order[(size_t)b] = b;
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const double cx = (double)Xs[x].nnz * ks[x], cy = (double)Xs[y].nnz * ks[y];
    return cx != cy ? cx > cy : x < y;
  });
  for (int c = 0; c < kWidthClasses; ++c)
    L->tile_rows[c] = o.batch_tile_rows > 0 ? o.batch_tile_rows : kBatchTileRows[c];
  for (int32_t b : order) {
    const Plan& P = L->plans[(size_t)b];
    const int wc = width_class(P.kp);
    for (int64_t r = 0; r < P.n; r += L->tile_rows[wc]) L->walk[wc].push_back({b, (int)r});
    for (int64_t r = 0; r < P.n; r += kBlock) L->rows256.push_back({b, (int)r});
    for (int32_t j = 0; j < P.k; ++j) L->centres.push_back({b, j});
    const int64_t ntt = (P.d + 63) / 64;
    for (int jt = 0; jt * 64 < P.k; ++jt)
      for (int64_t tg = 0; tg < ntt; tg += kTransposeGroup) L->tiles.push_back({b, jt, (int)tg, 0});
    if (P.gram) {
      const int nt = (P.k + 63) / 64;
      for (int pr = 0; pr < nt * (nt + 1) / 2; ++pr)
        for (int sl = 0; sl < P.nslice; ++sl) L->pairs.push_back({b, pr, sl, 0});
    }
  }
  size_t ic = 0;
  auto put = [&](size_t bytes) {
    const size_t o2 = ic;
    ic += align256(bytes);
    return o2;
  };
  L->off_rows256 = put(L->rows256.size() * sizeof(int2));
  L->off_centres = put(L->centres.size() * sizeof(int2));
  for (int c = 0; c < kWidthClasses; ++c) L->off_walk[c] = put(L->walk[c].size() * sizeof(int2));
  L->off_tiles = put(L->tiles.size() * sizeof(int4));
  L->off_pairs = put(L->pairs.size() * sizeof(int4));
  L->items_bytes = ic;
  L->items = cur;
  cur += align256(ic);
  L->total = cur;
  for (int c = 0; c < kWidthClasses; ++c)
    if (L->walk[c].size() > (size_t)INT32_MAX) return fail(SKM_ERR_UNSUPPORTED, "too many tiles");
  return SKM_OK;
}

int fit_batched_lockstep(int32_t nprob, const skm_matrix* Xs, const int32_t* ks,
                         const float* const* inits, int32_t variant, const int32_t* max_iters,
                         const skm_options& o, void* ws, const Lockstep& L,
                         int32_t* const* assign_outs, float* const* centers_outs,
                         skm_stats* stats, hipStream_t s) {
  int rc = SKM_OK;
  const size_t np = (size_t)nprob;
  const bool gram = variant == SKM_HAMERLY;
  const bool lloyd = variant == SKM_LLOYD;
  char* W = static_cast<char*>(ws);
  FitView* dV = reinterpret_cast<FitView*>(W + L.views);
  AssignArgs* dA = reinterpret_cast<AssignArgs*>(W + L.args);
  char* dctl = W + L.ctl;
  Counters* dcnt = reinterpret_cast<Counters*>(W + L.cnt);
  unsigned int* dq = reinterpret_cast<unsigned int*>(W + L.queues);
  char* ditems = W + L.items;
  const int2* d_rows256 = reinterpret_cast<const int2*>(ditems + L.off_rows256);
  const int2* d_centres = reinterpret_cast<const int2*>(ditems + L.off_centres);
  const int4* d_tiles = reinterpret_cast<const int4*>(ditems + L.off_tiles);
  const int4* d_pairs = reinterpret_cast<const int4*>(ditems + L.off_pairs);
  const int n_rows256 = (int)L.rows256.size(), n_centres = (int)L.centres.size(),
            n_tiles = (int)L.tiles.size(), n_pairs = (int)L.pairs.size();

  // host images of the views, walk arguments and items
  std::vector<FitView> hV(np);
  std::vector<AssignArgs> hA(np * kArgSlots);
  std::vector<char> hitems(L.items_bytes);
  for (size_t b = 0; b < np; ++b) {
    const Plan& P = L.plans[b];
    void* base = W + L.base[b];
    FitView& f = hV[b];
    f = FitView{};
    f.rp = Xs[b].row_ptr;
    f.ci = Xs[b].col_idx;
    f.v = Xs[b].val;
    f.n = P.n;
    f.d = P.d;
    f.k = P.k;
    f.kp = P.kp;
    f.init = inits[b];
    f.CT = at<float>(base, P.CT);
    f.C64 = at<double>(base, P.C64);
    f.S = at<long long>(base, P.S);
    f.eta = at<float>(base, P.eta);
    f.a = assign_outs[b];
    f.a_old = at<int32_t>(base, P.a_old);
    f.norm64 = at<double>(base, P.norm64);
    f.part = at<double>(base, P.part);
    f.part_sq = at<double>(base, P.part_sq);
    f.pc = at<double>(base, P.pc);
    f.ps = at<double>(base, P.ps);
    f.dirty = at<int32_t>(base, P.dirty);
    f.mm = at<MoveMin>(base, P.mm);
    f.G = P.gram ? at<double>(base, P.G) : nullptr;
    f.gmax = P.gram ? at<double>(base, P.gmax) : nullptr;
    f.gpart = P.gram ? at<double>(base, P.gpart) : nullptr;
    f.cnt = dcnt + b * kStepChunk * kCounterSlots;
    f.per = reinterpret_cast<Persist*>(dctl + b * kCtlBytes);
    f.ctl = reinterpret_cast<StepCtl*>(dctl + b * kCtlBytes + sizeof(Persist));
    f.rec = reinterpret_cast<StepRec*>(dctl + b * kCtlBytes + sizeof(Persist) + sizeof(StepCtl));
    f.maxeta = at<float>(base, P.maxeta);
    f.initnorm = at<double>(base, P.initnorm);
    f.nchunk = P.nchunk;
    f.nslice = P.nslice;
    f.slice_len = P.slice_len;
    f.fx = fixed_point_scale(P.n);
    f.fx_inv = 1.0 / f.fx;
    f.delta_c = (double)(P.d + 8) * kU64 * 1.01 + 1e-300;
    f.delta_g = (double)(P.d + 2) * 2.0 * kU64 * 1.01 + 2.0 * f.delta_c + 1e-15;
    // the same test and tightening thresholds as a single fit (FP32 copy)
    const double walk_lines = (double)P.kp * 4.0 / 128.0;
    f.tight_min = std::min(0.9, std::max(0.02, 1.25 / walk_lines));
    f.test_min = std::min(0.2, std::max(0.01, 0.4 / walk_lines));
    if (o.schedule == 1) f.test_min = f.tight_min = -1e300;
    f.gram = P.gram ? 1 : 0;
    f.max_iter = max_iters[b];
    for (int slot = 0; slot < kArgSlots; ++slot) {
      AssignArgs A{};
      A.rp = f.rp;
      A.ci = f.ci;
      A.v = f.v;
      A.CT = f.CT;
      A.negflag = at<int32_t>(base, P.negflag);
      A.C64 = f.C64;
      A.d = P.d;
      A.k = P.k;
      A.kp = P.kp;
      A.n_rows = P.n;
      A.a = f.a;
      A.read_prev = slot > 0 ? 1 : 0;
      A.l = P.bounds ? at<float>(base, P.l) : nullptr;
      A.u = P.bounds ? at<float>(base, P.u) : nullptr;
      A.eta = f.eta;
      A.delta_c = f.delta_c;
      const int c = slot == 0 ? 0 : (slot - 1) / 2;
      A.cnt = f.cnt + (size_t)c * kCounterSlots;
      A.ctl = f.ctl;
      A.pc = f.pc;
      A.ps = f.ps;
      A.mm = f.mm;
      A.gmax = f.gmax;
      A.simplified = variant == SKM_SIMP_HAMERLY;
      A.Gm = f.G;
      A.delta_g = f.delta_g;
      A.bound_form = o.bound_form;
      // step 0 and Lloyd: always (gate 0); else tested (1) / plain (2) twins
      A.gate = (slot == 0 || lloyd) ? 0 : ((slot - 1) % 2 == 0 ? 1 : 2);
      hA[b * kArgSlots + (size_t)slot] = A;
    }
  }
  memcpy(hitems.data() + L.off_rows256, L.rows256.data(), L.rows256.size() * sizeof(int2));
  memcpy(hitems.data() + L.off_centres, L.centres.data(), L.centres.size() * sizeof(int2));
  for (int c = 0; c < kWidthClasses; ++c)
    memcpy(hitems.data() + L.off_walk[c], L.walk[c].data(), L.walk[c].size() * sizeof(int2));
  memcpy(hitems.data() + L.off_tiles, L.tiles.data(), L.tiles.size() * sizeof(int4));
  memcpy(hitems.data() + L.off_pairs, L.pairs.data(), L.pairs.size() * sizeof(int4));

  std::vector<char> hctl(np * kCtlBytes);
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int32_t> iters(np, 0), conv(np, 0);
  std::vector<int64_t> sims(np, 0), rechecks(np, 0), rows(np, 0), nnz(np, 0);
  auto walk_step = [&](int slot_tested, int slot_plain, int qbase, hipStream_t st) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int c = 0; c < kWidthClasses && e == hipSuccess; ++c) {
      const int nit = (int)L.walk[c].size();
      if (nit == 0) continue;
      const int2* it = reinterpret_cast<const int2*>(ditems + L.off_walk[c]);
      const int kp = 16 << c;
      if (slot_tested >= 0)
        e = launch_assign_batched(dA, kArgSlots, slot_tested, it, nit, L.tile_rows[c], kp,
                                  kModeHamerly, dq + qbase + 2 * c, st);
      if (e == hipSuccess)
        e = launch_assign_batched(dA, kArgSlots, slot_plain, it, nit, L.tile_rows[c], kp,
                                  kModeFit, dq + qbase + 2 * c + 1, st);
    }
    return e;
  };
  auto centre_step = [&](hipStream_t st) -> hipError_t {
    hipError_t e;
    if ((e = launch_b_update_scan(dV, d_rows256, n_rows256, st)) != hipSuccess) return e;
    if ((e = launch_b_sumsq(dV, d_centres, n_centres, st)) != hipSuccess) return e;
    if ((e = launch_b_normalize(dV, d_centres, n_centres, st)) != hipSuccess) return e;
    if ((e = launch_b_finalize(dV, nprob, st)) != hipSuccess) return e;
    if ((e = launch_b_transpose(dV, d_tiles, n_tiles, 1, st)) != hipSuccess) return e;
    if (gram) e = launch_b_gram(dV, d_pairs, n_pairs, d_centres, n_centres, st);
    return e;
  };
  // reads every problem's control block and adds the records of the last
  // `steps` steps; returns true while a problem still runs
  auto collect = [&](int steps) -> int {
    hipError_t e = hipMemcpyAsync(hctl.data(), dctl, np * kCtlBytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return -1;
    int running = 0;
    for (size_t b = 0; b < np; ++b) {
      const char* blk = hctl.data() + b * kCtlBytes;
      const StepCtl* c = reinterpret_cast<const StepCtl*>(blk + sizeof(Persist));
      const StepRec* r = reinterpret_cast<const StepRec*>(blk + sizeof(Persist) + sizeof(StepCtl));
      for (int q = 0; q < steps; ++q) {
        if (!r[q].valid) break;
        const int32_t t = iters[b];
        sims[b] += (int64_t)r[q].sims;
        rechecks[b] += (int64_t)r[q].rechecks;
        rows[b] += (int64_t)r[q].rows_done;
        nnz[b] += (int64_t)r[q].nnz_done;
        skm_stats* S = stats ? &stats[b] : nullptr;
        if (S && t < S->per_iter_len) {
          if (S->changed_per_iter) S->changed_per_iter[t] = (int64_t)r[q].changed;
          if (S->sims_per_iter) S->sims_per_iter[t] = (int64_t)r[q].sims;
          if (S->objective_per_iter && t > 0) S->objective_per_iter[t - 1] = r[q].objective;
        }
        iters[b] = t + 1;
      }
      conv[b] = c->stop == 1;
      running += c->stop == 0 ? 1 : 0;
    }
    return running;
  };
  {
    SKM_HIP(hipMemcpyAsync(dV, hV.data(), np * sizeof(FitView), hipMemcpyHostToDevice, s));
    SKM_HIP(hipMemcpyAsync(dA, hA.data(), hA.size() * sizeof(AssignArgs), hipMemcpyHostToDevice,
                           s));
    SKM_HIP(hipMemcpyAsync(ditems, hitems.data(), hitems.size(), hipMemcpyHostToDevice, s));
    // initial state of every problem, as skm_fit sets it up
    for (size_t b = 0; b < np; ++b) {
      const Plan& P = L.plans[b];
      SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(hV[b].CT), P.d * (int64_t)P.kp, 0, s));
      SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(hV[b].S), 2 * P.d * (int64_t)P.k, 0, s));
      SKM_HIP(launch_fill_i32(hV[b].a_old, P.n, -1, s));
      SKM_HIP(launch_fill_i32(hV[b].dirty, P.k, 0, s));
      SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(hV[b].norm64), 2 * (int64_t)P.k, 0, s));
      SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(hV[b].maxeta), kCounterSlots, 0, s));
    }
    SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(dctl), (int64_t)(np * kCtlBytes / 4), 0,
                            s));
    SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(dcnt), (int64_t)(L.cnt_bytes / 4), 0, s));
    SKM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(dq), (int64_t)L.queue_count, 0, s));
    SKM_HIP(launch_b_row_eta(dV, d_rows256, n_rows256, s));
    SKM_HIP(launch_b_init_centres(dV, d_centres, n_centres, s));
    SKM_HIP(launch_b_transpose(dV, d_tiles, n_tiles, 0, s));
    SKM_HIP(launch_b_step_init(dV, nprob, s));
    // step 0: exhaustive for every problem
    SKM_HIP(walk_step(-1, 0, 0, s));
    SKM_HIP(launch_b_step_end(dV, nprob, 0, s));
    SKM_HIP(centre_step(s));
    int running = collect(1);
    if (running < 0) {
      rc = fail(SKM_ERR_HIP, "reading the step records failed");
      goto done;
    }
    if (running > 0) {
      // steps in chunks of kStepChunk from one captured graph
      SKM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      SKM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      {
        hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(dcnt),
                                       (int64_t)(L.cnt_bytes / 4), 0, cs);
        if (e == hipSuccess)
          e = launch_fill_i32(reinterpret_cast<int32_t*>(dq), (int64_t)L.queue_count, 0, cs);
        for (int c = 0; c < kStepChunk && e == hipSuccess; ++c) {
          const int qb = (1 + c) * kWidthClasses * 2;
          e = walk_step(lloyd ? -1 : 1 + 2 * c, lloyd ? 1 + 2 * c : 2 + 2 * c, qb, cs);
          if (e == hipSuccess) e = launch_b_step_end(dV, nprob, c, cs);
          if (e == hipSuccess) e = centre_step(cs);
        }
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        graph = g;
        SKM_HIP(e);
        SKM_HIP(e2);
      }
      SKM_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      int32_t longest = 0;
      for (size_t b = 0; b < np; ++b) longest = std::max(longest, max_iters[b]);
      for (int32_t t0 = 1; t0 < longest && running > 0; t0 += kStepChunk) {
        SKM_HIP(hipGraphLaunch(exec, s));
        running = collect(kStepChunk);
        if (running < 0) {
          rc = fail(SKM_ERR_HIP, "reading the step records failed");
          goto done;
        }
      }
    }
    for (size_t b = 0; b < np; ++b)
      if (centers_outs && centers_outs[b])
        SKM_HIP(launch_c64_to_f32(hV[b].C64, (int64_t)L.plans[b].k * L.plans[b].d,
                                  centers_outs[b], s));
    SKM_HIP(hipMemcpyAsync(hctl.data(), dctl, np * kCtlBytes, hipMemcpyDeviceToHost, s));
    SKM_HIP(hipStreamSynchronize(s));
    if (stats)
      for (size_t b = 0; b < np; ++b) {
        const Persist* per = reinterpret_cast<const Persist*>(hctl.data() + b * kCtlBytes);
        skm_stats& S = stats[b];
        S.iterations = iters[b];
        S.converged = conv[b];
        S.objective = per->objective;
        S.sims_point_center = sims[b];
        S.sims_center_center = (int64_t)per->ccsims;
        S.rechecks = rechecks[b];
        if (S.objective_per_iter && iters[b] - 1 < S.per_iter_len && iters[b] > 0)
          S.objective_per_iter[iters[b] - 1] = per->objective;
        S.sim_kernel_launches = iters[b];
        S.sim_kernel_rows = rows[b];
        S.sim_kernel_nnz = nnz[b];
        S.sim_kernel_ms = 0.0;
      }
  }
done:
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cs) (void)hipStreamDestroy(cs);
  return rc;
}

}  // namespace
}  // namespace skm

using namespace skm;

extern "C" {

int skm_version(void) { return 10000; }

const char* skm_status_string(int status) {
  switch (status) {
    case SKM_OK: return "ok";
    case SKM_ERR_INVALID_ARG: return "invalid argument";
    case SKM_ERR_NOT_NORMALIZED: return "input not normalised";
    case SKM_ERR_OUT_OF_MEMORY: return "out of memory";
    case SKM_ERR_HIP: return "HIP runtime error";
    case SKM_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* skm_last_error(void) { return g_last_error.c_str(); }

size_t skm_workspace_size(const skm_matrix* X, int32_t k, int32_t variant,
                          const skm_options* opt) {
  if (X && X->fmt == SKM_DENSE_F32) {
    DensePlan D;
    if (make_dense_plan(X, k, variant, opt ? opt->precision : 0, &D) != SKM_OK) return 0;
    return D.total;
  }
  Plan P;
  if (opt && (opt->chunk_walk < 0 || opt->chunk_walk > 2)) {
    fail(SKM_ERR_INVALID_ARG, "chunk_walk must be 0, 1 or 2");
    return 0;
  }
  if (make_plan(X, k, variant, opt ? opt->precision : 0, &P, opt ? opt->chunk_walk : 0) !=
      SKM_OK)
    return 0;
  return P.total;
}

size_t skm_assign_workspace_size(const skm_matrix* X, int32_t k) {
  if (X && X->fmt == SKM_DENSE_F32) {
    DensePlan D;
    if (make_dense_plan(X, k, SKM_LLOYD, 0, &D) != SKM_OK) return 0;
    return D.total;
  }
  if (check_matrix(X) != SKM_OK) return 0;
  if (k < 1) {
    fail(SKM_ERR_INVALID_ARG, "need k >= 1");
    return 0;
  }
  const Geometry g = pick_geometry(k);
  if (g.G == 0) {
    fail(SKM_ERR_UNSUPPORTED, "k = %d exceeds the supported 4096", (int)k);
    return 0;
  }
  if (check_ct_size(X->d, g.kp) != SKM_OK) return 0;
  return align256((size_t)X->d * g.kp * sizeof(float)) +
         align256((size_t)k * X->d * sizeof(double));
}

int skm_assign(const skm_matrix* X, int32_t k, const float* centers, int32_t* assign_out,
               float* best_sim_out, float* second_sim_out, void* workspace,
               size_t workspace_bytes, void* stream) {
  g_last_error.clear();
  int rc = check_matrix(X);
  if (rc != SKM_OK) return rc;
  if (k < 1) return fail(SKM_ERR_INVALID_ARG, "need k >= 1");
  if (!centers || !assign_out) return fail(SKM_ERR_INVALID_ARG, "centers/assign_out NULL");
  if (X->fmt == SKM_DENSE_F32)
    return assign_dense(X, k, centers, assign_out, best_sim_out, second_sim_out, workspace,
                        workspace_bytes, static_cast<hipStream_t>(stream));
  const Geometry g = pick_geometry(k);
  if (g.G == 0) return fail(SKM_ERR_UNSUPPORTED, "k = %d exceeds the supported 4096", (int)k);
  rc = check_ct_size(X->d, g.kp);
  if (rc != SKM_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = skm_assign_workspace_size(X, k);
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, need, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", need);
    owned = true;
  } else if (workspace_bytes < need) {
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                need);
  }
  rc = assign_csr(X, k, g.kp, centers, assign_out, best_sim_out, second_sim_out, ws, s);
  if (owned) (void)hipFreeAsync(ws, s);
  return rc;
}

int skm_assign_noalloc(const skm_matrix* X, int32_t k, const float* centers,
                       int32_t* assign_out, float* best_sim_out, float* second_sim_out,
                       void* stream) {
  g_last_error.clear();
  int rc = check_matrix(X);
  if (rc != SKM_OK) return rc;
  if (X->fmt != SKM_CSR_F32)
    return fail(SKM_ERR_UNSUPPORTED, "skm_assign_noalloc takes CSR input");
  if (k < 1) return fail(SKM_ERR_INVALID_ARG, "need k >= 1");
  if (!centers || !assign_out) return fail(SKM_ERR_INVALID_ARG, "centers/assign_out NULL");
  const Geometry g = pick_geometry(k);
  if (g.G == 0) return fail(SKM_ERR_UNSUPPORTED, "k = %d exceeds the supported 4096", (int)k);
  rc = check_ct_size(X->d, g.kp);
  if (rc != SKM_OK) return rc;
  const size_t need = skm_assign_workspace_size(X, k);
  if (need > (size_t)SKM_NOALLOC_SCRATCH_BYTES)
    return fail(SKM_ERR_UNSUPPORTED, "d = %lld, k = %d need %zu bytes of centre copies; the "
                "no-allocation buffer holds %zu", (long long)X->d, (int)k, need,
                (size_t)SKM_NOALLOC_SCRATCH_BYTES);
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  rc = scratch_address(s, &ws);
  if (rc != SKM_OK) return rc;
  return assign_csr(X, k, g.kp, centers, assign_out, best_sim_out, second_sim_out, ws, s);
}

int skm_fit(const skm_matrix* X, int32_t k, const float* init_centers, int32_t variant,
            int32_t max_iter, const skm_options* opt, void* workspace, size_t workspace_bytes,
            int32_t* assign_out, float* centers_out, double* centers64_out, skm_stats* stats,
            void* stream) {
  g_last_error.clear();
  if (!X) return fail(SKM_ERR_INVALID_ARG, "X is NULL");
  if (!init_centers || !assign_out) return fail(SKM_ERR_INVALID_ARG, "init/assign_out NULL");
  if (max_iter < 1) return fail(SKM_ERR_INVALID_ARG, "need max_iter >= 1");
  skm_options o{};
  if (opt) o = *opt;
  if (o.norm_tol <= 0.0) o.norm_tol = 1e-4;
  if (o.bound_form != 0 && o.bound_form != 1)
    return fail(SKM_ERR_INVALID_ARG, "bound_form must be 0 or 1");
  if (o.schedule != 0 && o.schedule != 1)
    return fail(SKM_ERR_INVALID_ARG, "schedule must be 0 or 1");
  if (o.walk_layout < 0 || o.walk_layout > 2)
    return fail(SKM_ERR_INVALID_ARG, "walk_layout must be 0, 1 or 2");
  if (o.chunk_walk < 0 || o.chunk_walk > 2)
    return fail(SKM_ERR_INVALID_ARG, "chunk_walk must be 0, 1 or 2");
  const int nwarm = (o.warm_assign != nullptr) + (o.warm_best != nullptr) +
                    (o.warm_second != nullptr);
  if (nwarm != 0 && nwarm != 3)
    return fail(SKM_ERR_INVALID_ARG, "warm_assign, warm_best and warm_second go together");
  const bool warm = nwarm == 3;
  if (X->fmt == SKM_DENSE_F32) {
    return fit_dense(X, k, init_centers, variant, max_iter, o, workspace, workspace_bytes,
                     assign_out, centers_out, centers64_out, stats, static_cast<hipStream_t>(stream));
  }
  Plan P;
  int rc = make_plan(X, k, variant, o.precision, &P, o.chunk_walk);
  if (rc != SKM_OK) return rc;
  if (workspace && workspace_bytes < P.total)
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                P.total);
  HostMirror* hm = host_mirror();
  if (!hm) return fail(SKM_ERR_HIP, "could not allocate pinned host memory");

  hipStream_t s = static_cast<hipStream_t>(stream);
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, P.total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", P.total);
    owned = true;
  } else if (workspace_bytes < P.total) {
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                P.total);
  }

  const int64_t n = P.n, d = P.d;
  const double delta_c = (double)(d + 8) * kU64 * 1.01 + 1e-300;
  // Gram entries on FP64 matrix cores: unit 2^-52 also covers accumulation
  // that truncates
  const double delta_g = (double)(d + 2) * 2.0 * kU64 * 1.01 + 2.0 * delta_c + 1e-15;
  const double fx = fixed_point_scale(n);
  const double fx_inv = 1.0 / fx;

  float* CT = at<float>(ws, P.CT);
  void* CT16 = P.half ? at<char>(ws, P.CT16) : nullptr;
  int32_t* negflag = at<int32_t>(ws, P.negflag);
  double* C64 = at<double>(ws, P.C64);
  long long* S = at<long long>(ws, P.S);
  float* eta = at<float>(ws, P.eta);
  int32_t* a_old = at<int32_t>(ws, P.a_old);
  float* l = P.bounds ? at<float>(ws, P.l) : nullptr;
  float* u = (P.bounds && !P.elkan && !P.yy) ? at<float>(ws, P.u) : nullptr;
  float* uy = P.yy ? at<float>(ws, P.uy) : nullptr;
  double* gpc = P.yy ? at<double>(ws, P.gpc) : nullptr;
  double* gps = P.yy ? at<double>(ws, P.gps) : nullptr;
  float* ue = P.elkan ? at<float>(ws, P.ue) : nullptr;
  double* norm64 = at<double>(ws, P.norm64);
  double* part = at<double>(ws, P.part);
  double* part_sq = at<double>(ws, P.part_sq);
  double* pc = at<double>(ws, P.pc);
  double* ps = at<double>(ws, P.ps);
  int32_t* dirty = at<int32_t>(ws, P.dirty);
  MoveMin* mm = at<MoveMin>(ws, P.mm);
  double* G = P.gram ? at<double>(ws, P.G) : nullptr;
  double* gmax = P.gram ? at<double>(ws, P.gmax) : nullptr;
  double* gpart = P.gram ? at<double>(ws, P.gpart) : nullptr;
  Counters* cnt = at<Counters>(ws, P.cnt);
  Persist* per = at<Persist>(ws, P.per);
  StepCtl* ctl = at<StepCtl>(ws, P.ctl);
  StepRec* rec = at<StepRec>(ws, P.rec);
  float* maxeta = at<float>(ws, P.maxeta);
  double* initnorm = at<double>(ws, P.initnorm);

  RowRun* rs = (P.chunk || P.chunk16 || P.pack_adapt) ? at<RowRun>(ws, P.rs) : nullptr;
  uint64_t* umask =
      ((P.chunk || P.chunk16 || P.pack_adapt) && P.elkan) ? at<uint64_t>(ws, P.umask) : nullptr;
  // Fits with pack_adapt: which walk their steps with tests (Lloyd and
  // Hamerly: all their walks) take.  The first chunk of steps times both
  // (HIP events around each step's walk; steps 2 and 5 whole rows, 3 and 4
  // slices, so that a trend over the steps favours neither), and the rest
  // of the fit (from step 6: the first chunk ends there) keeps the faster:
  // packed slices pay where the tests leave few centres per row, and slices
  // of a large copy where the rows' terms spread the gathers over it, which
  // the rows' structure decides, not the problem's shape.
  int pack_choice = 0;  // 0 timing both, 1 whole rows, 2 packed slices
  bool pack_step = false;
  // [without, with bound tests][whole rows, slices]
  double pack_ms[2][2] = {};
  int pack_steps[2][2] = {};
  const int pack_mode = P.elkan ? kModeElkan : kModeYinYang;
  // one assignment-step walk in `mode`: one launch, or one per chunk of
  // centres with the running per-row results in rs
  auto walk = [&](AssignArgs& A, int mode) -> hipError_t {
    if (P.chunk16 && (mode == kModeYinYang || mode == kModeElkan)) {
      for (int q = 0; q < P.nq16; ++q) {
        A.j0 = q * P.chunk16;
        A.chunk_last = q == P.nq16 - 1 ? 1 : 0;
        A.rs = rs;
        A.umask = umask;
        const hipError_t e = launch_assign_chunk(A, mode, s);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    if (!P.chunk && !(pack_step && (P.pack_all || mode == pack_mode)))
      return launch_assign(A, mode, s);
    // slices need the running record and a copy at least one slice wide
    if (rs == nullptr || P.kp < kChunkF32) return hipErrorInvalidValue;
    for (int q = 0; q < P.nq; ++q) {
      A.j0 = q * kChunkF32;
      A.chunk_last = q == P.nq - 1 ? 1 : 0;
      A.rs = rs;
      A.umask = umask;
      const hipError_t e = launch_assign_chunk(A, mode, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  int32_t iterations = 0, converged = 0;
  int64_t tot_sims = 0, tot_rechecks = 0, sk_launches = 0, sk_rows = 0, sk_nnz = 0;
  double sk_ms = 0.0;
  const bool prof = o.profile != 0;
  // Bounded fits on rows under 20 stored entries: a row's walk is a few
  // gathers, and the tests' bookkeeping can cost more than the walks they
  // save however much they prune.  Step 2 runs plain (the walk that
  // refreshes every bound, as after the step control switched the tests
  // off); if the steps with tests of steps 2-5 were not at least 5% faster
  // than the plain ones, the rest of the fit keeps the tests off but for
  // the step control's own widening probes (its threshold rises above any
  // pruning rate).
  const bool test_probe = P.bounds && o.schedule == 0 && !P.pack_adapt &&
                          row_class(n, X->nnz) == 0;
  int test_choice = 0;  // 0 timing, 1 decided
  double test_ms[2] = {0.0, 0.0};
  int test_steps[2] = {0, 0};
  const double tests_off_min = 2.0;  // above any pruned share
  const bool timed = prof || P.pack_adapt || test_probe;
  hipEvent_t ev0[kStepChunk] = {}, ev1[kStepChunk] = {};
  // timed walk choice: an event between the two gated walks of a step (the
  // one whose kernel works takes nearly all the time: steps with and
  // without bound tests are told apart) and whether the step was gated
  hipEvent_t evm[kStepChunk] = {};
  bool gated[kStepChunk] = {};
  double objective = 0.0;
  {
    // centre step: member sums of the moved rows, renormalisation and
    // movement, the transposed copies, and the centre-centre products as
    // the step control decided (exact, carried, or nothing after a stop)
    auto centre_update = [&](bool gram) -> hipError_t {
      hipError_t e;
      if ((e = launch_update_scan(X->row_ptr, X->col_idx, X->val, assign_out, a_old, n, d, fx,
                                  S, dirty, s)) != hipSuccess)
        return e;
      if ((e = launch_sumsq_partial(S, k, d, fx_inv, dirty, part_sq, P.nchunk, s)) != hipSuccess)
        return e;
      if ((e = launch_normalize_move(S, k, d, fx_inv, dirty, part_sq, C64, part, P.nchunk, s)) !=
          hipSuccess)
        return e;
      if ((e = launch_centre_finalize(k, d, dirty, norm64, part_sq, part, P.nchunk, delta_c, pc,
                                      ps, mm, per, s)) != hipSuccess)
        return e;
      if (P.yy && (e = launch_group_move(pc, ps, k, P.ng, gpc, gps, s)) != hipSuccess) return e;
      if ((e = launch_transpose(C64, k, d, P.kp, dirty, CT, s, CT16)) != hipSuccess) return e;
      if (P.gram && gram) {
        if ((e = launch_gram(C64, k, d, dirty, 0, gpart, P.nslice, P.slice_len, G, gmax, delta_g,
                             per, s, ctl)) != hipSuccess)
          return e;
        if ((e = launch_gram_carry(G, k, pc, ps, delta_g, gmax, s, ctl)) != hipSuccess) return e;
      }
      return hipSuccess;
    };
    if (o.validate >= 2) {
      rc = validate_input(X, at<unsigned long long>(ws, P.vbad), s);
      if (rc != SKM_OK) goto done;
    }
    if (timed)
      for (int c = 0; c < kStepChunk; ++c) {
        SKM_HIP(hipEventCreate(&ev0[c]));
        SKM_HIP(hipEventCreate(&ev1[c]));
        if (P.pack_adapt || test_probe) SKM_HIP(hipEventCreate(&evm[c]));
      }
    SKM_HIP(hipMemsetAsync(CT, 0, (size_t)d * P.kp * sizeof(float), s));
    SKM_HIP(hipMemsetAsync(S, 0, (size_t)k * d * sizeof(long long), s));
    SKM_HIP(hipMemsetAsync(per, 0, sizeof(Persist), s));
    SKM_HIP(launch_fill_i32(a_old, n, -1, s));
    SKM_HIP(hipMemsetAsync(dirty, 0, (size_t)k * sizeof(int32_t), s));
    SKM_HIP(hipMemsetAsync(norm64, 0, (size_t)k * sizeof(double), s));
    SKM_HIP(hipMemsetAsync(maxeta, 0, kCounterSlots * sizeof(float), s));
    SKM_HIP(launch_row_eta(X->row_ptr, X->val, n, eta, maxeta, s));
    SKM_HIP(launch_init_centres(init_centers, k, d, 1, C64, initnorm, s));
    SKM_HIP(hipMemsetAsync(negflag, 0, sizeof(int32_t), s));
    if (P.half) {
      SKM_HIP(hipMemsetAsync(CT16, 0, (size_t)d * P.kp * 2, s));
      SKM_HIP(launch_neg_scan(X->val, X->nnz, init_centers, (int64_t)k * d, negflag, s));
    }
    SKM_HIP(launch_transpose(C64, k, d, P.kp, nullptr, CT, s, CT16));
    if (o.validate >= 1) {
      rc = check_init_norms(initnorm, k, o.norm_tol, s);
      if (rc != SKM_OK) goto done;
      float hslots[kCounterSlots];
      float hmax = 0.f;
      SKM_HIP(hipMemcpyAsync(hslots, maxeta, sizeof(hslots), hipMemcpyDeviceToHost, s));
      SKM_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < kCounterSlots; ++q) hmax = std::max(hmax, hslots[q]);
      if (o.validate >= 2 && !((double)hmax <= o.norm_tol)) {
        rc = fail(SKM_ERR_NOT_NORMALIZED, "a data row deviates from unit norm by %.3g", hmax);
        goto done;
      }
    }

    // Steps are queued kStepChunk at a time: the stop flag and the Gram and
    // tightening decisions live on the device (StepCtl), and the host reads
    // the step records once per chunk.  Steps queued after the fit stopped
    // find nothing to do.
    {
      // tightening reads about one line per stored entry, a row walk
      // kp * (bytes per centre) / 128; it pays when it prunes more often
      // than their ratio
      const double walk_lines = (double)P.kp * (P.half ? 2.0 : 4.0) / 128.0;
      double tight_min = std::min(0.9, std::max(0.02, 1.25 / walk_lines));
      // the tests of a row cost about a fifth of its walk where the walk is
      // shortest (two lines per entry) and proportionally less for longer
      // walks; they run while they prune at least that share of the rows
      double test_min = std::min(0.2, std::max(0.01, 0.4 / walk_lines));
      // schedule 1: tests and tightening at every step (never switched off)
      if (o.schedule == 1) test_min = tight_min = -1e300;
      SKM_HIP(launch_step_init(ctl, P.gram ? 1 : 0, warm ? 1 : 0, test_min, tight_min, s));
    }
    if (warm) {
      // the first step's assignment and FP64 top-2 are given: bounds only
      SKM_HIP(launch_warm_start(X->row_ptr, n, k, P.kp, o.warm_assign, o.warm_best,
                                o.warm_second, eta, delta_c, assign_out, l, u, ue, uy, P.ng, s));
      if (stats && stats->changed_per_iter && stats->per_iter_len > 0)
        stats->changed_per_iter[0] = n;
      if (stats && stats->sims_per_iter && stats->per_iter_len > 0) stats->sims_per_iter[0] = 0;
      iterations = 1;
      SKM_HIP(centre_update(true));
    }
    // steps before off_until are known (from the last read-back) to run
    // without bound tests: only the plain walk is queued for them, and no
    // Gram kernels before them
    int64_t off_until = INT64_MIN;
    const int32_t layout = walk_layout_for(o, P.kp, n, X->nnz);
    for (int32_t t0 = warm ? 1 : 0; t0 < max_iter;) {
      int ch = (int)std::min<int64_t>(kStepChunk, (int64_t)max_iter - t0);
      // a timed walk choice ends the first chunk with its last timing step,
      // so the chosen walk starts at step 6
      if ((P.pack_adapt && pack_choice == 0) || (test_probe && test_choice == 0))
        if (t0 < 6) ch = std::min(ch, 6 - (int)t0);
      SKM_HIP(hipMemsetAsync(cnt, 0, (size_t)ch * kCounterSlots * sizeof(Counters), s));
      for (int c = 0; c < ch; ++c) {
        const int32_t t = t0 + c;
        Counters* cs = cnt + (size_t)c * kCounterSlots;
        const bool exhaustive = (t == 0) || variant == SKM_LLOYD;
        pack_step = P.pack_adapt && (pack_choice == 2 || (pack_choice == 0 && (t == 3 || t == 4)));
        if (timed) SKM_HIP(hipEventRecord(ev0[c], s));
        AssignArgs A{};
        A.rp = X->row_ptr;
        A.ci = X->col_idx;
        A.v = X->val;
        A.CT = CT;
        A.CT16 = CT16;
        A.negflag = negflag;
        A.C64 = C64;
        A.d = d;
        A.k = k;
        A.kp = P.kp;
        A.n_rows = n;
        A.a = assign_out;
        A.read_prev = t > 0 ? 1 : 0;
        A.l = l;
        A.u = u;
        A.ue = ue;
        A.eta = eta;
        A.delta_c = delta_c;
        A.cnt = cs;
        A.ctl = ctl;
        A.pc = pc;
        A.ps = ps;
        A.mm = mm;
        A.gmax = gmax;
        A.simplified = variant == SKM_SIMP_HAMERLY || variant == SKM_SIMP_ELKAN;
        A.Gm = G;
        A.delta_g = delta_g;
        A.bound_form = o.bound_form;
        A.uy = uy;
        A.ng = P.ng;
        A.gpc = gpc;
        A.gps = gps;
        A.layout = layout;
        const int plain = P.elkan ? kModeFitElkanInit : kModeFit;
        gated[c] = !(exhaustive || t < off_until || (test_probe && test_choice == 0 && t == 2));
        if (!gated[c]) {
          SKM_HIP(walk(A, plain));
        } else {
          // with the bound tests, or (switched off by the step control) a
          // full walk that refreshes every bound: the plain fit kernel
          A.gate = 1;
          SKM_HIP(walk(A, P.elkan ? kModeElkan : P.yy ? kModeYinYang : kModeHamerly));
          if (P.pack_adapt || test_probe) SKM_HIP(hipEventRecord(evm[c], s));
          A.gate = 2;
          SKM_HIP(walk(A, P.elkan ? kModeFitElkanInit : kModeFit));
        }
        if (timed) SKM_HIP(hipEventRecord(ev1[c], s));
        const bool gram = (int64_t)t + 1 >= off_until;
        SKM_HIP(launch_step_end(cs, ctl, rec + c, per, t, n, dirty, k, gram ? 1 : 0, s));
        SKM_HIP(centre_update(gram));
      }
      SKM_HIP(hipMemcpyAsync(&hm->per, per,
                             sizeof(Persist) + sizeof(StepCtl) + (size_t)ch * sizeof(StepRec),
                             hipMemcpyDeviceToHost, s));
      SKM_HIP(hipStreamSynchronize(s));
      for (int c = 0; c < ch; ++c) {
        const StepRec& r = hm->rec[c];
        if (!r.valid) break;
        const int32_t t = t0 + c;
        if (timed) {
          float ms = 0.f;
          SKM_HIP(hipEventElapsedTime(&ms, ev0[c], ev1[c]));
          if (prof) sk_ms += ms;
          if (P.pack_adapt && pack_choice == 0 && t >= 2 && t <= 5) {
            const int w = (t == 3 || t == 4) ? 1 : 0;
            int tested = 0;
            if (gated[c]) {
              float m1 = 0.f;
              SKM_HIP(hipEventElapsedTime(&m1, ev0[c], evm[c]));
              tested = m1 > ms - m1 ? 1 : 0;
            }
            // Lloyd and Hamerly: time per computed similarity (a step with
            // tests walks fewer rows); Elkan and Yin-Yang: time, since
            // computing fewer similarities is what their packed slices are for
            pack_ms[tested][w] +=
                P.pack_all ? (double)ms / (double)std::max<uint64_t>(r.sims, 1) : ms;
            pack_steps[tested][w] += 1;
          }
          if (test_probe && test_choice == 0 && t >= 2 && t <= 5) {
            int tested = 0;
            if (gated[c]) {
              float m1 = 0.f;
              SKM_HIP(hipEventElapsedTime(&m1, ev0[c], evm[c]));
              tested = m1 > ms - m1 ? 1 : 0;
            }
            test_ms[tested] += ms;
            test_steps[tested] += 1;
          }
        }
        sk_launches += 1;
        sk_rows += (int64_t)r.rows_done;
        sk_nnz += (int64_t)r.nnz_done;
        tot_sims += (int64_t)r.sims;
        tot_rechecks += (int64_t)r.rechecks;
        if (stats && t < stats->per_iter_len) {
          if (stats->changed_per_iter) stats->changed_per_iter[t] = (int64_t)r.changed;
          if (stats->sims_per_iter) stats->sims_per_iter[t] = (int64_t)r.sims;
          if (stats->objective_per_iter && t > 0) stats->objective_per_iter[t - 1] = r.objective;
        }
        iterations = t + 1;
      }
      if (hm->ctl.stop) {
        converged = 1;
        break;
      }
      t0 += ch;
      off_until = hm->ctl.tests ? INT64_MIN : (int64_t)hm->ctl.test_next;
      // after the timing steps: compare steps of one kind (Elkan and
      // Yin-Yang: with tests, the only walks they pack; Lloyd and Hamerly:
      // plain first), slices only where clearly faster (3%); no comparable
      // pair: whole rows
      if (test_probe && test_choice == 0 && t0 >= 6) {
        test_choice = 1;
        if (test_steps[0] > 0 && test_steps[1] > 0 &&
            test_ms[1] / test_steps[1] > 0.95 * (test_ms[0] / test_steps[0])) {
          // nothing runs on the stream now (the records were just read)
          SKM_HIP(hipMemcpyAsync(&ctl->test_min, &tests_off_min, sizeof(double),
                                 hipMemcpyHostToDevice, s));
        }
      }
      if (P.pack_adapt && pack_choice == 0 && t0 >= 6) {
        pack_choice = 1;
        const int order[2] = {P.pack_all ? 0 : 1, P.pack_all ? 1 : -1};
        for (int q : order) {
          if (q < 0 || pack_steps[q][0] == 0 || pack_steps[q][1] == 0) continue;
          const double whole = pack_ms[q][0] / pack_steps[q][0];
          const double sliced = pack_ms[q][1] / pack_steps[q][1];
          pack_choice = sliced < 0.97 * whole ? 2 : 1;
          break;
        }
      }
    }
    // final objective (after the last update) and centre-centre count
    SKM_HIP(hipMemcpyAsync(&hm->per, per, sizeof(Persist), hipMemcpyDeviceToHost, s));
    if (centers_out) SKM_HIP(launch_c64_to_f32(C64, (int64_t)k * d, centers_out, s));
    if (centers64_out)
      SKM_HIP(hipMemcpyAsync(centers64_out, C64, (size_t)k * d * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    SKM_HIP(hipStreamSynchronize(s));
    objective = hm->per.objective;
    if (stats) {
      stats->iterations = iterations;
      stats->converged = converged;
      stats->objective = objective;
      stats->sims_point_center = tot_sims;
      stats->sims_center_center = (int64_t)hm->per.ccsims;
      stats->rechecks = tot_rechecks;
      if (stats->objective_per_iter && iterations - 1 < stats->per_iter_len)
        stats->objective_per_iter[iterations - 1] = objective;
      stats->sim_kernel_launches = sk_launches;
      stats->sim_kernel_rows = sk_rows;
      stats->sim_kernel_nnz = sk_nnz;
      stats->sim_kernel_ms = sk_ms;
    }
  }
done:
  for (int c = 0; c < kStepChunk; ++c) {
    if (ev0[c]) (void)hipEventDestroy(ev0[c]);
    if (ev1[c]) (void)hipEventDestroy(ev1[c]);
    if (evm[c]) (void)hipEventDestroy(evm[c]);
  }
  if (owned) {
    (void)hipFreeAsync(ws, s);
    if (rc == SKM_OK) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = fail(SKM_ERR_HIP, "final synchronise: %s", hipGetErrorString(e));
    }
  }
  return rc;
}


namespace {
struct SeedPlan {
  size_t taken = 0, a = 0, best = 0, second = 0, w = 0, part = 0, c64 = 0, u = 0, centres = 0,
         chosen_dummy = 0, total = 0;
};

// Dense rows for the seeding kernels (nullptr: CSR).
const float* dense_rows(const skm_matrix* X) {
  return X->fmt == SKM_DENSE_F32 ? X->dense : nullptr;
}

int make_seed_plan(const skm_matrix* X, int32_t k, SeedPlan* S) {
  int rc = check_matrix(X);
  if (rc != SKM_OK) return rc;
  if (k < 1 || k > X->n) return fail(SKM_ERR_INVALID_ARG, "need 1 <= k <= n (k = %d)", (int)k);
  const size_t n = (size_t)X->n, d = (size_t)X->d, nb = (n + kBlock - 1) / kBlock;
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += align256(bytes);
    return o;
  };
  S->taken = take(n);
  S->a = take(n * 4);
  S->best = take(n * 8);
  S->second = take(n * 8);
  S->w = take(n * 8);
  S->part = take(nb * 8);
  S->c64 = take(d * 8);
  S->u = take((size_t)k * 8);
  S->centres = take((size_t)k * d * 4);
  S->total = cur;
  return SKM_OK;
}
}  // namespace

size_t skm_seed_workspace_size(const skm_matrix* X, int32_t k) {
  g_last_error.clear();
  SeedPlan S;
  if (make_seed_plan(X, k, &S) != SKM_OK) return 0;
  return S.total;
}

int skm_seed_kmeanspp(const skm_matrix* X, int32_t k, double alpha, const double* uniforms,
                      int32_t* chosen_out, float* centers_out, int32_t* assign_out,
                      double* best_out, double* second_out, void* workspace,
                      size_t workspace_bytes, void* stream) {
  g_last_error.clear();
  SeedPlan S;
  int rc = make_seed_plan(X, k, &S);
  if (rc != SKM_OK) return rc;
  if (!uniforms || !chosen_out) return fail(SKM_ERR_INVALID_ARG, "uniforms/chosen_out NULL");
  if (!(alpha >= 1.0) || !std::isfinite(alpha))
    return fail(SKM_ERR_INVALID_ARG, "need alpha >= 1 (got %g)", alpha);
  for (int32_t t = 0; t < k; ++t)
    if (!(uniforms[t] >= 0.0 && uniforms[t] < 1.0))
      return fail(SKM_ERR_INVALID_ARG, "uniform %d = %g is not in [0, 1)", (int)t, uniforms[t]);
  if (workspace && workspace_bytes < S.total)
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                S.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, S.total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", S.total);
    owned = true;
  }
  {
    const int64_t n = X->n, d = X->d;
    uint8_t* taken = at<uint8_t>(ws, S.taken);
    int32_t* a = assign_out ? assign_out : at<int32_t>(ws, S.a);
    double* best = best_out ? best_out : at<double>(ws, S.best);
    double* second = second_out ? second_out : at<double>(ws, S.second);
    float* centres = centers_out ? centers_out : at<float>(ws, S.centres);
    double* u_dev = at<double>(ws, S.u);
    SKM_HIP(hipMemcpyAsync(u_dev, uniforms, (size_t)k * sizeof(double), hipMemcpyHostToDevice, s));
    SKM_HIP(hipMemsetAsync(taken, 0, (size_t)n, s));
    SKM_HIP(hipMemsetAsync(centres, 0, (size_t)k * d * sizeof(float), s));
    SKM_HIP(launch_fill_i32(a, n, -1, s));
    SKM_HIP(launch_fill_f64(best, n, -INFINITY, s));
    SKM_HIP(launch_fill_f64(second, n, -INFINITY, s));
    for (int32_t t = 0; t < k; ++t)
      SKM_HIP(launch_kpp_step(X->row_ptr, X->col_idx, X->val, dense_rows(X), X->ld, n, d, t,
                              alpha, u_dev, taken,
                              chosen_out, centres, at<double>(ws, S.c64), a, best, second,
                              at<double>(ws, S.w), at<double>(ws, S.part), s));
  }
done:
  if (owned) (void)hipFreeAsync(ws, s);
  return rc;
}

namespace {
struct AfkPlan {
  size_t w = 0, W = 0, prefix = 0, cand = 0, dcand = 0, C64 = 0, u = 0, centres = 0, total = 0;
  size_t nu = 0;
};

int make_afk_plan(const skm_matrix* X, int32_t k, int32_t chain, AfkPlan* S) {
  int rc = check_matrix(X);
  if (rc != SKM_OK) return rc;
  if (k < 1 || k > X->n) return fail(SKM_ERR_INVALID_ARG, "need 1 <= k <= n (k = %d)", (int)k);
  if (chain < 1 || chain > (1 << 20))
    return fail(SKM_ERR_INVALID_ARG, "need 1 <= chain <= 2^20 (chain = %d)", (int)chain);
  const size_t n = (size_t)X->n, d = (size_t)X->d;
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += align256(bytes);
    return o;
  };
  S->nu = 1 + (size_t)(k - 1) * (2 * (size_t)chain - 1);
  S->w = take(n * 8);
  S->W = take(8);
  S->prefix = take(n * 8);
  S->cand = take((size_t)chain * 4);
  S->dcand = take((size_t)chain * 8);
  S->C64 = take((size_t)k * d * 8);
  S->u = take(S->nu * 8);
  S->centres = take((size_t)k * d * 4);
  S->total = cur;
  return SKM_OK;
}
}  // namespace

size_t skm_seed_afkmc2_workspace_size(const skm_matrix* X, int32_t k, int32_t chain) {
  g_last_error.clear();
  AfkPlan S;
  if (make_afk_plan(X, k, chain, &S) != SKM_OK) return 0;
  return S.total;
}

int skm_seed_afkmc2(const skm_matrix* X, int32_t k, int32_t chain, double alpha,
                    const double* uniforms, int32_t* chosen_out, float* centers_out,
                    void* workspace, size_t workspace_bytes, void* stream) {
  g_last_error.clear();
  AfkPlan S;
  int rc = make_afk_plan(X, k, chain, &S);
  if (rc != SKM_OK) return rc;
  if (!uniforms || !chosen_out) return fail(SKM_ERR_INVALID_ARG, "uniforms/chosen_out NULL");
  if (!(alpha >= 1.0) || !std::isfinite(alpha))
    return fail(SKM_ERR_INVALID_ARG, "need alpha >= 1 (got %g)", alpha);
  for (size_t q = 0; q < S.nu; ++q)
    if (!(uniforms[q] >= 0.0 && uniforms[q] < 1.0))
      return fail(SKM_ERR_INVALID_ARG, "uniform %zu = %g is not in [0, 1)", q, uniforms[q]);
  if (workspace && workspace_bytes < S.total)
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                S.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, S.total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", S.total);
    owned = true;
  }
  {
    float* centres = centers_out ? centers_out : at<float>(ws, S.centres);
    double* u_dev = at<double>(ws, S.u);
    SKM_HIP(hipMemcpyAsync(u_dev, uniforms, S.nu * sizeof(double), hipMemcpyHostToDevice, s));
    SKM_HIP(hipMemsetAsync(centres, 0, (size_t)k * X->d * sizeof(float), s));
    SKM_HIP(launch_afkmc2(X->row_ptr, X->col_idx, X->val, dense_rows(X), X->ld, X->n, X->d, k,
                          chain, alpha, u_dev,
                          chosen_out, centres, at<double>(ws, S.C64), at<double>(ws, S.w),
                          at<double>(ws, S.W), at<double>(ws, S.prefix), at<int32_t>(ws, S.cand),
                          at<double>(ws, S.dcand), s));
  }
done:
  if (owned) (void)hipFreeAsync(ws, s);
  return rc;
}

size_t skm_fit_batched_workspace_size(int32_t nprob, const skm_matrix* Xs, const int32_t* ks,
                                      int32_t variant, const skm_options* opt,
                                      int32_t workers) {
  g_last_error.clear();
  if (nprob < 1 || !Xs || !ks) {
    fail(SKM_ERR_INVALID_ARG, "need nprob >= 1 and non-NULL Xs, ks");
    return 0;
  }
  skm_options o{};
  if (opt) o = *opt;
  if (workers == 0 && lockstep_eligible(nprob, Xs, variant, o)) {
    Lockstep L;
    if (plan_lockstep(nprob, Xs, ks, variant, o, &L) != SKM_OK) return 0;
    return L.total;
  }
  size_t slot = 0;
  for (int32_t b = 0; b < nprob; ++b) {
    const size_t need = skm_workspace_size(&Xs[b], ks[b], variant, opt);
    if (need == 0) {
      const std::string m = g_last_error;
      fail(SKM_ERR_INVALID_ARG, "problem %d: %s", (int)b, m.c_str());
      return 0;
    }
    slot = std::max(slot, align256(need));
  }
  return slot * (size_t)batch_workers(workers, nprob);
}

int skm_fit_batched(int32_t nprob, const skm_matrix* Xs, const int32_t* ks,
                    const float* const* inits, int32_t variant, const int32_t* max_iters,
                    const skm_options* opt, int32_t workers, void* workspace,
                    size_t workspace_bytes, int32_t* const* assign_outs,
                    float* const* centers_outs, skm_stats* stats, void* stream) {
  g_last_error.clear();
  if (nprob < 1) return fail(SKM_ERR_INVALID_ARG, "need nprob >= 1");
  if (!Xs || !ks || !inits || !max_iters || !assign_outs)
    return fail(SKM_ERR_INVALID_ARG, "Xs, ks, inits, max_iters and assign_outs must be non-NULL");
  if (workers < 0) return fail(SKM_ERR_INVALID_ARG, "workers must be >= 0");
  for (int32_t b = 0; b < nprob; ++b) {
    if (!inits[b] || !assign_outs[b])
      return fail(SKM_ERR_INVALID_ARG, "problem %d: init or assign_out NULL", (int)b);
    if (max_iters[b] < 1) return fail(SKM_ERR_INVALID_ARG, "problem %d: max_iter < 1", (int)b);
  }
  skm_options o{};
  if (opt) o = *opt;
  if (variant < SKM_LLOYD || variant > SKM_YINYANG)
    return fail(SKM_ERR_INVALID_ARG, "unknown variant %d", (int)variant);
  if (o.bound_form != 0 && o.bound_form != 1)
    return fail(SKM_ERR_INVALID_ARG, "bound_form must be 0 or 1");
  if (o.schedule != 0 && o.schedule != 1)
    return fail(SKM_ERR_INVALID_ARG, "schedule must be 0 or 1");
  if (o.walk_layout < 0 || o.walk_layout > 2)
    return fail(SKM_ERR_INVALID_ARG, "walk_layout must be 0, 1 or 2");
  if (o.chunk_walk < 0 || o.chunk_walk > 2)
    return fail(SKM_ERR_INVALID_ARG, "chunk_walk must be 0, 1 or 2");
  if (workers == 0 && lockstep_eligible(nprob, Xs, variant, o)) {
    Lockstep L;
    int rc = plan_lockstep(nprob, Xs, ks, variant, o, &L);
    if (rc != SKM_OK) return rc;
    for (int32_t b = 0; b < nprob; ++b)
      if (!Xs[b].row_ptr || (Xs[b].nnz > 0 && (!Xs[b].col_idx || !Xs[b].val)))
        return fail(SKM_ERR_INVALID_ARG, "problem %d: CSR arrays must not be NULL", (int)b);
    if (workspace && workspace_bytes < L.total)
      return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                  L.total);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = workspace;
    if (!ws && hipMallocAsync(&ws, L.total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", L.total);
    rc = fit_batched_lockstep(nprob, Xs, ks, inits, variant, max_iters, o, ws, L, assign_outs,
                              centers_outs, stats, s);
    if (!workspace) (void)hipFreeAsync(ws, s);
    return rc;
  }
  const int W = batch_workers(workers, nprob);
  const size_t total = skm_fit_batched_workspace_size(nprob, Xs, ks, variant, opt, workers);
  if (total == 0) return g_last_error.empty() ? fail(SKM_ERR_INVALID_ARG, "bad problem") :
                                               SKM_ERR_INVALID_ARG;
  if (workspace && workspace_bytes < total)
    return fail(SKM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, %zu needed", workspace_bytes,
                total);
  const size_t slot = total / (size_t)W;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(SKM_ERR_HIP, "hipGetDevice failed");
  bool owned = false;
  void* ws = workspace;
  if (!ws) {
    if (hipMallocAsync(&ws, total, s) != hipSuccess)
      return fail(SKM_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of workspace", total);
    owned = true;
  }
  hipEvent_t start = nullptr;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(start, s) != hipSuccess) {
    if (start) (void)hipEventDestroy(start);
    if (owned) (void)hipFreeAsync(ws, s);
    return fail(SKM_ERR_HIP, "could not record the start event");
  }
  // most expensive problems first (the vectors below are small; an
  // allocation failure here ends the process like any other host OOM)
  std::vector<int32_t> order(nprob);
  std::vector<double> cost(nprob);
  for (int32_t b = 0; b < nprob; ++b) {
    order[b] = b;
    const double entries =
        Xs[b].fmt == SKM_DENSE_F32 ? (double)Xs[b].n * (double)Xs[b].d : (double)Xs[b].nnz;
    cost[b] = entries * (double)ks[b] * (double)max_iters[b];
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
  std::atomic<int32_t> next{0};
  std::atomic<bool> abort{false};
  std::vector<int> status(nprob, SKM_OK);
  std::vector<std::string> msg(nprob);
  std::vector<int> wstatus(W, SKM_OK);
  std::vector<std::string> wmsg(W);
  auto work = [&](int w) {
    if (hipSetDevice(device) != hipSuccess) {
      wstatus[w] = SKM_ERR_HIP;
      wmsg[w] = "hipSetDevice failed in a worker";
      abort = true;
      return;
    }
    hipStream_t ws_stream = nullptr;
    if (hipStreamCreateWithFlags(&ws_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamWaitEvent(ws_stream, start, 0) != hipSuccess) {
      wstatus[w] = SKM_ERR_HIP;
      wmsg[w] = "could not create a worker stream";
      abort = true;
      if (ws_stream) (void)hipStreamDestroy(ws_stream);
      return;
    }
    void* slot_ptr = static_cast<char*>(ws) + (size_t)w * slot;
    for (;;) {
      const int32_t i = next.fetch_add(1);
      if (i >= nprob || abort.load()) break;
      const int32_t b = order[i];
      const int rc = skm_fit(&Xs[b], ks[b], inits[b], variant, max_iters[b], opt, slot_ptr, slot,
                             assign_outs[b], centers_outs ? centers_outs[b] : nullptr, nullptr,
                             stats ? &stats[b] : nullptr, ws_stream);
      if (rc != SKM_OK) {
        status[b] = rc;
        msg[b] = g_last_error;
        abort = true;
      }
    }
    (void)hipStreamSynchronize(ws_stream);
    (void)hipStreamDestroy(ws_stream);
    release_host_mirror();
  };
  std::vector<std::thread> pool;
  int rc = SKM_OK;
  try {
    pool.reserve(W);
    for (int w = 0; w < W; ++w) pool.emplace_back(work, w);
  } catch (...) {  // thread creation failed: stop the started workers
    abort = true;
    rc = fail(SKM_ERR_OUT_OF_MEMORY, "could not start %d worker threads", W);
  }
  for (auto& t : pool) t.join();
  (void)hipEventDestroy(start);
  for (int32_t b = 0; b < nprob && rc == SKM_OK; ++b)
    if (status[b] != SKM_OK) rc = fail(status[b], "problem %d: %s", (int)b, msg[b].c_str());
  for (int w = 0; w < W && rc == SKM_OK; ++w)
    if (wstatus[w] != SKM_OK) rc = fail(wstatus[w], "%s", wmsg[w].c_str());
  if (owned) (void)hipFreeAsync(ws, s);
  return rc;
}

}  // extern "C"
