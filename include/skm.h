/*
 * skm.h -- C ABI of the MI355X (gfx950) spherical k-means library.
 *
 * Method: Schubert, Lang, Feher, "Accelerating Spherical k-Means"
 * (arXiv 2107.04074).  The library runs the assignment step
 *     a(i) <- argmax_j <x(i), c(j)>                 (Section 5)
 * over unit-length rows x(i), optionally pruned by the cosine-domain bounds
 * of Section 4 (Eq. (6), (7)) in the forms of Elkan (Sections 5.1-5.2) and
 * Hamerly (Sections 5.3-5.4, Eq. (9)), and the centre step
 *     c(j) <- sum_{a(i)=j} x(i) / |sum_{a(i)=j} x(i)| (Section 5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer unless its comment says [host].
 *    The caller owns all inputs, outputs and the workspace; the library never
 *    frees or reallocates caller memory.
 *  - All work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *    the default stream).  skm_assign returns without synchronising;
 *    skm_fit queues assignment steps eight at a time (the stop test and
 *    the other per-step decisions are taken on the GPU), synchronises with
 *    `stream` once per eight steps to read the step records, and returns
 *    after the fit completed.
 *  - Every function returns an skm_status; no C++ exception crosses the ABI.
 *    On error the outputs are unspecified and skm_last_error() describes the
 *    failure (thread-local string, valid until the next call on the thread).
 *  - Workspace: pass a device buffer of at least skm_workspace_size() bytes,
 *    256-byte aligned, or NULL to let the call allocate (stream-ordered
 *    hipMallocAsync) and free it before returning.  A smaller buffer fails
 *    with SKM_ERR_OUT_OF_MEMORY.
 *  - Concurrent calls on distinct workspaces and streams are safe.
 *
 * Input matrix (skm_matrix)
 * -------------------------
 *  SKM_CSR_F32:   row_ptr int64[n+1] (row_ptr[0] = 0, non-decreasing,
 *                 row_ptr[n] = nnz), col_idx int32[nnz] in [0, d), val
 *                 float[nnz].  Column ids strictly ascending within a row
 *                 is the expected layout (the paper stores sparse vectors as
 *                 sorted (index, value) pairs, Section 2); options.validate
 *                 = 2 checks all of this.  d * k_padded (k rounded up
 *                 to a power of two, at least 16: the width of the centre
 *                 copy the row kernels read) must stay below 2^32 (else
 *                 SKM_ERR_UNSUPPORTED).
 *  SKM_DENSE_F32: dense float[n * ld], row-major, ld >= d.
 *  Rows must have unit L2 norm (Section 5: samples are normalised during
 *  initialisation).  Float rounding of the norm is tolerated: internal
 *  bounds account for each row's measured deviation.
 *
 * Numerics
 * --------
 *  Similarities are evaluated in FP32 (sparse: FMA chains over the stored
 *  entries, a few partial chains per (row, centre) added in a fixed order;
 *  dense: MFMA); the error bound used holds for any summation order.  Whenever the best
 *  and second best FP32 values lie within the rigorous FP32 error bound of
 *  each other, the candidates are re-evaluated in FP64 against the FP64
 *  master centres, so every assignment equals the argmax of the FP64 dot
 *  products.  Ties are resolved by keeping the previous assignment if it
 *  attains the maximum, else by the lowest centre index.  Pruning tests use
 *  bounds on true cosines with outward rounding and margins, so the bounded
 *  variants produce exactly the assignments of SKM_LLOYD.
 */
#ifndef SKM_H_
#define SKM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SKM_LLOYD = 0,        /* exhaustive spherical Lloyd (Section 5)            */
  SKM_ELKAN = 1,        /* per-centre bounds + centre-centre tests (5.2)     */
  SKM_HAMERLY = 2,      /* one upper and one lower bound + s(a) test (5.3)   */
  SKM_SIMP_ELKAN = 3,   /* Elkan without centre-centre tests (5.1)           */
  SKM_SIMP_HAMERLY = 4, /* Hamerly without the s(a) test (5.4)               */
  SKM_YINYANG = 5       /* one upper bound per group of 32 consecutive
                           centres (5.5); CSR input                          */
} skm_variant;

typedef enum {
  SKM_OK = 0,
  SKM_ERR_INVALID_ARG = 1,    /* null pointer, size out of range, bad enum   */
  SKM_ERR_NOT_NORMALIZED = 2, /* validation found a row that is not unit     */
  SKM_ERR_OUT_OF_MEMORY = 3,  /* workspace too small or allocation failed    */
  SKM_ERR_HIP = 4,            /* a HIP runtime call failed                   */
  SKM_ERR_UNSUPPORTED = 5     /* valid request the library does not handle   */
} skm_status;

typedef enum { SKM_CSR_F32 = 0, SKM_DENSE_F32 = 1 } skm_format;

typedef struct {
  int32_t fmt;              /* skm_format                                     */
  int32_t reserved0;
  int64_t n, d, nnz;        /* rows, columns, stored entries (CSR)            */
  const int64_t* row_ptr;   /* CSR                                            */
  const int32_t* col_idx;   /* CSR                                            */
  const float* val;         /* CSR                                            */
  const float* dense;       /* DENSE: n x ld row-major                        */
  int64_t ld;               /* DENSE leading dimension (>= d)                 */
} skm_matrix;

typedef struct {            /* [host]; an all-zero struct means defaults      */
  int32_t bound_form;       /* Hamerly upper-bound update: 0 = guarded Eq. (7)
                               with p'(a) = min_{j!=a} p(j) (default);
                               1 = Eq. (9) where valid (u, p' >= 0)           */
  int32_t precision;        /* 0 = FP32 similarities; 1 = BF16 MFMA (dense
                               input only); 2 = FP16 copy of the centres for
                               the CSR row walk (k >= 65); every precision
                               keeps the same exact-argmax guarantee          */
  int32_t validate;         /* 0 = none; 1 = initial centres must be unit
                               within norm_tol (else SKM_ERR_NOT_NORMALIZED);
                               2 = also every data row unit within norm_tol,
                               and, before any kernel walks the rows, the
                               layout: CSR row_ptr[0] = 0, non-decreasing,
                               row_ptr[n] = nnz, column ids in [0, d) and
                               strictly ascending within each row; every
                               value finite (CSR and dense).  A layout
                               violation returns SKM_ERR_INVALID_ARG naming
                               the first offending row.  Without validate =
                               2 a malformed matrix is undefined behaviour. */
  int32_t profile;          /* 1 = time every launch of the similarity kernel
                               with HIP events on `stream` (fills the
                               sim_kernel_* statistics; adds event records) */
  double norm_tol;          /* default 1e-4                                   */
  /* Warm start (CSR or dense input; all three set or all NULL): the
     result of the first assignment step against init_centers, as
     skm_seed_kmeanspp returns it -- assignment int32[n] and the FP64 best
     and second-best similarities double[n] in the canonical order.  skm_fit then takes
     that step from these arrays instead of recomputing it and sets its
     bounds from them, so pruning starts with the second step (the
     seeding/bounds synergy named in the paper's conclusion). */
  const int32_t* warm_assign;
  const double* warm_best;
  const double* warm_second;
  int32_t schedule;         /* Bounded variants.  0 (default): the bound
                               tests (Sections 5.1-5.5) and the tightening of
                               l(i) run only while they prune enough to pay
                               for themselves, otherwise the step walks every
                               row and refreshes every bound exactly (on rows
                               under 20 stored entries the fit also times a
                               plain step against steps with tests and keeps
                               the tests off when they are not faster); 1:
                               they run at every step, as in the paper.
                               Results are the same either way; only work
                               differs.                                    */
  int32_t batch_tile_rows;  /* skm_fit_batched in lockstep (workers = 0): rows
                               per work item of the batched row walk; 0 takes
                               the table compiled into the library (the
                               lockstep driver is switched off in this
                               build, so the value is not used) */
  int32_t walk_layout;      /* Lloyd, Hamerly and simplified Hamerly fits on
                               CSR rows with the FP32 centre copy, 16 < k
                               <= 512, whole-row walks: 0 = the layout the
                               library's tuning table (measured by
                               tune_walk.py) picks for k and the mean row
                               length; 1 = the default layout; 2 = the
                               alternative (one row per wave at k <= 64,
                               four rows per wave above).  Results are
                               identical; only speed differs.  Other fits
                               ignore it.                                 */
  int32_t chunk_walk;       /* CSR rows, FP32 centre copy, 256 < k <= 4096:
                               0 = walk the centres 256 at a time (one
                               launch per slice; Elkan and Yin-Yang pack
                               each slice's surviving centres) or whole rows
                               (one launch) as the library's tuning table
                               (measured by tune_walk.py) picks for the
                               variant, k and the mean row length, always
                               sliced when the copy exceeds 256 MB;
                               Yin-Yang at k > 128 and Elkan at k > 256
                               where whole rows are picked (and rows hold
                               20 or more stored entries on average) time
                               their steps with tests both ways (whole
                               rows, packed slices) in the first eight
                               steps and keep the faster, as do Lloyd and
                               Hamerly (every walk) for copies of 64 MB
                               to 256 MB where the table picks whole rows;
                               1 = always sliced, and Elkan and Yin-Yang
                               at 128 < k <= 256 walk their one slice
                               packed (only the centres whose bounds fail;
                               faster where the bounds prune most pairs,
                               slower where they do not); 2 = always whole
                               rows.  Results are identical; only speed
                               and workspace size differ.                 */
} skm_options;

typedef struct {            /* [host] filled by skm_fit                       */
  int32_t iterations;       /* assignment steps executed                      */
  int32_t converged;        /* 1 if the last step changed no assignment       */
  double objective;         /* sum_i <x(i), c(a(i))> for the returned centres */
  int64_t sims_point_center;  /* point-centre similarities evaluated         */
  int64_t sims_center_center; /* centre-centre inner products evaluated      */
  int64_t rechecks;         /* rows whose decision was re-evaluated in FP64   */
  /* optional per-iteration records, [host] arrays of per_iter_len entries
     (nullable); entry t describes assignment step t+1 */
  int64_t* changed_per_iter;
  int64_t* sims_per_iter;
  double* objective_per_iter; /* objective after the update following step t
                                 (the previous value when nothing changed)  */
  int32_t per_iter_len;
  int32_t reserved0;
  /* work of the dominant similarity kernel: for CSR input the row-walk
     kernel of each assignment step (one or two launches per step: with and
     without bound tests, one of which returns at once; where the FP32 walk
     slices the centres (k > 256, see chunk_walk) that many per 256-centre
     slice), for dense input the
     first MFMA similarity pass of each step; steps, rows walked and their
     stored entries (rows x d for dense), and (profile = 1) the summed
     duration from HIP events recorded around each step's launches on
     `stream` */
  int64_t sim_kernel_launches;
  int64_t sim_kernel_rows;
  int64_t sim_kernel_nnz;
  double sim_kernel_ms;
} skm_stats;

/* Bytes of workspace skm_fit needs for this problem (0 on invalid input;
 * then skm_last_error() says why).  opt may be NULL. */
size_t skm_workspace_size(const skm_matrix* X, int32_t k, int32_t variant,
                          const skm_options* opt);

/* Bytes of workspace skm_assign needs. */
size_t skm_assign_workspace_size(const skm_matrix* X, int32_t k);

/* Spherical k-means from the given initial centres.
 *   k              1 <= k <= n, at most 4096 (SKM_ERR_UNSUPPORTED above).
 *   init_centers   float[k*d] row-major; rows are rescaled to unit length in
 *                  FP64 before the first step (the paper's centres are unit
 *                  vectors; rows picked from float data are unit only to
 *                  rounding).
 *   variant        skm_variant.
 *   max_iter       >= 1; counts assignment steps.  The fit stops early when
 *                  a step changes no assignment.  After every step that
 *                  changed something the centres are updated, so the returned
 *                  centres are the normalised member sums of the returned
 *                  assignment; a cluster that loses all members keeps its
 *                  previous centre.
 *   assign_out     int32[n]: final assignment (also used as working state).
 *   centers_out    float[k*d] row-major (nullable): final centres.
 *   centers64_out  double[k*d] row-major (nullable): final FP64 centres.
 *   stats          [host] (nullable).
 */
int skm_fit(const skm_matrix* X, int32_t k, const float* init_centers,
            int32_t variant, int32_t max_iter, const skm_options* opt,
            void* workspace, size_t workspace_bytes, int32_t* assign_out,
            float* centers_out, double* centers64_out, skm_stats* stats,
            void* stream);

/* One assignment step against fixed centres (Section 5, assignment
 * equation), for every row.
 *   centers          float[k*d] row-major, used as given (not rescaled).
 *   assign_out       int32[n]; ties go to the lowest index.
 *   best_sim_out     float[n] (nullable): <x(i), c(a(i))>.
 *   second_sim_out   float[n] (nullable): largest similarity to any other
 *                    centre (FP32 value; -inf when k = 1).
 * Asynchronous: returns after enqueueing. */
int skm_assign(const skm_matrix* X, int32_t k, const float* centers,
               int32_t* assign_out, float* best_sim_out, float* second_sim_out,
               void* workspace, size_t workspace_bytes, void* stream);

/* skm_assign for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same assignment step as skm_assign on CSR input (same kernels, same
 * results), but the centre copies live in a buffer the library owns: one
 * static device array of SKM_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * library's load until the process ends.  The call allocates nothing, frees
 * nothing and enqueues only kernels on `stream` (the buffer is cleared by a
 * fill kernel, not hipMemset); the first call on a device looks the
 * buffer's address up (hipGetSymbolAddress, host only).
 *   Size limit: align256(d * k_padded * 4) + align256(k * d * 8) bytes (the
 *   skm_assign_workspace_size of the same problem) must not exceed
 *   SKM_NOALLOC_SCRATCH_BYTES, else SKM_ERR_UNSUPPORTED and nothing is
 *   enqueued.  Dense input: SKM_ERR_UNSUPPORTED.
 *   Sharing: every call on one GPU uses that GPU's buffer, which keeps the
 *   last call's contents.  Calls that overlap on one GPU (several streams or
 *   host threads) race and give undefined results; order them on one
 *   stream.
 * Arguments and outputs as in skm_assign.  Asynchronous. */
#define SKM_NOALLOC_SCRATCH_BYTES (64u << 20)
int skm_assign_noalloc(const skm_matrix* X, int32_t k, const float* centers,
                       int32_t* assign_out, float* best_sim_out, float* second_sim_out,
                       void* stream);

/* Bytes of workspace skm_seed_kmeanspp needs. */
size_t skm_seed_workspace_size(const skm_matrix* X, int32_t k);

/* Spherical k-means++ seeding (Section 5.6, "Spherical k-means++"): centre 0
 * is row floor(u[0] n); centre t >= 1 is drawn with probability
 * proportional to alpha - max_c <x(i), c> over the centres chosen so far
 * (alpha = 1: cosine dissimilarity; alpha = 1.5: the metric form), as the
 * first row whose running weight sum exceeds u[t] W (W = total weight).
 * Rows already chosen have weight 0 (no row is drawn twice); when W = 0 the
 * lowest-index row not yet chosen is taken.  CSR or dense input (a dense
 * row is treated as the CSR row that stores every column, so both give the
 * same values).
 *   alpha          >= 1.
 *   uniforms       [host] double[k], each in [0, 1): the caller's draws.
 *   chosen_out     int32[k]: the chosen row indices in draw order.
 *   centers_out    float[k*d] row-major (nullable): the chosen rows.
 *   assign_out, best_out, second_out (nullable; int32[n], double[n],
 *                  double[n]): the assignment step against the chosen rows
 *                  rescaled to unit length, cached during the seeding
 *                  (ties to the lower index); skm_fit can start from it
 *                  (skm_options.warm_*), so pruning already works in the
 *                  first step.
 * Asynchronous: returns after enqueueing. */
int skm_seed_kmeanspp(const skm_matrix* X, int32_t k, double alpha,
                      const double* uniforms, int32_t* chosen_out,
                      float* centers_out, int32_t* assign_out, double* best_out,
                      double* second_out, void* workspace, size_t workspace_bytes,
                      void* stream);

/* Bytes of workspace skm_seed_afkmc2 needs. */
size_t skm_seed_afkmc2_workspace_size(const skm_matrix* X, int32_t k, int32_t chain);

/* AFK-MC2 seeding in the spherical form (Section 5.6 cites it with the
 * dissimilarity alpha - <x, c>): centre 0 is row floor(u[0] n) and fixes the
 * proposal distribution q(x) = w(x)/(2W) + 1/(2n), w(x) = max(0, alpha -
 * <x, c0>), W = sum of w (q = 1/n if W = 0).  Each further centre is the end
 * of a Markov chain over `chain` proposals drawn from q by inverse transform
 * (the first row whose running q sum exceeds the draw): the chain starts at
 * the first proposal and moves to proposal y when d(y) q(x) > u d(x) q(y),
 * with d(.) = max(0, alpha - max_c <., c>) over the centres chosen so far.
 * A row can be chosen twice.  CSR or dense input.
 *   chain          >= 1 proposals per centre.
 *   alpha          >= 1.
 *   uniforms       [host] double[1 + (k-1)(2 chain - 1)] in [0, 1): u[0],
 *                  then per centre the `chain` proposal draws followed by the
 *                  chain - 1 acceptance draws.
 *   chosen_out     int32[k]: chosen rows in draw order.
 *   centers_out    float[k*d] (nullable): the chosen rows.
 * Asynchronous: returns after enqueueing. */
int skm_seed_afkmc2(const skm_matrix* X, int32_t k, int32_t chain, double alpha,
                    const double* uniforms, int32_t* chosen_out, float* centers_out,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Many independent problems in one call (the batched setting: hundreds of
 * small clustering problems, each solved as in skm_fit; results and
 * statistics are identical to calling skm_fit on each problem).
 *   workers = 0, CSR input, SKM_LLOYD / SKM_HAMERLY / SKM_SIMP_HAMERLY, FP32
 *     similarities, no validate / profile / warm start: lockstep.  All
 *     problems advance one assignment step at a time on `stream`; every
 *     kernel of a step serves all problems (work items name the problem):
 *     the row walk is one persistent launch per centre-copy width that takes
 *     (problem, row tile) items from a device queue, with tile sizes from a
 *     table measured on this GPU (options.batch_tile_rows overrides it), and
 *     the centre step is one launch per kernel.  Steps after the first are
 *     queued eight at a time as one captured HIP graph, replayed until every
 *     problem has stopped.
 *   otherwise (or workers >= 1): `workers` host threads (0: min(nprob, 4)),
 *     each with its own HIP stream on the caller's current device and its
 *     own slice of the workspace, run skm_fit on the problems, most
 *     expensive (stored entries x k) first.
 *   nprob            >= 1 problems.
 *   Xs, ks           [host] arrays of nprob matrices and centre counts.
 *   inits            [host] array of nprob device pointers (float[k_b*d_b]).
 *   variant, opt     as in skm_fit, shared by all problems (opt nullable).
 *   max_iters        [host] int32[nprob], each >= 1.
 *   workspace        >= skm_fit_batched_workspace_size() bytes (same
 *                    arguments) or NULL.
 *   assign_outs      [host] array of nprob device pointers (int32[n_b]).
 *   centers_outs     [host] array (nullable; entries nullable) of float[k_b*d_b].
 *   stats            [host] skm_stats[nprob] (nullable), as in skm_fit
 *                    (sim_kernel_ms stays 0 in lockstep).
 * Ordering: work starts after what is already enqueued on `stream`; the
 * call returns after every problem finished.  On error the first failing
 * problem (lowest index) is reported and problems not yet started are
 * skipped. */
size_t skm_fit_batched_workspace_size(int32_t nprob, const skm_matrix* Xs,
                                      const int32_t* ks, int32_t variant,
                                      const skm_options* opt, int32_t workers);
int skm_fit_batched(int32_t nprob, const skm_matrix* Xs, const int32_t* ks,
                    const float* const* inits, int32_t variant,
                    const int32_t* max_iters, const skm_options* opt,
                    int32_t workers, void* workspace, size_t workspace_bytes,
                    int32_t* const* assign_outs, float* const* centers_outs,
                    skm_stats* stats, void* stream);

const char* skm_status_string(int status);
const char* skm_last_error(void);

/* Version of this ABI (major * 10000 + minor * 100 + patch). */
int skm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SKM_H_ */
