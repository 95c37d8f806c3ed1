// Internal declarations shared by the kernel translation units and the
// host driver of libskm.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace skm {

// Unit roundoff of float and double.
constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53

constexpr int kBlock = 256;       // threads per block for every kernel
constexpr int kMaxGridBlocks = 2048;  // persistent grids: 8 blocks per CU

// Per-step statistics.  Kernels add into slot (blockIdx.x % kCounterSlots)
// so that no single address takes more than a few atomics; the host sums
// the slots after each step and clears them before the next.
constexpr int kCounterSlots = 64;
constexpr int kRcSlots = 16;      // slots of the largest BF16 centre-copy error
struct Counters {                 // one 128-byte line
  unsigned long long changed;     // rows whose assignment changed
  unsigned long long sims;        // point-centre similarities evaluated
  unsigned long long rechecks;    // rows re-decided in FP64
  unsigned long long tightened;   // rows whose lower bound was recomputed
  unsigned long long tight_saved; // tightenings that pruned the row
  unsigned long long rows_done;   // rows walked by the similarity kernel
  unsigned long long nnz_done;    // their stored entries
  unsigned long long reserved[9];
};

// Values that persist across steps (written by single threads).
struct Persist {
  double objective;               // sum_j |S_j| after the last update
  unsigned long long ccsims;      // centre-centre inner products (whole fit)
  unsigned long long list_total;  // rows of the current step's row list
  unsigned long long near_total;  // rows re-decided from candidates
  unsigned long long scan_dummy;
  double pad[11];
};

// Steps queued between two host reads of the step records.
constexpr int kStepChunk = 8;

// Totals of one assignment step, summed from its counter slots on the device.
struct StepRec {
  unsigned long long changed, sims, rechecks, tightened, tight_saved, rows_done, nnz_done;
  double objective;               // sum_j |S_j| after the previous centre update
  int32_t valid;                  // 1: the step ran (the fit had not stopped before it)
  int32_t pad[7];
};

// State and decisions of the step loop kept on the device, so that steps are
// queued without a host round trip: the stop flag (no assignment changed);
// whether the next assignment step runs the bound tests at all (when too few
// rows were pruned they cost more than they save: the step then walks every
// row and refreshes every bound exactly); whether the coming centre update
// recomputes the centre-centre products, carries them as bounds, or skips
// them (no tests next step); and whether the next step tightens lower
// bounds.  None of these decisions changes a result, only the work.
struct StepCtl {
  int32_t stop;
  int32_t gram_on;                // the variant keeps centre-centre products
  int32_t gram_mode;              // coming centre update: 0 none, 1 exact, 2 carried
  int32_t gram_force;             // the exact update recomputes every tile
  int32_t gram_updates;           // exact or carried updates so far
  int32_t gram_since_exact;       // carried updates since the last exact one
  int32_t gram_stale;             // a centre update was skipped since the last one
  int32_t tests;                  // the next assignment step runs the bound tests
  int32_t test_next;              // step of the next test probe
  int32_t test_gap;               // probe interval, doubled after each failed probe
  int32_t tighten;                // the next assignment step tightens
  int32_t tight_next;             // step of the next tightening probe
  int32_t tight_gap;              // probe interval, doubled after each failed probe
  int32_t step;                   // batched fits: assignment steps taken so far
  double test_min;                // pruned-row fraction below which tests are switched off
  double tight_rate;              // pruned / tightened when last measured
  double tight_min;               // rate below which tightening is switched off
  int32_t max_iter;               // batched fits: the problem's step limit (stop = 2 there)
  int32_t pad1;
  double pad[5];
};
static_assert(sizeof(StepRec) == 96 && sizeof(StepCtl) == 128, "record layout");

__device__ __forceinline__ Counters* counter_slot(Counters* base) {
  return base + (blockIdx.x % kCounterSlots);
}

// Smallest and second smallest movement cosine over all centres, with the
// sine of the same (upper-bounded) movement angle.
struct MoveMin {
  double pc1, ps1, pc2, ps2;
  int32_t idx1;
  int32_t pad;
};

// Group geometry of the row kernels: G lanes per row, each lane owning R
// float4 chunks of centres, so kp = 4 * G * R padded centres per CT row.
struct Geometry {
  int G, R, kp;
};
Geometry pick_geometry(int k);

enum AssignMode {
  kModeAssign = 0,        // skm_assign: a, best, second
  kModeFit = 1,           // exhaustive step of a fit: a, l, u
  kModeFitElkanInit = 2,  // first step of an Elkan fit: also u(i, j) for all j
  kModeHamerly = 3,       // Hamerly step: bound update and tests, walk if needed
  kModeYinYang = 4,       // Yin-Yang step: group bounds, tests, walk if needed
  kModeElkan = 5          // Elkan step: pair bounds, point and pair tests, walk if needed
};

// Running result of a row across the launches of a chunked walk (the
// centres walked a chunk at a time): the best value so far (the canonical
// FP64 value when exact, else the FP32 one with error bound err), the
// largest value of every other centre seen so far (FP32 or FP64), the largest
// FP32 error bound of any chunk, the best centre, flags (bit 0: the row
// is walked in this step; bit 1: best is exact; bit 2: some FP64
// re-decision was made for the row; bit 3: best is the FP32 winner of a
// chunk whose top two lie within their error bounds), and for Yin-Yang the
// groups (bit f of surv0, then surv1) that this step's filters left to walk.
struct RowRun {
  double best, second, err, errmax;
  int32_t bj, flags;
  uint64_t surv0, surv1;
};

struct AssignArgs {
  const int64_t* rp;
  const int32_t* ci;
  const float* v;
  const float* CT;      // d x kp float, centre-minor
  const void* CT16;     // d x kp FP16 copy (nullable): the row walk reads it
  const int32_t* negflag;  // nonzero if any row or initial centre has a negative value
  const double* C64;    // k x d double, row-major
  int64_t d;
  int32_t k, kp;
  int64_t n_rows;
  int32_t* a;                 // prev (read when read_prev) and new assignment
  int32_t read_prev;
  // assign mode
  float* best_out;
  float* second_out;
  // fit modes
  float* l;
  float* u;
  float* ue;                  // Elkan upper bounds n x kp (init mode)
  const float* eta;           // per-row bound on | |x| - 1 |
  double delta_c;             // bound on | |c| - 1 | of the FP64 centres
  Counters* cnt;              // kCounterSlots slots (nullable in assign mode)
  // Hamerly mode
  const double* pc;
  const double* ps;
  const MoveMin* mm;
  const double* gmax;         // per centre max_{j != a} <c_a, c_j> + delta_G
  int32_t simplified;
  int32_t bound_form;
  int32_t try_tighten;
  // nullable: the fit's step control (stop flag; tightening decided there)
  const StepCtl* ctl;
  // with ctl: 0 always runs, 1 only when the step runs the bound tests,
  // 2 only when it does not (a full walk that refreshes every bound)
  int32_t gate;
  // Elkan: k x k centre inner products (full variant) and their bound
  const double* Gm;
  double delta_g;
  // Yin-Yang: n x ng group upper bounds (also written by the first step's
  // fit mode when set) and the cosine/sine of each group's largest movement
  float* uy;
  int32_t ng;
  const double* gpc;
  const double* gps;
  // chunked walks (FP32 copy at large k): this launch walks centres j0 ...
  // j0 + chunk - 1 (kp stays the row stride of the centre copies);
  // chunk_last marks the launch of the last chunk; rs holds every row's
  // running result between the launches
  int32_t j0;
  int32_t chunk_last;
  RowRun* rs;
  // chunked Elkan: per row kp / 256 words, bit q of word t set when the
  // 4-centre unit 64 t + q holds a centre whose pair tests failed (or the
  // assigned centre); written by the first launch of a step
  uint64_t* umask;
  // row-walk layout of the FP32 copy at kp = 32 ... 512 for the fit and
  // Hamerly modes (0 default, 1 alternative; see walk_tuning.h)
  int32_t layout;
};
constexpr int kYYGroup = 32;  // centres per Yin-Yang group
// Centres per launch of a chunked walk (FP32 centre copy): 1 KB of every
// centre row, which is what the row walk streams fastest.
constexpr int kChunkF32 = 256;
// The same 1 KB per centre row with the FP16 copy (Yin-Yang steps).
constexpr int kChunkF16 = 512;


struct DenseSimArgs {
  const void* X;              // rows: bf16 (padded copy) or f32 (caller), n x ldx
  int64_t ldx;
  const void* C;              // packed centres: bf16 or f32, kpad x dp
  int32_t k, kpad, dp, d;
  const int32_t* rows;        // nullable: identity
  const unsigned long long* rows_count;  // nullable: n_rows
  int64_t n_rows;
  float* best;                // per slot (top-2 mode)
  int32_t* best_j;
  float* second;
  const float* thr;           // per slot (candidate mode)
  int32_t* cand;              // slot x cand_cap
  int32_t* cand_n;
  int32_t cand_cap;
};

struct DensePostArgs {
  const int32_t* rows;
  const unsigned long long* rows_count;
  int64_t n_rows;
  int32_t k, dp;
  int32_t bf16;
  int32_t read_prev;
  const float* best;
  const int32_t* best_j;
  const float* second;
  const float* eta;
  const float* xr;            // BF16: per-row |x^ - x| (nullable: worst case)
  const float* rcmax;         // BF16: largest centre-copy error, kRcSlots slots (nullable: worst case)
  double delta_c;
  int32_t* a;
  float* l;
  float* u;
  int32_t* near;              // per slot flag
  float* thr;                 // per slot threshold of the candidate pass
  float* best_out;            // nullable raw outputs (assign entry point)
  float* second_out;
  Counters* cnt;
};

struct DenseExactArgs {
  const float* X;             // caller's FP32 rows
  int64_t ldx;
  const double* C64;
  int32_t k, d, dp;
  int32_t bf16;
  int32_t read_prev;
  const int32_t* rows;        // slot -> row of the similarity pass (nullable)
  const int32_t* near_list;   // candidate-pass index -> slot
  const unsigned long long* near_count;
  const int32_t* cand;
  const int32_t* cand_n;
  int32_t cand_cap;
  const float* best;          // per slot
  const int32_t* best_j;
  const float* eta;
  const float* xr;            // as in DensePostArgs
  const float* rcmax;
  double delta_c;
  int32_t* a;
  float* l;
  float* u;
  float* best_out;            // nullable raw outputs (assign entry point)
  float* second_out;
  Counters* cnt;
};

struct DenseHamerlyArgs {
  const float* X;
  int64_t ldx;
  const double* C64;
  int32_t k, d;
  int64_t n;
  const int32_t* a;
  float* l;
  float* u;
  const float* eta;
  const double* pc;
  const double* ps;
  const MoveMin* mm;
  const double* gmax;
  double delta_c;
  int32_t simplified, bound_form, try_tighten;
  int32_t* flag;
  Counters* cnt;
};

// ------------------------------------------------------------------------
// Batched fits: many small CSR problems advance in lockstep, one assignment
// step at a time, each kernel of a step serving every problem (work items
// name the problem).  Everything a kernel needs of problem p is in FitView p.
// ------------------------------------------------------------------------
struct FitView {
  const int64_t* rp;
  const int32_t* ci;
  const float* v;
  int64_t n, d;
  int32_t k, kp;
  const float* init;          // caller's initial centres, k x d
  float* CT;                  // d x kp FP32 centre copy
  double* C64;                // k x d
  long long* S;               // k x d fixed-point member sums
  float* eta;
  int32_t* a;
  int32_t* a_old;
  double* norm64;
  double* part;
  double* part_sq;
  double* pc;
  double* ps;
  int32_t* dirty;
  MoveMin* mm;
  double* G;                  // Gram variants only
  double* gmax;
  double* gpart;
  Counters* cnt;              // kStepChunk x kCounterSlots
  Persist* per;
  StepCtl* ctl;
  StepRec* rec;               // kStepChunk records
  float* maxeta;              // kCounterSlots
  double* initnorm;           // k
  int32_t nchunk, nslice;
  int64_t slice_len;
  double fx, fx_inv, delta_c, delta_g;
  double test_min, tight_min;
  int32_t gram;               // the variant keeps centre-centre products
  int32_t max_iter;
};

// Work items of the batched kernels: .x names the problem.
//  rows      (p, first row): 256 rows (row_eta, update) or the tuned tile (walk)
//  centres   (p, centre j)
//  transpose (p, centre tile, first column tile, 0): kTransposeGroup column tiles
//  gram      (p, tile pair, column slice, 0)
constexpr int kTransposeGroup = 16;
hipError_t launch_b_row_eta(const FitView* V, const int2* items, int n_items, hipStream_t s);
hipError_t launch_b_init_centres(const FitView* V, const int2* items, int n_items,
                                 hipStream_t s);
hipError_t launch_b_transpose(const FitView* V, const int4* items, int n_items, int use_dirty,
                              hipStream_t s);
hipError_t launch_b_step_init(const FitView* V, int nprob, hipStream_t s);
hipError_t launch_b_step_end(const FitView* V, int nprob, int slot, hipStream_t s);
hipError_t launch_b_update_scan(const FitView* V, const int2* items, int n_items, hipStream_t s);
hipError_t launch_b_sumsq(const FitView* V, const int2* items, int n_items, hipStream_t s);
hipError_t launch_b_normalize(const FitView* V, const int2* items, int n_items, hipStream_t s);
hipError_t launch_b_finalize(const FitView* V, int nprob, hipStream_t s);
hipError_t launch_b_gram(const FitView* V, const int4* pair_items, int n_pair_items,
                         const int2* centre_items, int n_centre_items, hipStream_t s);
// Row walk of one assignment step for every problem of one centre-copy width
// (kp): a persistent grid takes (problem, row tile) items from an atomic
// queue (*queue must be 0 at launch).  args[item.x * arg_stride + arg_off]
// are the walk arguments of the item's problem; mode as in launch_assign.
hipError_t launch_assign_batched(const AssignArgs* args, int arg_stride, int arg_off,
                                 const int2* items, int n_items, int tile_rows, int kp,
                                 int mode, unsigned int* queue, hipStream_t s);

// ---- launchers (kernels_dense.hip) ----
size_t dense_sim_lds_bytes(bool bf16, int dp);
hipError_t launch_dense_sim(const DenseSimArgs& A, bool bf16, int mode, hipStream_t s);
hipError_t launch_dense_post(const DensePostArgs& A, hipStream_t s);
hipError_t launch_dense_exact(const DenseExactArgs& A, int64_t max_rows, hipStream_t s);
hipError_t launch_dense_hamerly(const DenseHamerlyArgs& A, hipStream_t s);
hipError_t launch_gather_near(const int32_t* near_list, const unsigned long long* cnt,
                              int64_t max_rows, const int32_t* rows, const float* thr_slot,
                              int32_t* out_rows, float* out_thr, hipStream_t s);
int compact_blocks(int64_t nmax);
hipError_t launch_compact(const int32_t* flags, const unsigned long long* nptr, int64_t nmax,
                          int32_t* bcnt, int32_t* boff, int32_t* list,
                          unsigned long long* total, int32_t* zero_at, hipStream_t s);
hipError_t launch_cluster_sums(const int32_t* a, int64_t n, int32_t k, const float* X,
                               int64_t ldx, int64_t d, double fx, int32_t* cnt, int32_t* start,
                               int32_t* cursor, int32_t* perm, long long* S, int32_t* dirty,
                               unsigned long long* scratch_total, hipStream_t s);
hipError_t launch_dense_update_scan(const float* X, int64_t ldx, const int32_t* a,
                                    int32_t* a_old, int64_t n, int64_t d, double fx,
                                    long long* S, int32_t* dirty, hipStream_t s);
hipError_t launch_copy_assign(const int32_t* a, int32_t* a_old, int64_t n, hipStream_t s);
hipError_t launch_pack_centres(const double* C64, int32_t k, int64_t d, int dp,
                               const int32_t* dirty, int bf16, void* out, float* rcmax,
                               hipStream_t s);
hipError_t launch_dense_prep(const float* X, int64_t ldx, int64_t n, int64_t d, int dp,
                             float* eta, float* max_eta, void* Xb, float* xr, hipStream_t s);

// ---- launchers (kernels_assign.hip) ----
hipError_t launch_assign(const AssignArgs& A, int mode, hipStream_t s);
// One launch of a chunked walk (fit, Hamerly, Yin-Yang, Elkan or Elkan-init
// mode with the FP32 centre copy, chunks of kChunkF32 centres; Yin-Yang mode
// with the FP16 copy, chunks of kChunkF16; A.j0, A.chunk_last and A.rs set,
// and A.umask for Elkan).
hipError_t launch_assign_chunk(const AssignArgs& A, int mode, hipStream_t s);


// ---- launchers (kernels_update.hip) ----
hipError_t launch_row_eta(const int64_t* rp, const float* v, int64_t n, float* eta,
                          float* max_eta, hipStream_t s);
hipError_t launch_init_centres(const float* init, int32_t k, int64_t d, int normalize,
                               double* C64, double* init_norm, hipStream_t s);
hipError_t launch_transpose(const double* C64, int32_t k, int64_t d, int32_t kp,
                            const int32_t* dirty, float* CT, hipStream_t s, void* CT16 = nullptr);
// Sets *flag (not cleared here) if any of v[0..nnz) or init[0..ninit) is negative.
hipError_t launch_neg_scan(const float* v, int64_t nnz, const float* init, int64_t ninit,
                           int32_t* flag, hipStream_t s);
// Input checks (validate = 2).  Each records the first violation as
// row * 8 + kind in *bad (atomic minimum; the caller fills it with ~0 first).
constexpr int kBadRowPtr = 1;   // row_ptr[0] != 0, decreasing, or row_ptr[n] != nnz
constexpr int kBadColumn = 2;   // column id outside [0, d)
constexpr int kBadOrder = 3;    // column ids not strictly ascending within the row
constexpr int kBadValue = 4;    // NaN or infinite value
hipError_t launch_check_rowptr(const int64_t* rp, int64_t n, int64_t nnz,
                               unsigned long long* bad, hipStream_t s);
// Only after launch_check_rowptr found row_ptr valid.
hipError_t launch_check_entries(const int64_t* rp, const int32_t* ci, const float* v, int64_t n,
                                int64_t d, unsigned long long* bad, hipStream_t s);
hipError_t launch_check_dense(const float* x, int64_t ld, int64_t n, int64_t d,
                              unsigned long long* bad, hipStream_t s);
hipError_t launch_update_scan(const int64_t* rp, const int32_t* ci, const float* v,
                              const int32_t* a, int32_t* a_old, int64_t n, int64_t d,
                              double fx_scale, long long* S, int32_t* dirty, hipStream_t s);
hipError_t launch_sumsq_partial(const long long* S, int32_t k, int64_t d, double fx_inv,
                               const int32_t* dirty, double* part_sq, int nchunk, hipStream_t s);
hipError_t launch_normalize_move(const long long* S, int32_t k, int64_t d, double fx_inv,
                                 const int32_t* dirty, const double* part_sq, double* C64,
                                 double* part, int nchunk, hipStream_t s);
hipError_t launch_centre_finalize(int32_t k, int64_t d, const int32_t* dirty, double* norm64,
                                  const double* part_sq, const double* part, int nchunk,
                                  double delta_c, double* pc, double* ps, MoveMin* mm,
                                  Persist* per, hipStream_t s);
hipError_t launch_clear_dirty(int32_t* dirty, int32_t k, hipStream_t s);
// Movement-bound update of G and gmax in place of an exact Gram.
hipError_t launch_gram_carry(double* G, int32_t k, const double* pc, const double* ps,
                             double delta_g, double* gmax, hipStream_t s,
                             const StepCtl* ctl = nullptr);
// Initial step control: gram_on as given; warm = the first centre update
// (after a warm start) is already decided as an exact, full one.
hipError_t launch_step_init(StepCtl* ctl, int gram_on, int warm, double test_min,
                            double tight_min, hipStream_t s);
// After assignment step t: clears the dirty flags of the previous centre
// update, sums the step's counter slots into rec, stops the fit when no
// assignment changed, and decides the coming centre-centre update, the next
// step's bound tests and tightening (see StepCtl).  gram_queued: the Gram
// kernels are queued for the coming centre update (else no tests that need
// them run in step t + 1).
hipError_t launch_step_end(const Counters* cnt, StepCtl* ctl, StepRec* rec, const Persist* per,
                           int32_t t, int64_t n, int32_t* dirty, int32_t k, int gram_queued,
                           hipStream_t s);
// Whether the centre step after assignment step t recomputes the Gram
// exactly (else it carries the bounds): the first two centre steps, every
// fourth after an exact one, and whenever more than 5% of the rows changed.
__host__ __device__ inline bool gram_exact_step(int updates_done, int since_exact,
                                                int64_t changed, int64_t n) {
  return updates_done < 2 || since_exact >= 3 || changed * 20 > n;
}
// First assignment step from a given assignment and FP64 top-2 (uy: the
// Yin-Yang group bounds, nullable, ng per row).  rp = nullptr: dense rows of
// dense_d columns.
hipError_t launch_warm_start(const int64_t* rp, int64_t n, int32_t k, int32_t kp,
                             const int32_t* wa, const double* wb, const double* ws2,
                             const float* eta, double delta_c, int32_t* a, float* l, float* u,
                             float* ue, float* uy, int32_t ng, hipStream_t s,
                             int64_t dense_d = 0);
// Cosine and sine of every Yin-Yang group's largest movement.
hipError_t launch_group_move(const double* pc, const double* ps, int32_t k, int32_t ng,
                             double* gpc, double* gps, hipStream_t s);
// One step of spherical k-means++ seeding: choose centre t, write it to
// centres (FP32 k x d, zeroed) and its unit FP64 copy to c64 (d), refresh
// every row's running top-2 (a, best, second), weights w and per-block
// weight sums part.
hipError_t launch_kpp_step(const int64_t* rp, const int32_t* ci, const float* v, const float* x,
                           int64_t ld, int64_t n, int64_t d, int32_t t, double alpha,
                           const double* u_dev,
                           uint8_t* taken, int32_t* chosen, float* centres, double* c64,
                           int32_t* a, double* best, double* second, double* w, double* part,
                           hipStream_t s);
// AFK-MC2 seeding: chooses k rows (chosen), writes them to centres (FP32
// k x d, zeroed by the caller) and their unit FP64 copies to C64 (k x d).
// Scratch: w, prefix (n each), W (1), cand (m), dcand (m).
hipError_t launch_afkmc2(const int64_t* rp, const int32_t* ci, const float* v, const float* x,
                         int64_t ld, int64_t n, int64_t d, int32_t k, int32_t m, double alpha,
                         const double* u_dev,
                         int32_t* chosen, float* centres, double* C64, double* w, double* W,
                         double* prefix, int32_t* cand, double* dcand, hipStream_t s);
// Gram slicing over d: number of column slices and their length.
void gram_slicing(int32_t k, int64_t d, int* nslice, int64_t* slice_len);
hipError_t launch_gram(const double* C64, int32_t k, int64_t d, const int32_t* dirty,
                       int force_all, double* part, int nslice, int64_t slice_len,
                       double* G, double* gmax, double delta_g, Persist* per,
                       hipStream_t s, const StepCtl* ctl = nullptr);
hipError_t launch_c64_to_f32(const double* C64, int64_t count, float* out, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t count, double value, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s);

}  // namespace skm
