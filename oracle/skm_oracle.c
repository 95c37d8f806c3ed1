/*
 * FP64 CPU oracle for accelerated spherical k-means (Schubert, Lang, Feher,
 * "Accelerating Spherical k-Means", arXiv 2107.04074).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code,
 * header, table or constant with the GPU library and must never be used as
 * a fallback for it.
 *
 * Everything is plain double-precision loops written for readability:
 *   - similarities are dot products of unit vectors (Section 2), summed
 *     sequentially over the stored entries of a row;
 *   - the assignment keeps argmax_j <x(i), c(j)> (Section 5, assignment
 *     equation) with a fixed tie rule (see ARGMAX below);
 *   - the update sets c(j) to the member sum scaled to unit length
 *     (Section 5, centre equation);
 *   - Elkan, simplified Elkan, Hamerly and simplified Hamerly follow the
 *     steps of Sections 5.1 to 5.4 with the bound updates of Eq. (6), (7)
 *     and (9) of Section 4 / 5.3.
 * The plain Lloyd iteration is the definition of the result; the bounded
 * variants exist to count similarity computations and to show that they
 * reach exactly the same assignments (the central claim of Section 4).
 *
 * Readings where the paper is silent (documented with the project design):
 *   ARGMAX   ties: keep the previous assignment if it attains the maximum,
 *            otherwise the lowest index among the maxima.
 *   STOP     an iteration is one assignment step; stop when no assignment
 *            changed or after max_iter steps; after every step that changed
 *            something the centres are updated, so the returned centres are
 *            always the normalised member sums of the returned assignment.
 *   EMPTY    a cluster without members keeps its previous centre (p = 1).
 *   GUARDS   Eq. (7) is cos(theta_u - theta_p) and only bounds while
 *            theta_u >= theta_p, so u <- 1 when u >= p; Eq. (6) is
 *            cos(theta_l + theta_p) and only bounds while the sum stays
 *            below pi, so l <- -1 when l <= -p.
 *   HAMERLY  the default upper-bound update applies the guarded Eq. (7)
 *            with p'(a) = min_{j != a} p(j); the guarded form is monotone in
 *            the movement angle, so the largest movement is the worst case.
 *            bound_form = 1 uses Eq. (9) instead where it is valid
 *            (u >= 0 and p' >= 0) and the guarded Eq. (7) elsewhere.
 *            bound_form = 2 applies Eq. (6)/(7) exactly as printed, without
 *            guards; it exists only so tests can show what the guards
 *            prevent and is never a correct configuration.
 *   MOVEMENT 1 - p(j) is evaluated as |c(j) - c'(j)|^2 / 2 (Eq. (2)
 *            relation) rather than 1 - <c, c'>, which cancels near 1.
 *   MARGIN   every pruning test leaves a margin DELTA = 1e-10 so that
 *            double rounding in the bounds can never prune a centre whose
 *            computed similarity could reach the maximum.
 *   INIT     the initial centres are rescaled to unit length in double
 *            precision before the first step: the paper's centres are unit
 *            vectors, and rows picked as initial centres are unit only up to
 *            float rounding.
 *   COSINE   stored rows are unit only up to float rounding, so bounds are
 *            kept on the cosine <x, c> / |x| (the definition of sim in
 *            Section 2), for which the triangle inequalities of Eq. (4)/(5)
 *            hold exactly; assignment decisions compare the dot products
 *            themselves, which rank centres the same way for a fixed row.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DELTA 1e-10

/* Threads the OpenMP loops of this library use. */
int oracle_threads(void) { return omp_get_max_threads(); }

enum { ORC_LLOYD = 0, ORC_ELKAN = 1, ORC_HAMERLY = 2, ORC_SIMP_ELKAN = 3,
       ORC_SIMP_HAMERLY = 4, ORC_YINYANG = 5 };

/* YINYANG reading (Section 5.5 names the method and states that the bounds
 * transfer unchanged): the centres are split into groups of YY_GROUP
 * consecutive indices; every point keeps l(i) and one upper bound u(i, f)
 * per group f >= max over the group's centres other than a(i).  The group
 * bounds follow the guarded Eq. (7) with the group's largest movement; a
 * point whose l(i) is at least every group bound is skipped (global
 * filter), otherwise l(i) is tightened and only the groups whose bound
 * still exceeds it are recomputed (group filter). */
#define YY_GROUP 32

typedef struct {
  int64_t n, d;
  const int64_t *rp;
  const int32_t *ci;
  const float *v;
} csr_t;

/* <x(i), c> with c a dense length-d vector, summed in stored-entry order. */
static double sim(const csr_t *X, int64_t i, const double *c) {
  double s = 0.0;
  for (int64_t e = X->rp[i]; e < X->rp[i + 1]; ++e)
    s += (double)X->v[e] * c[X->ci[e]];
  return s;
}

static void all_sims(const csr_t *X, int64_t i, int32_t k, const double *C,
                     double *s) {
  for (int32_t j = 0; j < k; ++j) s[j] = sim(X, i, C + (size_t)j * X->d);
}

/* ARGMAX reading; *second = max over j != result (or -inf when k == 1). */
static int32_t argmax_rule(const double *s, int32_t k, int32_t prev,
                           double *best, double *second) {
  double mx = -INFINITY;
  for (int32_t j = 0; j < k; ++j)
    if (s[j] > mx) mx = s[j];
  int32_t a = -1;
  if (prev >= 0 && prev < k && s[prev] == mx) {
    a = prev;
  } else {
    for (int32_t j = 0; j < k; ++j)
      if (s[j] == mx) { a = j; break; }
  }
  double sc = -INFINITY;
  for (int32_t j = 0; j < k; ++j)
    if (j != a && s[j] > sc) sc = s[j];
  *best = mx;
  *second = sc;
  return a;
}

/* -------------------------------------------------------------------- */
/* exported single steps                                                 */
/* -------------------------------------------------------------------- */

/* Assignment step from given centres C (k x d, row-major).  a_prev may be
 * NULL (first iteration).  Outputs: a, best similarity, second best. */
void oracle_assign(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                   const float *v, int32_t k, const double *C,
                   const int32_t *a_prev, int32_t *a_out, double *s1_out,
                   double *s2_out) {
  csr_t X = {n, d, rp, ci, v};
#pragma omp parallel
  {
    double *s = (double *)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      double b, sc;
      all_sims(&X, i, k, C, s);
      a_out[i] = argmax_rule(s, k, a_prev ? a_prev[i] : -1, &b, &sc);
      if (s1_out) s1_out[i] = b;
      if (s2_out) s2_out[i] = sc;
    }
    free(s);
  }
}

/* The same assignment step with the centres stored transposed: CT is d x k,
 * CT[t * k + j] = c(j)_t.  Every similarity is the same sequential sum over
 * the row's stored entries, in storage order and with the same operations
 * as in oracle_assign, so the results are identical bit for bit; only the
 * memory layout differs (each stored entry reads one contiguous column of
 * the centres, which keeps the largest sparse workloads feasible here). */
void oracle_assign_ct(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                      const float *v, int32_t k, const double *CT,
                      const int32_t *a_prev, int32_t *a_out, double *s1_out,
                      double *s2_out) {
  (void)d;
#pragma omp parallel
  {
    double *s = (double *)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      double b, sc;
      for (int32_t j = 0; j < k; ++j) s[j] = 0.0;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const double x = (double)v[e];
        const double *c = CT + (size_t)ci[e] * (size_t)k;
        for (int32_t j = 0; j < k; ++j) s[j] += x * c[j];
      }
      a_out[i] = argmax_rule(s, k, a_prev ? a_prev[i] : -1, &b, &sc);
      if (s1_out) s1_out[i] = b;
      if (s2_out) s2_out[i] = sc;
    }
    free(s);
  }
}

/* INIT reading: rescale every centre row of C (k x d) to unit length in
 * double precision (rows of zeros stay as they are). */
void oracle_init_centres(int32_t k, int64_t d, double *C) {
  for (int32_t j = 0; j < k; ++j) {
    double *c = C + (size_t)j * (size_t)d, ss = 0.0;
    for (int64_t t = 0; t < d; ++t) ss += c[t] * c[t];
    if (ss > 0.0) {
      const double nrm = sqrt(ss);
      for (int64_t t = 0; t < d; ++t) c[t] /= nrm;
    }
  }
}

/* Similarities of the listed rows to all centres: out is m x k. */
void oracle_sims(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                 const float *v, int32_t k, const double *C,
                 const int64_t *rows, int64_t m, double *out) {
  csr_t X = {n, d, rp, ci, v};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < m; ++q) all_sims(&X, rows[q], k, C, out + (size_t)q * k);
}

/* Centre step: c(j) = S(j) / |S(j)| with S(j) the member sum; an empty
 * cluster keeps C_prev(j).  norms_out (nullable) receives |S(j)|.  Returns
 * sum_j |S(j)|, which equals sum_i <x(i), c(a(i))> after the update. */
double oracle_update(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                     const float *v, int32_t k, const int32_t *a,
                     const double *C_prev, double *C_out, double *norms_out) {
  double *S = (double *)calloc((size_t)k * (size_t)d, sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    double *Sj = S + (size_t)a[i] * (size_t)d;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) Sj[ci[e]] += (double)v[e];
  }
  double obj = 0.0;
  for (int32_t j = 0; j < k; ++j) {
    const double *Sj = S + (size_t)j * (size_t)d;
    double ss = 0.0;
    for (int64_t t = 0; t < d; ++t) ss += Sj[t] * Sj[t];
    const double nrm = sqrt(ss);
    if (norms_out) norms_out[j] = nrm;
    obj += nrm;
    double *Cj = C_out + (size_t)j * (size_t)d;
    if (nrm > 0.0) {
      for (int64_t t = 0; t < d; ++t) Cj[t] = Sj[t] / nrm;
    } else if (Cj != C_prev + (size_t)j * (size_t)d) {
      memcpy(Cj, C_prev + (size_t)j * (size_t)d, sizeof(double) * (size_t)d);
    }
  }
  free(S);
  return obj;
}

/* -------------------------------------------------------------------- */
/* spherical k-means++ seeding (Section 5.6, "Spherical k-means++")        */
/* -------------------------------------------------------------------- */

/* The first centre is row floor(u[0] n); centre t >= 1 is drawn with
 * probability proportional to alpha - max_c <x(i), c> over the centres
 * chosen so far (alpha = 1 is the cosine form, alpha = 1.5 the metric form
 * the section mentions), by inverse transform sampling with u[t]: the first
 * row whose running weight sum exceeds u[t] * W, W the total.  Readings
 * (SEED): rows already chosen get weight 0, so no row is drawn twice;
 * negative weights count as 0; if W = 0 the lowest-index row not yet chosen
 * is taken.  Centres are the chosen rows rescaled to unit length (INIT
 * reading).  The maximum over the chosen centres is cached per row and
 * updated once per new centre (the O(nk) scheme of the section); on return
 * best/assign/second hold the assignment step against all k centres
 * (ARGMAX with no previous assignment: the lowest index among maxima). */
void oracle_kmeanspp(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                     const float *v, int32_t k, double alpha, const double *u,
                     int32_t *chosen, int32_t *assign, double *best, double *second) {
  csr_t X = {n, d, rp, ci, v};
  double *c = (double *)calloc((size_t)d, sizeof(double));
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  char *taken = (char *)calloc((size_t)n, 1);
  for (int64_t i = 0; i < n; ++i) {
    best[i] = -INFINITY;
    second[i] = -INFINITY;
    assign[i] = -1;
  }
  int64_t p = (int64_t)floor(u[0] * (double)n);
  if (p > n - 1) p = n - 1;
  for (int32_t t = 0; t < k; ++t) {
    if (t > 0) {
      double W = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const double wi = taken[i] ? 0.0 : alpha - best[i];
        w[i] = wi > 0.0 ? wi : 0.0;
        W += w[i];
      }
      p = -1;
      if (W > 0.0) {
        const double target = u[t] * W;
        double run = 0.0;
        int64_t last = -1;
        for (int64_t i = 0; i < n; ++i) {
          if (w[i] > 0.0) last = i;
          run += w[i];
          if (run > target) { p = i; break; }
        }
        if (p < 0) p = last; /* rounding left the target unreached */
      }
      if (p < 0)
        for (int64_t i = 0; i < n; ++i)
          if (!taken[i]) { p = i; break; }
    }
    chosen[t] = (int32_t)p;
    taken[p] = 1;
    /* centre t: row p scaled to unit length */
    memset(c, 0, sizeof(double) * (size_t)d);
    double ss = 0.0;
    for (int64_t e = rp[p]; e < rp[p + 1]; ++e) {
      c[ci[e]] = (double)v[e];
      ss += (double)v[e] * (double)v[e];
    }
    if (ss > 0.0) {
      const double nrm = sqrt(ss);
      for (int64_t e = rp[p]; e < rp[p + 1]; ++e) c[ci[e]] /= nrm;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const double s = sim(&X, i, c);
      if (s > best[i]) {
        second[i] = best[i];
        best[i] = s;
        assign[i] = t;
      } else if (s > second[i]) {
        second[i] = s;
      }
    }
  }
  free(c);
  free(w);
  free(taken);
}

/* AFK-MC2 seeding in its spherical form (Section 5.6 cites it with the
 * dissimilarity alpha - <x, c>): centre 0 is row floor(u[0] n) and fixes the
 * proposal distribution q(x) = w(x) / (2 W) + 1 / (2 n), w(x) = max(0,
 * alpha - <x, c0>), W = sum w (q = 1/n when W = 0).  Centre t >= 1 comes
 * from a Markov chain of length m over proposals y_1 .. y_m drawn from q by
 * inverse transform sampling (the first row whose running q sum exceeds the
 * uniform; the last row if rounding leaves it unreached): the chain starts
 * at y_1 and moves to y_j when d(y_j) q(x) > u d(x) q(y_j), d(.) =
 * max(0, alpha - max_c <., c>) over the centres chosen so far, u the j-th
 * acceptance uniform (SEED-MC reading: the multiplied form decides the
 * 0/0 case as "stay").  Uniforms: u[0] for centre 0, then per centre t the
 * m proposal draws followed by the m - 1 acceptance draws.  Centres are the
 * chosen rows rescaled to unit length (INIT).  Rows may be chosen twice (the
 * chain does not exclude centres); the fit then keeps an empty cluster. */
static void unit_row_centre(const csr_t *X, int64_t p, double *c) {
  memset(c, 0, sizeof(double) * (size_t)X->d);
  double ss = 0.0;
  for (int64_t e = X->rp[p]; e < X->rp[p + 1]; ++e) {
    c[X->ci[e]] = (double)X->v[e];
    ss += (double)X->v[e] * (double)X->v[e];
  }
  if (ss > 0.0) {
    const double nrm = sqrt(ss);
    for (int64_t e = X->rp[p]; e < X->rp[p + 1]; ++e) c[X->ci[e]] /= nrm;
  }
}

void oracle_afkmc2(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                   const float *v, int32_t k, int32_t m, double alpha, const double *u,
                   int32_t *chosen) {
  csr_t X = {n, d, rp, ci, v};
  double *C = (double *)malloc(sizeof(double) * (size_t)k * (size_t)d);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  int64_t p = (int64_t)floor(u[0] * (double)n);
  if (p > n - 1) p = n - 1;
  chosen[0] = (int32_t)p;
  unit_row_centre(&X, p, C);
  double W = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double w = alpha - sim(&X, i, C);
    q[i] = w > 0.0 ? w : 0.0;
    W += q[i];
  }
  for (int64_t i = 0; i < n; ++i)
    q[i] = W > 0.0 ? 0.5 * q[i] / W + 0.5 / (double)n : 1.0 / (double)n;
  const double *ut = u + 1;
  for (int32_t t = 1; t < k; ++t, ut += 2 * m - 1) {
    int64_t x = -1;
    double dx = 0.0;
    for (int32_t j = 0; j < m; ++j) {
      /* proposal j by inverse transform on q */
      double run = 0.0;
      int64_t y = n - 1;
      for (int64_t i = 0; i < n; ++i) {
        run += q[i];
        if (run > ut[j]) { y = i; break; }
      }
      double best = -INFINITY;
      for (int32_t c = 0; c < t; ++c) {
        const double s = sim(&X, y, C + (size_t)c * (size_t)d);
        if (s > best) best = s;
      }
      double dy = alpha - best;
      if (!(dy > 0.0)) dy = 0.0;
      if (j == 0 || dy * q[x] > ut[m + j - 1] * dx * q[y]) {
        x = y;
        dx = dy;
      }
    }
    chosen[t] = (int32_t)x;
    unit_row_centre(&X, x, C + (size_t)t * (size_t)d);
  }
  free(C);
  free(q);
}

/* -------------------------------------------------------------------- */
/* bound updates (Section 4 and 5.3), exported for the tests             */
/* -------------------------------------------------------------------- */

static double clamp1(double x) { return x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x); }

/* Eq. (6) with the GUARDS reading; omp = 1 - p. */
double oracle_lower_update(double l, double p, double omp) {
  l = clamp1(l);
  if (l <= -p) return -1.0;
  return clamp1(l * p - sqrt((1.0 - l) * (1.0 + l) * omp * (1.0 + p)));
}

/* Eq. (7) with the GUARDS reading; omp = 1 - p. */
double oracle_upper_update(double u, double p, double omp) {
  u = clamp1(u);
  if (u >= p) return 1.0;
  return clamp1(u * p + sqrt((1.0 - u) * (1.0 + u) * omp * (1.0 + p)));
}

/* Eq. (9), valid for u >= 0 and p >= 0; elsewhere the guarded Eq. (7). */
double oracle_upper_eq9(double u, double p, double omp) {
  u = clamp1(u);
  if (u < 0.0 || p < 0.0) return oracle_upper_update(u, p, omp);
  return clamp1(u + sqrt((1.0 - u) * (1.0 + u) * omp * (1.0 + p)));
}

/* The printed forms without guards, for tests that show why guards exist. */
double oracle_lower_unguarded(double l, double p) {
  return l * p - sqrt((1.0 - l * l) * (1.0 - p * p));
}
double oracle_upper_unguarded(double u, double p) {
  return u * p + sqrt((1.0 - u * u) * (1.0 - p * p));
}

/* Centre-centre half-angle bound of Section 5.2: cc = sqrt((<ci,cj>+1)/2). */
double oracle_cc(double g) { return sqrt((clamp1(g) + 1.0) / 2.0); }

/* -------------------------------------------------------------------- */
/* full fit                                                              */
/* -------------------------------------------------------------------- */

/* p(j) and 1 - p(j) from old and new centres (MOVEMENT reading). */
static void movement(int32_t k, int64_t d, const double *Cold,
                     const double *Cnew, double *p, double *omp) {
  for (int32_t j = 0; j < k; ++j) {
    const double *a = Cold + (size_t)j * (size_t)d, *b = Cnew + (size_t)j * (size_t)d;
    double ss = 0.0;
    for (int64_t t = 0; t < d; ++t) {
      const double q = b[t] - a[t];
      ss += q * q;
    }
    omp[j] = 0.5 * ss;
    p[j] = 1.0 - omp[j];
  }
}

/* cc(j, j') for all pairs and s(j) = max_{j' != j} cc(j, j'). */
static void center_bounds(int32_t k, int64_t d, const double *C, double *cc,
                          double *s) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t j = 0; j < k; ++j) {
    for (int32_t q = 0; q < k; ++q) {
      if (q == j) { cc[(size_t)j * k + q] = 1.0; continue; }
      const double *a = C + (size_t)j * (size_t)d, *b = C + (size_t)q * (size_t)d;
      double g = 0.0;
      for (int64_t t = 0; t < d; ++t) g += a[t] * b[t];
      cc[(size_t)j * k + q] = oracle_cc(g);
    }
  }
  for (int32_t j = 0; j < k; ++j) {
    double m = -INFINITY;
    for (int32_t q = 0; q < k; ++q)
      if (q != j && cc[(size_t)j * k + q] > m) m = cc[(size_t)j * k + q];
    s[j] = m;
  }
}

/* Runs spherical k-means from C_init (k x d) with the given variant.
 * Per-iteration traces (each of length max_iter, nullable):
 *   changed    number of points whose assignment changed in the step
 *   sims       point-centre similarities computed in the step
 *   ccsims     centre-centre similarities computed in the step
 *   obj_assign sum_i <x(i), c(a(i))> with the centres used in the step
 *              (Lloyd only; NaN for the bounded variants)
 *   obj_update sum_j |S(j)| after the following update (NaN if none)
 *   a_trace    n x max_iter assignments (column t = step t+1)
 * check_bounds != 0 recomputes every similarity before each step's tests
 * and counts bound violations (l above its similarity, u below) into
 * *violations.  Returns the number of assignment steps executed. */
int32_t oracle_fit(int64_t n, int64_t d, const int64_t *rp, const int32_t *ci,
                   const float *v, int32_t k, const double *C_init,
                   int32_t variant, int32_t max_iter, int32_t bound_form,
                   int32_t check_bounds, int32_t *a_out, double *C_out,
                   int64_t *changed_tr, int64_t *sims_tr, int64_t *ccsims_tr,
                   double *obj_assign_tr, double *obj_update_tr,
                   int32_t *a_trace, int64_t *violations, int32_t *converged) {
  csr_t X = {n, d, rp, ci, v};
  const int elkan = variant == ORC_ELKAN || variant == ORC_SIMP_ELKAN;
  const int hamerly = variant == ORC_HAMERLY || variant == ORC_SIMP_HAMERLY;
  const int simplified = variant == ORC_SIMP_ELKAN || variant == ORC_SIMP_HAMERLY;
  const int yy = variant == ORC_YINYANG;
  const int ng = (k + YY_GROUP - 1) / YY_GROUP;

  double *C = (double *)malloc(sizeof(double) * (size_t)k * (size_t)d);
  double *Cold = (double *)malloc(sizeof(double) * (size_t)k * (size_t)d);
  memcpy(C, C_init, sizeof(double) * (size_t)k * (size_t)d);
  oracle_init_centres(k, d, C);
  int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) a[i] = -1;
  double *l = (double *)malloc(sizeof(double) * (size_t)n);
  double *uh = hamerly ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
  double *ue = elkan ? (double *)malloc(sizeof(double) * (size_t)n * (size_t)k) : NULL;
  double *uy = yy ? (double *)malloc(sizeof(double) * (size_t)n * (size_t)ng) : NULL;
  double *pg = yy ? (double *)malloc(sizeof(double) * (size_t)ng) : NULL;
  double *ompg = yy ? (double *)malloc(sizeof(double) * (size_t)ng) : NULL;
  double *p = (double *)malloc(sizeof(double) * (size_t)k);
  double *omp = (double *)malloc(sizeof(double) * (size_t)k);
  double *cc = (!simplified && (elkan || hamerly))
                   ? (double *)malloc(sizeof(double) * (size_t)k * (size_t)k) : NULL;
  double *sthr = (double *)malloc(sizeof(double) * (size_t)k);
  double *rn = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    double ss = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) ss += (double)v[e] * (double)v[e];
    rn[i] = sqrt(ss);
  }
  int64_t viol = 0;
  int32_t t, done = 0;

  for (t = 0; t < max_iter; ++t) {
    int64_t changed = 0, sims = 0, ccsims = 0;
    double obj_assign = NAN;

    if (variant == ORC_LLOYD || t == 0) {
      /* exhaustive step: Lloyd, and the first step of every variant */
      double oa = 0.0;
#pragma omp parallel reduction(+ : changed, oa)
      {
        double *s = (double *)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
          double b, sc;
          all_sims(&X, i, k, C, s);
          const int32_t na = argmax_rule(s, k, a[i], &b, &sc);
          if (na != a[i]) changed += 1;
          a[i] = na;
          oa += b;
          if (elkan || hamerly || yy) l[i] = b / rn[i];
          if (hamerly) uh[i] = sc / rn[i];
          if (yy)
            for (int32_t f = 0; f < ng; ++f) {
              double gm = -1.0; /* no other centre in the group: any bound holds */
              for (int32_t j = f * YY_GROUP; j < k && j < (f + 1) * YY_GROUP; ++j)
                if (j != na && s[j] / rn[i] > gm) gm = s[j] / rn[i];
              uy[(size_t)i * ng + f] = gm;
            }
          if (elkan)
            for (int32_t j = 0; j < k; ++j) ue[(size_t)i * k + j] = s[j] / rn[i];
        }
        free(s);
      }
      sims = n * (int64_t)k;
      obj_assign = oa;
    } else {
      /* bounded step: p and omp describe the last centre update */
      if (cc) {
        center_bounds(k, d, C, cc, sthr);
        ccsims = (int64_t)k * (k - 1) / 2;
      }
      /* p'(j) = min_{j' != j} p(j') for Hamerly: smallest and second
       * smallest movement cosine */
      int32_t jmin = -1;
      double pmin = INFINITY, pmin2 = INFINITY, ompmin = 0.0, ompmin2 = 0.0;
      for (int32_t j = 0; j < k; ++j) {
        if (p[j] < pmin) {
          pmin2 = pmin; ompmin2 = ompmin;
          pmin = p[j]; ompmin = omp[j]; jmin = j;
        } else if (p[j] < pmin2) {
          pmin2 = p[j]; ompmin2 = omp[j];
        }
      }
      if (k == 1) { pmin2 = 1.0; ompmin2 = 0.0; }
      /* YINYANG: the largest movement (smallest p) of every group */
      if (yy)
        for (int32_t f = 0; f < ng; ++f) {
          pg[f] = INFINITY;
          for (int32_t j = f * YY_GROUP; j < k && j < (f + 1) * YY_GROUP; ++j)
            if (p[j] < pg[f]) { pg[f] = p[j]; ompg[f] = omp[j]; }
        }

#pragma omp parallel reduction(+ : changed, sims, viol)
      {
        double *s = check_bounds ? (double *)malloc(sizeof(double) * (size_t)k) : NULL;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
          const int32_t prev = a[i];
          int32_t cur = prev;
          /* Eq. (6) for l(i) */
          const int raw = bound_form == 2;
          l[i] = raw ? oracle_lower_unguarded(l[i], p[cur])
                     : oracle_lower_update(l[i], p[cur], omp[cur]);
          if (yy) {
            /* Eq. (7) with every group's largest movement */
            double *ug = uy + (size_t)i * ng;
            for (int32_t f = 0; f < ng; ++f)
              ug[f] = raw ? oracle_upper_unguarded(ug[f], pg[f])
                          : oracle_upper_update(ug[f], pg[f], ompg[f]);
          } else if (elkan) {
            /* Eq. (7) for every u(i, j) */
            double *ui = ue + (size_t)i * k;
            for (int32_t j = 0; j < k; ++j)
              ui[j] = raw ? oracle_upper_unguarded(ui[j], p[j])
                          : oracle_upper_update(ui[j], p[j], omp[j]);
          } else {
            const double pp = (cur == jmin) ? pmin2 : pmin;
            const double oo = (cur == jmin) ? ompmin2 : ompmin;
            uh[i] = raw ? oracle_upper_unguarded(uh[i], pp)
                        : bound_form == 1 ? oracle_upper_eq9(uh[i], pp, oo)
                                          : oracle_upper_update(uh[i], pp, oo);
          }
          if (s) {
            all_sims(&X, i, k, C, s);
            for (int32_t j = 0; j < k; ++j) s[j] /= rn[i];
            if (l[i] > s[cur] + 1e-12) viol += 1;
            if (yy) {
              for (int32_t j = 0; j < k; ++j)
                if (j != cur && uy[(size_t)i * ng + j / YY_GROUP] < s[j] - 1e-12) viol += 1;
            } else if (elkan) {
              for (int32_t j = 0; j < k; ++j)
                if (ue[(size_t)i * k + j] < s[j] - 1e-12) viol += 1;
            } else {
              for (int32_t j = 0; j < k; ++j)
                if (j != cur && uh[i] < s[j] - 1e-12) { viol += 1; break; }
            }
          }

          if (yy) {
            double *ug = uy + (size_t)i * ng;
            double umax = -INFINITY;
            for (int32_t f = 0; f < ng; ++f) umax = ug[f] > umax ? ug[f] : umax;
            if (umax <= l[i] - DELTA) continue; /* global filter */
            const double sa = sim(&X, i, C + (size_t)cur * d);
            l[i] = sa / rn[i];
            sims += 1;
            if (umax <= l[i] - DELTA) continue;
            /* group filter: recompute the groups whose bound exceeds l */
            double best = sa;
            int32_t bj = cur;
            char *open = (char *)calloc((size_t)ng, 1);
            double *gs = (double *)malloc(sizeof(double) * (size_t)k);
            for (int32_t f = 0; f < ng; ++f) {
              if (ug[f] <= l[i] - DELTA) continue;
              open[f] = 1;
              for (int32_t j = f * YY_GROUP; j < k && j < (f + 1) * YY_GROUP; ++j) {
                if (j == cur) { gs[j] = sa; continue; }
                gs[j] = sim(&X, i, C + (size_t)j * d);
                sims += 1;
                /* ARGMAX: a switch needs a strictly larger value, ties go to
                 * the lower index among the challengers */
                if (gs[j] > best || (gs[j] == best && bj != cur && j < bj)) {
                  best = gs[j];
                  bj = j;
                }
              }
            }
            cur = bj;
            l[i] = best / rn[i];
            for (int32_t f = 0; f < ng; ++f) {
              if (!open[f]) continue;
              double gm = -1.0;
              for (int32_t j = f * YY_GROUP; j < k && j < (f + 1) * YY_GROUP; ++j)
                if (j != cur && gs[j] / rn[i] > gm) gm = gs[j] / rn[i];
              ug[f] = gm;
            }
            /* the old centre is now an ordinary member of its group */
            if (cur != prev) {
              const int32_t fo = prev / YY_GROUP;
              if (sa / rn[i] > ug[fo]) ug[fo] = sa / rn[i];
            }
            free(gs);
            free(open);
          } else if (elkan) {
            /* Sections 5.1 / 5.2 */
            if (!simplified && sthr[cur] <= l[i] - DELTA) continue;
            double *ui = ue + (size_t)i * k;
            int tight = 0;
            double best_raw = 0.0; /* dot product with c(cur) once tight */
            for (int32_t j = 0; j < k; ++j) {
              if (j == cur) continue;
              if (ui[j] <= l[i] - DELTA) continue;
              if (!simplified && cc[(size_t)cur * k + j] <= l[i] - DELTA) continue;
              if (!tight) {
                best_raw = sim(&X, i, C + (size_t)cur * d);
                l[i] = best_raw / rn[i];
                ui[cur] = l[i];
                sims += 1;
                tight = 1;
                if (ui[j] <= l[i] - DELTA) continue;
                if (!simplified && cc[(size_t)cur * k + j] <= l[i] - DELTA) continue;
              }
              const double sj = sim(&X, i, C + (size_t)j * d);
              ui[j] = sj / rn[i];
              sims += 1;
              if (sj > best_raw) {
                cur = j;
                best_raw = sj;
                l[i] = ui[j];
              }
            }
          } else {
            /* Sections 5.3 / 5.4 */
            if (uh[i] <= l[i] - DELTA) continue;
            if (!simplified && sthr[cur] <= l[i] - DELTA) continue;
            l[i] = sim(&X, i, C + (size_t)cur * d) / rn[i];
            sims += 1;
            if (uh[i] <= l[i] - DELTA) continue;
            if (!simplified && sthr[cur] <= l[i] - DELTA) continue;
            double best = -INFINITY, second = -INFINITY;
            double *sv = (double *)malloc(sizeof(double) * (size_t)k);
            all_sims(&X, i, k, C, sv);
            sims += k - 1;
            cur = argmax_rule(sv, k, prev, &best, &second);
            free(sv);
            l[i] = best / rn[i];
            uh[i] = second / rn[i];
          }
          if (cur != prev) changed += 1;
          a[i] = cur;
        }
        free(s);
      }
    }

    if (changed_tr) changed_tr[t] = changed;
    if (sims_tr) sims_tr[t] = sims;
    if (ccsims_tr) ccsims_tr[t] = ccsims;
    if (obj_assign_tr) obj_assign_tr[t] = obj_assign;
    if (a_trace)
      for (int64_t i = 0; i < n; ++i) a_trace[(size_t)i * max_iter + t] = a[i];

    if (changed == 0) {
      if (obj_update_tr) obj_update_tr[t] = NAN;
      done = 1;
      t += 1;
      break;
    }
    memcpy(Cold, C, sizeof(double) * (size_t)k * (size_t)d);
    const double ou = oracle_update(n, d, rp, ci, v, k, a, Cold, C, NULL);
    if (obj_update_tr) obj_update_tr[t] = ou;
    movement(k, d, Cold, C, p, omp);
  }

  memcpy(a_out, a, sizeof(int32_t) * (size_t)n);
  memcpy(C_out, C, sizeof(double) * (size_t)k * (size_t)d);
  if (violations) *violations = viol;
  if (converged) *converged = done;
  free(rn); free(sthr); free(cc); free(omp); free(p); free(ue); free(uh); free(l);
  free(uy); free(pg); free(ompg);
  free(a); free(Cold); free(C);
  return t;
}
