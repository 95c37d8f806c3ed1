/*
 * Seeded synthetic inputs for spherical k-means: sparse tf-idf document
 * vectors and dense von Mises-Fisher mixtures.
 *
 * This file holds input generation only.  Nothing here evaluates
 * similarities, assignments, centres or bounds; both the CPU oracle and the
 * GPU library consume its output.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to key + counter * golden-gamma, where
 * the key is derived from (seed, stream, row).  Every row has its own
 * reproducible stream, so rows are generated in parallel and the result does
 * not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t key;
  uint64_t ctr;
} rng_t;

static inline rng_t rng_make(uint64_t seed, uint64_t stream, uint64_t row) {
  rng_t r;
  r.key = mix64(seed ^ mix64(stream * GOLDEN_GAMMA + 0x632BE59BD9B4E019ULL) ^
                mix64(row + 0x2545F4914F6CDD1DULL));
  r.ctr = 0;
  return r;
}

static inline uint64_t rng_u64(rng_t *r) {
  r->ctr += 1;
  return mix64(r->key + r->ctr * GOLDEN_GAMMA);
}

/* uniform on the open interval (0,1) with 53 random bits */
static inline double rng_unif(rng_t *r) {
  return ((double)(rng_u64(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* standard normal by Box-Muller (one output per call) */
static inline double rng_normal(rng_t *r) {
  double u1 = rng_unif(r), u2 = rng_unif(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Gamma(alpha, 1) for alpha >= 1 by Marsaglia and Tsang (2000). */
static double rng_gamma(rng_t *r, double alpha) {
  const double dd = alpha - 1.0 / 3.0, cc = 1.0 / sqrt(9.0 * dd);
  for (;;) {
    double x = rng_normal(r), v = 1.0 + cc * x;
    if (v <= 0.0) continue;
    v = v * v * v;
    double u = rng_unif(r);
    if (log(u) < 0.5 * x * x + dd - dd * v + dd * log(v)) return dd * v;
  }
}

enum { STREAM_LEN = 1, STREAM_TERMS = 2, STREAM_PERM = 3, STREAM_VMF = 4,
       STREAM_MEANS = 5, STREAM_TOPIC = 6, STREAM_TOPIC_PERM = 7 };

/* ------------------------------------------------------------------------ */
/* sparse tf-idf rows                                                        */
/* ------------------------------------------------------------------------ */

/* Row lengths m_i = clip(round(LogNormal(mu, sigma)), 1, d) with
 * mu = ln(mean) - sigma^2/2, so that `mean` is the arithmetic mean before
 * clipping.  Returns sum(m_i). */
int64_t skmgen_row_lengths(int64_t n, int64_t d, double mean, double sigma,
                           uint64_t seed, int32_t *m_out) {
  const double mu = log(mean) - 0.5 * sigma * sigma;
  int64_t total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    rng_t r = rng_make(seed, STREAM_LEN, (uint64_t)i);
    double z = rng_normal(&r);
    double m = floor(exp(mu + sigma * z) + 0.5);
    if (m < 1.0) m = 1.0;
    if (m > (double)d) m = (double)d;
    m_out[i] = (int32_t)m;
    total += (int64_t)m;
  }
  return total;
}

typedef struct {
  int32_t c;
  float v;
} entry_t;

static int cmp_entry(const void *a, const void *b) {
  const int32_t x = ((const entry_t *)a)->c, y = ((const entry_t *)b)->c;
  return (x > y) - (x < y);
}

/* Fills CSR rows.  For every row: m_i distinct term ranks drawn one at a time
 * from a Zipf(s) law truncated to 1..d (a repeat is rejected and redrawn),
 * ranks mapped to column ids by a seeded permutation, term frequency
 * tf ~ Geometric(1/2) on {1,2,...}, weight ln(1+tf) * idf with
 * idf_t = ln(n / df_t).  Zero-valued entries (terms present in every row)
 * are dropped, as are rows left empty.  Rows are L2-normalised in double and
 * stored as float with ascending column ids.
 *
 * row_ptr has n+1 slots, col/val have sum(m) slots.  Returns the final nnz;
 * *n_out receives the number of rows kept, *dropped the number removed.
 * idf_out (nullable, d slots) receives idf per column. */
static int64_t sparse_fill(int64_t n, int64_t d, double zipf_s, uint64_t seed,
                           int32_t topics, double topic_share, const int32_t *m,
                           int64_t *row_ptr, int32_t *col, float *val, int64_t *n_out,
                           int64_t *dropped, double *idf_out);

int64_t skmgen_sparse_fill(int64_t n, int64_t d, double zipf_s, uint64_t seed,
                           const int32_t *m, int64_t *row_ptr, int32_t *col,
                           float *val, int64_t *n_out, int64_t *dropped,
                           double *idf_out) {
  return sparse_fill(n, d, zipf_s, seed, 0, 0.0, m, row_ptr, col, val, n_out, dropped,
                     idf_out);
}

/* The same rows with topic structure: every row draws one of `topics`
 * topics (uniformly), and each of its terms takes, with probability
 * topic_share, its column from the topic's own seeded rank -> column
 * permutation instead of the shared one, so rows of one topic share their
 * frequent terms.  topics = 0 gives exactly skmgen_sparse_fill's rows. */
int64_t skmgen_sparse_fill_topics(int64_t n, int64_t d, double zipf_s, uint64_t seed,
                                  int32_t topics, double topic_share, const int32_t *m,
                                  int64_t *row_ptr, int32_t *col, float *val,
                                  int64_t *n_out, int64_t *dropped, double *idf_out) {
  return sparse_fill(n, d, zipf_s, seed, topics, topic_share, m, row_ptr, col, val, n_out,
                     dropped, idf_out);
}

static int64_t sparse_fill(int64_t n, int64_t d, double zipf_s, uint64_t seed,
                           int32_t topics, double topic_share, const int32_t *m,
                           int64_t *row_ptr, int32_t *col, float *val, int64_t *n_out,
                           int64_t *dropped, double *idf_out) {
  double *cdf = (double *)malloc(sizeof(double) * (size_t)d);
  double acc = 0.0;
  for (int64_t r = 0; r < d; ++r) {
    acc += pow((double)(r + 1), -zipf_s);
    cdf[r] = acc;
  }
  const double total_w = acc;

  /* rank -> column id permutation (Fisher-Yates) */
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)d);
  for (int64_t r = 0; r < d; ++r) perm[r] = (int32_t)r;
  {
    rng_t pr = rng_make(seed, STREAM_PERM, 0);
    for (int64_t r = d - 1; r > 0; --r) {
      int64_t j = (int64_t)(rng_u64(&pr) % (uint64_t)(r + 1));
      int32_t t = perm[r];
      perm[r] = perm[j];
      perm[j] = t;
    }
  }

  /* per-topic rank -> column permutations */
  int32_t *tperm = NULL;
  if (topics > 0) {
    tperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)d * (size_t)topics);
    for (int32_t t = 0; t < topics; ++t) {
      int32_t *pt = tperm + (size_t)t * (size_t)d;
      for (int64_t r = 0; r < d; ++r) pt[r] = (int32_t)r;
      rng_t pr = rng_make(seed, STREAM_TOPIC_PERM, (uint64_t)t);
      for (int64_t r = d - 1; r > 0; --r) {
        int64_t j = (int64_t)(rng_u64(&pr) % (uint64_t)(r + 1));
        int32_t x = pt[r];
        pt[r] = pt[j];
        pt[j] = x;
      }
    }
  }

  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  off[0] = 0;
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + m[i];
  const int64_t cap = off[n];
  double *w = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));

  /* draw terms and term frequencies */
#pragma omp parallel
  {
    uint8_t *used = (uint8_t *)calloc((size_t)d, 1);
    int32_t *ranks = (int32_t *)malloc(sizeof(int32_t) * (size_t)d);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      rng_t r = rng_make(seed, STREAM_TERMS, (uint64_t)i);
      const int64_t base = off[i];
      const int32_t mi = m[i];
      const int32_t *tp = NULL;
      rng_t rt;
      if (topics > 0) {
        rt = rng_make(seed, STREAM_TOPIC, (uint64_t)i);
        tp = tperm + (size_t)(rng_u64(&rt) % (uint64_t)topics) * (size_t)d;
      }
      int32_t got = 0;
      while (got < mi) {
        const double target = rng_unif(&r) * total_w;
        int64_t lo = 0, hi = d - 1; /* smallest r with cdf[r] >= target */
        while (lo < hi) {
          int64_t mid = (lo + hi) >> 1;
          if (cdf[mid] >= target) hi = mid; else lo = mid + 1;
        }
        /* repeats are rejected by column (by rank without topics) */
        const int32_t c =
            (tp != NULL && rng_unif(&rt) < topic_share) ? tp[lo] : perm[lo];
        const int64_t key = tp != NULL ? (int64_t)c : lo;
        if (used[key]) continue;
        used[key] = 1;
        ranks[got] = (int32_t)key;
        uint64_t bits = rng_u64(&r);
        int tf = 1 + (bits ? __builtin_ctzll(bits) : 63);
        col[base + got] = c;
        w[base + got] = log1p((double)tf);
        ++got;
      }
      for (int32_t q = 0; q < mi; ++q) used[ranks[q]] = 0;
    }
    free(ranks);
    free(used);
  }

  /* document frequencies and idf */
  int64_t *df = (int64_t *)calloc((size_t)d, sizeof(int64_t));
  for (int64_t e = 0; e < cap; ++e) df[col[e]] += 1;
  double *idf = (double *)malloc(sizeof(double) * (size_t)d);
  for (int64_t t = 0; t < d; ++t)
    idf[t] = df[t] > 0 ? log((double)n / (double)df[t]) : 0.0;
  if (idf_out) memcpy(idf_out, idf, sizeof(double) * (size_t)d);

  /* weights, drop zeros, normalise, sort; rows are written in place into a
   * per-row compacted region [off[i], off[i] + kept_i) */
  int64_t *kept = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel
  {
    entry_t *buf = (entry_t *)malloc(sizeof(entry_t) * (size_t)d);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t base = off[i];
      int32_t q = 0;
      double ss = 0.0;
      for (int32_t e = 0; e < m[i]; ++e) {
        const double x = w[base + e] * idf[col[base + e]];
        if (x == 0.0) continue;
        w[base + q] = x;
        col[base + q] = col[base + e];
        ss += x * x;
        ++q;
      }
      const double inv = q > 0 ? 1.0 / sqrt(ss) : 0.0;
      for (int32_t e = 0; e < q; ++e) {
        buf[e].c = col[base + e];
        buf[e].v = (float)(w[base + e] * inv);
      }
      qsort(buf, (size_t)q, sizeof(entry_t), cmp_entry);
      for (int32_t e = 0; e < q; ++e) {
        col[base + e] = buf[e].c;
        val[base + e] = buf[e].v;
      }
      kept[i] = q;
    }
    free(buf);
  }

  /* compact rows to the front, dropping empty rows */
  int64_t nnz = 0, rows = 0;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (kept[i] == 0) continue;
    if (nnz != off[i]) {
      memmove(col + nnz, col + off[i], sizeof(int32_t) * (size_t)kept[i]);
      memmove(val + nnz, val + off[i], sizeof(float) * (size_t)kept[i]);
    }
    nnz += kept[i];
    rows += 1;
    row_ptr[rows] = nnz;
  }
  *n_out = rows;
  *dropped = n - rows;

  free(kept);
  free(idf);
  free(df);
  free(w);
  free(off);
  free(perm);
  free(tperm);
  free(cdf);
  return nnz;
}

/* ------------------------------------------------------------------------ */
/* dense von Mises-Fisher mixture                                            */
/* ------------------------------------------------------------------------ */

/* Draws the cosine w = <x, mu> of a vMF(mu, kappa) sample on the unit sphere
 * in R^p with the rejection scheme of Wood (1994), "Simulation of the von
 * Mises Fisher distribution". */
static double vmf_cosine(rng_t *r, double kappa, int64_t p) {
  const double pm1 = (double)(p - 1);
  const double b = (-2.0 * kappa + sqrt(4.0 * kappa * kappa + pm1 * pm1)) / pm1;
  const double x0 = (1.0 - b) / (1.0 + b);
  const double c = kappa * x0 + pm1 * log(1.0 - x0 * x0);
  for (;;) {
    const double g1 = rng_gamma(r, 0.5 * pm1), g2 = rng_gamma(r, 0.5 * pm1);
    const double z = g1 / (g1 + g2);
    const double wv = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z);
    const double u = rng_unif(r);
    if (kappa * wv + pm1 * log(1.0 - x0 * wv) - c >= log(u)) return wv;
  }
}

/* n points in R^d from an equal-weight mixture of n_means vMF components.
 * Mean directions are normalised standard normal vectors; concentrations are
 * uniform on [kappa_lo, kappa_hi].  Each point: w from Wood's sampler, a
 * tangent direction uniform on the sphere orthogonal to mu, x = w mu +
 * sqrt(1-w^2) v, renormalised in double and stored as float (row-major n x
 * d).  means_out (n_means x d, float), kappa_out and comp_out are
 * nullable. */
void skmgen_vmf(int64_t n, int64_t d, int32_t n_means, double kappa_lo,
                double kappa_hi, uint64_t seed, float *X, float *means_out,
                double *kappa_out, int32_t *comp_out) {
  double *mu = (double *)malloc(sizeof(double) * (size_t)n_means * (size_t)d);
  double *kap = (double *)malloc(sizeof(double) * (size_t)n_means);
#pragma omp parallel for schedule(static)
  for (int32_t c = 0; c < n_means; ++c) {
    rng_t r = rng_make(seed, STREAM_MEANS, (uint64_t)c);
    double ss = 0.0;
    double *m = mu + (size_t)c * (size_t)d;
    for (int64_t t = 0; t < d; ++t) {
      m[t] = rng_normal(&r);
      ss += m[t] * m[t];
    }
    const double inv = 1.0 / sqrt(ss);
    for (int64_t t = 0; t < d; ++t) m[t] *= inv;
    kap[c] = kappa_lo + (kappa_hi - kappa_lo) * rng_unif(&r);
  }
  if (means_out)
    for (size_t e = 0; e < (size_t)n_means * (size_t)d; ++e)
      means_out[e] = (float)mu[e];
  if (kappa_out) memcpy(kappa_out, kap, sizeof(double) * (size_t)n_means);

#pragma omp parallel
  {
    double *v = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      rng_t r = rng_make(seed, STREAM_VMF, (uint64_t)i);
      const int32_t c = (int32_t)(rng_u64(&r) % (uint64_t)n_means);
      const double *m = mu + (size_t)c * (size_t)d;
      const double wv = vmf_cosine(&r, kap[c], d);
      double dot = 0.0;
      for (int64_t t = 0; t < d; ++t) {
        v[t] = rng_normal(&r);
        dot += v[t] * m[t];
      }
      double ss = 0.0;
      for (int64_t t = 0; t < d; ++t) {
        v[t] -= dot * m[t];
        ss += v[t] * v[t];
      }
      const double sv = sqrt(1.0 - wv * wv) / sqrt(ss);
      double xs = 0.0;
      for (int64_t t = 0; t < d; ++t) {
        v[t] = wv * m[t] + sv * v[t];
        xs += v[t] * v[t];
      }
      const double inv = 1.0 / sqrt(xs);
      float *x = X + (size_t)i * (size_t)d;
      for (int64_t t = 0; t < d; ++t) x[t] = (float)(v[t] * inv);
      if (comp_out) comp_out[i] = c;
    }
    free(v);
  }
  free(kap);
  free(mu);
}
