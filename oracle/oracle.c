/*
 * oracle.c -- plain CPU reference for the ternary EVP search path of
 * "Ultra-Quantisation: Efficient Embedding Search via 1.58-bit Encodings"
 * (Connor, Dearle, Claydon; arXiv 2506.00528).
 *
 * TEST INFRASTRUCTURE.  This file exists only so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against an independent, slow, obviously correct implementation.  No product
 * code links it, includes it, or calls it; it shares no source with the HIP
 * library (no headers, helpers, tables or constants).
 *
 * What it computes, and where the paper defines it:
 *   encode : nearest {x,d} EVP vertex of a float vector (Sec. 2.4, "Mapping to
 *            the vertex space"): take the x largest-magnitude coordinates, give
 *            them the sign of the coordinate, set the rest to zero.  Done here
 *            by an explicit sort of the coordinate indices.
 *   pack   : the two bit vectors v+ / v- of Sec. 5.1.2 and Table 3 (bit i of
 *            v+ set iff v_i = +1, bit i of v- set iff v_i = -1).
 *   delta  : the b2sp function of Sec. 5.1.2, i.e. the scalar product of two
 *            ternary vectors; computed here on the unpacked int8 vectors as a
 *            plain integer dot product (the paper states b2sp equals it).
 *   knn    : exhaustive kNN in the proxy space (problem statement of Sec. 1.1
 *            and Table 1; "closest n" of Sec. 5.3): score every database
 *            vector, order all of them, keep the first k.
 *   rerank : the n proxy candidates of a query ordered by the scalar product
 *            of the original float vectors (the search that the k@n recall of
 *            Sec. 5.3 measures), the first k kept.
 *   masked : exhaustive kNN of a float query against the ternary vectors by
 *            masked addition (Sec. 5.1.2; the asymmetric variant of Sec. 6).
 *   b1.58  : the absmean ternary quantisation the paper compares against
 *            (Sec. 4.3), per embedding.
 *   knn_l2 : exhaustive kNN by the euclidean distance between ternary vectors,
 *            the distance a search over codes of varying non-zero counts
 *            (b1.58) needs (Sec. 1.1, Sec. 4.3).
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *   - equal magnitudes at the x-th place: the lower coordinate index wins;
 *   - a selected coordinate that is zero (+0.0 or -0.0) gets +1, because the
 *     rule is "-1 iff u_i < 0";
 *   - equal Delta scores in the top-k: the lower database id wins;
 *   - packed layout: W = ceil(d/32) 32-bit words per plane, coordinate i is bit
 *     (i mod 32) of word (i / 32) (least significant bit first), a row is the
 *     W plus-plane words followed by the W minus-plane words, unused bits 0.
 *
 * All entry points return 0 on success, ORACLE_EINVAL (-1) for bad sizes and
 * ORACLE_ENONFINITE (-2) when an input float is NaN or infinite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_EINVAL (-1)
#define ORACLE_ENONFINITE (-2)
#define ORACLE_ENOMEM (-3)

/* Deliberately planted mistakes, compiled in only when the test suite builds
 * a mutant copy of this file to prove that the pins catch them. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

int oracle_words_per_plane(int d) { return (d + 31) / 32; }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Encode (Sec. 2.4)                                                         */
/* ------------------------------------------------------------------------ */

/* Coordinate a comes before coordinate b in the "largest absolute elements"
 * order: larger magnitude first; on equal magnitude the lower index first. */
static int comes_before(const float *u, int a, int b) {
  float ma = fabsf(u[a]);
  float mb = fabsf(u[b]);
  if (ma != mb) return ma > mb;
#if ORACLE_MUTANT == 1
  return a > b; /* planted: ties to the higher index */
#else
  return a < b;
#endif
}

/* Plain top-down merge sort of idx[lo, hi) by comes_before(). */
static void merge_sort(const float *u, int *idx, int *tmp, int lo, int hi) {
  if (hi - lo < 2) return;
  int mid = lo + (hi - lo) / 2;
  merge_sort(u, idx, tmp, lo, mid);
  merge_sort(u, idx, tmp, mid, hi);
  int i = lo, j = mid, o = lo;
  while (i < mid && j < hi) {
    if (comes_before(u, idx[j], idx[i]))
      tmp[o++] = idx[j++];
    else
      tmp[o++] = idx[i++];
  }
  while (i < mid) tmp[o++] = idx[i++];
  while (j < hi) tmp[o++] = idx[j++];
  for (o = lo; o < hi; ++o) idx[o] = tmp[o];
}

/* Nearest {x,d} EVP vertex of every row of X (n rows of d floats, row-major).
 * V receives n rows of d int8 values in {-1, 0, +1}. */
int oracle_encode(const float *X, int64_t n, int d, int x, int8_t *V) {
  if (n < 0 || d < 1 || x < 1 || x > d) return ORACLE_EINVAL;
  if (n == 0) return 0;
  for (int64_t e = 0; e < n * (int64_t)d; ++e)
    if (!isfinite(X[e])) return ORACLE_ENONFINITE;
  int failed = 0;
#pragma omp parallel
  {
    int *idx = (int *)malloc(sizeof(int) * (size_t)d);
    int *tmp = (int *)malloc(sizeof(int) * (size_t)d);
    if (!idx || !tmp) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 256)
      for (int64_t r = 0; r < n; ++r) {
        const float *u = X + r * (int64_t)d;
        int8_t *v = V + r * (int64_t)d;
        /* step 1: order the coordinates by magnitude, largest first */
        for (int i = 0; i < d; ++i) idx[i] = i;
        merge_sort(u, idx, tmp, 0, d);
        /* step 3: every coordinate outside the chosen set is 0 */
        for (int i = 0; i < d; ++i) v[i] = 0;
        /* step 2: the x largest get +1 if positive, -1 if negative */
        for (int s = 0; s < x; ++s) {
          int i = idx[s];
#if ORACLE_MUTANT == 2
          v[i] = (u[i] <= 0.0f) ? -1 : 1; /* planted: zero gets -1 */
#else
          v[i] = (u[i] < 0.0f) ? -1 : 1;
#endif
        }
      }
    }
    free(idx);
    free(tmp);
  }
  return failed ? ORACLE_ENOMEM : 0;
}

/* ------------------------------------------------------------------------ */
/* Bit planes (Sec. 5.1.2, Table 3)                                          */
/* ------------------------------------------------------------------------ */

int oracle_pack(const int8_t *V, int64_t n, int d, uint32_t *codes) {
  if (n < 0 || d < 1) return ORACLE_EINVAL;
  int W = oracle_words_per_plane(d);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    const int8_t *v = V + r * (int64_t)d;
    uint32_t *plus = codes + r * (int64_t)(2 * W);
    uint32_t *minus = plus + W;
    for (int w = 0; w < W; ++w) plus[w] = minus[w] = 0;
    for (int i = 0; i < d; ++i) {
#if ORACLE_MUTANT == 5
      uint32_t bit = 1u << (31 - (i % 32)); /* planted: most significant bit first */
#else
      uint32_t bit = 1u << (i % 32);
#endif
      if (v[i] == 1) plus[i / 32] |= bit;
      if (v[i] == -1) minus[i / 32] |= bit;
    }
  }
  return 0;
}

/* Inverse of oracle_pack.  Rejects (ORACLE_EINVAL) a code with a coordinate set
 * in both planes or a set bit beyond coordinate d-1. */
int oracle_unpack(const uint32_t *codes, int64_t n, int d, int8_t *V) {
  if (n < 0 || d < 1) return ORACLE_EINVAL;
  int W = oracle_words_per_plane(d);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t r = 0; r < n; ++r) {
    const uint32_t *plus = codes + r * (int64_t)(2 * W);
    const uint32_t *minus = plus + W;
    int8_t *v = V + r * (int64_t)d;
    for (int i = 0; i < W * 32; ++i) {
      int p = (int)((plus[i / 32] >> (i % 32)) & 1u);
      int m = (int)((minus[i / 32] >> (i % 32)) & 1u);
      if (i >= d) {
        if (p || m) bad = 1;
        continue;
      }
      if (p && m) bad = 1;
      v[i] = (int8_t)(p - m);
    }
  }
  return bad ? ORACLE_EINVAL : 0;
}

/* ------------------------------------------------------------------------ */
/* Delta = b2sp = ternary scalar product (Sec. 5.1.2)                        */
/* ------------------------------------------------------------------------ */

static int32_t ternary_dot(const int8_t *a, const int8_t *b, int d) {
  int32_t s = 0;
  for (int i = 0; i < d; ++i) {
#if ORACLE_MUTANT == 3
    int32_t t = (int32_t)a[i] * (int32_t)b[i];
    s += t > 0 ? t : 0; /* planted: the disagreeing (negative) terms are dropped */
#else
    s += (int32_t)a[i] * (int32_t)b[i];
#endif
  }
  return s;
}

/* D[q*n + i] = Delta(Q_q, V_i) for nq queries against n database vectors. */
int oracle_delta(const int8_t *Q, int64_t nq, const int8_t *V, int64_t n, int d, int32_t *D) {
  if (nq < 0 || n < 0 || d < 1) return ORACLE_EINVAL;
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t q = 0; q < nq; ++q)
    for (int64_t i = 0; i < n; ++i)
      D[q * n + i] = ternary_dot(Q + q * (int64_t)d, V + i * (int64_t)d, d);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive kNN in the proxy space                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t score;
  int32_t id;
} scored_t;

/* a is nearer than b: larger Delta first; on equal Delta the lower id first */
static int nearer(scored_t a, scored_t b) {
  if (a.score != b.score) return a.score > b.score;
#if ORACLE_MUTANT == 4
  return a.id > b.id; /* planted: ties to the higher id */
#else
  return a.id < b.id;
#endif
}

static void merge_sort_scored(scored_t *s, scored_t *tmp, int64_t lo, int64_t hi) {
  if (hi - lo < 2) return;
  int64_t mid = lo + (hi - lo) / 2;
  merge_sort_scored(s, tmp, lo, mid);
  merge_sort_scored(s, tmp, mid, hi);
  int64_t i = lo, j = mid, o = lo;
  while (i < mid && j < hi) {
    if (nearer(s[j], s[i]))
      tmp[o++] = s[j++];
    else
      tmp[o++] = s[i++];
  }
  while (i < mid) tmp[o++] = s[i++];
  while (j < hi) tmp[o++] = s[j++];
  for (o = lo; o < hi; ++o) s[o] = tmp[o];
}

/* For each of nq queries: score all n database vectors with Delta, sort them
 * all (nearest first), and write the first k ids and scores (row-major nq x k). */
int oracle_knn(const int8_t *Q, int64_t nq, const int8_t *V, int64_t n, int d, int k,
               int32_t *ids, int32_t *scores) {
  if (nq < 0 || n < 1 || n > INT32_MAX || d < 1 || k < 1 || k > n) return ORACLE_EINVAL;
  scored_t *all = (scored_t *)malloc(sizeof(scored_t) * (size_t)n);
  scored_t *tmp = (scored_t *)malloc(sizeof(scored_t) * (size_t)n);
  if (!all || !tmp) {
    free(all);
    free(tmp);
    return ORACLE_ENOMEM;
  }
  for (int64_t q = 0; q < nq; ++q) {
    const int8_t *qv = Q + q * (int64_t)d;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      all[i].score = ternary_dot(qv, V + i * (int64_t)d, d);
      all[i].id = (int32_t)i;
    }
    merge_sort_scored(all, tmp, 0, n);
    for (int j = 0; j < k; ++j) {
      ids[q * k + j] = all[j].id;
      scores[q * k + j] = all[j].score;
    }
  }
  free(all);
  free(tmp);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive kNN by euclidean distance between ternary vectors              */
/* ------------------------------------------------------------------------ */
/*
 * Codes with a varying number of non-zeros (the b1.58 quantisation of
 * Sec. 4.3) have varying norms, and the scalar product orders vectors by
 * distance only when the norms are equal (Sec. 1.1 relates l2 and the scalar
 * product for normalised vectors).  This search orders the database by the
 * squared euclidean distance between the ternary vectors, taken coordinate by
 * coordinate: nearest first, the lower id on equal distances.  The score it
 * reports is nnz(q) - distance, so that larger means nearer, as for Delta
 * (it equals 2 Delta - nnz(v)).
 */
static int32_t ternary_sqdist(const int8_t *a, const int8_t *b, int d) {
  int32_t s = 0;
  for (int i = 0; i < d; ++i) {
    const int32_t t = (int32_t)a[i] - (int32_t)b[i];
#if ORACLE_MUTANT == 10
    s += t != 0; /* planted: counts differing coordinates (a Hamming distance) */
#else
    s += t * t;
#endif
  }
  return s;
}

static int32_t ternary_nnz(const int8_t *a, int d) {
  int32_t s = 0;
  for (int i = 0; i < d; ++i) s += a[i] != 0;
  return s;
}

int oracle_knn_l2(const int8_t *Q, int64_t nq, const int8_t *V, int64_t n, int d, int k,
                  int32_t *ids, int32_t *scores) {
  if (nq < 0 || n < 1 || n > INT32_MAX || d < 1 || k < 1 || k > n) return ORACLE_EINVAL;
  scored_t *all = (scored_t *)malloc(sizeof(scored_t) * (size_t)n);
  scored_t *tmp = (scored_t *)malloc(sizeof(scored_t) * (size_t)n);
  if (!all || !tmp) {
    free(all);
    free(tmp);
    return ORACLE_ENOMEM;
  }
  for (int64_t q = 0; q < nq; ++q) {
    const int8_t *qv = Q + q * (int64_t)d;
    const int32_t nnzq = ternary_nnz(qv, d);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      all[i].score = nnzq - ternary_sqdist(qv, V + i * (int64_t)d, d);
      all[i].id = (int32_t)i;
    }
    merge_sort_scored(all, tmp, 0, n);
    for (int j = 0; j < k; ++j) {
      ids[q * k + j] = all[j].id;
      scores[q * k + j] = all[j].score;
    }
  }
  free(all);
  free(tmp);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Refinement of proxy candidates with the original vectors                 */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 5.3 measures k@n recall: how many of the k true nearest neighbours
 * are among the n nearest in the proxy space.  The search that this protects
 * takes those n proxy candidates and orders them by the original similarity.
 * For l2-normalised vectors (Sec. 1.1) the nearest in l2 distance are the
 * largest scalar products, so each candidate is scored with the double
 * precision scalar product of the float vectors (products and sums in
 * double, in coordinate order), and the k best are kept: larger score first,
 * the lower id on equal scores.  A candidate id outside [0, n) is skipped;
 * missing results are written as id -1 with score -infinity.
 */
typedef struct {
  double score;
  int32_t id;
} refined_t;

static int refined_before(refined_t a, refined_t b) {
#if ORACLE_MUTANT == 6
  if (a.score != b.score) return a.score < b.score; /* planted: the worst first */
#else
  if (a.score != b.score) return a.score > b.score;
#endif
#if ORACLE_MUTANT == 7
  return a.id > b.id; /* planted: ties to the higher id */
#else
  return a.id < b.id;
#endif
}

static void merge_sort_refined(refined_t *s, refined_t *tmp, int lo, int hi) {
  if (hi - lo < 2) return;
  int mid = lo + (hi - lo) / 2;
  merge_sort_refined(s, tmp, lo, mid);
  merge_sort_refined(s, tmp, mid, hi);
  int i = lo, j = mid, o = lo;
  while (i < mid && j < hi) {
    if (refined_before(s[j], s[i]))
      tmp[o++] = s[j++];
    else
      tmp[o++] = s[i++];
  }
  while (i < mid) tmp[o++] = s[i++];
  while (j < hi) tmp[o++] = s[j++];
  for (o = lo; o < hi; ++o) s[o] = tmp[o];
}

int oracle_rerank(const float *X, int64_t n, int d, const float *Q, int64_t nq, const int32_t *cand, int ncand,
                  int k, int32_t *ids, double *scores) {
  if (n < 1 || d < 1 || nq < 0 || ncand < 1 || k < 1 || k > ncand) return ORACLE_EINVAL;
  int rc = 0;
#pragma omp parallel for schedule(dynamic) reduction(min : rc)
  for (int64_t q = 0; q < nq; ++q) {
    refined_t *all = (refined_t *)malloc(sizeof(refined_t) * (size_t)ncand);
    refined_t *tmp = (refined_t *)malloc(sizeof(refined_t) * (size_t)ncand);
    if (!all || !tmp) {
      free(all);
      free(tmp);
      rc = ORACLE_ENOMEM;
      continue;
    }
    const float *qv = Q + q * (int64_t)d;
    int m = 0;
    for (int c = 0; c < ncand; ++c) {
      const int32_t id = cand[q * (int64_t)ncand + c];
      if (id < 0 || (int64_t)id >= n) continue;
      const float *xv = X + (int64_t)id * d;
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += (double)qv[i] * (double)xv[i];
      all[m].score = s;
      all[m].id = id;
      ++m;
    }
    merge_sort_refined(all, tmp, 0, m);
    for (int j = 0; j < k; ++j) {
      ids[q * k + j] = j < m ? all[j].id : -1;
      scores[q * k + j] = j < m ? all[j].score : -INFINITY;
    }
    free(all);
    free(tmp);
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Masked addition: a float query against ternary database vectors          */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 5.1.2: the scalar product of a ternary v with any vector w is the sum
 * of w over the coordinates where v+ is set minus the sum of w where v- is
 * set (no multiplications); Sec. 6 notes that comparing the ternary database
 * with the original float query is the more accurate variant.  The two sums
 * are taken here in double precision, coordinate by coordinate in index
 * order; the score is their difference rounded once to float, and the k
 * largest scores are kept (the lower id on equal float scores).  The exact
 * double difference is also returned, for tolerance checks.
 */
typedef struct {
  float score;
  double exact;
  int32_t id;
} masked_t;

static int masked_before(masked_t a, masked_t b) {
  if (a.score != b.score) return a.score > b.score;
  return a.id < b.id;
}

static void merge_sort_masked(masked_t *s, masked_t *tmp, int64_t lo, int64_t hi) {
  if (hi - lo < 2) return;
  int64_t mid = lo + (hi - lo) / 2;
  merge_sort_masked(s, tmp, lo, mid);
  merge_sort_masked(s, tmp, mid, hi);
  int64_t i = lo, j = mid, o = lo;
  while (i < mid && j < hi) {
    if (masked_before(s[j], s[i]))
      tmp[o++] = s[j++];
    else
      tmp[o++] = s[i++];
  }
  while (i < mid) tmp[o++] = s[i++];
  while (j < hi) tmp[o++] = s[j++];
  for (o = lo; o < hi; ++o) s[o] = tmp[o];
}

static double masked_addition(const float *w, const int8_t *v, int d) {
  double plus = 0.0, minus = 0.0;
  for (int i = 0; i < d; ++i) {
#if ORACLE_MUTANT == 8
    if (v[i] != 0) plus += (double)w[i]; /* planted: the sign of v ignored */
#else
    if (v[i] > 0) plus += (double)w[i];
    if (v[i] < 0) minus += (double)w[i];
#endif
  }
  return plus - minus;
}

int oracle_masked_knn(const float *Q, int64_t nq, const int8_t *V, int64_t n, int d, int k, int32_t *ids,
                      float *scores, double *exact) {
  if (nq < 0 || n < 1 || n > INT32_MAX || d < 1 || k < 1 || k > n) return ORACLE_EINVAL;
  masked_t *all = (masked_t *)malloc(sizeof(masked_t) * (size_t)n);
  masked_t *tmp = (masked_t *)malloc(sizeof(masked_t) * (size_t)n);
  if (!all || !tmp) {
    free(all);
    free(tmp);
    return ORACLE_ENOMEM;
  }
  for (int64_t q = 0; q < nq; ++q) {
    const float *qv = Q + q * (int64_t)d;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const double s = masked_addition(qv, V + i * (int64_t)d, d);
      all[i].exact = s;
      all[i].score = (float)s;
      all[i].id = (int32_t)i;
    }
    merge_sort_masked(all, tmp, 0, n);
    for (int j = 0; j < k; ++j) {
      ids[q * k + j] = all[j].id;
      scores[q * k + j] = all[j].score;
      exact[q * k + j] = all[j].exact;
    }
  }
  free(all);
  free(tmp);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* b1.58 quantisation (Sec. 4.3), one embedding at a time                   */
/* ------------------------------------------------------------------------ */
/*
 * gamma = the mean of |u_i| over the vector (the paper's mean over a weight
 * matrix, taken per embedding here), then v_i = max(-1, min(1, round(u_i /
 * gamma))).  gamma is summed in double in index order, the division is in
 * double, and round() is to nearest with ties to even (the IEEE default; the
 * paper does not say).  The paper's epsilon only keeps an all-zero matrix
 * from dividing by zero: an all-zero row gives the zero vector here.
 */
int oracle_encode_b158(const float *X, int64_t n, int d, int8_t *V) {
  if (n < 0 || d < 1) return ORACLE_EINVAL;
  int rc = 0;
#pragma omp parallel for schedule(static) reduction(min : rc)
  for (int64_t r = 0; r < n; ++r) {
    const float *u = X + r * (int64_t)d;
    int8_t *v = V + r * (int64_t)d;
    double gamma = 0.0;
    int finite = 1;
    for (int i = 0; i < d; ++i) {
      if (!isfinite(u[i])) finite = 0;
      gamma += fabs((double)u[i]);
    }
    if (!finite) {
      rc = ORACLE_ENONFINITE;
      memset(v, 0, (size_t)d);
      continue;
    }
    gamma /= (double)d;
    for (int i = 0; i < d; ++i) {
      if (gamma == 0.0) {
        v[i] = 0;
        continue;
      }
#if ORACLE_MUTANT == 9
      double q = round((double)u[i] / gamma); /* planted: ties away from zero */
#else
      double q = nearbyint((double)u[i] / gamma);
#endif
      if (q > 1.0) q = 1.0;
      if (q < -1.0) q = -1.0;
      v[i] = (int8_t)q;
    }
  }
  return rc;
}
