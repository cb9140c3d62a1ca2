/*
 * oracle/orc.c -- plain, slow FP64 reference for sliding-window cumulant
 * tensors (Domino & Gawron, "Algorithm for an arbitrary-order cumulant tensor
 * calculation in a sliding window of data streams", arXiv:1701.06446).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or generator
 * with the HIP library.
 *
 * Storage convention (the paper's block structure, Sec. 2.3 and Sec. 4.1):
 *   - columns are zero-padded to N = nbar*b with nbar = ceil(n/b);
 *   - an order-k tensor is kept as the blocks whose block multi-index
 *     (j_1 <= ... <= j_k) is non-decreasing, listed in lexicographic order;
 *   - every block is a full b^k array, row-major in (a_1, ..., a_k), a_1
 *     slowest; element (j, a) sits at global index i_m = j_m*b + a_m.
 *
 * Functions and the passages they follow:
 *   orc_sums_add    Eq. (mom) summed over rows, and the window slide of
 *                   Eq. (momupdate): new rows enter with +1, dropped rows
 *                   with -1.  Neumaier-compensated FP64 accumulation.
 *   orc_moms2cums   Alg. 3 (moms2cums) with Alg. 4 (symmetrized outer
 *                   product): for s = 1..d, C_s = M_s - A, where A sums, over
 *                   every partition of {1..s} into sigma = 2..s parts, the
 *                   product of lower-order cumulants at the sub-multi-indices.
 *                   All partitions, singletons included (Sec. 2.6, item 2).
 *   orc_norms       Alg. 5 with exponent 2 (Eq. (me)) and Eq. (mef):
 *                   ||C_k||^2 = sum over stored blocks of k!/prod(r_l!) times
 *                   the block's sum of squares; nu_k = ||C_k|| / ||C_2||^(k/2).
 *
 * Every function here is pinned by the CPU test-suite against brute-force
 * full tensors, textbook closed forms and invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 8

/* Number of non-decreasing k-tuples over {0..nbar-1}, counted by walking
 * them (the closed form C(nbar+k-1, k) is checked by the tests). */
int64_t orc_count_tuples(int nbar, int k) {
  if (k == 0) return 1;
  if (nbar <= 0 || k < 0 || k > ORC_MAXK) return 0;
  int j[ORC_MAXK];
  for (int m = 0; m < k; ++m) j[m] = 0;
  int64_t count = 0;
  for (;;) {
    ++count;
    int m = k - 1;
    while (m >= 0 && j[m] == nbar - 1) --m;
    if (m < 0) break;
    j[m] += 1;
    for (int q = m + 1; q < k; ++q) j[q] = j[m];
  }
  return count;
}

/* Writes the non-decreasing k-tuples in lexicographic order, k ints each. */
void orc_tuples(int nbar, int k, int *out) {
  if (k == 0 || nbar <= 0) return;
  int j[ORC_MAXK];
  for (int m = 0; m < k; ++m) j[m] = 0;
  int64_t row = 0;
  for (;;) {
    for (int m = 0; m < k; ++m) out[row * k + m] = j[m];
    ++row;
    int m = k - 1;
    while (m >= 0 && j[m] == nbar - 1) --m;
    if (m < 0) break;
    j[m] += 1;
    for (int q = m + 1; q < k; ++q) j[q] = j[m];
  }
}

static int64_t ipow(int b, int k) {
  int64_t r = 1;
  for (int m = 0; m < k; ++m) r *= b;
  return r;
}

/* Dense lookup from a non-decreasing block tuple to its lexicographic rank,
 * built by walking the tuple list: table[sum_m j_m * nbar^(k-1-m)] = rank. */
static int64_t *rank_table(int nbar, int k) {
  int64_t nt = orc_count_tuples(nbar, k);
  int64_t cells = ipow(nbar, k);
  int64_t *tab = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cells > 0 ? cells : 1));
  int *tup = (int *)malloc(sizeof(int) * (size_t)(nt * k + 1));
  if (!tab || !tup) { free(tab); free(tup); return NULL; }
  for (int64_t c = 0; c < cells; ++c) tab[c] = -1;
  orc_tuples(nbar, k, tup);
  for (int64_t r = 0; r < nt; ++r) {
    int64_t key = 0;
    for (int m = 0; m < k; ++m) key = key * nbar + tup[r * k + m];
    tab[key] = r;
  }
  free(tup);
  return tab;
}

/*
 * S, comp: order-k pyramid (orc_count_tuples(nbar,k) * b^k values each).
 * For every stored element adds sign * sum_rows prod_m x[row, i_m] into the
 * Neumaier pair (S, comp).  X is row-major rows x n (FP64); columns n..N-1
 * are the zero padding and contribute exact zeros.
 */
void orc_sums_add(const double *X, int64_t rows, int n, int b, int k, double sign,
                  double *S, double *comp) {
  int nbar = (n + b - 1) / b;
  int64_t nt = orc_count_tuples(nbar, k);
  int64_t bk = ipow(b, k);
  int *tup = (int *)malloc(sizeof(int) * (size_t)(nt * k + 1));
  if (!tup) return;
  orc_tuples(nbar, k, tup);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t blk = 0; blk < nt; ++blk) {
    int cols[ORC_MAXK];
    for (int64_t e = 0; e < bk; ++e) {
      /* decode the within-block offset, a_1 slowest */
      int64_t rem = e;
      int valid = 1;
      for (int m = k - 1; m >= 0; --m) {
        int a = (int)(rem % b);
        rem /= b;
        cols[m] = tup[blk * k + m] * b + a;
        if (cols[m] >= n) valid = 0;
      }
      double s = S[blk * bk + e], c = comp[blk * bk + e];
      if (valid) {
        for (int64_t l = 0; l < rows; ++l) {
          double p = sign;
          for (int m = 0; m < k; ++m) p *= X[l * n + cols[m]];
          /* Neumaier compensated add of p into (s, c) */
          double t = s + p;
          if (fabs(s) >= fabs(p)) c += (s - t) + p;
          else c += (p - t) + s;
          s = t;
        }
      }
      S[blk * bk + e] = s;
      comp[blk * bk + e] = c;
    }
  }
  free(tup);
}

/* Partitions of {0..s-1} as restricted growth strings: rgs[m] is the part of
 * element m, rgs[0] = 0 and rgs[m] <= 1 + max(rgs[0..m-1]).  Calls visit()
 * once per partition with its number of parts. */
typedef void (*orc_visit)(const int *rgs, int s, int parts, void *ctx);
static void rgs_walk(int s, orc_visit visit, void *ctx) {
  int rgs[ORC_MAXK], mx[ORC_MAXK];
  for (int m = 0; m < s; ++m) { rgs[m] = 0; mx[m] = 0; }
  for (;;) {
    int parts = 0;
    for (int m = 0; m < s; ++m) if (rgs[m] + 1 > parts) parts = rgs[m] + 1;
    visit(rgs, s, parts, ctx);
    int m = s - 1;
    while (m > 0 && rgs[m] == mx[m - 1] + 1) --m;
    if (m <= 0) break;
    rgs[m] += 1;
    mx[m] = mx[m - 1] > rgs[m] ? mx[m - 1] : rgs[m];
    for (int q = m + 1; q < s; ++q) { rgs[q] = 0; mx[q] = mx[m]; }
  }
}

/* A flat list of the partitions of {0..s-1} with sigma = 2..s parts, grouped
 * by sigma in increasing order as in Alg. 4's outer loop.  For each partition:
 * its parts as bitmasks. */
typedef struct { int count; int parts[4200]; unsigned masks[4200][ORC_MAXK]; } plist;
typedef struct { plist *pl; int sigma; } pctx;
static void collect(const int *rgs, int s, int parts, void *vctx) {
  pctx *c = (pctx *)vctx;
  if (parts != c->sigma) return;
  plist *pl = c->pl;
  pl->parts[pl->count] = parts;
  for (int q = 0; q < parts; ++q) pl->masks[pl->count][q] = 0u;
  for (int m = 0; m < s; ++m) pl->masks[pl->count][rgs[m]] |= 1u << m;
  pl->count += 1;
}
static void partitions_sigma_ge2(int s, plist *pl) {
  pl->count = 0;
  for (int sigma = 2; sigma <= s; ++sigma) {
    pctx c = {pl, sigma};
    rgs_walk(s, collect, &c);
  }
}

/* Number of partitions of {0..s-1} into exactly sigma parts, by walking. */
int64_t orc_count_partitions(int s, int sigma) {
  if (s < 1 || s > ORC_MAXK) return 0;
  plist *pl = (plist *)malloc(sizeof(plist));
  if (!pl) return -1;
  pctx c = {pl, sigma};
  pl->count = 0;
  rgs_walk(s, collect, &c);
  int64_t r = pl->count;
  free(pl);
  return r;
}

/*
 * Alg. 3 / Alg. 4.  M[k-1] and C[k-1] point at the order-k pyramids
 * (k = 1..d), FP64.  Computes C_1..C_d in increasing order; C_s uses only
 * C_1..C_{s-1}.  Returns 0, or -1 on allocation failure.
 */
int orc_moms2cums(int n, int b, int d, const double *const *M, double *const *C) {
  if (d < 1 || d > 6 || b < 1 || n < 1) return -1;
  int nbar = (n + b - 1) / b;
  int64_t *rt[ORC_MAXK + 1] = {0};
  for (int k = 1; k <= d; ++k) {
    rt[k] = rank_table(nbar, k);
    if (!rt[k]) { for (int q = 1; q < k; ++q) free(rt[q]); return -1; }
  }
  plist *pl = (plist *)malloc(sizeof(plist));
  if (!pl) { for (int k = 1; k <= d; ++k) free(rt[k]); return -1; }
  for (int s = 1; s <= d; ++s) {
    partitions_sigma_ge2(s, pl);
    int64_t nt = orc_count_tuples(nbar, s);
    int64_t bs = ipow(b, s);
    int *tup = (int *)malloc(sizeof(int) * (size_t)(nt * s + 1));
    if (!tup) { free(pl); for (int k = 1; k <= d; ++k) free(rt[k]); return -1; }
    orc_tuples(nbar, s, tup);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < nt; ++blk) {
      for (int64_t e = 0; e < bs; ++e) {
        int idx[ORC_MAXK];
        int64_t rem = e;
        for (int m = s - 1; m >= 0; --m) {
          idx[m] = tup[blk * s + m] * b + (int)(rem % b);
          rem /= b;
        }
        double A = 0.0;
        for (int p = 0; p < pl->count; ++p) {
          double a = 1.0;
          for (int q = 0; q < pl->parts[p]; ++q) {
            unsigned mask = pl->masks[p][q];
            /* the sub-multi-index i_B, sorted (super-symmetry) */
            int sub[ORC_MAXK], len = 0;
            for (int m = 0; m < s; ++m)
              if (mask & (1u << m)) sub[len++] = idx[m];
            for (int u = 1; u < len; ++u) {
              int v = sub[u], w = u - 1;
              while (w >= 0 && sub[w] > v) { sub[w + 1] = sub[w]; --w; }
              sub[w + 1] = v;
            }
            int64_t key = 0, off = 0;
            for (int m = 0; m < len; ++m) {
              key = key * nbar + sub[m] / b;
              off = off * b + sub[m] % b;
            }
            int64_t r = rt[len][key];
            a *= C[len - 1][r * ipow(b, len) + off];
          }
          A += a;
        }
        C[s - 1][blk * bs + e] = M[s - 1][blk * bs + e] - A;
      }
    }
    free(tup);
  }
  free(pl);
  for (int k = 1; k <= d; ++k) free(rt[k]);
  return 0;
}

/* Alg. 5 (k = 2) for one order: fro = sqrt(sum_blocks mult * sum_e e^2). */
double orc_block_norm(int n, int b, int k, const double *A) {
  int nbar = (n + b - 1) / b;
  int64_t nt = orc_count_tuples(nbar, k);
  int64_t bk = ipow(b, k);
  int *tup = (int *)malloc(sizeof(int) * (size_t)(nt * k + 1));
  if (!tup) return NAN;
  orc_tuples(nbar, k, tup);
  double kfact = 1.0;
  for (int m = 2; m <= k; ++m) kfact *= m;
  double z = 0.0;
  for (int64_t blk = 0; blk < nt; ++blk) {
    /* multiplicity k!/prod(r_l!) over the runs of equal block indices */
    double denom = 1.0;
    int run = 1;
    for (int m = 1; m <= k; ++m) {
      if (m < k && tup[blk * k + m] == tup[blk * k + m - 1]) {
        ++run;
      } else {
        for (int q = 2; q <= run; ++q) denom *= q;
        run = 1;
      }
    }
    double sq = 0.0;
    for (int64_t e = 0; e < bk; ++e) {
      double v = A[blk * bk + e];
      sq += v * v;
    }
    z += (kfact / denom) * sq;
  }
  free(tup);
  return sqrt(z);
}

/* Eq. (mef): fro[k] = ||C_k|| (k = 1..d), nu[k] = fro[k] / fro[2]^(k/2) for
 * k >= 3 (NaN when ||C_2|| = 0); nu[0..2] are set to NaN.  fro[0] is unused (NaN). */
void orc_norms(int n, int b, int d, const double *const *C, double *fro, double *nu) {
  fro[0] = NAN;
  for (int k = 1; k <= d; ++k) fro[k] = orc_block_norm(n, b, k, C[k - 1]);
  for (int k = 0; k <= d; ++k) {
    if (k < 3 || d < 2 || !(fro[2] > 0.0)) nu[k] = NAN;  /* no scale: ||C_2|| = 0 */
    else nu[k] = fro[k] / pow(fro[2], 0.5 * k);
  }
}

/* Threads the OpenMP loops above use. */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
#else
int orc_num_threads(void) { return 1; }
#endif
