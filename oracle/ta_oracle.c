/*
 * ta_oracle.c -- plain, slow, obviously-correct CPU oracle for the trace ->
 * rank x iteration x region tensor method and its statistics.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code, header or table with the HIP path.
 *
 * Paper: "Enhancing Performance Insight at Scale: A Heterogeneous Framework for
 * Exascale Diagnostics" (arXiv 2605.03561).
 *
 * Everything here is the plain definition written out, event by event:
 *   - durations and exclusive cost:   Sec. II (traces are series of timed
 *     calling-context-tree node events; HPCToolkit samples the call stack), and
 *     Sec. VI-B ("inclusive and exclusive costs" per CCT node);
 *   - inclusive cost:                 an ancestor walk up the parent tree
 *     (Sec. VI-B, bottom-up call-path traversal from a leaf id);
 *   - iteration boundaries and the re-materialised per-iteration profile:
 *     Sec. V and Fig. 2 (scan traces for iterative boundaries, rebuild one
 *     profile per interval, index node x trace x iteration);
 *   - per-iteration cross-rank statistics {mean, min, max, std}: the groupby
 *     listing of Sec. VI-A (pandas semantics, so std uses ddof = 1);
 *   - global balance ratio (mean over ranks / max over ranks): Sec. VI-A
 *     (GPU imbalance quantification) and Sec. VI-B;
 *   - coefficient of variation across / within ranks: Sec. VI-A, Table IV;
 *   - potential savings = average max - average mean per iteration, times the
 *     iteration count, divided by application time: Sec. VI-A, Table V;
 *   - execution share: Table IV, column 2.
 * The outlier statistic (robust z from median / MAD) is not in the paper; it is
 * the textbook modified z-score (Iglewicz-Hoaglin), written out per column.
 *
 * Readings where the paper is silent are listed in the design notes; the ones
 * that change arithmetic are restated at the function that uses them.
 *
 * Precision: int64 for all times (ns), __int128 for sums of squares, FP64 for
 * every statistic; FP accumulations of many FP64 terms are long double, except
 * where the result feeds a difference that can cancel (the second-stage
 * means and deviations of the outlier scores, the topology means): those sums
 * are exact, rounded once (tao_fsum).
 * Build: gcc -O2 -ffp-contract=off (no FMA contraction), optional -fopenmp
 * (only the independent per-rank loop is parallel; results do not depend on it).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status codes: the numeric values are the library's documented ABI values. */
enum {
  TAO_OK = 0,
  TAO_ERR_INVALID_ARG = 1,
  TAO_ERR_BAD_TREE = 2,
  TAO_ERR_CTX_RANGE = 3,
  TAO_ERR_UNSORTED = 4,
  TAO_ERR_ITER_OVERFLOW = 5,
  TAO_ERR_SIZE_OVERFLOW = 6
};

typedef __int128 i128;

/* ------------------------------------------------------------------------ */
/* Tree helpers                                                              */
/* ------------------------------------------------------------------------ */

/* A parent array is a valid forest iff every node reaches a root (-1) in at
 * most N steps and every parent id is in range. */
int tao_check_tree(int32_t N, const int32_t *parent) {
  if (N <= 0 || parent == NULL) return TAO_ERR_INVALID_ARG;
  for (int32_t v = 0; v < N; v++) {
    int32_t u = v;
    int32_t steps = 0;
    while (u != -1) {
      if (u < -1 || u >= N) return TAO_ERR_BAD_TREE;
      if (steps > N) return TAO_ERR_BAD_TREE; /* cycle */
      u = parent[u];
      steps++;
    }
  }
  return TAO_OK;
}

/* Is `a` an ancestor-or-self of `c`?  Plain walk to the root. */
static int is_anc_or_self(const int32_t *parent, int32_t a, int32_t c) {
  for (int32_t u = c; u != -1; u = parent[u])
    if (u == a) return 1;
  return 0;
}

/* Region of a node: the region whose root is the NEAREST ancestor-or-self of
 * c among the region roots; -1 if none.  Plain walk, checking every region at
 * each step (O(depth * G)). */
static int32_t region_of_node(const int32_t *parent, int32_t c, int32_t G,
                              const int32_t *region_nodes) {
  for (int32_t u = c; u != -1; u = parent[u])
    for (int32_t g = 0; g < G; g++)
      if (region_nodes[g] == u) return g;
  return -1;
}

/* Number of OpenMP threads for the next calls (n < 1: leave as is); returns
 * the number in use.  Only the timing of the oracle uses it: results do not
 * depend on the thread count. */
int tao_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Input checks shared by attribute and segment                              */
/* ------------------------------------------------------------------------ */

static int check_traces(int64_t R, const int64_t *off, const int64_t *ts,
                        const int32_t *ctx, int32_t N) {
  if (R < 0 || off == NULL) return TAO_ERR_INVALID_ARG;
  if (off[0] != 0) return TAO_ERR_INVALID_ARG;
  for (int64_t r = 0; r < R; r++)
    if (off[r + 1] < off[r]) return TAO_ERR_INVALID_ARG;
  int64_t E = off[R];
  if (E > 0 && (ts == NULL || ctx == NULL)) return TAO_ERR_INVALID_ARG;
  for (int64_t k = 0; k < E; k++)
    if (ctx[k] < 0 || ctx[k] >= N) return TAO_ERR_CTX_RANGE;
  for (int64_t r = 0; r < R; r++)
    for (int64_t k = off[r]; k + 1 < off[r + 1]; k++)
      if (ts[k + 1] < ts[k]) return TAO_ERR_UNSORTED;
  return TAO_OK;
}

/* Duration of event k of a rank whose events are [b, e): the time until the
 * next sample of the same rank; the last sample of a rank gets 0 (sampling
 * semantics, Sec. II; the interval [t_k, t_k+1) belongs to ctx_k). */
static int64_t duration(const int64_t *ts, int64_t k, int64_t e) {
  return (k + 1 < e) ? ts[k + 1] - ts[k] : 0;
}

/* ------------------------------------------------------------------------ */
/* Attribution: exclusive and inclusive cost per CCT node per rank           */
/* ------------------------------------------------------------------------ */

/* excl[r][v] = sum of durations of rank r's events whose context is v.
 * incl[r][v] = sum of excl[r][u] over every u whose ancestor-or-self set holds
 *              v (computed by walking from each u to the root).
 * Either output may be NULL. */
int tao_attribute(int64_t R, const int64_t *off, const int64_t *ts,
                  const int32_t *ctx, int32_t N, const int32_t *parent,
                  int64_t *excl, int64_t *incl) {
  int st = tao_check_tree(N, parent);
  if (st) return st;
  st = check_traces(R, off, ts, ctx, N);
  if (st) return st;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < R; r++) {
    int64_t *ex = excl ? excl + r * (int64_t)N : NULL;
    int64_t *local = NULL;
    if (!ex) {
      local = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
      ex = local;
    }
    for (int32_t v = 0; v < N; v++) ex[v] = 0;
    for (int64_t k = off[r]; k < off[r + 1]; k++)
      ex[ctx[k]] += duration(ts, k, off[r + 1]);
    if (incl) {
      int64_t *in = incl + r * (int64_t)N;
      for (int32_t v = 0; v < N; v++) in[v] = 0;
      for (int32_t u = 0; u < N; u++)
        for (int32_t a = u; a != -1; a = parent[a]) in[a] += ex[u];
    }
    free(local);
  }
  return TAO_OK;
}

/* ------------------------------------------------------------------------ */
/* Segmentation: iteration boundaries and the rank x iteration x region      */
/* tensor (Sec. V, Fig. 2)                                                   */
/* ------------------------------------------------------------------------ */

/* Reading of the iteration boundary (the paper gives no rule): an event is a
 * boundary when its context lies in the marker's subtree and the previous event
 * of the same rank (if any) does not.  The iteration index of an event is the
 * number of boundaries at or before it, minus one; events before the first
 * boundary (index -1) and events outside every region go to `outside`.  The
 * last iteration runs to the end of the trace.
 *
 * tensor[(r*I + i)*G + g] = sum of d_k over rank r's events k with iteration i
 *                           and region g.
 * iters_found[r] = number of boundaries; more than I -> TAO_ERR_ITER_OVERFLOW.
 * span[r] = t_last - t_first (0 for an empty rank), outside[r] = span - sum T.
 * outside and span may be NULL. */
int tao_segment(int64_t R, const int64_t *off, const int64_t *ts,
                const int32_t *ctx, int32_t N, const int32_t *parent,
                int32_t marker, int32_t G, const int32_t *region_nodes,
                int32_t I, int64_t *tensor, int32_t *iters_found,
                int64_t *outside, int64_t *span) {
  int st = tao_check_tree(N, parent);
  if (st) return st;
  if (marker < 0 || marker >= N || G < 0 || I < 0 || tensor == NULL ||
      iters_found == NULL || (G > 0 && region_nodes == NULL))
    return TAO_ERR_INVALID_ARG;
  for (int32_t g = 0; g < G; g++) {
    if (region_nodes[g] < 0 || region_nodes[g] >= N) return TAO_ERR_INVALID_ARG;
    for (int32_t h = 0; h < g; h++)
      if (region_nodes[h] == region_nodes[g]) return TAO_ERR_INVALID_ARG;
  }
  st = check_traces(R, off, ts, ctx, N);
  if (st) return st;

  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : overflow)
  for (int64_t r = 0; r < R; r++) {
    int64_t *row = tensor + r * (int64_t)I * G;
    for (int64_t j = 0; j < (int64_t)I * G; j++) row[j] = 0;
    int64_t b = off[r], e = off[r + 1];
    int64_t out = 0;
    int32_t it = -1;   /* iteration index of the current event */
    int prev_in = 0;   /* was the previous event inside the marker subtree? */
    for (int64_t k = b; k < e; k++) {
      int32_t c = ctx[k];
      int in_m = is_anc_or_self(parent, marker, c);
      if (in_m && (k == b || !prev_in)) it++;
      prev_in = in_m;
      int64_t d = duration(ts, k, e);
      int32_t g = region_of_node(parent, c, G, region_nodes);
      if (it < 0 || g < 0) {
        out += d;
      } else if (it < I) {
        row[(int64_t)it * G + g] += d;
      }
      /* it >= I: overflow, reported below; the value is not stored. */
    }
    iters_found[r] = it + 1;
    if (it + 1 > I) overflow = 1;
    int64_t sp = (e > b) ? ts[e - 1] - ts[b] : 0;
    if (span) span[r] = sp;
    if (outside) outside[r] = out;
  }
  return overflow ? TAO_ERR_ITER_OVERFLOW : TAO_OK;
}

/* ------------------------------------------------------------------------ */
/* Imbalance statistics (Sec. VI-A, Tables IV and V, groupby listing)        */
/* ------------------------------------------------------------------------ */

/* int128 -> double, correctly rounded (gcc's conversion is). */
static double d128(i128 x) { return (double)x; }

/* The valid ranks of iteration i are those that found more than i iterations
 * (ranks with fewer iterations are left out of that iteration's statistics).
 * With iters_found == NULL every rank is valid for every iteration. */
static int valid(const int32_t *iters_found, int64_t r, int32_t i) {
  return iters_found == NULL || i < iters_found[r];
}

/* Per (i,g), over the valid ranks, with n = count:
 *   s1 = sum x (int64), s2 = sum x^2 (int128), mn, mx
 *   mean           = s1 / n
 *   std            = sqrt((n*s2 - s1^2) / (n*(n - ddof)))     (NaN if n<=ddof)
 *   max_minus_mean = (n*mx - s1) / n
 * computed as one FP64 operation on exact integers each.  Empty columns give
 * mean = std = max_minus_mean = NaN and min = max = 0.
 *
 * Per region g, over I' = {i : n_i > 0}:
 *   avg_mean         = (1/|I'|) sum_i mean_i
 *   avg_max          = (1/|I'|) sum_i max_i
 *   savings_per_iter = (1/|I'|) sum_i (max_i - mean_i)       [= avg_max - avg_mean]
 *   total_savings    = savings_per_iter * |I'|
 *   balance_ratio    = (sum_r S[r,g] / R) / max_r S[r,g],   S[r,g] = sum_i x
 *   cv_across        = mean over {i : n_i > ddof, mean_i > 0} of std_i / mean_i
 *   cv_within        = mean over {r : n_r > ddof, S[r,g] > 0} of the rank's
 *                      std over its iterations / its mean over its iterations
 *   share            = sum of region g's cells / sum of all cells
 * and potential_speedup = sum_g total_savings_g / t_app (fraction of time).
 * FP sums of many FP64 terms accumulate in long double, in ascending index.
 * t_app <= 0: use max_r span[r] if span != NULL, else NaN. */
int tao_imbalance(const int64_t *T, int64_t R, int32_t I, int32_t G,
                  const int32_t *iters_found, int32_t ddof, double t_app,
                  const int64_t *span,
                  /* [I*G] */ double *mean, double *stdv, double *max_minus_mean,
                  int64_t *minv, int64_t *maxv,
                  /* [G] */ double *avg_mean, double *avg_max,
                  double *savings_per_iter, double *total_savings,
                  double *balance_ratio, double *cv_across, double *cv_within,
                  double *share,
                  /* [1] */ double *potential_speedup) {
  if (R < 0 || I < 0 || G <= 0 || ddof < 0 || T == NULL) return TAO_ERR_INVALID_ARG;
  const double nan = NAN;
  int64_t grand = 0;
#pragma omp parallel for reduction(+ : grand)
  for (int64_t r = 0; r < R; r++)
    for (int32_t i = 0; i < I; i++)
      if (valid(iters_found, r, i))
        for (int32_t g = 0; g < G; g++) grand += T[((int64_t)r * I + i) * G + g];

  /* Regions are independent (threads take whole regions); each region's
   * total savings is kept and the total is summed in ascending g below. */
  double *tot_g = (double *)malloc(sizeof(double) * (size_t)G);
  int *has_g = (int *)malloc(sizeof(int) * (size_t)G);
  if (!tot_g || !has_g) {
    free(tot_g);
    free(has_g);
    return TAO_ERR_SIZE_OVERFLOW;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t g = 0; g < G; g++) {
    long double acc_mean = 0.0L, acc_mm = 0.0L, acc_cv = 0.0L;
    int64_t acc_max = 0, n_iters = 0, n_cv = 0;
    for (int32_t i = 0; i < I; i++) {
      int64_t n = 0, s1 = 0, mn = 0, mx = 0;
      i128 s2 = 0;
      for (int64_t r = 0; r < R; r++) {
        if (!valid(iters_found, r, i)) continue;
        int64_t x = T[((int64_t)r * I + i) * G + g];
        if (n == 0 || x < mn) mn = x;
        if (n == 0 || x > mx) mx = x;
        n++;
        s1 += x;
        s2 += (i128)x * x;
      }
      double m = nan, sd = nan, mm = nan;
      if (n > 0) {
        m = (double)s1 / (double)n;
        mm = d128((i128)n * mx - s1) / (double)n;
        if (n > ddof) {
          double var = d128((i128)n * s2 - (i128)s1 * s1) /
                       ((double)n * (double)(n - ddof));
          sd = sqrt(var);
        }
        acc_mean += m;
        acc_mm += mm;
        acc_max += mx;
        n_iters++;
        if (n > ddof && m > 0.0) {
          acc_cv += sd / m;
          n_cv++;
        }
      }
      int64_t j = (int64_t)i * G + g;
      if (mean) mean[j] = m;
      if (stdv) stdv[j] = sd;
      if (max_minus_mean) max_minus_mean[j] = mm;
      if (minv) minv[j] = mn;
      if (maxv) maxv[j] = mx;
    }
    double spi = n_iters ? (double)(acc_mm / (long double)n_iters) : nan;
    double tot = n_iters ? spi * (double)n_iters : nan;
    if (avg_mean) avg_mean[g] = n_iters ? (double)(acc_mean / (long double)n_iters) : nan;
    if (avg_max) avg_max[g] = n_iters ? (double)acc_max / (double)n_iters : nan;
    if (savings_per_iter) savings_per_iter[g] = spi;
    if (total_savings) total_savings[g] = tot;
    tot_g[g] = tot;
    has_g[g] = n_iters > 0;
    if (cv_across) cv_across[g] = n_cv ? (double)(acc_cv / (long double)n_cv) : nan;

    /* Per-rank totals over the rank's valid iterations. */
    int64_t ssum = 0, smax = 0, gsum = 0;
    long double acc_w = 0.0L;
    int64_t n_w = 0;
    for (int64_t r = 0; r < R; r++) {
      int64_t s = 0, nr = 0;
      i128 q = 0;
      for (int32_t i = 0; i < I; i++) {
        if (!valid(iters_found, r, i)) continue;
        int64_t x = T[((int64_t)r * I + i) * G + g];
        s += x;
        q += (i128)x * x;
        nr++;
      }
      ssum += s;
      if (r == 0 || s > smax) smax = s;
      gsum += s;
      if (nr > ddof && s > 0) {
        double mr = (double)s / (double)nr;
        double vr = d128((i128)nr * q - (i128)s * s) / ((double)nr * (double)(nr - ddof));
        acc_w += sqrt(vr) / mr;
        n_w++;
      }
    }
    if (balance_ratio)
      balance_ratio[g] = (R > 0 && smax != 0)
                             ? ((double)ssum / (double)R) / (double)smax
                             : nan;
    if (cv_within) cv_within[g] = n_w ? (double)(acc_w / (long double)n_w) : nan;
    if (share) share[g] = grand ? (double)gsum / (double)grand : nan;
  }
  long double sum_total = 0.0L;
  for (int32_t g = 0; g < G; g++)
    if (has_g[g]) sum_total += tot_g[g];
  free(tot_g);
  free(has_g);
  if (potential_speedup) {
    double tapp = t_app;
    if (!(tapp > 0.0)) {
      tapp = nan;
      if (span && R > 0) {
        int64_t mx = span[0];
        for (int64_t r = 1; r < R; r++)
          if (span[r] > mx) mx = span[r];
        tapp = (double)mx;
      }
    }
    potential_speedup[0] = (double)sum_total / tapp;
  }
  return TAO_OK;
}

/* ------------------------------------------------------------------------ */
/* Outliers: robust z (median / MAD) and plain z scores                      */
/* ------------------------------------------------------------------------ */

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}
static int cmp_f64(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Twice the median of n sorted integers: 2*x[n/2] for odd n, the sum of the
 * two middle values for even n (exact in int64). */
static int64_t twice_median_sorted(const int64_t *s, int64_t n) {
  return (n & 1) ? 2 * s[n / 2] : s[n / 2 - 1] + s[n / 2];
}

/* Exact sum of n doubles (every `stride`-th of v), rounded once to nearest
 * (ties to even); exact zero gives +0.0 and any non-finite term gives NaN.
 * Shewchuk's algorithm (Adaptive Precision Floating-Point Arithmetic, 1997):
 * the running sum is kept as a list of non-overlapping partials, each new term
 * is folded in by exact two-sum steps (sum rounded + its exact error), and the
 * partials are added from the largest down; the last step checks whether the
 * remaining partials push an exact halfway case up or down. */
double tao_fsum(const double *v, int64_t n, int64_t stride) {
  double part[256];  /* non-overlapping: far fewer than 2,100 / 53 + 2 are live */
  int np = 0;
  for (int64_t k = 0; k < n; k++) {
    double x = v[k * stride];
    if (!isfinite(x)) return NAN;
    int j = 0;
    for (int i = 0; i < np; i++) {
      double y = part[i];
      if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
      double hi = x + y;
      double lo = y - (hi - x);
      if (lo != 0.0) part[j++] = lo;
      x = hi;
    }
    part[j++] = x;
    np = j;
  }
  if (np == 0) return 0.0;
  double hi = part[--np], lo = 0.0;
  while (np > 0) {
    double x = hi, y = part[--np];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  /* hi + lo is exact and hi = round(hi + lo); if lo is exactly half an ulp of
   * hi and the next partial has the same sign, the true sum lies beyond the
   * halfway point, so round away from hi. */
  if (np > 0 && ((lo < 0.0 && part[np - 1] < 0.0) || (lo > 0.0 && part[np - 1] > 0.0))) {
    double y = lo * 2.0, x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi == 0.0 ? 0.0 : hi;
}

/* Robust z of one integer column (n values, already gathered):
 *   med2 = 2*median,  dev_r = |2x_r - med2| (= 2|x - med|),
 *   mad4 = 2*median(dev) (= 4*MAD),
 *   z_r  = (4x_r - 2*med2) / (1.4826 * mad4)            when mad4 > 0,
 *   z_r  = (2x_r - med2)*n / (1.253314 * sum_r dev_r)   when mad4 == 0 and
 *                                                       the mean abs dev > 0,
 *   z_r  = 0                                            otherwise (all equal).
 * 1.4826 = 1/Phi^-1(3/4) makes MAD consistent with the normal sigma;
 * 1.253314 = sqrt(pi/2) does the same for the mean absolute deviation. */
static void robust_z_int(const int64_t *x, int64_t n, double *z, int64_t *work) {
  memcpy(work, x, sizeof(int64_t) * (size_t)n);
  qsort(work, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t med2 = twice_median_sorted(work, n);
  int64_t sumdev = 0;
  for (int64_t r = 0; r < n; r++) {
    int64_t dv = 2 * x[r] - med2;
    work[r] = dv < 0 ? -dv : dv;
    sumdev += work[r];
  }
  qsort(work, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t mad4 = twice_median_sorted(work, n);
  for (int64_t r = 0; r < n; r++) {
    if (mad4 > 0) {
      z[r] = (double)(4 * x[r] - 2 * med2) / (1.4826 * (double)mad4);
    } else if (sumdev > 0) {
      z[r] = ((double)(2 * x[r] - med2) * (double)n) / (1.253314 * (double)sumdev);
    } else {
      z[r] = 0.0;
    }
  }
}

/* The same robust z for FP64 values: med = middle value (odd n) or
 * 0.5*(a + b) (even n); MAD = median of |v - med| by the same rule;
 * z = (v - med) / (1.4826*MAD); MAD == 0 -> 1.253314 * mean|v - med| (the
 * exact sum of the |v - med|, rounded, over n); both zero -> 0. */
static void robust_z_f64(const double *v, int64_t n, double *z, double *work) {
  memcpy(work, v, sizeof(double) * (size_t)n);
  qsort(work, (size_t)n, sizeof(double), cmp_f64);
  double med = (n & 1) ? work[n / 2] : 0.5 * (work[n / 2 - 1] + work[n / 2]);
  for (int64_t r = 0; r < n; r++) work[r] = fabs(v[r] - med);
  double mean_ad = tao_fsum(work, n, 1) / (double)n;
  qsort(work, (size_t)n, sizeof(double), cmp_f64);
  double mad = (n & 1) ? work[n / 2] : 0.5 * (work[n / 2 - 1] + work[n / 2]);
  for (int64_t r = 0; r < n; r++) {
    if (mad > 0.0)
      z[r] = (v[r] - med) / (1.4826 * mad);
    else if (mean_ad > 0.0)
      z[r] = (v[r] - med) / (1.253314 * mean_ad);
    else
      z[r] = 0.0;
  }
}

/* Plain z with ddof: (x - mean)/std over the n values; std from exact sums for
 * integers; std == 0 or n <= ddof -> 0. */
static void plain_z_int(const int64_t *x, int64_t n, int32_t ddof, double *z) {
  int64_t s1 = 0;
  i128 s2 = 0;
  for (int64_t r = 0; r < n; r++) {
    s1 += x[r];
    s2 += (i128)x[r] * x[r];
  }
  double sd = 0.0;
  if (n > ddof)
    sd = sqrt(d128((i128)n * s2 - (i128)s1 * s1) / ((double)n * (double)(n - ddof)));
  for (int64_t r = 0; r < n; r++)
    z[r] = (sd > 0.0) ? d128((i128)n * x[r] - s1) / ((double)n * sd) : 0.0;
}
/* FP64 values: mean = (exact sum, rounded) / n; the squared deviations
 * (v - mean)^2 are rounded to FP64 and summed exactly (rounded once);
 * std = sqrt(that / (n - ddof)).  `work` holds n doubles. */
static void plain_z_f64(const double *v, int64_t n, int32_t ddof, double *z, double *work) {
  double m = tao_fsum(v, n, 1) / (double)n;
  for (int64_t r = 0; r < n; r++) work[r] = (v[r] - m) * (v[r] - m);
  double q = tao_fsum(work, n, 1);
  double sd = (n > ddof) ? sqrt(q / (double)(n - ddof)) : 0.0;
  for (int64_t r = 0; r < n; r++) z[r] = (sd > 0.0) ? (v[r] - m) / sd : 0.0;
}

/* Outlier scan over the tensor.  Ranks with iters_found == 0 take no part and
 * get score 0 / flag 0.  (Not in the paper, which clusters ranks instead; this
 * is the exact scan that judges the learned pre-screen.)
 *
 * mode 0 (FULL):   per column (i,g), a score z(r,i,g) over the ranks valid in
 *                  iteration i; m(r,g) = mean over the rank's valid iterations
 *                  of z (FP64 sum in ascending i); then per region a second
 *                  robust z over ranks of m(r,g).
 * mode 1 (TOTALS): per region, one score over ranks of S[r,g] (the sum of the
 *                  rank's valid cells).
 * kind 0: robust (median/MAD) z;  kind 1: plain z with ddof 1.
 * rank_score[r] = max_g |z2(r,g)|,  rank_flag[r] = rank_score > tau,
 * region_score[r*G+g] = z2(r,g) (signed; may be NULL). */
int tao_outliers(const int64_t *T, int64_t R, int32_t I, int32_t G,
                 const int32_t *iters_found, int32_t mode, int32_t kind,
                 double tau, double *rank_score, uint8_t *rank_flag,
                 int64_t *n_flagged, double *region_score) {
  if (R < 0 || I < 0 || G <= 0 || T == NULL || rank_score == NULL ||
      rank_flag == NULL || (mode != 0 && mode != 1) || (kind != 0 && kind != 1))
    return TAO_ERR_INVALID_ARG;
  int64_t *who = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R + 1));
  double *m = (double *)calloc((size_t)R * (size_t)G + 1, sizeof(double));
  double *zr = (double *)malloc(sizeof(double) * ((size_t)R * (size_t)G + 1));
  if (!who || !m || !zr) {
    free(who); free(m); free(zr);
    return TAO_ERR_SIZE_OVERFLOW;
  }

  /* Active ranks: at least one iteration. */
  int64_t na = 0;
  for (int64_t r = 0; r < R; r++)
    if (iters_found == NULL ? I > 0 : iters_found[r] > 0) who[na++] = r;

  /* Regions are independent: threads take whole regions, each with its own
   * column buffers; within a region the iterations go in ascending order. */
  int nomem = 0;
#pragma omp parallel reduction(| : nomem)
  {
    int64_t *col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R + 1));
    int64_t *iwork = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R + 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    double *fwork = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    double *fcol = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    int ok = col && iwork && z && fwork && fcol;
    if (!ok) nomem = 1;
#pragma omp for schedule(dynamic, 1)
    for (int32_t g = 0; g < G; g++) {
      if (!ok) continue;
      if (mode == 0) {
        /* Stage 1: per-cell score, summed over i in ascending order per (r,g). */
        for (int32_t i = 0; i < I; i++) {
          int64_t n = 0;
          for (int64_t a = 0; a < na; a++) {
            int64_t r = who[a];
            if (valid(iters_found, r, i)) col[n++] = T[((int64_t)r * I + i) * G + g];
          }
          if (n == 0) continue;
          if (kind == 0) robust_z_int(col, n, z, iwork);
          else plain_z_int(col, n, 1, z);
          n = 0;
          for (int64_t a = 0; a < na; a++) {
            int64_t r = who[a];
            if (valid(iters_found, r, i)) m[r * G + g] += z[n++];
          }
        }
        for (int64_t a = 0; a < na; a++) {
          int64_t r = who[a];
          double cnt = (double)(iters_found ? iters_found[r] : I);
          if (iters_found && iters_found[r] > I) cnt = (double)I;
          m[r * G + g] = m[r * G + g] / cnt;
        }
        /* Stage 2: score of m(r,g) over active ranks. */
        for (int64_t a = 0; a < na; a++) fcol[a] = m[who[a] * G + g];
        if (na > 0) {
          if (kind == 0) robust_z_f64(fcol, na, z, fwork);
          else plain_z_f64(fcol, na, 1, z, fwork);
        }
      } else {
        for (int64_t a = 0; a < na; a++) {
          int64_t r = who[a], s = 0;
          for (int32_t i = 0; i < I; i++)
            if (valid(iters_found, r, i)) s += T[((int64_t)r * I + i) * G + g];
          col[a] = s;
        }
        if (na > 0) {
          if (kind == 0) robust_z_int(col, na, z, iwork);
          else plain_z_int(col, na, 1, z);
        }
      }
      for (int64_t a = 0; a < na; a++) zr[who[a] * G + g] = z[a];
    }
    free(col); free(iwork); free(z); free(fwork); free(fcol);
  }
  if (nomem) {
    free(who); free(m); free(zr);
    return TAO_ERR_SIZE_OVERFLOW;
  }

  int64_t nf = 0;
  for (int64_t r = 0; r < R; r++) {
    rank_score[r] = 0.0;
    rank_flag[r] = 0;
    if (region_score)
      for (int32_t g = 0; g < G; g++) region_score[r * G + g] = 0.0;
  }
  for (int64_t a = 0; a < na; a++) {
    int64_t r = who[a];
    double best = 0.0;
    for (int32_t g = 0; g < G; g++) {
      double v = fabs(zr[r * G + g]);
      if (v > best) best = v;
      if (region_score) region_score[r * G + g] = zr[r * G + g];
    }
    rank_score[r] = best;
    rank_flag[r] = best > tau;
    nf += rank_flag[r];
  }
  if (n_flagged) n_flagged[0] = nf;
  free(who); free(m); free(zr);
  return TAO_OK;
}

/* ------------------------------------------------------------------------ */
/* Topology aggregation (Sec. VI-B: ranks -> compute nodes -> racks/chassis) */
/* ------------------------------------------------------------------------ */

/* Per rack and per chassis: number of flagged ranks, max score and mean score
 * over the ranks placed there (NaN where none). */
int tao_topology(const double *rank_score, const uint8_t *rank_flag, int64_t R,
                 const int32_t *rank_node, const int32_t *node_rack,
                 const int32_t *node_chassis, int32_t n_nodes, int32_t n_racks,
                 int32_t n_chassis, int64_t *flagged_rack, double *max_rack,
                 double *mean_rack, int64_t *flagged_chassis,
                 double *max_chassis, double *mean_chassis) {
  if (R < 0 || n_racks <= 0 || n_chassis <= 0 || n_nodes <= 0) return TAO_ERR_INVALID_ARG;
  for (int64_t r = 0; r < R; r++) {
    int32_t nd = rank_node[r];
    if (nd < 0 || nd >= n_nodes) return TAO_ERR_INVALID_ARG;
    if (node_rack[nd] < 0 || node_rack[nd] >= n_racks) return TAO_ERR_INVALID_ARG;
    if (node_chassis[nd] < 0 || node_chassis[nd] >= n_chassis) return TAO_ERR_INVALID_ARG;
  }
  for (int pass = 0; pass < 2; pass++) {
    int32_t K = pass ? n_chassis : n_racks;
    const int32_t *key = pass ? node_chassis : node_rack;
    int64_t *fl = pass ? flagged_chassis : flagged_rack;
    double *mx = pass ? max_chassis : max_rack;
    double *mn = pass ? mean_chassis : mean_rack;
    double *sel = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    if (!sel) return TAO_ERR_SIZE_OVERFLOW;
    for (int32_t k = 0; k < K; k++) {
      int64_t cnt = 0, nfl = 0;
      double best = -INFINITY;
      for (int64_t r = 0; r < R; r++) {
        if (key[rank_node[r]] != k) continue;
        sel[cnt++] = rank_score[r];
        nfl += rank_flag[r] ? 1 : 0;
        if (rank_score[r] > best) best = rank_score[r];
      }
      if (fl) fl[k] = nfl;
      if (mx) mx[k] = cnt ? best : NAN;
      /* mean = (exact sum of the scores, rounded) / count */
      if (mn) mn[k] = cnt ? tao_fsum(sel, cnt, 1) / (double)cnt : NAN;
    }
    free(sel);
  }
  return TAO_OK;
}

/* ------------------------------------------------------------------------- */
/* Pruning (Sec. III: pruning strategies are evaluated once on the summary    */
/* profile -- the aggregate of all parallel profiles -- and propagated to     */
/* every profile; Sec. VI: negligible code regions, less than 1 % of the      */
/* total runtime, are removed).                                               */
/* ------------------------------------------------------------------------- */

/* Summary profile: sums over ranks of excl[R][N] and incl[R][N] (either input
 * may be NULL, then its output is left alone). */
int tao_summary(int64_t R, int32_t N, const int64_t *excl, const int64_t *incl,
                int64_t *sum_excl, int64_t *sum_incl) {
  if (R < 0 || N <= 0) return TAO_ERR_INVALID_ARG;
  for (int32_t v = 0; v < N; v++) {
    int64_t se = 0, si = 0;
    for (int64_t r = 0; r < R; r++) {
      if (excl) se += excl[r * N + v];
      if (incl) si += incl[r * N + v];
    }
    if (excl && sum_excl) sum_excl[v] = se;
    if (incl && sum_incl) sum_incl[v] = si;
  }
  return TAO_OK;
}

/* Kept nodes: v with (double)sum_incl[v] >= fraction * (double)total, total =
 * sum over v of sum_excl[v]; listed in ascending node id. */
int tao_prune(int32_t N, const int64_t *sum_excl, const int64_t *sum_incl, double fraction,
              int32_t *kept, int32_t *n_kept) {
  if (N <= 0 || !sum_excl || !sum_incl || !kept || !n_kept || !(fraction >= 0.0))
    return TAO_ERR_INVALID_ARG;
  int64_t total = 0;
  for (int32_t v = 0; v < N; v++) total += sum_excl[v];
  const double cut = fraction * (double)total;
  int32_t k = 0;
  for (int32_t v = 0; v < N; v++)
    if ((double)sum_incl[v] >= cut) kept[k++] = v;
  *n_kept = k;
  return TAO_OK;
}

/* Nearest ancestor-or-self of u that is kept (is_kept[] = index in kept or
 * -1), or -1.  Plain walk. */
static int32_t nearest_kept(const int32_t *parent, const int32_t *is_kept, int32_t u) {
  for (; u != -1; u = parent[u])
    if (is_kept[u] >= 0) return is_kept[u];
  return -1;
}

/* Profiles on the pruned tree, per rank: p_excl[r][k] = sum of excl[r][u] over
 * the nodes u whose nearest kept ancestor-or-self is kept[k] (the cost of pruned
 * descendants folds into the nearest kept ancestor); p_incl[r][k] = sum of
 * excl[r][u] over the subtree of kept[k]. */
int tao_pruned(int64_t R, int32_t N, const int32_t *parent, const int64_t *excl, int32_t K,
               const int32_t *kept, int64_t *p_excl, int64_t *p_incl) {
  if (R < 0 || N <= 0 || K <= 0 || !parent || !excl || !kept) return TAO_ERR_INVALID_ARG;
  int32_t *is_kept = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  if (!is_kept) return TAO_ERR_INVALID_ARG;
  for (int32_t v = 0; v < N; v++) is_kept[v] = -1;
  for (int32_t k = 0; k < K; k++) {
    if (kept[k] < 0 || kept[k] >= N || is_kept[kept[k]] >= 0) {
      free(is_kept);
      return TAO_ERR_INVALID_ARG;
    }
    is_kept[kept[k]] = k;
  }
  for (int64_t r = 0; r < R; r++) {
    int64_t *pe = p_excl ? p_excl + r * K : NULL;
    int64_t *pi = p_incl ? p_incl + r * K : NULL;
    for (int32_t k = 0; k < K; k++) {
      if (pe) pe[k] = 0;
      if (pi) pi[k] = 0;
    }
    for (int32_t u = 0; u < N; u++) {
      const int64_t x = excl[r * N + u];
      if (x == 0) continue;
      const int32_t k = nearest_kept(parent, is_kept, u);
      if (pe && k >= 0) pe[k] += x;
      if (pi)
        for (int32_t w = u; w != -1; w = parent[w])
          if (is_kept[w] >= 0) pi[is_kept[w]] += x;
    }
  }
  free(is_kept);
  return TAO_OK;
}

/* Inclusive version of a rank x iteration x region tensor whose regions are
 * nested (e.g. the kept nodes of a pruned tree): out[r][i][g] = sum of T[r][i][h]
 * over the regions h whose node lies in the subtree of region g's node. */
int tao_tensor_inclusive(const int64_t *T, int64_t R, int32_t I, int32_t G, int32_t N,
                         const int32_t *parent, const int32_t *region_nodes, int64_t *out) {
  if (!T || !out || R < 0 || I < 0 || G <= 0 || N <= 0 || !parent || !region_nodes)
    return TAO_ERR_INVALID_ARG;
  int32_t *is_reg = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  if (!is_reg) return TAO_ERR_INVALID_ARG;
  for (int32_t v = 0; v < N; v++) is_reg[v] = -1;
  for (int32_t g = 0; g < G; g++) is_reg[region_nodes[g]] = g;
  for (int64_t c = 0; c < R * I; c++) {
    const int64_t *row = T + c * G;
    int64_t *o = out + c * G;
    for (int32_t g = 0; g < G; g++) o[g] = 0;
    for (int32_t h = 0; h < G; h++)
      for (int32_t w = region_nodes[h]; w != -1; w = parent[w])
        if (is_reg[w] >= 0) o[is_reg[w]] += row[h];
  }
  free(is_reg);
  return TAO_OK;
}

/* ---- Clustering of ranks (Sec. VI-B: DBSCAN over the ranks, K-Means with
 * 2..5 groups, and the compute nodes whose ranks fall in two groups). ---- */

/* K-Means (Lloyd) on integer feature rows X[R][D], K clusters from the given
 * centroids C0[K][D].  An iteration assigns every row to the centroid with the
 * smallest squared distance, summed over d in ascending order of
 * ((double)x_d - c_d)^2 with every product and sum rounded (no fused
 * multiply-add), ties to the smaller k; then each centroid becomes the mean of
 * its rows, (double)(exact int64 sum) / count, and keeps its value when no row
 * chose it.  Iterations stop after the first one in which no row changes
 * cluster, or after max_iter.  Outputs: labels[R], C[K][D], counts[K],
 * *n_iter (iterations run). */
int tao_kmeans(const int64_t *X, int64_t R, int32_t D, int32_t K, const double *C0,
               int32_t max_iter, int32_t *labels, double *C, int64_t *counts, int32_t *n_iter) {
  if (R < 0 || D < 1 || K < 1 || max_iter < 1 || !C0 || !C || !n_iter || (R > 0 && (!X || !labels)))
    return TAO_ERR_INVALID_ARG;
  memcpy(C, C0, sizeof(double) * (size_t)K * (size_t)D);
  int64_t *sum = (int64_t *)malloc(sizeof(int64_t) * (size_t)K * (size_t)D);
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
  if (!sum || !cnt) {
    free(sum);
    free(cnt);
    return TAO_ERR_INVALID_ARG;
  }
  for (int64_t r = 0; r < R; r++) labels[r] = -1;
  int32_t it = 0;
  for (;;) {
    it++;
    int64_t changed = 0;
    for (int64_t r = 0; r < R; r++) {
      const int64_t *x = X + r * D;
      int32_t best = 0;
      double bestd = 0.0;
      for (int32_t k = 0; k < K; k++) {
        double dist = 0.0;
        for (int32_t d = 0; d < D; d++) {
          const double t = (double)x[d] - C[(size_t)k * D + d];
          const double sq = t * t;
          dist = dist + sq;
        }
        if (k == 0 || dist < bestd) {
          best = k;
          bestd = dist;
        }
      }
      if (labels[r] != best) changed++;
      labels[r] = best;
    }
    memset(sum, 0, sizeof(int64_t) * (size_t)K * (size_t)D);
    memset(cnt, 0, sizeof(int64_t) * (size_t)K);
    for (int64_t r = 0; r < R; r++) {
      cnt[labels[r]]++;
      for (int32_t d = 0; d < D; d++)
        sum[(size_t)labels[r] * D + d] = (int64_t)((uint64_t)sum[(size_t)labels[r] * D + d] + (uint64_t)X[r * D + d]);
    }
    for (int32_t k = 0; k < K; k++)
      if (cnt[k] > 0)
        for (int32_t d = 0; d < D; d++)
          C[(size_t)k * D + d] = (double)sum[(size_t)k * D + d] / (double)cnt[k];
    if (changed == 0 || it >= max_iter) break;
  }
  if (counts)
    for (int32_t k = 0; k < K; k++) counts[k] = cnt[k];
  *n_iter = it;
  free(sum);
  free(cnt);
  return TAO_OK;
}

typedef struct {
  int64_t x;
  int64_t i;
} tao_xi;

static int cmp_xi(const void *a, const void *b) {
  const tao_xi *p = (const tao_xi *)a, *q = (const tao_xi *)b;
  if (p->x != q->x) return p->x < q->x ? -1 : 1;
  return p->i < q->i ? -1 : (p->i > q->i);
}

/* DBSCAN on one integer feature per row.  The neighbours of row i are the rows
 * j with |x_j - x_i| <= eps (i itself included); i is a core row when it has
 * at least min_pts neighbours.  Clusters are the connected components of the
 * core rows under the neighbour relation, numbered 0, 1, ... by increasing
 * value.  A non-core row with a core neighbour (a border row) joins the cluster
 * of its nearest core neighbour, the smaller cluster number on a tie; any
 * other row is noise (-1).  Works on the rows sorted by (value, index). */
int tao_dbscan1d(const int64_t *x, int64_t R, int64_t eps, int64_t min_pts, int32_t *labels,
                 int32_t *n_clusters, uint8_t *core) {
  if (R < 0 || eps < 0 || min_pts < 1 || !n_clusters || (R > 0 && (!x || !labels)))
    return TAO_ERR_INVALID_ARG;
  *n_clusters = 0;
  if (R == 0) return TAO_OK;
  tao_xi *s = (tao_xi *)malloc(sizeof(tao_xi) * (size_t)R);
  uint8_t *is_core = (uint8_t *)malloc((size_t)R);
  int32_t *cl = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
  if (!s || !is_core || !cl) {
    free(s);
    free(is_core);
    free(cl);
    return TAO_ERR_INVALID_ARG;
  }
  for (int64_t i = 0; i < R; i++) {
    s[i].x = x[i];
    s[i].i = i;
  }
  qsort(s, (size_t)R, sizeof(tao_xi), cmp_xi);
  /* neighbour counts by two pointers over the sorted values */
  int64_t lo = 0, hi = 0;
  for (int64_t j = 0; j < R; j++) {
    while (s[lo].x < s[j].x - eps) lo++;
    while (hi + 1 < R && s[hi + 1].x <= s[j].x + eps) hi++;
    if (hi < j) hi = j;
    is_core[j] = (hi - lo + 1) >= min_pts;
  }
  /* core rows: a new cluster starts where the previous core row is more than
   * eps below */
  int32_t c = -1;
  int64_t prev = -1;
  for (int64_t j = 0; j < R; j++) {
    cl[j] = -1;
    if (!is_core[j]) continue;
    if (prev < 0 || s[j].x - s[prev].x > eps) c++;
    cl[j] = c;
    prev = j;
  }
  *n_clusters = c + 1;
  /* border rows: nearest core on either side in sorted order (next_core[j] =
   * the first core row after j, found by one backward pass) */
  int64_t *next_core = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
  if (!next_core) {
    free(s);
    free(is_core);
    free(cl);
    return TAO_ERR_INVALID_ARG;
  }
  int64_t nc = -1;
  for (int64_t j = R - 1; j >= 0; j--) {
    next_core[j] = nc;
    if (is_core[j]) nc = j;
  }
  int64_t left = -1;
  for (int64_t j = 0; j < R; j++) {
    if (is_core[j]) {
      left = j;
      continue;
    }
    const int64_t right = next_core[j];
    const int64_t dl = left >= 0 ? s[j].x - s[left].x : INT64_MAX;
    const int64_t dr = right >= 0 ? s[right].x - s[j].x : INT64_MAX;
    if (dl <= eps && dl <= dr) cl[j] = cl[left];
    else if (dr <= eps) cl[j] = cl[right];
  }
  for (int64_t j = 0; j < R; j++) {
    labels[s[j].i] = cl[j];
    if (core) core[s[j].i] = is_core[j];
  }
  free(next_core);
  free(s);
  free(is_core);
  free(cl);
  return TAO_OK;
}

/* Compute nodes shared by clusters: pair[a][b] (K x K, symmetric, zero
 * diagonal) = number of compute nodes holding ranks of both cluster a and
 * cluster b; node_clusters[n] = number of distinct clusters among node n's
 * ranks.  Ranks labelled -1 are ignored. */
int tao_node_intersections(const int32_t *labels, const int32_t *rank_node, int64_t R, int32_t n_nodes,
                           int32_t K, int64_t *pair, int32_t *node_clusters) {
  if (R < 0 || n_nodes < 1 || K < 1 || !pair || (R > 0 && (!labels || !rank_node)))
    return TAO_ERR_INVALID_ARG;
  uint8_t *has = (uint8_t *)calloc((size_t)n_nodes * (size_t)K, 1);
  if (!has) return TAO_ERR_INVALID_ARG;
  for (int64_t r = 0; r < R; r++) {
    if (rank_node[r] < 0 || rank_node[r] >= n_nodes || labels[r] >= K) {
      free(has);
      return TAO_ERR_INVALID_ARG;
    }
    if (labels[r] >= 0) has[(size_t)rank_node[r] * K + labels[r]] = 1;
  }
  memset(pair, 0, sizeof(int64_t) * (size_t)K * (size_t)K);
  for (int32_t n = 0; n < n_nodes; n++) {
    int32_t c = 0;
    for (int32_t a = 0; a < K; a++) {
      if (!has[(size_t)n * K + a]) continue;
      c++;
      for (int32_t b = 0; b < K; b++)
        if (b != a && has[(size_t)n * K + b]) pair[(size_t)a * K + b]++;
    }
    if (node_clusters) node_clusters[n] = c;
  }
  free(has);
  return TAO_OK;
}

/* ---- Time-window profile (Sec. II: a calling context tree for a trace
 * interval of any subset of ranks). ---- */

/* For the ranks rank_ids[0 .. n_sel) (all R ranks, in order, when rank_ids is
 * NULL; a rank listed twice counts twice), the interval of every event,
 * [t_k, t_{k+1}) (a rank's last event lasts 0), clipped to the window [t0, t1),
 * is summed per context node: excl[v]; incl[v] = the sum of excl over the
 * subtree of v (ancestor walks). */
int tao_window_profile(int64_t R, const int64_t *off, const int64_t *ts, const int32_t *ctx,
                       int32_t N, const int32_t *parent, const int32_t *rank_ids, int64_t n_sel,
                       int64_t t0, int64_t t1, int64_t *excl, int64_t *incl) {
  if (N <= 0 || !parent || !excl || t1 < t0 || n_sel < 0) return TAO_ERR_INVALID_ARG;
  int st = tao_check_tree(N, parent);
  if (st) return st;
  st = check_traces(R, off, ts, ctx, N);
  if (st) return st;
  for (int32_t v = 0; v < N; v++) excl[v] = 0;
  const int64_t n = rank_ids ? n_sel : R;
  for (int64_t i = 0; i < n; i++) {
    const int64_t r = rank_ids ? rank_ids[i] : i;
    if (r < 0 || r >= R) return TAO_ERR_INVALID_ARG;
    const int64_t b = off[r], e = off[r + 1];
    for (int64_t k = b; k < e; k++) {
      const int64_t s = ts[k];
      const int64_t f = s + duration(ts, k, e);
      const int64_t lo = s > t0 ? s : t0;
      const int64_t hi = f < t1 ? f : t1;
      if (hi > lo) excl[ctx[k]] += hi - lo;
    }
  }
  if (incl) {
    for (int32_t v = 0; v < N; v++) incl[v] = 0;
    for (int32_t v = 0; v < N; v++)
      if (excl[v] != 0)
        for (int32_t w = v; w != -1; w = parent[w]) incl[w] += excl[v];
  }
  return TAO_OK;
}

/* ---- Sparse per-rank profiles (Sec. I: stored densely, GPU profiles can be
 * over 1000x larger than sparsely; Sec. VI-B: 97,833 calling contexts). ---- */

/* For each rank r, the nodes with a non-zero exclusive time (the sum of the
 * durations of r's events in that context), in ascending node id, stored at
 * node_ids[off[r] + j], excl[off[r] + j] for j < counts[r] (counts[r] <= the
 * rank's event count, so each rank's entries fit in its own event range). */
int tao_sparse_profiles(int64_t R, const int64_t *off, const int64_t *ts, const int32_t *ctx,
                        int32_t N, int64_t *counts, int32_t *node_ids, int64_t *excl) {
  if (N <= 0 || !counts) return TAO_ERR_INVALID_ARG;
  int st = check_traces(R, off, ts, ctx, N);
  if (st) return st;
  int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  if (!row) return TAO_ERR_INVALID_ARG;
  for (int64_t r = 0; r < R; r++) {
    const int64_t b = off[r], e = off[r + 1];
    for (int32_t v = 0; v < N; v++) row[v] = 0;
    for (int64_t k = b; k < e; k++) row[ctx[k]] += duration(ts, k, e);
    int64_t j = 0;
    for (int32_t v = 0; v < N; v++)
      if (row[v] != 0) {
        node_ids[b + j] = v;
        excl[b + j] = row[v];
        j++;
      }
    counts[r] = j;
  }
  free(row);
  return TAO_OK;
}

/* ---- Node x rank x iteration model (Sec. V: per-iteration profiles indexed
 * by calling-context node, trace and iteration; the Thicket model keeps
 * inclusive and exclusive metrics per node). ---- */

/* For rank r and iteration i < iters_found[r] (iterations as in tao_segment:
 * entry into the marker's subtree opens one; events before the first boundary
 * belong to none):
 *   excl(r,i,v) = sum of d_k over rank r's events k of iteration i with
 *                 context v,
 *   incl(r,i,v) = sum of excl(r,i,u) over the subtree of v (walk from each u
 *                 up to its root).
 * Row (r,i) of the sparse model is stored at index q = r*I + i: the nodes with
 * a non-zero excl, in the tree's preorder (every node before its descendants;
 * the children of a node, and the roots of a forest, in ascending id), at
 * node_x[row_off_x[q] + j] / val_x[...] for j < nnz_x[q]; likewise the nodes
 * with a non-zero incl, in the same order, in node_i / val_i.  Rows i >= iters_found[r] are empty.  nnz_x[R*I] and
 * nnz_i[R*I] are always written; the rows are written when row_off_x (and
 * node_x, val_x) and row_off_i (and node_i, val_i) are given.  More than I
 * boundaries in a rank -> TAO_ERR_ITER_OVERFLOW (nothing of that rank past
 * iteration I-1 is stored). */
int tao_node_model(int64_t R, const int64_t *off, const int64_t *ts, const int32_t *ctx,
                   int32_t N, const int32_t *parent, int32_t marker, int32_t I,
                   int64_t *nnz_x, int64_t *nnz_i, const int64_t *row_off_x, int32_t *node_x,
                   int64_t *val_x, const int64_t *row_off_i, int32_t *node_i, int64_t *val_i) {
  int st = tao_check_tree(N, parent);
  if (st) return st;
  if (marker < 0 || marker >= N || I < 1 || !nnz_x || !nnz_i) return TAO_ERR_INVALID_ARG;
  if (row_off_x && (!node_x || !val_x)) return TAO_ERR_INVALID_ARG;
  if (row_off_i && (!node_i || !val_i)) return TAO_ERR_INVALID_ARG;
  st = check_traces(R, off, ts, ctx, N);
  if (st) return st;
  /* the preorder: children grouped by parent in ascending id (counting sort),
   * then a depth-first walk from each root in ascending id */
  int32_t *first = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
  int32_t *kids = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int32_t *stk = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  if (!first || !kids || !fill || !order || !stk) {
    free(first); free(kids); free(fill); free(order); free(stk);
    return TAO_ERR_INVALID_ARG;
  }
  for (int32_t v = 0; v < N; v++)
    if (parent[v] >= 0) first[parent[v] + 1]++;
  for (int32_t v = 0; v < N; v++) first[v + 1] += first[v];
  for (int32_t v = 0; v < N; v++) fill[v] = first[v];
  for (int32_t v = 0; v < N; v++)
    if (parent[v] >= 0) kids[fill[parent[v]]++] = v;
  int32_t n_ord = 0;
  for (int32_t root = 0; root < N; root++) {
    if (parent[root] != -1) continue;
    int32_t top = 0;
    stk[top++] = root;
    while (top > 0) {
      const int32_t v = stk[--top];
      order[n_ord++] = v;
      /* push the children in descending id so the smallest is visited next */
      for (int32_t c = first[v + 1] - 1; c >= first[v]; c--) stk[top++] = kids[c];
    }
  }
  free(first); free(kids); free(fill); free(stk);
  int overflow = 0;
#pragma omp parallel reduction(| : overflow)
  {
    int64_t *ex = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *in = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < R; r++) {
      for (int32_t i = 0; i < I; i++) {
        nnz_x[r * I + i] = 0;
        nnz_i[r * I + i] = 0;
      }
      const int64_t b = off[r], e = off[r + 1];
      int32_t it = -1;
      int prev_in = 0;
      int64_t k = b;
      /* prologue: events before the first boundary */
      while (k < e) {
        const int in_m = is_anc_or_self(parent, marker, ctx[k]);
        if (in_m && (k == b || !prev_in)) break;
        prev_in = in_m;
        k++;
      }
      while (k < e) {
        /* k opens iteration it + 1; find the end of that iteration */
        it++;
        int64_t k_end = k + 1;
        prev_in = 1;
        while (k_end < e) {
          const int in_m = is_anc_or_self(parent, marker, ctx[k_end]);
          if (in_m && !prev_in) break;
          prev_in = in_m;
          k_end++;
        }
        if (it >= I) {
          overflow = 1;
          break;
        }
        for (int32_t v = 0; v < N; v++) ex[v] = in[v] = 0;
        for (int64_t j = k; j < k_end; j++) ex[ctx[j]] += duration(ts, j, e);
        for (int32_t u = 0; u < N; u++)
          if (ex[u] != 0)
            for (int32_t a = u; a != -1; a = parent[a]) in[a] += ex[u];
        const int64_t q = r * I + it;
        int64_t nx = 0, ni = 0;
        for (int32_t j = 0; j < N; j++) {
          const int32_t v = order[j];
          if (ex[v] != 0) {
            if (row_off_x) {
              node_x[row_off_x[q] + nx] = v;
              val_x[row_off_x[q] + nx] = ex[v];
            }
            nx++;
          }
          if (in[v] != 0) {
            if (row_off_i) {
              node_i[row_off_i[q] + ni] = v;
              val_i[row_off_i[q] + ni] = in[v];
            }
            ni++;
          }
        }
        nnz_x[q] = nx;
        nnz_i[q] = ni;
        k = k_end;
      }
    }
    free(ex);
    free(in);
  }
  free(order);
  return overflow ? TAO_ERR_ITER_OVERFLOW : TAO_OK;
}
