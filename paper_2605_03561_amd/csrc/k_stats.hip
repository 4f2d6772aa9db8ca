// k_stats.hip -- imbalance statistics over the rank x iteration x region tensor
// and topology aggregation.
//
// Column pass: every column (i,g) of the tensor is reduced over ranks with
// exact integer sums (int64 sum, unsigned 128-bit sum of squares, min, max).
// Threads own columns, so each row read is contiguous; ranks are split into
// chunks across workgroups and the chunk partials are combined in chunk
// order.  The FP64 values are then one or two correctly rounded operations on
// exact integers (Sec. VI-A: mean / min / max / std per iteration across
// ranks, ddof as in pandas).  Per-region summaries (Tables IV and V) use
// fixed-tree reductions, so repeated runs give identical bits.
#include "ta_device.h"
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int CT = 256;  // threads per column block

struct ColWs {
  int64_t *p_n, *p_s1, *p_mn, *p_mx;  // [RC][IG]
  uint64_t *p_lo, *p_hi;              // [RC][IG]
  int64_t *n, *s1, *mx;               // [IG]
  double *mean, *std, *mmm;           // [IG]
  int64_t *S;                         // [R*G]   (when computed here)
  uint64_t *Q;                        // [R*G*2]
  int64_t *ssum;                      // [G]
  double *tot;                        // [G]
  int32_t *has;                       // [G]
};

__global__ __launch_bounds__(CT) void colstats_partial(const int64_t *__restrict__ T, int64_t R,
                                                       int IG, int G, const int32_t *it,
                                                       int64_t rpc, ColWs w) {
  const int c = blockIdx.x * CT + threadIdx.x;
  const int rc = blockIdx.y;
  if (c >= IG) return;
  const int ic = c / G;
  const int64_t r0 = (int64_t)rc * rpc;
  const int64_t r1 = (r0 + rpc < R) ? r0 + rpc : R;
  int64_t n = 0, s1 = 0, mn = INT64_MAX, mx = INT64_MIN;
  u128 s2 = 0;
  int64_t r = r0;
  for (; r + 4 <= r1; r += 4) {
    int64_t x[4];
    bool v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      x[u] = T[(r + u) * IG + c];
      v[u] = (it == nullptr) || ic < it[r + u];
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (v[u]) {
        n++;
        s1 += x[u];
        s2 += (u128)((i128)x[u] * x[u]);
        mn = x[u] < mn ? x[u] : mn;
        mx = x[u] > mx ? x[u] : mx;
      }
  }
  for (; r < r1; r++) {
    if (it != nullptr && ic >= it[r]) continue;
    int64_t x = T[r * IG + c];
    n++;
    s1 += x;
    s2 += (u128)((i128)x * x);
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
  }
  const int64_t p = (int64_t)rc * IG + c;
  w.p_n[p] = n;
  w.p_s1[p] = s1;
  w.p_lo[p] = (uint64_t)s2;
  w.p_hi[p] = (uint64_t)(s2 >> 64);
  w.p_mn[p] = mn;
  w.p_mx[p] = mx;
}

__global__ __launch_bounds__(CT) void colstats_final(int IG, int RC, int ddof, ColWs w,
                                                     ta_imbalance_out o) {
  const int c = blockIdx.x * CT + threadIdx.x;
  if (c >= IG) return;
  int64_t n = 0, s1 = 0, mn = INT64_MAX, mx = INT64_MIN;
  u128 s2 = 0;
  for (int rc = 0; rc < RC; rc++) {
    const int64_t p = (int64_t)rc * IG + c;
    n += w.p_n[p];
    s1 += w.p_s1[p];
    s2 += ((u128)w.p_hi[p] << 64) | w.p_lo[p];
    mn = w.p_mn[p] < mn ? w.p_mn[p] : mn;
    mx = w.p_mx[p] > mx ? w.p_mx[p] : mx;
  }
  const double nan = nan_f64();
  double mean = nan, sd = nan, mmm = nan;
  if (n > 0) {
    const double dn = (double)n;
    mean = i64_to_f64(s1) / dn;
    mmm = i128_to_f64((i128)n * mx - s1) / dn;
    if (n > ddof) {
      const i128 num = (i128)((u128)n * s2) - (i128)s1 * s1;
      const double var = i128_to_f64(num) / (dn * (double)(n - ddof));
      sd = sqrt(var);
    }
  } else {
    mn = 0;
    mx = 0;
  }
  w.n[c] = n;
  w.s1[c] = s1;
  w.mx[c] = mx;
  w.mean[c] = mean;
  w.std[c] = sd;
  w.mmm[c] = mmm;
  if (o.mean) o.mean[c] = mean;
  if (o.std) o.std[c] = sd;
  if (o.max_minus_mean) o.max_minus_mean[c] = mmm;
  if (o.min) o.min[c] = mn;
  if (o.max) o.max[c] = mx;
}

// Per-(rank, region) totals over the rank's valid iterations, when the
// segmentation pass did not provide them.
__global__ __launch_bounds__(CT) void rank_stats(const int64_t *__restrict__ T, int64_t R, int I,
                                                 int G, const int32_t *it, int64_t *S,
                                                 uint64_t *Q) {
  const int64_t p = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (p >= R * G) return;
  const int64_t r = p / G;
  const int g = (int)(p % G);
  int ni = it ? it[r] : I;
  if (ni > I) ni = I;
  int64_t s = 0;
  u128 q = 0;
  const int64_t *row = T + r * (int64_t)I * G + g;
  for (int i = 0; i < ni; i++) {
    int64_t x = row[(int64_t)i * G];
    s += x;
    q += (u128)((i128)x * x);
  }
  S[p] = s;
  Q[2 * p] = (uint64_t)q;
  Q[2 * p + 1] = (uint64_t)(q >> 64);
}

constexpr int RT = 256;

__global__ __launch_bounds__(RT) void region_stats(int64_t R, int I, int G, const int32_t *it,
                                                   const int64_t *S, const uint64_t *Q, int ddof,
                                                   ColWs w, ta_imbalance_out o) {
  __shared__ double fb[RT];
  __shared__ int64_t ib[RT];
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  // Over iterations (ascending within each thread, then a fixed tree).
  double a_mean = 0.0, a_mmm = 0.0, a_cv = 0.0;
  int64_t a_max = 0, n_it = 0, n_cv = 0;
  for (int i = t; i < I; i += RT) {
    const int c = i * G + g;
    const int64_t n = w.n[c];
    if (n > 0) {
      a_mean += w.mean[c];
      a_mmm += w.mmm[c];
      a_max += w.mx[c];
      n_it++;
      if (n > ddof && w.mean[c] > 0.0) {
        a_cv += w.std[c] / w.mean[c];
        n_cv++;
      }
    }
  }
  a_mean = block_sum_f64<RT>(a_mean, fb);
  a_mmm = block_sum_f64<RT>(a_mmm, fb);
  a_cv = block_sum_f64<RT>(a_cv, fb);
  a_max = block_sum_i64<RT>(a_max, ib);
  n_it = block_sum_i64<RT>(n_it, ib);
  n_cv = block_sum_i64<RT>(n_cv, ib);
  // Over ranks.
  int64_t ssum = 0, smax = INT64_MIN, n_w = 0;
  double a_w = 0.0;
  for (int64_t r = t; r < R; r += RT) {
    const int64_t s = S[r * G + g];
    ssum += s;
    smax = s > smax ? s : smax;
    int64_t nr = it ? it[r] : I;
    if (nr > I) nr = I;
    if (nr > ddof && s > 0) {
      const u128 q = ((u128)Q[2 * (r * G + g) + 1] << 64) | Q[2 * (r * G + g)];
      const double mr = i64_to_f64(s) / (double)nr;
      const i128 num = (i128)((u128)nr * q) - (i128)s * s;
      const double vr = i128_to_f64(num) / ((double)nr * (double)(nr - ddof));
      a_w += sqrt(vr) / mr;
      n_w++;
    }
  }
  ssum = block_sum_i64<RT>(ssum, ib);
  smax = block_max_i64<RT>(smax, ib);
  n_w = block_sum_i64<RT>(n_w, ib);
  a_w = block_sum_f64<RT>(a_w, fb);
  if (t == 0) {
    const double nan = nan_f64();
    const double dn = (double)n_it;
    const double spi = n_it ? a_mmm / dn : nan;
    const double tot = n_it ? spi * dn : nan;
    if (o.avg_mean) o.avg_mean[g] = n_it ? a_mean / dn : nan;
    if (o.avg_max) o.avg_max[g] = n_it ? i64_to_f64(a_max) / dn : nan;
    if (o.savings_per_iter) o.savings_per_iter[g] = spi;
    if (o.total_savings) o.total_savings[g] = tot;
    if (o.cv_across) o.cv_across[g] = n_cv ? a_cv / (double)n_cv : nan;
    if (o.cv_within) o.cv_within[g] = n_w ? a_w / (double)n_w : nan;
    if (o.balance_ratio)
      o.balance_ratio[g] = (R > 0 && smax != 0) ? (i64_to_f64(ssum) / (double)R) / i64_to_f64(smax)
                                                : nan;
    w.ssum[g] = ssum;
    w.tot[g] = tot;
    w.has[g] = n_it > 0;
  }
}

__global__ __launch_bounds__(RT) void imbalance_final(int64_t R, int G, const int64_t *span,
                                                      double t_app, ColWs w,
                                                      ta_imbalance_out o) {
  __shared__ int64_t ib[RT];
  const int t = threadIdx.x;
  int64_t smax = INT64_MIN;
  if (span)
    for (int64_t r = t; r < R; r += RT) smax = span[r] > smax ? span[r] : smax;
  smax = block_max_i64<RT>(smax, ib);
  if (t == 0) {
    const double nan = nan_f64();
    int64_t grand = 0;
    double tot = 0.0;
    for (int g = 0; g < G; g++) {
      grand += w.ssum[g];
      if (w.has[g]) tot += w.tot[g];
    }
    if (o.share)
      for (int g = 0; g < G; g++)
        o.share[g] = grand ? i64_to_f64(w.ssum[g]) / i64_to_f64(grand) : nan;
    double tapp = t_app;
    if (!(tapp > 0.0)) tapp = (span && R > 0) ? i64_to_f64(smax) : nan;
    if (o.potential_speedup) o.potential_speedup[0] = tot / tapp;
  }
}

// ---- topology -----------------------------------------------------------

__global__ __launch_bounds__(RT) void topo_kernel(TopoArgs a) {
  __shared__ double fb[RT];
  __shared__ int64_t ib[RT];
  __shared__ int64_t xacc[(RT / 64) * XL];
  __shared__ uint32_t xbad;
  const int k = blockIdx.x;
  const bool chassis = k >= a.n_racks;
  const int key = chassis ? k - a.n_racks : k;
  const int32_t *map = chassis ? a.node_chassis : a.node_rack;
  const int lim = chassis ? a.n_chassis : a.n_racks;
  int64_t cnt = 0, nfl = 0;
  double best = -__builtin_inf();
  uint32_t bad = 0;
  xsum_clear<RT>(xacc, &xbad);
  int64_t *xw = xacc + (threadIdx.x >> 6) * XL;
  // uniform trip count: every lane of a wave takes part in the exact sum
  for (int64_t r0 = 0; r0 < a.R; r0 += RT) {
    const int64_t r = r0 + threadIdx.x;
    bool mine = false;
    double sc = 0.0;
    if (r < a.R) {
      const int32_t nd = a.rank_node[r];
      const int32_t kk = (nd < 0 || nd >= a.n_nodes) ? -1 : map[nd];
      if (kk < 0 || kk >= lim) {
        bad = 1;
      } else if (kk == key) {
        mine = true;
        sc = a.score[r];
        cnt++;
        nfl += a.flag[r] ? 1 : 0;
        best = sc > best ? sc : best;
      }
    }
    xsum_add_wave(xw, sc, mine, &xbad);
  }
  const double s = xsum_block_result<RT>(xacc, &xbad, fb);  // exact sum of the scores
  cnt = block_sum_i64<RT>(cnt, ib);
  nfl = block_sum_i64<RT>(nfl, ib);
  best = block_max_f64<RT>(best, fb);
  if (bad) atomicOr(a.err, ERRBIT_OFFSETS);
  if (threadIdx.x == 0) {
    const double nan = nan_f64();
    int64_t *fl = chassis ? a.fl_ch : a.fl_rack;
    double *mx = chassis ? a.mx_ch : a.mx_rack;
    double *mn = chassis ? a.mn_ch : a.mn_rack;
    if (fl) fl[key] = nfl;
    if (mx) mx[key] = cnt ? best : nan;
    if (mn) mn[key] = cnt ? s / (double)cnt : nan;
  }
}

struct WsCursor {
  char *p;
  size_t used = 0;
  template <class T>
  T *take(size_t n) {
    size_t bytes = (n * sizeof(T) + 255) & ~(size_t)255;
    T *r = reinterpret_cast<T *>(p + used);
    used += bytes;
    return r;
  }
};

int rank_chunks(int64_t R, int IG) {
  const int cb = (IG + CT - 1) / CT;
  int64_t rc = (2048 + cb - 1) / cb;
  if (rc > R) rc = R;
  if (rc < 1) rc = 1;
  if (rc > 256) rc = 256;
  return (int)rc;
}

ColWs carve(void *ws, int64_t R, int I, int G, bool rankst, size_t *used, int rc_ext = 0) {
  const int IG = I * G;
  const int RC = rc_ext > 0 ? rc_ext : rank_chunks(R, IG);
  WsCursor c{(char *)ws};
  ColWs w;
  w.p_n = c.take<int64_t>((size_t)RC * IG);
  w.p_s1 = c.take<int64_t>((size_t)RC * IG);
  w.p_mn = c.take<int64_t>((size_t)RC * IG);
  w.p_mx = c.take<int64_t>((size_t)RC * IG);
  w.p_lo = c.take<uint64_t>((size_t)RC * IG);
  w.p_hi = c.take<uint64_t>((size_t)RC * IG);
  w.n = c.take<int64_t>(IG);
  w.s1 = c.take<int64_t>(IG);
  w.mx = c.take<int64_t>(IG);
  w.mean = c.take<double>(IG);
  w.std = c.take<double>(IG);
  w.mmm = c.take<double>(IG);
  w.S = rankst ? c.take<int64_t>((size_t)R * G) : nullptr;
  w.Q = rankst ? c.take<uint64_t>((size_t)R * G * 2) : nullptr;
  w.ssum = c.take<int64_t>(G);
  w.tot = c.take<double>(G);
  w.has = c.take<int32_t>(G);
  *used = c.used;
  return w;
}

}  // namespace

size_t imbalance_ws_bytes(int64_t R, int32_t I, int32_t G, bool need_rank_stats, int rc_ext) {
  size_t used = 0;
  carve((void *)0x100, R, I, G, need_rank_stats, &used, rc_ext);
  return used + 256;
}

ColPartials imbalance_partials(void *ws, int64_t R, int32_t I, int32_t G, bool need_rank_stats,
                               int rc_ext) {
  size_t used = 0;
  ColWs w = carve(ws, R, I, G, need_rank_stats, &used, rc_ext);
  ColPartials p{};
  p.n = w.p_n;
  p.s1 = w.p_s1;
  p.mn = w.p_mn;
  p.mx = w.p_mx;
  p.lo = w.p_lo;
  p.hi = w.p_hi;
  p.rc = rc_ext;
  return p;
}

hipError_t launch_imbalance(const ImbArgs &a, void *ws, size_t ws_bytes, hipStream_t s, int rc_ext) {
  const bool rankst = a.rank_sum == nullptr || a.rank_sumsq == nullptr;
  size_t used = 0;
  ColWs w = carve(ws, a.R, a.I, a.G, rankst, &used, rc_ext);
  if (used > ws_bytes) return hipErrorInvalidValue;
  const int IG = a.I * a.G;
  const int RC = rc_ext > 0 ? rc_ext : rank_chunks(a.R, IG);
  const int64_t rpc = (a.R + RC - 1) / RC;
  if (rc_ext > 0) {
    // partials already written (by the FULL scan's transpose)
  } else if (IG > 0 && a.R > 0) {
    hipLaunchKernelGGL(colstats_partial, dim3((IG + CT - 1) / CT, RC), dim3(CT), 0, s, a.T, a.R,
                       IG, a.G, a.it, rpc, w);
  } else if (IG > 0) {
    // No ranks: one empty chunk.
    hipLaunchKernelGGL(colstats_partial, dim3((IG + CT - 1) / CT, 1), dim3(CT), 0, s, a.T,
                       (int64_t)0, IG, a.G, a.it, (int64_t)1, w);
  }
  if (IG > 0)
    hipLaunchKernelGGL(colstats_final, dim3((IG + CT - 1) / CT), dim3(CT), 0, s, IG,
                       a.R > 0 ? RC : 1, a.ddof, w, a.o);
  const int64_t *S = a.rank_sum;
  const uint64_t *Q = a.rank_sumsq;
  if (rankst) {
    if (a.R > 0)
      hipLaunchKernelGGL(rank_stats, dim3((unsigned)((a.R * a.G + CT - 1) / CT)), dim3(CT), 0, s,
                         a.T, a.R, a.I, a.G, a.it, w.S, w.Q);
    S = w.S;
    Q = w.Q;
  }
  hipLaunchKernelGGL(region_stats, dim3(a.G), dim3(RT), 0, s, a.R, a.I, a.G, a.it, S, Q, a.ddof, w,
                     a.o);
  hipLaunchKernelGGL(imbalance_final, dim3(1), dim3(RT), 0, s, a.R, a.G, a.span, a.t_app, w, a.o);
  return hipGetLastError();
}

hipError_t launch_topology(const TopoArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(topo_kernel, dim3(a.n_racks + a.n_chassis), dim3(RT), 0, s, a);
  return hipGetLastError();
}

}  // namespace ta
