// k_outliers.hip -- exact outlier scan over the rank x iteration x region tensor.
//
// Robust (modified) z-score: z = (x - median) / (1.4826 * MAD), with the
// mean-absolute-deviation fallback when MAD is 0.  Medians are found exactly
// by most-significant-digit radix selection (8-bit digits) with LDS
// histograms; no sort, no approximation.  For an even count the upper middle
// value is either a repeat of the lower one, the next non-empty bucket of the
// last digit, or the smallest key above the lower median's prefix group (kept
// during the last pass), so no extra pass is needed.
//
// FULL scan:   stage 1  per column (i,g): median and MAD over ranks
//              scoring  m(r,g) = mean over the rank's iterations of z(r,i,g),
//                       summed in ascending i (bit-reproducible)
//              stage 2  per region g: median / MAD over ranks of m(r,g)
// TOTALS scan: stage 2 only, on the rank totals S(r,g).
#include "ta_device.h"
#include "ta_internal.h"

namespace ta {
namespace {

constexpr uint64_t SIGN = 0x8000000000000000ull;

// ----------------------------------------------------------------------------
// Stage 1: 64 columns per workgroup, all selection passes in one launch.
// ----------------------------------------------------------------------------
constexpr int SC = 64;
constexpr int ST = 256;
constexpr int SWV = ST / 64;
constexpr int UNR = 8;

struct ColSel {
  int64_t *med2, *mad4, *sumdev, *n;  // [IG]
};

__device__ inline int nbits64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

__global__ __launch_bounds__(ST) void sel_columns(const int64_t *__restrict__ T, int64_t R, int IG,
                                                  int G, const int32_t *it, ColSel out) {
  __shared__ uint32_t hist[SC][257];
  __shared__ int64_t red0[SWV][SC], red1[SWV][SC], red2[SWV][SC];
  __shared__ uint64_t s_base[SC], s_pref[SC], s_v1[SC], s_v2[SC];
  __shared__ int64_t s_krem[SC], s_n[SC], s_med2[SC];
  __shared__ int s_np[SC];
  __shared__ int s_maxnp;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int c = blockIdx.x * SC + lane;
  const bool col_ok = c < IG;
  const int ic = col_ok ? c / G : 0;
  const int64_t *colp = T + (col_ok ? c : 0);

  for (int k = tid; k < SC * 257; k += ST) (&hist[0][0])[k] = 0;

  // ---- pass A: count, min, max --------------------------------------------
  {
    int64_t n = 0, mn = INT64_MAX, mx = INT64_MIN;
    for (int64_t r0 = wid; r0 < R; r0 += SWV * UNR) {
      int64_t x[UNR];
      bool v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const int64_t r = r0 + (int64_t)u * SWV;
        v[u] = col_ok && r < R && (it == nullptr || ic < it[r]);
        x[u] = v[u] ? colp[r * IG] : 0;
      }
#pragma unroll
      for (int u = 0; u < UNR; u++)
        if (v[u]) {
          n++;
          mn = x[u] < mn ? x[u] : mn;
          mx = x[u] > mx ? x[u] : mx;
        }
    }
    red0[wid][lane] = n;
    red1[wid][lane] = mn;
    red2[wid][lane] = mx;
    __syncthreads();
    if (wid == 0) {
      int64_t nn = 0, a = INT64_MAX, b = INT64_MIN;
      for (int w = 0; w < SWV; w++) {
        nn += red0[w][lane];
        a = red1[w][lane] < a ? red1[w][lane] : a;
        b = red2[w][lane] > b ? red2[w][lane] : b;
      }
      if (nn == 0) a = b = 0;
      s_n[lane] = nn;
      s_base[lane] = (uint64_t)a;
      const int np = (nbits64((uint64_t)b - (uint64_t)a) + 7) / 8;
      s_np[lane] = nn > 0 ? np : 0;
      s_pref[lane] = 0;
      s_krem[lane] = nn > 0 ? (nn - 1) / 2 : 0;
      s_v1[lane] = s_v2[lane] = 0;
      s_med2[lane] = (int64_t)a + (int64_t)b;  // placeholder until selected
      red2[0][lane] = b;                        // keep max for the MAD range
      int m = np;
      for (int d = 32; d >= 1; d >>= 1) {
        int o = __shfl_xor(m, d, 64);
        m = o > m ? o : m;
      }
      if (lane == 0) s_maxnp = m;
    }
    __syncthreads();
  }
  const int64_t colmax = red2[0][lane];
  __syncthreads();

  // ---- two selections: median of x (phase 0), median of |2x - med2| (1) ----
  for (int phase = 0; phase < 2; phase++) {
    const int maxnp = s_maxnp;
    const uint64_t base = phase == 0 ? s_base[lane] : 0;
    const int64_t med2 = s_med2[lane];
    const int np = s_np[lane];
    int64_t sumdev = 0;
    for (int p = 0; p < maxnp; p++) {
      const bool act = col_ok && p < np;
      const int sh = 8 * (np - 1 - p);
      const uint64_t pref = s_pref[lane];
      const bool last = act && sh == 0;
      uint64_t mgt = ~0ull;
      for (int64_t r0 = wid; r0 < R; r0 += SWV * UNR) {
        int64_t x[UNR];
        bool v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
          const int64_t r = r0 + (int64_t)u * SWV;
          v[u] = act && r < R && (it == nullptr || ic < it[r]);
          x[u] = v[u] ? colp[r * IG] : 0;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++)
          if (v[u]) {
            uint64_t key;
            if (phase == 0) {
              key = (uint64_t)x[u] - base;
            } else {
              const int64_t dv = 2 * x[u] - med2;
              key = (uint64_t)(dv < 0 ? -dv : dv);
              if (p == 0) sumdev += (int64_t)key;
            }
            const uint64_t ks = key >> sh;
            const uint64_t hiK = ks >> 8;
            if (hiK == pref) atomicAdd(&hist[lane][(uint32_t)(ks & 255)], 1u);
            else if (last && hiK > pref) mgt = key < mgt ? key : mgt;
          }
      }
      red0[wid][lane] = (int64_t)mgt;
      if (phase == 1 && p == 0) red1[wid][lane] = sumdev;
      __syncthreads();
      if (wid == 0 && act) {
        if (phase == 1 && p == 0) {
          int64_t sd = 0;
          for (int w = 0; w < SWV; w++) sd += red1[w][lane];
          red1[0][lane] = sd;
        }
        uint64_t mg = ~0ull;
        for (int w = 0; w < SWV; w++) mg = (uint64_t)red0[w][lane] < mg ? (uint64_t)red0[w][lane] : mg;
        int64_t k = s_krem[lane];
        int64_t cum = 0;
        int b = 0;
        for (; b < 256; b++) {
          const int64_t cnt = hist[lane][b];
          if (cum + cnt > k) break;
          cum += cnt;
        }
        const int64_t cntb = hist[lane][b];
        k -= cum;
        const uint64_t np_pref = (pref << 8) | (uint64_t)b;
        if (last) {
          s_v1[lane] = np_pref;
          if (k + 1 < cntb) {
            s_v2[lane] = np_pref;
          } else {
            int b2 = b + 1;
            while (b2 < 256 && hist[lane][b2] == 0) b2++;
            s_v2[lane] = b2 < 256 ? ((pref << 8) | (uint64_t)b2) : mg;
          }
        }
        s_pref[lane] = np_pref;
        s_krem[lane] = k;
        for (int bb = 0; bb < 256; bb++) hist[lane][bb] = 0;
      }
      __syncthreads();
    }
    if (wid == 0) {
      const int64_t nn = s_n[lane];
      // Columns needing no pass have all keys equal to 0 (relative to base).
      // For an odd count the lower middle value is the median itself.
      const uint64_t v1 = s_np[lane] ? s_v1[lane] : 0;
      const uint64_t v2 = s_np[lane] ? ((nn & 1) ? v1 : s_v2[lane]) : 0;
      if (phase == 0) {
        const int64_t m2 = (int64_t)(base + v1) + (int64_t)(base + v2);
        s_med2[lane] = m2;
        // min <= median <= max, so the largest deviation is at an end.
        const uint64_t dlo = (uint64_t)(m2 - 2 * (int64_t)base);
        const uint64_t dhi = (uint64_t)(2 * colmax - m2);
        const uint64_t dmax = dlo > dhi ? dlo : dhi;
        const int np2 = nn > 0 ? (nbits64(dmax) + 7) / 8 : 0;
        s_np[lane] = np2;
        s_pref[lane] = 0;
        s_krem[lane] = nn > 0 ? (nn - 1) / 2 : 0;
        s_v1[lane] = s_v2[lane] = 0;
        red1[0][lane] = 0;  // sumdev when no MAD pass runs (all deviations 0)
        int m = col_ok ? np2 : 0;
        for (int d = 32; d >= 1; d >>= 1) {
          int o = __shfl_xor(m, d, 64);
          m = o > m ? o : m;
        }
        if (lane == 0) s_maxnp = m;
      } else if (col_ok) {
        out.med2[c] = s_med2[lane];
        out.mad4[c] = (int64_t)(v1 + v2);
        out.sumdev[c] = s_np[lane] ? red1[0][lane] : 0;
        out.n[c] = nn;
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// Plain moments per column (TA_SCORE_Z): n, sum, sum of squares -> std.
// ----------------------------------------------------------------------------
struct ColMom {
  int64_t *n, *s1;
  double *sd;
};

__global__ __launch_bounds__(256) void col_moments(const int64_t *__restrict__ T, int64_t R, int IG,
                                                   int G, const int32_t *it, ColMom out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= IG) return;
  const int ic = c / G;
  int64_t n = 0, s1 = 0;
  u128 s2 = 0;
  for (int64_t r = 0; r < R; r++) {
    if (it && ic >= it[r]) continue;
    const int64_t x = T[r * IG + c];
    n++;
    s1 += x;
    s2 += (u128)((i128)x * x);
  }
  double sd = 0.0;
  if (n > 1)
    sd = sqrt(i128_to_f64((i128)((u128)n * s2) - (i128)s1 * s1) / ((double)n * (double)(n - 1)));
  out.n[c] = n;
  out.s1[c] = s1;
  out.sd[c] = sd;
}

// ----------------------------------------------------------------------------
// Scoring: m(r,g) = (1/n_r) sum_{i < n_r} z(r,i,g), written transposed [G][R].
// ----------------------------------------------------------------------------
template <bool MAD>
__global__ __launch_bounds__(256) void score_cells(const int64_t *__restrict__ T, int64_t R, int I,
                                                   int G, const int32_t *it, ColSel cs, ColMom cm,
                                                   double *m_t) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= R * G) return;
  const int64_t r = p / G;
  const int g = (int)(p % G);
  int ni = it ? it[r] : I;
  if (ni > I) ni = I;
  const int64_t *row = T + r * (int64_t)I * G + g;
  double acc = 0.0;
  for (int i = 0; i < ni; i++) {
    const int c = i * G + g;
    const int64_t x = row[(int64_t)i * G];
    double z;
    if (MAD) {
      const int64_t med2 = cs.med2[c], mad4 = cs.mad4[c];
      if (mad4 > 0) {
        z = (double)(4 * x - 2 * med2) / (1.4826 * (double)mad4);
      } else {
        const int64_t sdv = cs.sumdev[c];
        z = sdv > 0 ? ((double)(2 * x - med2) * (double)cs.n[c]) / (1.253314 * (double)sdv) : 0.0;
      }
    } else {
      const double sd = cm.sd[c];
      const int64_t n = cm.n[c];
      z = sd > 0.0 ? i128_to_f64((i128)n * x - cm.s1[c]) / ((double)n * sd) : 0.0;
    }
    acc += z;
  }
  m_t[(int64_t)g * R + r] = ni > 0 ? acc / (double)ni : 0.0;
}

// Rank totals S(r,g), transposed [G][R].
__global__ __launch_bounds__(256) void rank_totals_t(const int64_t *__restrict__ T, int64_t R, int I,
                                                     int G, const int32_t *it, int64_t *S_t) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= R * G) return;
  const int64_t r = p / G;
  const int g = (int)(p % G);
  int ni = it ? it[r] : I;
  if (ni > I) ni = I;
  const int64_t *row = T + r * (int64_t)I * G + g;
  int64_t s = 0;
  for (int i = 0; i < ni; i++) s += row[(int64_t)i * G];
  S_t[(int64_t)g * R + r] = s;
}

// ----------------------------------------------------------------------------
// Stage 2: one workgroup per region, values contiguous over ranks.
// ----------------------------------------------------------------------------
constexpr int RT = 1024;
constexpr int RW = RT / 64;

__device__ inline uint64_t key_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  return (u & SIGN) ? ~u : (u | SIGN);
}
__device__ inline double dec_f64(uint64_t k) {
  const uint64_t u = (k & SIGN) ? (k & ~SIGN) : ~k;
  return __longlong_as_double((long long)u);
}

__device__ inline bool rank_active(const int32_t *it, int I, int64_t r) {
  return it ? it[r] > 0 : I > 0;
}

// Exact k-th smallest (k = (n-1)/2) of keys given by `keyf(r)` over active
// ranks, and the next order statistic.  Returns both through v1/v2.
template <class KeyF>
__device__ void block_select(int64_t R, const int32_t *it, int I, int64_t n, KeyF keyf,
                             uint32_t (*hist)[256], uint32_t *tot, uint64_t *sh_u64,
                             uint64_t &v1, uint64_t &v2) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  uint64_t pref = 0;
  int64_t k = (n - 1) / 2;
  for (int sh = 56; sh >= 0; sh -= 8) {
    const bool last = sh == 0;
    uint64_t mgt = ~0ull;
    for (int64_t r = tid; r < R; r += RT) {
      if (!rank_active(it, I, r)) continue;
      const uint64_t key = keyf(r);
      const uint64_t ks = key >> sh;
      const uint64_t hk = ks >> 8;
      if (hk == pref) atomicAdd(&hist[wid][(uint32_t)(ks & 255)], 1u);
      else if (last && hk > pref) mgt = key < mgt ? key : mgt;
    }
    // reduce the min-above-group over the block
    for (int d = 32; d >= 1; d >>= 1) {
      const uint64_t o = __shfl_xor(mgt, d, 64);
      mgt = o < mgt ? o : mgt;
    }
    if (lane == 0) sh_u64[wid] = mgt;
    __syncthreads();
    if (tid < 256) {
      uint32_t s = 0;
      for (int w = 0; w < RW; w++) {
        s += hist[w][tid];
        hist[w][tid] = 0;
      }
      tot[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
      int64_t cum = 0;
      int b = 0;
      for (; b < 256; b++) {
        if (cum + (int64_t)tot[b] > k) break;
        cum += tot[b];
      }
      k -= cum;
      const uint64_t np = (pref << 8) | (uint64_t)b;
      if (last) {
        uint64_t mg = ~0ull;
        for (int w = 0; w < RW; w++) mg = sh_u64[w] < mg ? sh_u64[w] : mg;
        uint64_t w2;
        if (k + 1 < (int64_t)tot[b]) {
          w2 = np;
        } else {
          int b2 = b + 1;
          while (b2 < 256 && tot[b2] == 0) b2++;
          w2 = b2 < 256 ? ((pref << 8) | (uint64_t)b2) : mg;
        }
        sh_u64[RW] = np;
        sh_u64[RW + 1] = w2;
      }
      sh_u64[RW + 2] = np;
      sh_u64[RW + 3] = (uint64_t)k;
    }
    __syncthreads();
    pref = sh_u64[RW + 2];
    k = (int64_t)sh_u64[RW + 3];
    __syncthreads();
  }
  v1 = sh_u64[RW];
  v2 = (n & 1) ? v1 : sh_u64[RW + 1];  // odd count: the median is the lower middle
  __syncthreads();
}

template <bool F64, bool MAD>
__global__ __launch_bounds__(RT) void sel_regions(const void *vals_t, int64_t R, int G,
                                                  const int32_t *it, int I, double *z_t,
                                                  double *region_score) {
  __shared__ uint32_t hist[RW][256];
  __shared__ uint32_t tot[256];
  __shared__ uint64_t sh_u64[RW + 4];
  __shared__ double fb[RT];
  __shared__ int64_t ib[RT];
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const double *vd = reinterpret_cast<const double *>(vals_t) + (int64_t)g * R;
  const int64_t *vi = reinterpret_cast<const int64_t *>(vals_t) + (int64_t)g * R;
  for (int k = tid; k < RW * 256; k += RT) (&hist[0][0])[k] = 0;

  int64_t n = 0;
  for (int64_t r = tid; r < R; r += RT) n += rank_active(it, I, r) ? 1 : 0;
  n = block_sum_i64<RT>(n, ib);

  // Centre and scale.
  double med = 0.0, scale = 0.0;
  int64_t med2 = 0;
  int mode = 0;  // 1: MAD, 2: mean AD / plain std, 0: all z = 0
  if (n > 0) {
    if (MAD) {
      uint64_t a, b;
      if (F64) {
        block_select(R, it, I, n, [&](int64_t r) { return key_f64(vd[r]); }, hist, tot, sh_u64, a, b);
        med = (n & 1) ? dec_f64(a) : 0.5 * (dec_f64(a) + dec_f64(b));
        block_select(R, it, I, n, [&](int64_t r) { return key_f64(fabs(vd[r] - med)); }, hist, tot,
                     sh_u64, a, b);
        const double mad = (n & 1) ? dec_f64(a) : 0.5 * (dec_f64(a) + dec_f64(b));
        if (mad > 0.0) {
          mode = 1;
          scale = 1.4826 * mad;
        } else {
          double s = 0.0;
          for (int64_t r = tid; r < R; r += RT)
            if (rank_active(it, I, r)) s += fabs(vd[r] - med);
          s = block_sum_f64<RT>(s, fb);
          const double mean_ad = s / (double)n;
          if (mean_ad > 0.0) {
            mode = 2;
            scale = 1.253314 * mean_ad;
          }
        }
      } else {
        block_select(R, it, I, n, [&](int64_t r) { return (uint64_t)vi[r] ^ SIGN; }, hist, tot,
                     sh_u64, a, b);
        med2 = (int64_t)(a ^ SIGN) + (int64_t)(b ^ SIGN);
        block_select(R, it, I, n,
                     [&](int64_t r) {
                       const int64_t d = 2 * vi[r] - med2;
                       return (uint64_t)(d < 0 ? -d : d);
                     },
                     hist, tot, sh_u64, a, b);
        const int64_t mad4 = (int64_t)(a + b);
        if (mad4 > 0) {
          mode = 1;
          scale = 1.4826 * (double)mad4;
        } else {
          int64_t s = 0;
          for (int64_t r = tid; r < R; r += RT)
            if (rank_active(it, I, r)) {
              const int64_t d = 2 * vi[r] - med2;
              s += d < 0 ? -d : d;
            }
          s = block_sum_i64<RT>(s, ib);
          if (s > 0) {
            mode = 2;
            scale = 1.253314 * (double)s;
          }
        }
      }
    } else {
      if (F64) {
        double s = 0.0;
        for (int64_t r = tid; r < R; r += RT)
          if (rank_active(it, I, r)) s += vd[r];
        s = block_sum_f64<RT>(s, fb);
        med = s / (double)n;
        double q = 0.0;
        for (int64_t r = tid; r < R; r += RT)
          if (rank_active(it, I, r)) q += (vd[r] - med) * (vd[r] - med);
        q = block_sum_f64<RT>(q, fb);
        const double sd = n > 1 ? sqrt(q / (double)(n - 1)) : 0.0;
        if (sd > 0.0) {
          mode = 2;
          scale = sd;
        }
      } else {
        int64_t s1 = 0;
        u128 q = 0;
        for (int64_t r = tid; r < R; r += RT)
          if (rank_active(it, I, r)) {
            s1 += vi[r];
            q += (u128)((i128)vi[r] * vi[r]);
          }
        s1 = block_sum_i64<RT>(s1, ib);
        // Exact 128-bit sum of squares: per-thread partial words, summed by
        // one thread in thread order.
        uint64_t *qlo = reinterpret_cast<uint64_t *>(ib);
        uint64_t *qhi = reinterpret_cast<uint64_t *>(fb);
        qlo[tid] = (uint64_t)q;
        qhi[tid] = (uint64_t)(q >> 64);
        __syncthreads();
        if (tid == 0) {
          u128 qs = 0;
          for (int t = 0; t < RT; t++) qs += ((u128)qhi[t] << 64) | qlo[t];
          const i128 num = (i128)((u128)n * qs) - (i128)s1 * s1;
          sh_u64[0] = (uint64_t)__double_as_longlong(
              n > 1 ? sqrt(i128_to_f64(num) / ((double)n * (double)(n - 1))) : 0.0);
        }
        __syncthreads();
        const double sd = __longlong_as_double((long long)sh_u64[0]);
        med2 = s1;  // the centre term of the plain score is the exact sum
        __syncthreads();
        if (sd > 0.0) {
          mode = 2;
          scale = (double)n * sd;
        }
      }
    }
  }

  // Scores.
  for (int64_t r = tid; r < R; r += RT) {
    double z = 0.0;
    if (rank_active(it, I, r) && mode != 0) {
      if (F64) {
        z = (vd[r] - med) / scale;
      } else if (MAD) {
        if (mode == 1) z = (double)(4 * vi[r] - 2 * med2) / scale;
        else z = ((double)(2 * vi[r] - med2) * (double)n) / scale;
      } else {
        z = i128_to_f64((i128)n * vi[r] - med2) / scale;
      }
    }
    z_t[(int64_t)g * R + r] = z;
    if (region_score) region_score[r * G + g] = z;
  }
}

// Per-rank maximum |z| over regions, flags, per-block flag counts.
__global__ __launch_bounds__(256) void rank_final(const double *z_t, int64_t R, int G,
                                                  const int32_t *it, int I, double tau,
                                                  double *score, uint8_t *flag, int64_t *part) {
  __shared__ int64_t ib[256];
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t f = 0;
  if (r < R) {
    double best = 0.0;
    if (rank_active(it, I, r))
      for (int g = 0; g < G; g++) {
        const double v = fabs(z_t[(int64_t)g * R + r]);
        if (v > best) best = v;
      }
    score[r] = best;
    f = best > tau ? 1 : 0;
    flag[r] = (uint8_t)f;
  }
  f = block_sum_i64<256>(f, ib);
  if (threadIdx.x == 0) part[blockIdx.x] = f;
}

__global__ __launch_bounds__(256) void count_final(const int64_t *part, int64_t nb, int64_t *out) {
  __shared__ int64_t ib[256];
  int64_t s = 0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) s += part[b];
  s = block_sum_i64<256>(s, ib);
  if (threadIdx.x == 0 && out) out[0] = s;
}

struct OWs {
  ColSel cs;
  ColMom cm;
  double *m_t;      // [G][R] doubles (FULL) -- also reused as z_t
  int64_t *S_t;     // [G][R] (TOTALS)
  double *z_t;      // [G][R]
  int64_t *part;    // [ceil(R/256)]
};

OWs carve(void *ws, int64_t R, int I, int G, int mode, int kind, size_t *used) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = (char *)ws + off;
    off += (bytes + 255) & ~(size_t)255;
    return (void *)p;
  };
  const size_t IG = (size_t)I * G;
  OWs w{};
  if (mode == TA_SCAN_FULL) {
    if (kind == TA_SCORE_MAD) {
      w.cs.med2 = (int64_t *)take(IG * 8);
      w.cs.mad4 = (int64_t *)take(IG * 8);
      w.cs.sumdev = (int64_t *)take(IG * 8);
      w.cs.n = (int64_t *)take(IG * 8);
    } else {
      w.cm.n = (int64_t *)take(IG * 8);
      w.cm.s1 = (int64_t *)take(IG * 8);
      w.cm.sd = (double *)take(IG * 8);
    }
    w.m_t = (double *)take((size_t)R * G * 8);
  } else {
    w.S_t = (int64_t *)take((size_t)R * G * 8);
  }
  w.z_t = (double *)take((size_t)R * G * 8);
  w.part = (int64_t *)take((size_t)((R + 255) / 256 + 1) * 8);
  *used = off;
  return w;
}

}  // namespace

size_t outliers_ws_bytes(int64_t R, int32_t I, int32_t G, int32_t mode, int32_t kind) {
  size_t used = 0;
  carve((void *)0x100, R, I, G, mode, kind, &used);
  return used + 256;
}

hipError_t launch_outliers(const OutArgs &a, void *ws, size_t ws_bytes, hipStream_t s) {
  size_t used = 0;
  OWs w = carve(ws, a.R, a.I, a.G, a.mode, a.kind, &used);
  if (used > ws_bytes) return hipErrorInvalidValue;
  const int IG = a.I * a.G;
  const unsigned nb = (unsigned)((a.R * a.G + 255) / 256);
  const bool mad = a.kind == TA_SCORE_MAD;
  if (a.R > 0) {
    if (a.mode == TA_SCAN_FULL) {
      if (IG > 0) {
        if (mad)
          hipLaunchKernelGGL(sel_columns, dim3((IG + SC - 1) / SC), dim3(ST), 0, s, a.T, a.R, IG,
                             a.G, a.it, w.cs);
        else
          hipLaunchKernelGGL(col_moments, dim3((IG + 255) / 256), dim3(256), 0, s, a.T, a.R, IG,
                             a.G, a.it, w.cm);
      }
      if (mad)
        hipLaunchKernelGGL((score_cells<true>), dim3(nb), dim3(256), 0, s, a.T, a.R, a.I, a.G,
                           a.it, w.cs, w.cm, w.m_t);
      else
        hipLaunchKernelGGL((score_cells<false>), dim3(nb), dim3(256), 0, s, a.T, a.R, a.I, a.G,
                           a.it, w.cs, w.cm, w.m_t);
      if (mad)
        hipLaunchKernelGGL((sel_regions<true, true>), dim3(a.G), dim3(RT), 0, s, (const void *)w.m_t,
                           a.R, a.G, a.it, a.I, w.z_t, a.region_score);
      else
        hipLaunchKernelGGL((sel_regions<true, false>), dim3(a.G), dim3(RT), 0, s,
                           (const void *)w.m_t, a.R, a.G, a.it, a.I, w.z_t, a.region_score);
    } else {
      hipLaunchKernelGGL(rank_totals_t, dim3(nb), dim3(256), 0, s, a.T, a.R, a.I, a.G, a.it, w.S_t);
      if (mad)
        hipLaunchKernelGGL((sel_regions<false, true>), dim3(a.G), dim3(RT), 0, s,
                           (const void *)w.S_t, a.R, a.G, a.it, a.I, w.z_t, a.region_score);
      else
        hipLaunchKernelGGL((sel_regions<false, false>), dim3(a.G), dim3(RT), 0, s,
                           (const void *)w.S_t, a.R, a.G, a.it, a.I, w.z_t, a.region_score);
    }
  }
  const unsigned nr = (unsigned)((a.R + 255) / 256);
  if (a.R > 0)
    hipLaunchKernelGGL(rank_final, dim3(nr), dim3(256), 0, s, w.z_t, a.R, a.G, a.it, a.I, a.tau,
                       a.rank_score, a.rank_flag, w.part);
  hipLaunchKernelGGL(count_final, dim3(1), dim3(256), 0, s, w.part, (int64_t)nr, a.n_flagged);
  return hipGetLastError();
}

}  // namespace ta
