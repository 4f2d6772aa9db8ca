// k_outliers.hip -- exact outlier scan over the rank x iteration x region tensor.
//
// Robust (modified) z-score: z = (x - median) / (1.4826 * MAD), with the
// mean-absolute-deviation fallback when MAD is 0.  Medians are found exactly
// by most-significant-digit radix selection with LDS histograms; no sort, no
// approximation.  For an even count the upper middle value is either a repeat
// of the lower one, the next non-empty bucket of the last digit, or the
// smallest key above the lower median's prefix group (kept during the last
// pass), so no extra pass is needed.
//
// FULL scan:   transpose the tensor to column-major [I*G][ranks] so that every
//              per-column pass streams contiguous memory
//              stage 1  per column (i,g): median and MAD over ranks (11-bit
//                       digits, one workgroup per column)
//              scoring  m(r,g) = mean over the rank's iterations of z(r,i,g),
//                       summed in ascending i (bit-reproducible)
//              stage 2  per region g: median / MAD over ranks of m(r,g)
// TOTALS scan: stage 2 only, on the rank totals S(r,g).
#include "ta_device.h"
#include "ta_internal.h"

namespace ta {
namespace {

constexpr uint64_t SIGN = 0x8000000000000000ull;

struct ColSel {
  int64_t *med2, *mad4, *sumdev, *n;  // [IG]
};

__device__ inline int nbits64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

// ----------------------------------------------------------------------------
// Column-major path for the robust FULL scan.
//   transpose_kernel  T[R][IG] -> Tt[IG][Rp] (Rp = R rounded up to 64) through
//                     64 x 64 LDS tiles; a cell of an iteration the rank does
//                     not have, and the padding, hold the sentinel INT64_MIN
//   col_select        one workgroup per column, streaming the contiguous column:
//                     count/min/max, radix selection of the lower median with
//                     11-bit digits, then of the MAD (the first MAD pass also
//                     sums the absolute deviations).  The next order statistic
//                     of an even count is the next non-empty bin of the last
//                     digit, else the smallest key above the prefix group
//   score_cols        a wave = 64 consecutive ranks of one region; the column
//                     parameters are uniform across the wave
// ----------------------------------------------------------------------------
constexpr int TT = 64;
constexpr int64_t SENT = INT64_MIN;

__host__ __device__ inline int64_t pad_ranks(int64_t R) { return (R + 63) & ~(int64_t)63; }

__global__ __launch_bounds__(256) void transpose_kernel(const int64_t *__restrict__ T, int64_t R,
                                                        int IG, int G, const int32_t *it,
                                                        int64_t *__restrict__ Tt) {
  __shared__ int64_t tile[TT][TT + 1];
  const int64_t r0 = (int64_t)blockIdx.x * TT;
  const int c0 = blockIdx.y * TT;
  const int64_t Rp = pad_ranks(R);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int k = ty; k < TT; k += 4) {
    const int64_t r = r0 + k;
    const int c = c0 + tx;
    int64_t v = SENT;
    if (r < R && c < IG && (it == nullptr || c / G < it[r])) v = __builtin_nontemporal_load(&T[r * IG + c]);
    tile[k][tx] = v;
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 4) {
    const int c = c0 + k;
    if (c < IG) Tt[(int64_t)c * Rp + r0 + tx] = tile[tx][k];
  }
}

constexpr int CS = 512;           // threads per column workgroup
constexpr int CWV = CS / 64;      // waves
constexpr int CU = 4;             // 16-byte loads in flight per thread
constexpr int DIG = 11;           // bits per digit
constexpr int NB = 1 << DIG;
constexpr int NHC = 2;            // histogram copies (waves alternate)
constexpr int BPT = NB / CS;      // bins per thread in the bin search

typedef long long v2ll __attribute__((ext_vector_type(2)));

__device__ inline uint64_t shr64(uint64_t x, int s) { return s >= 64 ? 0 : x >> s; }

struct ColSelLds {
  uint32_t hist[NHC][NB];
  int64_t red[CS];
  uint64_t ured[CS];
  int64_t wtot[CWV];
  uint64_t state[4];
};

// f(x) for every cell of the padded column, sentinels included.
template <class F>
__device__ __forceinline__ void sweep(const int64_t *__restrict__ col, int64_t Rp, F &&f) {
  const int64_t t2 = 2 * (int64_t)threadIdx.x;
  for (int64_t b = 0; b < Rp; b += (int64_t)CS * 2 * CU) {
    v2ll v[CU];
#pragma unroll
    for (int u = 0; u < CU; u++) {
      const int64_t r = b + (int64_t)u * CS * 2 + t2;
      v[u] = r < Rp ? *reinterpret_cast<const v2ll *>(col + r) : v2ll{SENT, SENT};
    }
#pragma unroll
    for (int u = 0; u < CU; u++) {
      f((int64_t)v[u].x);
      f((int64_t)v[u].y);
    }
  }
}

__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t *buf) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int st = CS / 2; st > 0; st >>= 1) {
    if (t < st && buf[t + st] < buf[t]) buf[t] = buf[t + st];
    __syncthreads();
  }
  const uint64_t r = buf[0];
  __syncthreads();
  return r;
}

__device__ inline int64_t block_minmax_i64(int64_t v, bool is_max, int64_t *buf) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int st = CS / 2; st > 0; st >>= 1) {
    if (t < st) {
      const int64_t o = buf[t + st];
      if (is_max ? o > buf[t] : o < buf[t]) buf[t] = o;
    }
    __syncthreads();
  }
  const int64_t r = buf[0];
  __syncthreads();
  return r;
}

// Lower median (rank (n-1)/2) of key(x) over the valid cells, keys in
// [0, 2^bits), and the next order statistic (equal to it for odd n).  With
// SUMD, also returns the sum of the keys (the first pass reads every cell).
template <bool SUMD, class KeyF>
__device__ void col_radix_select(const int64_t *__restrict__ col, int64_t Rp, int64_t n, int bits,
                                 KeyF keyf, ColSelLds &L, uint64_t &v1, uint64_t &v2,
                                 int64_t &ksum) {
  const int t = threadIdx.x, wid = t >> 6, lane = t & 63;
  uint32_t *hist = L.hist[wid & (NHC - 1)];
  uint64_t pref = 0;
  int64_t k = (n - 1) / 2;
  int hi = bits;
  bool first = true;
  ksum = 0;
  while (hi > 0) {
    const int w = hi < DIG ? hi : DIG;
    const int lo = hi - w;
    const bool last = lo == 0;
    const uint64_t mask = (1ull << w) - 1;
    uint64_t mgt = ~0ull;
    int64_t sk = 0;
    const bool sumd = SUMD && first;
    sweep(col, Rp, [&](int64_t x) {
      if (x == SENT) return;
      const uint64_t key = keyf(x);
      if (sumd) sk += (int64_t)key;
      const uint64_t top = shr64(key, hi);
      if (top == pref)
        atomicAdd(&hist[(uint32_t)((key >> lo) & mask)], 1u);
      else if (last && top > pref && key < mgt)
        mgt = key;
    });
    if (sumd) ksum = block_sum_i64<CS>(sk, L.red);
    if (last) mgt = block_min_u64(mgt, L.ured);  // includes the barrier
    else __syncthreads();
    // Bin search: thread t owns bins [t*BPT, t*BPT + BPT) (merged copies).
    uint32_t cnt[BPT];
    int64_t own = 0;
#pragma unroll
    for (int j = 0; j < BPT; j++) {
      const int bb = t * BPT + j;
      uint32_t c = 0;
#pragma unroll
      for (int q = 0; q < NHC; q++) c += L.hist[q][bb];
      cnt[j] = (bb >> w) ? 0u : c;  // bins beyond this digit's width are empty
      own += cnt[j];
    }
    int64_t incl = own;  // inclusive scan over the wave
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(incl, d, 64);
      if (lane >= d) incl += o;
    }
    if (lane == 63) L.wtot[wid] = incl;
    __syncthreads();
    int64_t excl = incl - own;
    for (int q = 0; q < wid; q++) excl += L.wtot[q];
    // Clear the histograms for the next pass (all reads above are done after
    // the barrier below; the merged counts live in registers).
    __syncthreads();
    for (int j = t; j < NHC * NB; j += CS) (&L.hist[0][0])[j] = 0;
    if (excl <= k && k < excl + own) {
      int64_t cum = excl;
      int j = 0;
      for (; j < BPT; j++) {
        if (cum + (int64_t)cnt[j] > k) break;
        cum += cnt[j];
      }
      const int64_t kk = k - cum;
      const int bsel = t * BPT + j;
      L.state[0] = (pref << w) | (uint64_t)bsel;
      L.state[1] = (uint64_t)kk;
      // Upper middle of an even count on the last digit: the same bin when it
      // holds another key, else the next non-empty bin (searched below).
      L.state[2] = (kk + 1 < (int64_t)cnt[j]) ? 1 : 0;
    }
    __syncthreads();
    const uint64_t np = L.state[0];
    const int64_t kk = (int64_t)L.state[1];
    if (last) {
      uint64_t nxt = ~0ull;  // smallest non-empty bin above the selected one
      if (L.state[2] == 0) {
        const int bsel = (int)(np & mask);
#pragma unroll
        for (int j = BPT - 1; j >= 0; j--) {
          const int bb = t * BPT + j;
          if (bb > bsel && cnt[j] > 0) nxt = (uint64_t)bb;
        }
      }
      nxt = block_min_u64(nxt, L.ured);
      v1 = np;
      if (L.state[2]) v2 = np;
      else if (nxt != ~0ull) v2 = (pref << w) | nxt;
      else v2 = mgt;
      __syncthreads();
    }
    pref = np;
    k = kk;
    hi = lo;
    first = false;
  }
  if (bits == 0) {
    v1 = v2 = 0;
    if (SUMD) ksum = 0;
  }
  if (n & 1) v2 = v1;
}

__global__ __launch_bounds__(CS) void col_select(const int64_t *__restrict__ Tt, int64_t R,
                                                 ColSel out) {
  __shared__ ColSelLds L;
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t Rp = pad_ranks(R);
  const int64_t *col = Tt + (int64_t)c * Rp;
  for (int j = t; j < NHC * NB; j += CS) (&L.hist[0][0])[j] = 0;
  int64_t n = 0, mn = INT64_MAX, mx = INT64_MIN;
  sweep(col, Rp, [&](int64_t x) {
    if (x == SENT) return;
    n++;
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
  });
  n = block_sum_i64<CS>(n, L.red);
  mn = block_minmax_i64(mn, false, L.red);
  mx = block_minmax_i64(mx, true, L.red);
  if (n == 0) {
    if (t == 0) {
      out.med2[c] = 0;
      out.mad4[c] = 0;
      out.sumdev[c] = 0;
      out.n[c] = 0;
    }
    return;
  }
  const uint64_t base = (uint64_t)mn;
  uint64_t a, b;
  int64_t unused;
  col_radix_select<false>(col, Rp, n, nbits64((uint64_t)mx - base),
                          [&](int64_t x) { return (uint64_t)x - base; }, L, a, b, unused);
  const int64_t med2 = (int64_t)(base + a) + (int64_t)(base + b);
  // Deviations |2x - med2|; the largest is at an end of the range.
  const uint64_t dlo = (uint64_t)(med2 - 2 * mn), dhi = (uint64_t)(2 * mx - med2);
  const uint64_t dmax = dlo > dhi ? dlo : dhi;
  int64_t sd = 0;
  col_radix_select<true>(col, Rp, n, nbits64(dmax),
                         [&](int64_t x) {
                           const int64_t d = 2 * x - med2;
                           return (uint64_t)(d < 0 ? -d : d);
                         },
                         L, a, b, sd);
  if (t == 0) {
    out.med2[c] = med2;
    out.mad4[c] = (int64_t)(a + b);
    out.sumdev[c] = sd;
    out.n[c] = n;
  }
}

// ----------------------------------------------------------------------------
// Plain moments per column (TA_SCORE_Z) over the column-major tensor:
// n, sum, 128-bit sum of squares -> std (ddof 1).
// ----------------------------------------------------------------------------
struct ColMom {
  int64_t *n, *s1;
  double *sd;
};

__global__ __launch_bounds__(CS) void col_moments(const int64_t *__restrict__ Tt, int64_t R,
                                                  ColMom out) {
  __shared__ u128 q[CS];
  __shared__ int64_t red[CS];
  const int c = blockIdx.x, t = threadIdx.x;
  const int64_t Rp = pad_ranks(R);
  int64_t n = 0, s1 = 0;
  u128 s2 = 0;
  sweep(Tt + (int64_t)c * Rp, Rp, [&](int64_t x) {
    if (x == SENT) return;
    n++;
    s1 += x;
    s2 += (u128)((i128)x * x);
  });
  n = block_sum_i64<CS>(n, red);
  s1 = block_sum_i64<CS>(s1, red);
  q[t] = s2;
  __syncthreads();
  for (int st = CS / 2; st > 0; st >>= 1) {
    if (t < st) q[t] += q[t + st];
    __syncthreads();
  }
  if (t == 0) {
    double sd = 0.0;
    if (n > 1)
      sd = sqrt(i128_to_f64((i128)((u128)n * q[0]) - (i128)s1 * s1) / ((double)n * (double)(n - 1)));
    out.n[c] = n;
    out.s1[c] = s1;
    out.sd[c] = sd;
  }
}

// m(r,g) = (1/n_r) sum_{i < n_r} z(r,i,g) (ascending i) from the column-major
// tensor, written [G][R]; one wave = 64 consecutive ranks of region g, so the
// column parameters are uniform across the wave.
template <bool MAD>
__global__ __launch_bounds__(256) void score_cols(const int64_t *__restrict__ Tt, int64_t R, int I,
                                                  int G, const int32_t *it, ColSel cs, ColMom cm,
                                                  double *m_t) {
  const int lane = threadIdx.x & 63;
  const int64_t rblocks = (R + 63) / 64;
  const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = (int)(wave / rblocks);
  if (g >= G) return;
  const int64_t Rp = pad_ranks(R);
  const int64_t r = (wave % rblocks) * 64 + lane;
  int ni = 0;
  if (r < R) {
    ni = it ? it[r] : I;
    ni = ni > I ? I : (ni < 0 ? 0 : ni);
  }
  double acc = 0.0;
  const int64_t *p = Tt + (int64_t)g * Rp + (r < R ? r : 0);
  for (int i = 0; i < I; i++) {
    const int c = i * G + g;
    if (i < ni) {
      const int64_t x = p[(int64_t)i * G * Rp];
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
  }
  if (r < R) m_t[(int64_t)g * R + r] = ni > 0 ? acc / (double)ni : 0.0;
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
  int64_t *Tt;      // [IG][Rp] column-major copy of the tensor (FULL)
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
    w.Tt = (int64_t *)take((size_t)pad_ranks(R) * IG * 8);
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
  if ((IG + TT - 1) / TT > 65535) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)((a.R * a.G + 255) / 256);
  const bool mad = a.kind == TA_SCORE_MAD;
  if (a.R > 0) {
    if (a.mode == TA_SCAN_FULL) {
      if (IG > 0) {
        hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(pad_ranks(a.R) / TT), (IG + TT - 1) / TT),
                           dim3(256), 0, s, a.T, a.R, IG, a.G, a.it, w.Tt);
        if (mad)
          hipLaunchKernelGGL(col_select, dim3(IG), dim3(CS), 0, s, w.Tt, a.R, w.cs);
        else
          hipLaunchKernelGGL(col_moments, dim3(IG), dim3(CS), 0, s, w.Tt, a.R, w.cm);
      }
      const unsigned nw = (unsigned)((a.G * ((a.R + 63) / 64) + 3) / 4);
      if (mad)
        hipLaunchKernelGGL((score_cols<true>), dim3(nw), dim3(256), 0, s, w.Tt, a.R, a.I, a.G, a.it,
                           w.cs, w.cm, w.m_t);
      else
        hipLaunchKernelGGL((score_cols<false>), dim3(nw), dim3(256), 0, s, w.Tt, a.R, a.I, a.G, a.it,
                           w.cs, w.cm, w.m_t);
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
