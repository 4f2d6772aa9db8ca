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
// FULL scan:   stage 1  per column (i,g): median and MAD over ranks
//                       - robust kind, long columns: on the row-major tensor,
//                         a sampled bracket per column, one streaming pass
//                         that counts and compacts the bracket interior, an
//                         exact selection over it (rm_* kernels below)
//                       - otherwise: transpose to column-major [I*G][ranks]
//                         and select per column (11-bit digits)
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
  double *zc, *zd;                    // [IG] row-major path: z = ((2x - med2) * zc) / zd
};

// The robust z of a cell in one division with per-column (zc, zd): when
// mad4 > 0, (2.0, 1.4826 * mad4) -- (2x - med2) * 2 converts to the same double
// as 4x - 2 med2; when only the mean absolute deviation is positive,
// (n, 1.253314 * sumdev); else (0, 1) (every cell is the median, z = 0).
__host__ __device__ inline void z_coefs(int64_t mad4, int64_t sumdev, int64_t n, double &zc, double &zd) {
  if (mad4 > 0) {
    zc = 2.0;
    zd = 1.4826 * (double)mad4;
  } else if (sumdev > 0) {
    zc = (double)n;
    zd = 1.253314 * (double)sumdev;
  } else {
    zc = 0.0;
    zd = 1.0;
  }
}

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
typedef long long v2ll __attribute__((ext_vector_type(2)));
typedef int v2i __attribute__((ext_vector_type(2)));
constexpr int64_t SENT = INT64_MIN;

__host__ __device__ inline int64_t pad_ranks(int64_t R) { return (R + 63) & ~(int64_t)63; }

// 64 columns x TG tiles of 64 ranks per workgroup, one tile at a time.  Reads:
// lane pairs of adjacent columns of one row (16-byte loads when rows are
// 16-byte aligned, i.e. I*G even); writes: lane pairs of adjacent ranks of one
// column (16-byte stores).  STATS: each column's valid cells (not sentinels)
// are also summed exactly over the workgroup's ranks -- count, int64 sum,
// unsigned 128-bit sum of squares, min, max -- and written as rank chunk
// blockIdx.x of the imbalance column partials (thread = column and quarter of
// a tile; the four quarters are combined through LDS at the end).
constexpr int TG = 16;

int transpose_groups_of(int64_t R) { return (int)((pad_ranks(R) / TT + TG - 1) / TG); }

template <bool STATS>
__global__ __launch_bounds__(256) void transpose_kernel(const int64_t *__restrict__ T, int64_t R,
                                                        int IG, int G, const int32_t *it,
                                                        int64_t *__restrict__ Tt, ColPartials ps) {
  __shared__ int64_t tile[TT][TT + 1];
  const int c0 = blockIdx.y * TT;
  const int64_t Rp = pad_ranks(R);
  const int p2 = 2 * (threadIdx.x & 31), k0 = threadIdx.x >> 5;
  const int ca = c0 + p2;  // this thread's columns ca, ca + 1 (read phase)
  const int ia = ca / G, ib = (ca + 1) / G;
  const bool vec = (IG & 1) == 0;
  const int sc = threadIdx.x & 63, sq = threadIdx.x >> 6;  // stats: column, quarter of a tile
  int64_t n = 0, s1 = 0, mn = INT64_MAX, mx = INT64_MIN;
  u128 s2 = 0;
  const int64_t n_tiles = Rp / TT;
  for (int64_t tl = (int64_t)blockIdx.x * TG; tl < n_tiles && tl < (int64_t)(blockIdx.x + 1) * TG; tl++) {
    const int64_t r0 = tl * TT;
    for (int k = k0; k < TT; k += 8) {
      const int64_t r = r0 + k;
      int64_t v0 = SENT, v1 = SENT;
      if (r < R) {
        const int nit = it ? it[r] : 0x7fffffff;
        const int64_t *row = T + r * IG;
        if (vec && ca + 1 < IG) {
          const v2ll q = __builtin_nontemporal_load(reinterpret_cast<const v2ll *>(row + ca));
          v0 = ia < nit ? (int64_t)q.x : SENT;
          v1 = ib < nit ? (int64_t)q.y : SENT;
        } else {
          if (ca < IG && ia < nit) v0 = __builtin_nontemporal_load(row + ca);
          if (ca + 1 < IG && ib < nit) v1 = __builtin_nontemporal_load(row + ca + 1);
        }
      }
      tile[k][p2] = v0;
      tile[k][p2 + 1] = v1;
    }
    __syncthreads();
    for (int k = k0; k < TT; k += 8) {
      const int c = c0 + k;
      if (c < IG) {
        const v2ll q = {tile[p2][k], tile[p2 + 1][k]};
        *reinterpret_cast<v2ll *>(Tt + (int64_t)c * Rp + r0 + p2) = q;
      }
    }
    if (STATS) {
#pragma unroll 4
      for (int k = sq * 16; k < sq * 16 + 16; k++) {
        const int64_t x = tile[k][sc];
        if (x != SENT) {
          n++;
          s1 += x;
          s2 += (u128)((i128)x * x);
          mn = x < mn ? x : mn;
          mx = x > mx ? x : mx;
        }
      }
    }
    __syncthreads();
  }
  if (STATS) {
    // combine the four quarters of each column (reusing the tile's LDS)
    int64_t *red = &tile[0][0];  // [6][4][64]
    const int b = sq * 64 + sc;
    red[0 * 256 + b] = n;
    red[1 * 256 + b] = s1;
    red[2 * 256 + b] = (int64_t)(uint64_t)s2;
    red[3 * 256 + b] = (int64_t)(uint64_t)(s2 >> 64);
    red[4 * 256 + b] = mn;
    red[5 * 256 + b] = mx;
    __syncthreads();
    if (threadIdx.x < 64 && c0 + sc < IG) {
      int64_t tn = 0, ts1 = 0, tmn = INT64_MAX, tmx = INT64_MIN;
      u128 ts2 = 0;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int j = q * 64 + sc;
        tn += red[0 * 256 + j];
        ts1 += red[1 * 256 + j];
        ts2 += ((u128)(uint64_t)red[3 * 256 + j] << 64) | (uint64_t)red[2 * 256 + j];
        tmn = red[4 * 256 + j] < tmn ? red[4 * 256 + j] : tmn;
        tmx = red[5 * 256 + j] > tmx ? red[5 * 256 + j] : tmx;
      }
      const int64_t p = (int64_t)blockIdx.x * IG + c0 + sc;
      ps.n[p] = tn;
      ps.s1[p] = ts1;
      ps.lo[p] = (uint64_t)ts2;
      ps.hi[p] = (uint64_t)(ts2 >> 64);
      ps.mn[p] = tmn;
      ps.mx[p] = tmx;
    }
  }
}

constexpr int CS = 256;           // threads per column workgroup
constexpr int CWV = CS / 64;      // waves
constexpr int CU = 4;             // 16-byte loads in flight per thread
constexpr int DIG = 11;           // bits per digit
constexpr int NB = 1 << DIG;
constexpr int NHC = 1;            // histogram copies
constexpr int BPT = NB / CS;      // bins per thread in the bin search

__device__ inline uint64_t shr64(uint64_t x, int s) { return s >= 64 ? 0 : x >> s; }

constexpr int MS = 2048;          // sample slots (LDS)
constexpr int SEL_GRID_MAX = 2048; // column workgroups (persistent, one scratch slot each)
constexpr int64_t SEL_BRACKET_MIN_RP = 32768;  // shorter columns: whole-column radix selection

// LDS of the radix selection (and of the column reductions).
struct SelLds {
  uint32_t hist[NHC][NB];
  int64_t red[CS];
  uint64_t ured[CS];
  int64_t wtot[CWV];
  uint64_t state[4];
};

struct ColSelLds : SelLds {
  int64_t samp[MS];
  uint32_t ns, cin;  // sample count, bracket count
};

// Scratch slot per column workgroup: the values inside a bracket (expected
// about BRACKET_SE / sqrt(2048) = 10 % of the column; the cap leaves room for
// skewed or tied columns).
__host__ __device__ inline int64_t sel_cap(int64_t R) {
  const int64_t Rp = pad_ranks(R);
  int64_t c = ((Rp * 45 / 100) + 63) & ~(int64_t)63;
  if (c < 4096) c = 4096;
  return c;
}

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

// Block reductions of the column workgroup: a shuffle reduction in each wave,
// one barrier, then every thread combines the CWV wave results in wave order,
// and a second barrier before the slots are reused.  `slots` holds CWV * K
// values.
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t *slots) {
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = slots[0];
  for (int q = 1; q < CWV; q++) r = slots[q] < r ? slots[q] : r;
  __syncthreads();
  return r;
}

// K sums, then (with MM) a minimum and a maximum, in one exchange.
template <int K, bool MM>
__device__ inline void block_stats(int64_t (&v)[K], int64_t &mn, int64_t &mx, int64_t *slots) {
  constexpr int W = K + (MM ? 2 : 0);
  for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
    for (int k = 0; k < K; k++) v[k] += __shfl_xor(v[k], d, 64);
    if (MM) {
      const int64_t a = __shfl_xor(mn, d, 64), b = __shfl_xor(mx, d, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) slots[wid * W + k] = v[k];
    if (MM) {
      slots[wid * W + K] = mn;
      slots[wid * W + K + 1] = mx;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    int64_t s = 0;
    for (int q = 0; q < CWV; q++) s += slots[q * W + k];
    v[k] = s;
  }
  if (MM) {
    mn = slots[K];
    mx = slots[K + 1];
    for (int q = 1; q < CWV; q++) {
      mn = slots[q * W + K] < mn ? slots[q * W + K] : mn;
      mx = slots[q * W + K + 1] > mx ? slots[q * W + K + 1] : mx;
    }
  }
  __syncthreads();
}

__device__ inline int64_t block_sum1(int64_t v, int64_t *slots) {
  int64_t a[1] = {v}, d0 = 0, d1 = 0;
  block_stats<1, false>(a, d0, d1, slots);
  return a[0];
}

// The k-th smallest key (k from 0) of the values a source visits, keys in
// [0, 2^bits), and with want_next the (k+1)-th (which must exist).  `visit(f)`
// calls f(x) for every value of this thread's share of the source; `keyf(x)`
// maps a value to its key.
template <class Visit, class KeyF>
__device__ void radix_select(Visit &&visit, int64_t k, bool want_next, int bits, KeyF keyf,
                             SelLds &L, uint64_t &v1, uint64_t &v2, int64_t *key_sum = nullptr) {
  const int t = threadIdx.x, wid = t >> 6, lane = t & 63;
  uint32_t *hist = L.hist[wid & (NHC - 1)];
  uint64_t pref = 0;
  int hi = bits;
  bool first = true;
  v1 = v2 = 0;
  if (key_sum && bits == 0) *key_sum = 0;
  while (hi > 0) {
    const int w = hi < DIG ? hi : DIG;
    const int lo = hi - w;
    const bool last = lo == 0;
    const uint64_t mask = (1ull << w) - 1;
    const bool sum_keys = key_sum != nullptr && first;
    uint64_t mgt = ~0ull;
    int64_t ks = 0;
    visit([&](int64_t x) {
      const uint64_t key = keyf(x);
      if (sum_keys) ks += (int64_t)key;
      const uint64_t top = shr64(key, hi);
      if (top == pref)
        atomicAdd(&hist[(uint32_t)((key >> lo) & mask)], 1u);
      else if (last && top > pref && key < mgt)
        mgt = key;
    });
    if (sum_keys) *key_sum = block_sum1(ks, L.red);
    first = false;
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
      cnt[j] = c;
      own += c;
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
    // All histogram reads above precede this barrier; clear for the next pass.
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
      L.state[0] = (pref << w) | (uint64_t)(t * BPT + j);
      L.state[1] = (uint64_t)kk;
      // On the last digit the (k+1)-th key is in the same bin when the bin
      // holds another key, else in the next non-empty bin (searched below).
      L.state[2] = (kk + 1 < (int64_t)cnt[j]) ? 1 : 0;
    }
    __syncthreads();
    const uint64_t np = L.state[0];
    const int64_t kk = (int64_t)L.state[1];
    if (last) {
      const bool same = L.state[2] != 0;
      uint64_t nxt = ~0ull;  // smallest non-empty bin above the selected one
      if (want_next && !same) {
        const int bsel = (int)(np & mask);
#pragma unroll
        for (int j = BPT - 1; j >= 0; j--) {
          const int bb = t * BPT + j;
          if (bb > bsel && cnt[j] > 0) nxt = (uint64_t)bb;
        }
      }
      nxt = block_min_u64(nxt, L.ured);
      v1 = np;
      if (!want_next || same) v2 = np;
      else if (nxt != ~0ull) v2 = (pref << w) | nxt;
      else v2 = mgt;
    }
    pref = np;
    k = kk;
    hi = lo;
  }
  if (!want_next) v2 = v1;
}

// f(x) for this thread's share of scr[0..c), eight loads in flight.
template <class F>
__device__ __forceinline__ void visit_scratch(const int64_t *__restrict__ scr, int64_t c, F &&f) {
  constexpr int U = 4;
  for (int64_t i0 = 0; i0 < c; i0 += (int64_t)CS * U) {
    int64_t v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t i = i0 + (int64_t)u * CS + threadIdx.x;
      v[u] = i < c ? scr[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (i0 + (int64_t)u * CS + threadIdx.x < c) f(v[u]);
  }
}

// Append v to scratch when `in` (all lanes of the wave call this together).
__device__ inline void wave_append(bool in, int64_t v, uint32_t *counter, int64_t *scr, int64_t cap) {
  const uint64_t m = __ballot(in);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  if (in) {
    const int64_t pos = (int64_t)base + __popcll(m & ((1ull << lane) - 1));
    if (pos < cap) scr[pos] = v;
  }
}

// Visits the m sample values held in LDS.
struct SampleVisit {
  const int64_t *samp;
  int m;
  template <class F>
  __device__ void operator()(F &&f) const {
    for (int j = threadIdx.x; j < m; j += CS) f(samp[j]);
  }
};

// Order statistics j1 and j2 of the m (> 0) sample values.
__device__ void sample_pick(ColSelLds &L, int m, int64_t j1, int64_t j2, int64_t &v1, int64_t &v2) {
  int64_t mnl = INT64_MAX, mxl = INT64_MIN;
  for (int j = threadIdx.x; j < m; j += CS) {
    const int64_t x = L.samp[j];
    mnl = x < mnl ? x : mnl;
    mxl = x > mxl ? x : mxl;
  }
  int64_t none[1] = {0}, mn = mnl, mx = mxl;
  block_stats<1, true>(none, mn, mx, L.red);
  const int bits = nbits64((uint64_t)mx - (uint64_t)mn);
  auto key = [&](int64_t x) { return (uint64_t)x - (uint64_t)mn; };
  const SampleVisit vs{L.samp, m};
  uint64_t a, b;
  if (j2 == j1 + 1) {
    radix_select(vs, j1, true, bits, key, L, a, b);
  } else {
    radix_select(vs, j1, false, bits, key, L, a, b);
    if (j2 != j1) radix_select(vs, j2, false, bits, key, L, b, b);
    else b = a;
  }
  v1 = (int64_t)((uint64_t)mn + a);
  v2 = (int64_t)((uint64_t)mn + b);
}

// Bracket [lo, hi] around the middle of the sample (m values): its order
// statistics (1/2 -/+ delta)(m - 1), delta = BRACKET_SE / (2 sqrt(m)).  A wider
// bracket misses less often; a narrower one compacts (and selects over) fewer
// cells per pass.  Exactness does not depend on it.  Measured at 100k ranks:
// +-3 standard errors (about 170 column gathers per scan) made the scan 2 ms
// slower than +-4.5.
constexpr double BRACKET_SE = 4.5;
__device__ inline void sample_bracket(ColSelLds &L, int m, int64_t &lo, int64_t &hi) {
  if (m <= 0) {
    lo = INT64_MAX;  // empty bracket: the caller falls back to full selection
    hi = INT64_MIN;
    return;
  }
  // the sample median's standard error in quantile units is 0.5 / sqrt(m): a
  // bracket of +-BRACKET_SE of them misses the median with probability
  // 2 * P(Z > BRACKET_SE) (then the caller selects over the whole column)
  const double dl = 0.5 * BRACKET_SE / sqrt((double)m);
  const double ca = (0.5 - dl) * (double)(m - 1), cb = (0.5 + dl) * (double)(m - 1);
  const int ia = ca <= 0.0 ? 0 : (int)floor(ca);
  const int ib = cb >= (double)(m - 1) ? m - 1 : (int)ceil(cb);
  sample_pick(L, m, ia, ib, lo, hi);
}

// The k-th smallest value of a column (and with `even` the (k+1)-th) from the
// counts of a bracket pass: clo values below qa, ceqa equal to qa, cmid strictly
// inside (qa, qb) -- compacted in the scratch that `vmid` visits -- and ceqb
// equal to qb (0 when qa == qb).  Returns false when a wanted rank lies outside
// the bracket or the interior overflowed the scratch.
template <class Visit>
__device__ bool bracket_pick(Visit &&vmid, int64_t clo, int64_t ceqa, int64_t cmid, int64_t ceqb,
                             int64_t qa, int64_t qb, int64_t cap, int64_t k, bool even,
                             SelLds &L, int64_t &x1, int64_t &x2) {
  auto where = [&](int64_t j) -> int {
    if (j < clo) return 0;
    j -= clo;
    if (j < ceqa) return 1;
    j -= ceqa;
    if (j < cmid) return 2;
    j -= cmid;
    return j < ceqb ? 3 : 0;
  };
  const int w1 = where(k), w2 = even ? where(k + 1) : w1;
  if (w1 == 0 || w2 == 0) return false;
  if ((w1 == 2 || w2 == 2) && cmid > cap) return false;
  const int64_t base = clo + ceqa;
  const int bits = nbits64((uint64_t)qb - (uint64_t)qa);
  auto key = [&](int64_t x) { return (uint64_t)x - (uint64_t)qa; };
  auto val = [&](uint64_t kv) { return (int64_t)((uint64_t)qa + kv); };
  uint64_t a1 = 0, a2 = 0;
  if (w1 == 2 && w2 == 2) {
    radix_select(vmid, k - base, even, bits, key, L, a1, a2);
    x1 = val(a1);
    x2 = val(a2);
    return true;
  }
  if (w1 == 2) {
    radix_select(vmid, k - base, false, bits, key, L, a1, a2);
    x1 = val(a1);
  } else {
    x1 = w1 == 1 ? qa : qb;
  }
  if (!even) {
    x2 = x1;
    return true;
  }
  if (w2 == 2) {
    radix_select(vmid, k + 1 - base, false, bits, key, L, a1, a2);
    x2 = val(a1);
  } else {
    x2 = w2 == 1 ? qa : qb;
  }
  return true;
}

// Per column (at least SEL_BRACKET_MIN_RP padded ranks; persistent grid, one
// scratch slot per workgroup): sample, then two streaming passes (median
// bracket, MAD bracket); exact selection over the compacted bracket values, or
// over the whole column when a bracket misses the middle or overflows the
// scratch.
constexpr int SEL_WGS_PER_CU = 4;  // column workgroups per CU (LDS 20 KB, at most 128 VGPRs each)

__global__ __launch_bounds__(CS, SEL_WGS_PER_CU) void col_select_bracket(const int64_t *__restrict__ Tt, int64_t R, int IG,
                                                 int64_t *__restrict__ scratch, int64_t cap,
                                                 ColSel out) {
  __shared__ ColSelLds L;
  const int t = threadIdx.x;
  const int64_t Rp = pad_ranks(R);
  int64_t *scr = scratch + (int64_t)blockIdx.x * cap;
  for (int j = t; j < NHC * NB; j += CS) (&L.hist[0][0])[j] = 0;
  for (int c = blockIdx.x; c < IG; c += gridDim.x) {
    const int64_t *col = Tt + (int64_t)c * Rp;
    auto vcol = [&](auto &&f) {
      sweep(col, Rp, [&](int64_t x) {
        if (x != SENT) f(x);
      });
    };
    // ---- sample: MS / 2 chunks of 2 consecutive cells (Rp >= 2 * MS) -------
    if (t == 0) {
      L.ns = 0;
      L.cin = 0;
    }
    __syncthreads();
    {
      constexpr int NCH = MS / 2;  // chunks of 2 consecutive cells, NCH / CS per thread
#pragma unroll
      for (int u = 0; u < NCH / CS; u++) {
        const int64_t j = (int64_t)t * (NCH / CS) + u;
        const int64_t s0 = ((j * Rp) / NCH) & ~(int64_t)1;
        const v2ll q = *reinterpret_cast<const v2ll *>(col + s0);
        if (q.x != SENT) L.samp[atomicAdd(&L.ns, 1u)] = q.x;
        if (q.y != SENT) L.samp[atomicAdd(&L.ns, 1u)] = q.y;
      }
    }
    __syncthreads();
    const int m = (int)L.ns;

    // ---- median ------------------------------------------------------------
    int64_t n, mn = 0, mx = 0, med2 = 0;
    {
      int64_t qa, qb;
      sample_bracket(L, m, qa, qb);
      int64_t nl = 0, cl = 0, cea = 0, ceb = 0, mnl = INT64_MAX, mxl = INT64_MIN;
      sweep(col, Rp, [&](int64_t x) {
        const bool ok = x != SENT;
        if (ok) {
          nl++;
          mnl = x < mnl ? x : mnl;
          mxl = x > mxl ? x : mxl;
          cl += x < qa ? 1 : 0;
          cea += x == qa ? 1 : 0;
          ceb += (x == qb && qb != qa) ? 1 : 0;
        }
        wave_append(ok && x > qa && x < qb, x, &L.cin, scr, cap);
      });
      int64_t cnt[4] = {nl, cl, cea, ceb};
      mn = mnl;
      mx = mxl;
      block_stats<4, true>(cnt, mn, mx, L.red);
      n = cnt[0];
      const int64_t clo = cnt[1], ceqa = cnt[2], ceqb = cnt[3];
      const int64_t cmid = (int64_t)L.cin;
      med2 = 0;
      if (n > 0) {
        const int64_t k = (n - 1) / 2;
        const bool even = (n & 1) == 0;
        const int64_t ci = cmid < cap ? cmid : cap;
        auto vscr = [&](auto &&f) { visit_scratch(scr, ci, f); };
        int64_t x1, x2;
        if (!bracket_pick(vscr, clo, ceqa, cmid, ceqb, qa, qb, cap, k, even, L, x1, x2)) {
          uint64_t a1, a2;
          radix_select(vcol, k, even, nbits64((uint64_t)mx - (uint64_t)mn),
                       [&](int64_t x) { return (uint64_t)x - (uint64_t)mn; }, L, a1, a2);
          x1 = (int64_t)((uint64_t)mn + a1);
          x2 = (int64_t)((uint64_t)mn + a2);
        }
        med2 = x1 + x2;
      }
    }
    if (n == 0) {
      if (t == 0) {
        out.med2[c] = 0;
        out.mad4[c] = 0;
        out.sumdev[c] = 0;
        out.n[c] = 0;
      }
      __syncthreads();
      continue;
    }

    // ---- MAD: the same on the deviations |2x - med2| -------------------------
    __syncthreads();  // every thread has read the sorted sample values it needs
    for (int j = t; j < m; j += CS) {
      const int64_t d = 2 * L.samp[j] - med2;
      L.samp[j] = d < 0 ? -d : d;
    }
    if (t == 0) L.cin = 0;
    __syncthreads();
    int64_t mad4, sd;
    {
      int64_t da, db;
      sample_bracket(L, m, da, db);
      int64_t sl = 0, cl = 0, cea = 0, ceb = 0;
      sweep(col, Rp, [&](int64_t x) {
        const bool ok = x != SENT;
        int64_t d = 2 * x - med2;
        d = d < 0 ? -d : d;
        if (ok) {
          sl += d;
          cl += d < da ? 1 : 0;
          cea += d == da ? 1 : 0;
          ceb += (d == db && db != da) ? 1 : 0;
        }
        wave_append(ok && d > da && d < db, d, &L.cin, scr, cap);
      });
      int64_t cnt[4] = {sl, cl, cea, ceb}, u0 = 0, u1 = 0;
      block_stats<4, false>(cnt, u0, u1, L.red);
      sd = cnt[0];
      const int64_t clo = cnt[1], ceqa = cnt[2], ceqb = cnt[3];
      const int64_t cmid = (int64_t)L.cin;
      const int64_t k = (n - 1) / 2;
      const bool even = (n & 1) == 0;
      const int64_t ci = cmid < cap ? cmid : cap;
      auto vscr = [&](auto &&f) { visit_scratch(scr, ci, f); };
      int64_t x1, x2;
      if (!bracket_pick(vscr, clo, ceqa, cmid, ceqb, da, db, cap, k, even, L, x1, x2)) {
        // Deviations lie in [0, max(med2 - 2 mn, 2 mx - med2)].
        const uint64_t dlo = (uint64_t)(med2 - 2 * mn), dhi = (uint64_t)(2 * mx - med2);
        const uint64_t dmax = dlo > dhi ? dlo : dhi;
        uint64_t a1, a2;
        radix_select(vcol, k, even, nbits64(dmax),
                     [&](int64_t x) {
                       const int64_t d = 2 * x - med2;
                       return (uint64_t)(d < 0 ? -d : d);
                     },
                     L, a1, a2);
        x1 = (int64_t)a1;
        x2 = (int64_t)a2;
      }
      mad4 = x1 + x2;
    }
    if (t == 0) {
      out.med2[c] = med2;
      out.mad4[c] = mad4;
      out.sumdev[c] = sd;
      out.n[c] = n;
    }
    __syncthreads();
  }
}

// Per column, one workgroup each (columns of up to SEL_BRACKET_MIN_RP padded
// ranks, which stay in the caches between passes): count/min/max, then radix
// selection over the whole column for the median and for the MAD (whose first
// pass also sums the absolute deviations).
__global__ __launch_bounds__(CS) void col_select_radix(const int64_t *__restrict__ Tt, int64_t R,
                                                       ColSel out) {
  __shared__ SelLds L;
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t Rp = pad_ranks(R);
  const int64_t *col = Tt + (int64_t)c * Rp;
  for (int j = t; j < NHC * NB; j += CS) (&L.hist[0][0])[j] = 0;
  auto vcol = [&](auto &&f) {
    sweep(col, Rp, [&](int64_t x) {
      if (x != SENT) f(x);
    });
  };
  int64_t n = 0, mn = INT64_MAX, mx = INT64_MIN;
  vcol([&](int64_t x) {
    n++;
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
  });
  {
    int64_t cnt[1] = {n};
    block_stats<1, true>(cnt, mn, mx, L.red);
    n = cnt[0];
  }
  if (n == 0) {
    if (t == 0) {
      out.med2[c] = 0;
      out.mad4[c] = 0;
      out.sumdev[c] = 0;
      out.n[c] = 0;
    }
    return;
  }
  const int64_t k = (n - 1) / 2;
  const bool even = (n & 1) == 0;
  uint64_t a1, a2;
  radix_select(vcol, k, even, nbits64((uint64_t)mx - (uint64_t)mn),
               [&](int64_t x) { return (uint64_t)x - (uint64_t)mn; }, L, a1, a2);
  const int64_t med2 = (int64_t)((uint64_t)mn + a1) + (int64_t)((uint64_t)mn + a2);
  const uint64_t dlo = (uint64_t)(med2 - 2 * mn), dhi = (uint64_t)(2 * mx - med2);
  const uint64_t dmax = dlo > dhi ? dlo : dhi;
  int64_t sd = 0;
  radix_select(vcol, k, even, nbits64(dmax),
               [&](int64_t x) {
                 const int64_t d = 2 * x - med2;
                 return (uint64_t)(d < 0 ? -d : d);
               },
               L, a1, a2, &sd);
  if (t == 0) {
    out.med2[c] = med2;
    out.mad4[c] = (int64_t)(a1 + a2);
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

// ----------------------------------------------------------------------------
// Row-major path for the robust FULL scan over long columns (no transpose).
//   rm_sample    MS cells of every column at fixed ranks (MS / 2 chunks of two
//                consecutive ranks, evenly spread), column-major Smp[IG][MS]
//   rm_brackets  per column, the sample's order statistics around its middle
//   rm_pass      one streaming pass over the row-major tensor: per column and
//                chunk of RCH ranks, the counts below / equal to the bracket
//                ends (and the imbalance partials, or the sum of deviations);
//                the bracket interior of each (chunk, column) goes to its own
//                scratch slot
//   rm_select    per column, exact selection over the compacted interior, or
//                over a gathered copy of the whole column when the bracket
//                misses the middle or the interior overflows the region; the
//                median step also brackets the MAD from the sample's
//                deviations
//   score_rows   m(r,g) from the row-major tensor, a wave = SRW ranks x 64
//                regions
// The same MAD pass runs on the deviations |2x - med2| once the medians are
// known.  Every count is an integer and every selection exact, so the results
// equal the column-major path's.
// ----------------------------------------------------------------------------
__host__ __device__ inline int64_t sample_rank(int j, int64_t Rp) {
  return ((((int64_t)(j >> 1)) * Rp / (MS / 2)) & ~(int64_t)1) + (j & 1);
}

__global__ __launch_bounds__(256) void rm_sample(const int64_t *__restrict__ T, int64_t R, int IG,
                                                 int G, const int32_t *it, int64_t *__restrict__ smp,
                                                 int32_t *esc) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) esc[threadIdx.x] = 0;  // before the median pass
  __shared__ int64_t tile[TT][TT + 1];
  const int c0 = blockIdx.y * TT;
  const int j0 = blockIdx.x * TT;
  const int64_t Rp = pad_ranks(R);
  const int p2 = 2 * (threadIdx.x & 31), k0 = threadIdx.x >> 5;
  const int ca = c0 + p2;
  const int ia = ca / G, ib = (ca + 1) / G;
  const bool vec = (IG & 1) == 0;
  for (int k = k0; k < TT; k += 8) {
    const int64_t r = sample_rank(j0 + k, Rp);
    int64_t v0 = SENT, v1 = SENT;
    if (r < R) {
      const int nit = it ? it[r] : 0x7fffffff;
      const int64_t *row = T + r * IG;
      if (vec && ca + 1 < IG) {
        const v2ll q = *reinterpret_cast<const v2ll *>(row + ca);
        v0 = ia < nit ? (int64_t)q.x : SENT;
        v1 = ib < nit ? (int64_t)q.y : SENT;
      } else {
        if (ca < IG && ia < nit) v0 = row[ca];
        if (ca + 1 < IG && ib < nit) v1 = row[ca + 1];
      }
    }
    tile[k][p2] = v0;
    tile[k][p2 + 1] = v1;
  }
  __syncthreads();
  for (int k = k0; k < TT; k += 8) {
    const int c = c0 + k;
    if (c < IG) {
      const v2ll q = {tile[p2][k], tile[p2 + 1][k]};
      *reinterpret_cast<v2ll *>(smp + (int64_t)c * MS + j0 + p2) = q;
    }
  }
}

// The valid sample values of column c into L.samp (as deviations |2x - med2|
// with DEV); returns their count.
template <bool DEV>
__device__ int load_sample(ColSelLds &L, const int64_t *__restrict__ s, int64_t med2) {
  if (threadIdx.x == 0) L.ns = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < MS; j += CS) {
    const int64_t x = s[j];
    if (x != SENT) {
      int64_t v = x;
      if (DEV) {
        const int64_t d = 2 * x - med2;
        v = d < 0 ? -d : d;
      }
      L.samp[atomicAdd(&L.ns, 1u)] = v;
    }
  }
  __syncthreads();
  return (int)L.ns;
}

__global__ __launch_bounds__(CS) void rm_brackets(const int64_t *__restrict__ smp, int c_lo,
                                                  int64_t *qa, int64_t *qb) {
  __shared__ ColSelLds L;
  const int c = c_lo + (int)blockIdx.x;
  for (int j = threadIdx.x; j < NHC * NB; j += CS) (&L.hist[0][0])[j] = 0;
  const int m = load_sample<false>(L, smp + (int64_t)c * MS, 0);
  int64_t a, b;
  sample_bracket(L, m, a, b);
  if (threadIdx.x == 0) {
    qa[c] = a;
    qb[c] = b;
  }
}

// Per (rank chunk, column) counts of one bracket pass.
struct RmPart {
  int32_t *n, *cl, *cea, *ceb, *cm;  // [chunks][IG]; cm: cells in the chunk's interior slot
  int64_t *sd;                       // [chunks][IG] (MAD pass)
};

// Bracket per column: (qa, qb) for the median pass; (da, db) and med2 for the
// MAD pass.
struct RmBr {
  const int64_t *a, *b, *med2;
};

constexpr int RCH = TG * TT;   // ranks per chunk (the imbalance partials' chunk)
constexpr int RPU = 8;         // rows in flight per thread
constexpr int SEG_MAX = 2048;  // chunks per column the selection can visit (LDS)

constexpr int RQ = 6;          // interior cells buffered per column
// Interior cells kept per (chunk, column) slot; a column with a fuller slot
// is selected over its gathered copy instead.  The bracket holds about a tenth
// of a column (60-110 cells of a chunk), so only skewed or tied columns reach it.
constexpr int SCAP = 256;

// The 32-bit copy of the tensor that the median pass writes for the later
// passes: a cell as its offset v from the column's median-bracket low end
// when |v| < 2^29, else CSENT, and then the half's flag is set and the later
// passes of that half read the int64 tensor.  The range leaves the MAD pass
// 32-bit keys: with |med2 - 2 * base| < 2^30 (checked when the median is
// known), |2x - med2| = |2v - (med2 - 2 * base)| < 2^31 - 2.
constexpr int32_t CSENT = INT32_MIN;
constexpr int64_t CX_LIM = (int64_t(1) << 29) - 1;  // largest |v| kept
constexpr int64_t CK_LIM = (int64_t(1) << 30) - 1;  // largest |med2 - 2 * base|
struct CxRange {
  int64_t lo, hi;  // the cells that fit
  __device__ explicit CxRange(int64_t base)
      : lo(base > INT64_MIN + CX_LIM ? base - CX_LIM : INT64_MIN),
        hi(base < INT64_MAX - CX_LIM ? base + CX_LIM : INT64_MAX) {}
  __device__ int32_t put(int64_t x, int64_t base) const {
    return (x >= lo && x <= hi) ? (int32_t)(x - base) : CSENT;
  }
};

// The MAD pass's counts on the 32-bit copy (the half's flag clear): key =
// |2v - K| with K = med2 - 2 * base, in [0, 2^31 - 3]; the bracket ends are
// clamped to [-1, INT32_MAX], which changes no comparison with such keys.
// Same counts, sums and interior cells as RmCol<true, false>.
struct RmMad32 {
  int32_t K = 0, a = 0, b = 0;
  bool bneq = false;
  int32_t n = 0, cl = 0, cea = 0, ceb = 0, cm = 0, qn = 0;
  int64_t sd = 0;
  uint32_t q[RQ];
  __device__ void set(int64_t a64, int64_t b64, int64_t k64) {
    auto clamp = [](int64_t x) { return (int32_t)(x < -1 ? -1 : (x > INT32_MAX ? INT32_MAX : x)); };
    a = clamp(a64);
    b = clamp(b64);
    bneq = a64 != b64;
    K = (int32_t)k64;
  }
  __device__ __forceinline__ void cell(int32_t v, bool ok) {
    const int32_t d = 2 * v - K;
    const int32_t key = d < 0 ? -d : d;
    sd += ok ? key : 0;
    cl += (ok && key < a) ? 1 : 0;
    cea += (ok && key == a) ? 1 : 0;
    ceb += (ok && key == b && bneq) ? 1 : 0;
    const bool in = ok && key > a && key < b;
#pragma unroll
    for (int e = RQ - 1; e > 0; e--) q[e] = in ? q[e - 1] : q[e];
    q[0] = in ? (uint32_t)key : q[0];
    qn += in ? 1 : 0;
  }
  __device__ __forceinline__ void drain(int64_t *__restrict__ slot) {
#pragma unroll
    for (int e = 0; e < RQ; e++)
      if (e < qn && cm + e < SCAP) slot[cm + e] = (int64_t)q[e];
    cm += qn;
    qn = 0;
  }
  __device__ __forceinline__ void flush(int64_t p, RmPart pp, ColPartials, int64_t *__restrict__ slot) {
    drain(slot);
    pp.cl[p] = cl;
    pp.cea[p] = cea;
    pp.ceb[p] = ceb;
    pp.cm[p] = cm;
    pp.sd[p] = sd;
  }
};

// Counts and compaction of one column's cells against its bracket.  Interior
// cells are buffered in registers (newest first, qn of them) and written out
// when the wave flushes: after any row in which some lane's buffer filled up,
// every lane writes what it holds (so a store instruction carries many lanes,
// not the one lane whose buffer happened to fill).  The order of the cells in
// a slot does not matter to the selection.  A cell is counted when `ok`, with
// selects rather than branches, so the row loads around it stay in one block.
template <bool MAD, bool STATS>
struct RmCol {
  int64_t a, b, m;
  int32_t n = 0, cl = 0, cea = 0, ceb = 0, cm = 0, qn = 0;
  int64_t sd = 0, s1 = 0, mn = INT64_MAX, mx = INT64_MIN;
  u128 s2 = 0;
  int64_t q[RQ];
  __device__ __forceinline__ void cell(int64_t x, bool ok) {
    int64_t key = x;
    if (MAD) {
      const int64_t d = 2 * x - m;
      key = d < 0 ? -d : d;
      sd += ok ? key : 0;
    }
    n += ok ? 1 : 0;
    cl += (ok && key < a) ? 1 : 0;
    cea += (ok && key == a) ? 1 : 0;
    ceb += (ok && key == b && b != a) ? 1 : 0;
    if (STATS && ok) {
      s1 += x;
      // the square: one 32 x 32 -> 64-bit product when |x| < 2^32 (times
      // below 4.3 s), the full 128-bit one otherwise
      const uint64_t ax = (uint64_t)(x < 0 ? -x : x);
      if ((ax >> 32) == 0)
        s2 += (u128)((uint64_t)(uint32_t)ax * (uint64_t)(uint32_t)ax);
      else
        s2 += (u128)((i128)x * x);
      mn = x < mn ? x : mn;
      mx = x > mx ? x : mx;
    }
    const bool in = ok && key > a && key < b;
#pragma unroll
    for (int e = RQ - 1; e > 0; e--) q[e] = in ? q[e - 1] : q[e];
    q[0] = in ? key : q[0];
    qn += in ? 1 : 0;
  }
  // Writes the buffered cells at slot[cm ..); every lane of the wave calls it
  // together.
  __device__ __forceinline__ void drain(int64_t *__restrict__ slot) {
#pragma unroll
    for (int e = 0; e < RQ; e++)
      if (e < qn && cm + e < SCAP) slot[cm + e] = q[e];
    cm += qn;
    qn = 0;
  }
  // the buffered remainder, then the counts
  __device__ __forceinline__ void flush(int64_t p, RmPart pp, ColPartials ps, int64_t *__restrict__ slot) {
    drain(slot);
    if (!MAD) pp.n[p] = n;
    pp.cl[p] = cl;
    pp.cea[p] = cea;
    pp.ceb[p] = ceb;
    pp.cm[p] = cm;
    if (MAD) pp.sd[p] = sd;
    if (STATS) {
      ps.n[p] = n;
      ps.s1[p] = s1;
      ps.lo[p] = (uint64_t)s2;
      ps.hi[p] = (uint64_t)(s2 >> 64);
      ps.mn[p] = mn;
      ps.mx[p] = mx;
    }
  }
};

template <bool S32>
struct RmRow {
  typedef v2ll T;  // two int64 cells
};
template <>
struct RmRow<true> {
  typedef v2i T;  // two cells of the 32-bit copy
};
template <bool MAD, bool STATS, bool S32>
struct RmColOf {
  typedef RmCol<MAD, STATS> T;
};
template <>
struct RmColOf<true, false, true> {
  typedef RmMad32 T;
};
template <bool S32>
struct RmCell {
  typedef long long T;
};
template <>
struct RmCell<true> {
  typedef int T;
};

// One streaming pass over the row-major tensor: a thread owns CPL adjacent
// columns (two: 16-byte loads when the row length is even, a wave reads 1 KB
// of a row; one: half the registers, so more waves) and walks the RCH ranks of
// chunk blockIdx.y, RPU rows in flight, counting in registers; the bracket
// interior of each (chunk, column) goes to its own slot of SCAP cells (no
// atomics; cells past SCAP are counted, not stored).  The median pass also
// writes the 32-bit copy of every cell it reads (cx, offsets from its bracket's
// low end) and sets its column half's flag *esc when a valid cell did not fit
// (the median selection sets it too when a column's MAD keys would not fit 32
// bits); the MAD pass then reads the copy with 32-bit keys (S32, half the
// bytes), or the int64 tensor when *esc is set: both forms are launched and
// the one that does not apply returns at once (one loop per kernel, so no load
// sits in a branch inside it).  No LDS and no barriers.  Rows past the chunk's
// end load its last row (in bounds) and are not counted.
template <bool MAD, bool STATS, bool VEC, int CPL, bool S32>
__global__ __launch_bounds__(256) void rm_pass(const int64_t *__restrict__ T, int64_t R, int IG, int G,
                                               const int32_t *it, int c_lo, int c_hi, RmBr br,
                                               int64_t *__restrict__ scr, RmPart pp, ColPartials ps,
                                               int32_t *__restrict__ cx, const int64_t *__restrict__ cbase,
                                               int32_t *esc) {
  static_assert(MAD || !S32, "the median pass reads the int64 tensor");
  static_assert(!(S32 && STATS), "the MAD pass takes no imbalance partials");
  if (MAD && (*esc == 0) != S32) return;
  const int ca = c_lo + ((int)blockIdx.x * 256 + (int)threadIdx.x) * CPL;
  if (ca >= c_hi) return;
  const int64_t ng = gridDim.y, ch = blockIdx.y;
  const bool two = CPL == 2 && ca + 1 < c_hi;
  const int ia = ca / G, ib = (ca + 1) / G;
  typename RmColOf<MAD, STATS, S32>::T c0, c1;
  if constexpr (MAD && S32) {
    // K = med2 - 2 * base (in range: the half's flag is clear)
    auto kof = [&](int c) { return (int64_t)((uint64_t)br.med2[c] - 2 * (uint64_t)cbase[c]); };
    c0.set(br.a[ca], br.b[ca], kof(ca));
    if (two)
      c1.set(br.a[ca + 1], br.b[ca + 1], kof(ca + 1));
    else
      c1.set(INT64_MAX, INT64_MIN, 0);
  } else {
    c0.a = br.a[ca];
    c0.b = br.b[ca];
    c0.m = MAD ? br.med2[ca] : 0;
    c1.a = two ? br.a[ca + 1] : INT64_MAX;
    c1.b = two ? br.b[ca + 1] : INT64_MIN;
    c1.m = (MAD && two) ? br.med2[ca + 1] : 0;
  }
  int64_t *slot0 = scr + ((int64_t)ca * ng + ch) * SCAP;
  int64_t *slot1 = scr + ((int64_t)(ca + 1) * ng + ch) * SCAP;
  const int64_t rb = ch * RCH, re = rb + RCH < R ? rb + RCH : R, last = re - 1;
  const int cb = two ? ca + 1 : ca;
  // the median pass: the copy's base per column (column cb is column ca again
  // without a second)
  const int64_t b0 = MAD ? 0 : (int64_t)c0.a;
  const int64_t b1 = MAD ? 0 : (two ? (int64_t)c1.a : (int64_t)c0.a);
  bool escaped = false;
  {
    typedef typename RmRow<S32>::T Row;
    const CxRange f0(b0), f1(b1);
    auto load_row = [&](int64_t r) -> Row {
      const int64_t rr = r < re ? r : last;
      if constexpr (S32) {
        const int32_t *row = cx + rr * IG;
        if (CPL == 1) return v2i{__builtin_nontemporal_load(row + ca), 0};
        if (VEC) return __builtin_nontemporal_load(reinterpret_cast<const v2i *>(row + ca));
        return v2i{__builtin_nontemporal_load(row + ca), __builtin_nontemporal_load(row + cb)};
      } else {
        const int64_t *row = T + rr * IG;
        if (CPL == 1) return v2ll{__builtin_nontemporal_load(row + ca), SENT};
        if (VEC) return __builtin_nontemporal_load(reinterpret_cast<const v2ll *>(row + ca));
        return v2ll{__builtin_nontemporal_load(row + ca), __builtin_nontemporal_load(row + cb)};
      }
    };
    // RPU rows in flight: the register of a row, once counted, loads the row
    // RPU further on (so the loads stay in flight while the counting runs)
    Row v[RPU];
#pragma unroll
    for (int u = 0; u < RPU; u++) v[u] = load_row(rb + u);
    for (int64_t r0 = rb; r0 < re; r0 += RPU) {
      int nit[RPU];
#pragma unroll
      for (int u = 0; u < RPU; u++) nit[u] = it ? it[r0 + u < re ? r0 + u : last] : 0x7fffffff;
#pragma unroll
      for (int u = 0; u < RPU; u++) {
        const bool rv = r0 + u < re;
        const bool ok0 = rv && ia < nit[u], ok1 = rv && two && ib < nit[u];
        int64_t x0 = 0, x1 = 0;
        if constexpr (!S32) {
          x0 = (int64_t)v[u].x;
          x1 = (int64_t)v[u].y;
        }
        if constexpr (!MAD) {
          // a row past the chunk's end rewrites the last row's copy with its
          // own values (no branch around the store)
          int32_t *crow = cx + (rv ? r0 + u : last) * IG;
          const int32_t y0 = f0.put(x0, b0);
          escaped |= ok0 && y0 == CSENT;
          if (CPL == 1) {
            __builtin_nontemporal_store(y0, crow + ca);
          } else {
            const int32_t y1 = f1.put(x1, b1);
            escaped |= ok1 && y1 == CSENT;
            if (VEC)
              __builtin_nontemporal_store(v2i{y0, y1}, reinterpret_cast<v2i *>(crow + ca));
            else {
              __builtin_nontemporal_store(y0, crow + ca);
              __builtin_nontemporal_store(y1, crow + cb);
            }
          }
        }
        if constexpr (S32) {
          c0.cell(v[u].x, ok0);
          c1.cell(v[u].y, ok1);
        } else {
          c0.cell(x0, ok0);
          c1.cell(x1, ok1);
        }
        v[u] = load_row(r0 + u + RPU);
        // a row adds at most one cell per column: drain the whole wave as
        // soon as one buffer is full
        if (__ballot(c0.qn == RQ || c1.qn == RQ)) {
          c0.drain(slot0);
          c1.drain(slot1);
        }
      }
    }
  }
  if (!MAD && escaped) *esc = 1;
  c0.flush(ch * IG + ca, pp, ps, slot0);
  if (two) c1.flush(ch * IG + ca + 1, pp, ps, slot1);
}

// Column c of the row-major tensor into slot[0..Rp) (SENT for cells of missing
// iterations and padding); returns the column's min and max over valid cells.
__device__ void gather_column(const int64_t *__restrict__ T, int64_t R, int IG, int G, const int32_t *it,
                              int c, int64_t *__restrict__ slot, SelLds &L, int64_t &mn, int64_t &mx) {
  constexpr int U = 8;
  const int64_t Rp = pad_ranks(R);
  const int i = c / G;
  int64_t mnl = INT64_MAX, mxl = INT64_MIN;
  for (int64_t r0 = 0; r0 < Rp; r0 += (int64_t)CS * U) {
    int64_t v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t r = r0 + (int64_t)u * CS + threadIdx.x;
      v[u] = SENT;
      if (r < R && (it ? it[r] : 0x7fffffff) > i) v[u] = T[r * IG + c];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t r = r0 + (int64_t)u * CS + threadIdx.x;
      if (r < Rp) slot[r] = v[u];
      if (v[u] != SENT) {
        mnl = v[u] < mnl ? v[u] : mnl;
        mxl = v[u] > mxl ? v[u] : mxl;
      }
    }
  }
  int64_t none[1] = {0};
  mn = mnl;
  mx = mxl;
  block_stats<1, true>(none, mn, mx, L.red);  // its barriers also order the slot writes
}

struct RmOut {
  int64_t *da, *db;  // MAD brackets, written by the median step
};

// Per column (persistent grid, a gather slot of Rp cells per workgroup).
constexpr int SU = 4;  // chunk slots read together by a wave

template <bool MAD>
__global__ __launch_bounds__(CS, SEL_WGS_PER_CU) void rm_select(
    const int64_t *__restrict__ T, int64_t R, int IG, int G, const int32_t *it,
    const int64_t *__restrict__ smp, int ng, int c_lo, int c_hi, RmPart pp, RmBr br,
    const int64_t *__restrict__ scr, int64_t *__restrict__ slots, RmOut ro, ColSel out, int32_t *esc) {
  __shared__ ColSelLds L;
  __shared__ int32_t segn[SEG_MAX];
  const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
  const int64_t Rp = pad_ranks(R);
  int64_t *slot = slots + (int64_t)blockIdx.x * Rp;
  for (int j = t; j < NHC * NB; j += CS) (&L.hist[0][0])[j] = 0;
  for (int c = c_lo + (int)blockIdx.x; c < c_hi; c += gridDim.x) {
    // the chunk partials, summed; the chunk slots' fill counts into LDS
    int64_t sums[6] = {0, 0, 0, 0, 0, 0};
    for (int g = t; g < ng; g += CS) {
      const int64_t p = (int64_t)g * IG + c;
      sums[0] += MAD ? pp.sd[p] : pp.n[p];
      sums[1] += pp.cl[p];
      sums[2] += pp.cea[p];
      sums[3] += pp.ceb[p];
      const int32_t cm = pp.cm[p];
      sums[4] += cm;
      sums[5] += cm > SCAP ? 1 : 0;  // a slot that could not hold its chunk's interior
      segn[g] = cm;
    }
    int64_t u0 = 0, u1 = 0;
    block_stats<6, false>(sums, u0, u1, L.red);  // its barriers publish segn
    const int64_t clo = sums[1], ceqa = sums[2], ceqb = sums[3], cmid = sums[4];
    const bool full = sums[5] > 0;
    const int64_t qa = br.a[c], qb = br.b[c];
    const int64_t n = MAD ? out.n[c] : sums[0];
    // the interior cells: wave wv reads chunk slots wv, wv + CWV, ..., SU of
    // them (two cells per lane each) per round trip
    const int64_t *colscr = scr + (int64_t)c * ng * SCAP;
    auto vscr = [&](auto &&f) {
      for (int g0 = wv; g0 < ng; g0 += CWV * SU) {
        int64_t v0[SU], v1[SU];
        int cn[SU];
#pragma unroll
        for (int u = 0; u < SU; u++) {
          const int g = g0 + u * CWV;
          cn[u] = g < ng ? segn[g] : 0;
          const int64_t *sp = colscr + (int64_t)g * SCAP;
          v0[u] = ln < cn[u] ? sp[ln] : 0;
          v1[u] = ln + 64 < cn[u] ? sp[ln + 64] : 0;
        }
#pragma unroll
        for (int u = 0; u < SU; u++) {
          if (ln < cn[u]) f(v0[u]);
          if (ln + 64 < cn[u]) f(v1[u]);
          if (cn[u] > 128) {
            const int64_t *sp = colscr + (int64_t)(g0 + u * CWV) * SCAP;
            for (int e = ln + 128; e < cn[u]; e += 64) f(sp[e]);
          }
        }
      }
    };
    auto vslot = [&](auto &&f) {
      sweep(slot, Rp, [&](int64_t x) {
        if (x != SENT) f(x);
      });
    };
    if (n == 0) {
      if (t == 0) {
        if (!MAD) {
          out.med2[c] = 0;
          out.n[c] = 0;
          ro.da[c] = INT64_MAX;  // empty bracket: the MAD pass compacts nothing
          ro.db[c] = INT64_MIN;
        } else {
          out.mad4[c] = 0;
          out.sumdev[c] = 0;
          out.zc[c] = 0.0;
          out.zd[c] = 1.0;
        }
      }
      __syncthreads();
      continue;
    }
    const int64_t k = (n - 1) / 2;
    const bool even = (n & 1) == 0;
    int64_t x1, x2;
    if (!MAD) {
      if (full || !bracket_pick(vscr, clo, ceqa, cmid, ceqb, qa, qb, INT64_MAX, k, even, L, x1, x2)) {
        int64_t mn, mx;
        gather_column(T, R, IG, G, it, c, slot, L, mn, mx);
        uint64_t a1, a2;
        radix_select(vslot, k, even, nbits64((uint64_t)mx - (uint64_t)mn),
                     [&](int64_t x) { return (uint64_t)x - (uint64_t)mn; }, L, a1, a2);
        x1 = (int64_t)((uint64_t)mn + a1);
        x2 = (int64_t)((uint64_t)mn + a2);
      }
      const int64_t med2 = x1 + x2;
      __syncthreads();  // the sample slots are rewritten below
      const int m = load_sample<true>(L, smp + (int64_t)c * MS, med2);
      int64_t da, db;
      sample_bracket(L, m, da, db);
      if (t == 0) {
        out.med2[c] = med2;
        out.n[c] = n;
        ro.da[c] = da;
        ro.db[c] = db;
        // the MAD pass's 32-bit keys need |med2 - 2 * base| <= CK_LIM (base:
        // the copy's base, the median bracket's low end)
        const i128 k = (i128)med2 - 2 * (i128)qa;
        if (k > CK_LIM || k < -CK_LIM) *esc = 1;
      }
    } else {
      const int64_t med2 = br.med2[c];
      if (full || !bracket_pick(vscr, clo, ceqa, cmid, ceqb, qa, qb, INT64_MAX, k, even, L, x1, x2)) {
        int64_t mn, mx;
        gather_column(T, R, IG, G, it, c, slot, L, mn, mx);
        const uint64_t dlo = (uint64_t)(med2 - 2 * mn), dhi = (uint64_t)(2 * mx - med2);
        const uint64_t dmax = dlo > dhi ? dlo : dhi;
        uint64_t a1, a2;
        radix_select(vslot, k, even, nbits64(dmax),
                     [&](int64_t x) {
                       const int64_t d = 2 * x - med2;
                       return (uint64_t)(d < 0 ? -d : d);
                     },
                     L, a1, a2);
        x1 = (int64_t)a1;
        x2 = (int64_t)a2;
      }
      if (t == 0) {
        out.mad4[c] = x1 + x2;
        out.sumdev[c] = sums[0];
        z_coefs(x1 + x2, sums[0], n, out.zc[c], out.zd[c]);
      }
    }
    __syncthreads();
  }
}

// m(r,g) = (1/n_r) sum_{i < n_r} z(r,i,g) (ascending i) from the median
// pass's 32-bit copy of the row-major tensor (the int64 cell where the copy
// holds CSENT), written [G][R]; a wave = SRW consecutive ranks x 64 regions
// (lane = region), so each row read is contiguous and the column parameters
// are read once per SRW ranks.  One launch adds the iterations [i_lo, i_hi): a launch
// with i_lo > 0 continues the running sums that the previous one left in m_t
// (the same additions in the same order), and the launch that reaches I
// divides by n_r.
constexpr int SRW = 8;

template <bool S32>
__global__ __launch_bounds__(256) void score_rows(const int64_t *__restrict__ T,
                                                  const int32_t *__restrict__ cx,
                                                  const int64_t *__restrict__ cxb, const int32_t *esc,
                                                  int64_t R, int I, int G, const int32_t *it, int i_lo,
                                                  int i_hi, ColSel cs, double *m_t) {
  // both forms are launched and one applies (without the flag: the int64 form)
  if (esc ? (*esc == 0) != S32 : S32) return;
  const int lane = threadIdx.x & 63;
  const int gbn = (G + 63) / 64;
  const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = (wave / gbn) * SRW;
  if (r0 >= R) return;
  const int g = (int)(wave % gbn) * 64 + lane;
  const bool gl = g < G;
  const int64_t IG = (int64_t)I * G;
  int ni[SRW];
  int nmax = 0;
#pragma unroll
  for (int q = 0; q < SRW; q++) {
    int v = 0;
    if (r0 + q < R) {
      v = it ? it[r0 + q] : I;
      v = v > I ? I : (v < 0 ? 0 : v);
    }
    ni[q] = v;
    nmax = v > nmax ? v : nmax;
  }
  double acc[SRW];
#pragma unroll
  for (int q = 0; q < SRW; q++) acc[q] = (i_lo > 0 && gl && r0 + q < R) ? m_t[(int64_t)g * R + r0 + q] : 0.0;
  const int gg = gl ? g : 0;
  const int ie = nmax < i_hi ? nmax : i_hi;
  // iteration i's cells and column parameters; those of i + 1 are loaded
  // before i is scored.  The cells come from the 32-bit copy (S32) unless
  // some valid cell did not fit in it (then from the int64 tensor).
  {
    typedef typename RmCell<S32>::T Cell;
    const Cell *base = S32 ? (const Cell *)(const void *)(cx + r0 * IG + gg)
                           : (const Cell *)(const void *)(T + r0 * IG + gg);
    Cell x[SRW];
    int64_t med2 = 0, cb = 0;
    double zc = 0.0, zd = 1.0;
    auto load = [&](int i) {
#pragma unroll
      for (int q = 0; q < SRW; q++)
        x[q] = i < ni[q] ? __builtin_nontemporal_load(base + q * IG + (int64_t)i * G) : 0;
      const int64_t c = (int64_t)i * G + gg;
      med2 = cs.med2[c];
      if (S32) cb = cxb[c];
      zc = cs.zc[c];
      zd = cs.zd[c];
    };
    if (i_lo < ie) load(i_lo);
    for (int i = i_lo; i < ie; i++) {
      Cell xc[SRW];
#pragma unroll
      for (int q = 0; q < SRW; q++) xc[q] = x[q];
      const int64_t m2 = med2, b = cb;
      const double a = zc, d = zd;
      if (i + 1 < ie) load(i + 1);
#pragma unroll
      for (int q = 0; q < SRW; q++)
        if (i < ni[q]) acc[q] += ((double)(2 * (b + (int64_t)xc[q]) - m2) * a) / d;
    }
  }
  if (gl) {
    const bool fin = i_hi >= I;
#pragma unroll
    for (int q = 0; q < SRW; q++)
      if (r0 + q < R) m_t[(int64_t)g * R + r0 + q] = !fin ? acc[q] : (ni[q] > 0 ? acc[q] / (double)ni[q] : 0.0);
  }
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
constexpr int SU2 = 8;  // keys in flight per thread in the stage-2 selection

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
    // SU2 keys per thread per round trip; a wave whose hits share one bin
    // adds them with one LDS atomic (the rule in the leading passes)
    for (int64_t r0 = tid; r0 < R; r0 += (int64_t)RT * SU2) {
      uint64_t kv[SU2];
      bool ok[SU2];
#pragma unroll
      for (int u = 0; u < SU2; u++) {
        const int64_t r = r0 + (int64_t)u * RT;
        ok[u] = r < R && rank_active(it, I, r);
        kv[u] = r < R ? keyf(r) : 0;
      }
#pragma unroll
      for (int u = 0; u < SU2; u++) {
        const uint64_t key = kv[u];
        const uint64_t ks = key >> sh;
        const uint64_t hk = ks >> 8;
        const bool hit = ok[u] && hk == pref;
        const uint32_t bin = (uint32_t)(ks & 255);
        const uint64_t hm = __ballot(hit);
        if (hm) {
          const int lead = __ffsll((long long)hm) - 1;
          const uint32_t b0 = (uint32_t)__shfl((int)bin, lead, 64);
          if (__ballot(hit && bin == b0) == hm) {
            if (lane == lead) atomicAdd(&hist[wid][b0], (uint32_t)__popcll(hm));
          } else if (hit) {
            atomicAdd(&hist[wid][bin], 1u);
          }
        }
        if (ok[u] && last && hk > pref) mgt = key < mgt ? key : mgt;
      }
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

// Stage-2 selection by bracket, for regions of at least S2_MIN_N active ranks:
// the keys of S2S evenly spaced ranks give a bracket [lo, hi] of +-BRACKET_SE
// standard errors around the sample median (as in the first stage); one pass
// over the region counts the keys below lo and equal to either end and
// compacts those strictly inside into LDS, where the selection finishes.  A
// wanted rank outside the bracket, or an interior larger than the LDS buffer,
// returns false and the caller runs the whole-region radix passes instead, so
// the result is the same exact order statistic either way (two passes over
// the region instead of eight).
constexpr int S2S = 4096;              // sample keys
constexpr int S2CAP = 14336;           // interior keys held in LDS (112 KB)
constexpr int64_t S2_MIN_N = 16384;    // fewer active ranks: radix passes only
constexpr size_t S2_LDS_BYTES = (size_t)S2CAP * sizeof(uint64_t);

// Appends v to buf (LDS) when `in`; all lanes of the wave call it together.
// The counter keeps counting past cap (the caller detects the overflow).
__device__ inline void wave_push(bool in, uint64_t v, uint32_t *counter, uint64_t *buf, int cap) {
  const uint64_t m = __ballot(in);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, leader, 64);
  const uint32_t pos = base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
  if (in && pos < (uint32_t)cap) buf[pos] = v;
}

// Block-wide (RT threads) sums of three counters, returned to every thread.
__device__ inline void block_sum3(int64_t &a, int64_t &b, int64_t &c, int64_t *slots) {
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
    c += __shfl_xor(c, d, 64);
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    slots[3 * wid] = a;
    slots[3 * wid + 1] = b;
    slots[3 * wid + 2] = c;
  }
  __syncthreads();
  a = b = c = 0;
  for (int w = 0; w < RW; w++) {
    a += slots[3 * w];
    b += slots[3 * w + 1];
    c += slots[3 * w + 2];
  }
  __syncthreads();
}

// Block-wide minimum and maximum, returned to every thread.
__device__ inline void block_minmax_u64(uint64_t &mn, uint64_t &mx, uint64_t *slots) {
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t a = __shfl_xor(mn, d, 64), b = __shfl_xor(mx, d, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    slots[2 * wid] = mn;
    slots[2 * wid + 1] = mx;
  }
  __syncthreads();
  for (int w = 0; w < RW; w++) {
    mn = slots[2 * w] < mn ? slots[2 * w] : mn;
    mx = slots[2 * w + 1] > mx ? slots[2 * w + 1] : mx;
  }
  __syncthreads();
}

// The k-th smallest (k from 0) of the cnt keys buf[0 .. cnt) in LDS, all in
// [base, base + 2^bits), and with want_next also the (k+1)-th, which must
// exist.  8-bit digits, a histogram per wave; st holds at least 4 + RW words.
// hist is zero on entry and on return.
__device__ void lds_select(const uint64_t *buf, int cnt, uint64_t base, int bits, int64_t k,
                           bool want_next, uint32_t (*hist)[256], uint32_t *tot, uint64_t *st,
                           uint64_t &v1, uint64_t &v2) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  uint64_t pref = 0, r1 = 0, r2 = 0;
  int hi = bits;
  while (hi > 0) {
    const int w = hi < 8 ? hi : 8;
    const int lo = hi - w;
    const bool last = lo == 0;
    const uint32_t mask = (1u << w) - 1;
    uint64_t mgt = ~0ull;  // smallest key above the prefix group (last digit)
    for (int i = tid; i < cnt; i += RT) {
      const uint64_t rel = buf[i] - base;
      const uint64_t top = shr64(rel, hi);
      if (top == pref)
        atomicAdd(&hist[wid][(uint32_t)(rel >> lo) & mask], 1u);
      else if (last && top > pref && rel < mgt)
        mgt = rel;
    }
    if (last && want_next) {
      for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(mgt, d, 64);
        mgt = o < mgt ? o : mgt;
      }
      if (lane == 0) st[4 + wid] = mgt;
    }
    __syncthreads();
    if (tid < 256) {
      uint32_t c = 0;
      for (int q = 0; q < RW; q++) {
        c += hist[q][tid];
        hist[q][tid] = 0;
      }
      tot[tid] = c;
    }
    __syncthreads();
    if (wid == 0) {
      // lane owns bins 4 lane .. 4 lane + 3
      uint32_t c[4];
      int64_t own = 0;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        c[j] = tot[4 * lane + j];
        own += c[j];
      }
      int64_t incl = own;
      for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
      }
      const int64_t excl = incl - own;
      const bool mine = excl <= k && k < excl + own;
      int b = 0, same = 0;
      int64_t kk = 0;
      if (mine) {
        int64_t cum = excl;
        int j = 0;
        for (; j < 3; j++) {
          if (cum + (int64_t)c[j] > k) break;
          cum += c[j];
        }
        b = 4 * lane + j;
        kk = k - cum;
        same = kk + 1 < (int64_t)c[j] ? 1 : 0;
      }
      const int owner = __ffsll((long long)__ballot(mine)) - 1;
      b = __shfl(b, owner, 64);
      kk = __shfl(kk, owner, 64);
      same = __shfl(same, owner, 64);
      uint32_t nxt = 0xffffffffu;  // smallest non-empty bin above b
      if (last && want_next && !same) {
#pragma unroll
        for (int j = 3; j >= 0; j--)
          if (4 * lane + j > b && c[j] > 0) nxt = (uint32_t)(4 * lane + j);
        for (int d = 32; d >= 1; d >>= 1) {
          const uint32_t o = (uint32_t)__shfl_xor((int)nxt, d, 64);
          nxt = o < nxt ? o : nxt;
        }
      }
      if (lane == 0) {
        st[0] = (pref << w) | (uint64_t)b;
        st[1] = (uint64_t)kk;
        st[2] = (uint64_t)same;
        st[3] = nxt;
      }
    }
    __syncthreads();
    const uint64_t np = st[0];
    const int64_t kn = (int64_t)st[1];
    if (last) {
      r1 = np;
      if (!want_next || st[2]) {
        r2 = np;
      } else if (st[3] != 0xffffffffu) {
        r2 = (pref << w) | st[3];
      } else {
        uint64_t mg = ~0ull;
        for (int q = 0; q < RW; q++) mg = st[4 + q] < mg ? st[4 + q] : mg;
        r2 = mg;
      }
    }
    pref = np;
    k = kn;
    hi = lo;
    __syncthreads();  // st is rewritten by the next digit
  }
  v1 = base + r1;
  v2 = base + (want_next ? r2 : r1);
}

// Order statistics (n-1)/2 and, for even n, n/2 of the keys keyf(r) over the
// active ranks (block_select's contract) through a bracket; false when the
// bracket misses or overflows (nothing written to v1, v2).
template <class KeyF>
__device__ bool bracket_select(int64_t R, const int32_t *it, int I, int64_t n, KeyF keyf,
                               uint64_t *buf, uint32_t (*hist)[256], uint32_t *tot, uint64_t *st,
                               int64_t *slots, uint32_t *counter, uint64_t &v1, uint64_t &v2) {
  const int tid = threadIdx.x;
  if (tid == 0) *counter = 0;
  __syncthreads();
  {
    constexpr int U = S2S / RT;
    uint64_t kv[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t j = (int64_t)u * RT + tid;
      const int64_t r = ((2 * j + 1) * R) / (2 * S2S);
      ok[u] = rank_active(it, I, r);
      kv[u] = keyf(r);
    }
#pragma unroll
    for (int u = 0; u < U; u++) wave_push(ok[u], kv[u], counter, buf, S2S);
  }
  __syncthreads();
  const int m = (int)*counter;
  if (m < 256) return false;
  uint64_t mn = ~0ull, mx = 0;
  for (int j = tid; j < m; j += RT) {
    mn = buf[j] < mn ? buf[j] : mn;
    mx = buf[j] > mx ? buf[j] : mx;
  }
  block_minmax_u64(mn, mx, reinterpret_cast<uint64_t *>(slots));
  const int sbits = nbits64(mx - mn);
  const double dl = 0.5 * BRACKET_SE / sqrt((double)m);
  const double ca = (0.5 - dl) * (double)(m - 1), cb = (0.5 + dl) * (double)(m - 1);
  const int ia = ca <= 0.0 ? 0 : (int)floor(ca);
  const int ib = cb >= (double)(m - 1) ? m - 1 : (int)ceil(cb);
  uint64_t lo, hi;
  lds_select(buf, m, mn, sbits, ia, ib == ia + 1, hist, tot, st, lo, hi);
  if (ib > ia + 1) lds_select(buf, m, mn, sbits, ib, false, hist, tot, st, hi, hi);
  else if (ib == ia) hi = lo;
  // buf now takes the interior
  if (tid == 0) *counter = 0;
  __syncthreads();
  int64_t clo = 0, ceqa = 0, ceqb = 0;
  for (int64_t r0 = tid; r0 < R; r0 += (int64_t)RT * SU2) {
    uint64_t kv[SU2];
    bool ok[SU2];
#pragma unroll
    for (int u = 0; u < SU2; u++) {
      const int64_t r = r0 + (int64_t)u * RT;
      ok[u] = r < R && rank_active(it, I, r);
      kv[u] = r < R ? keyf(r) : 0;
    }
#pragma unroll
    for (int u = 0; u < SU2; u++) {
      const uint64_t key = kv[u];
      clo += (ok[u] && key < lo) ? 1 : 0;
      ceqa += (ok[u] && key == lo) ? 1 : 0;
      ceqb += (ok[u] && key == hi && hi != lo) ? 1 : 0;
      wave_push(ok[u] && key > lo && key < hi, key, counter, buf, S2CAP);
    }
  }
  block_sum3(clo, ceqa, ceqb, slots);
  const int64_t cmid = (int64_t)*counter;
  __syncthreads();  // every thread has read the counter
  const int64_t k = (n - 1) / 2;
  const bool even = (n & 1) == 0;
  auto where = [&](int64_t j) -> int {
    if (j < clo) return 0;
    j -= clo;
    if (j < ceqa) return 1;
    j -= ceqa;
    if (j < cmid) return 2;
    j -= cmid;
    return j < ceqb ? 3 : 0;
  };
  const int w1 = where(k), w2 = even ? where(k + 1) : w1;
  if (w1 == 0 || w2 == 0) return false;
  if ((w1 == 2 || w2 == 2) && cmid > S2CAP) return false;
  const int64_t base = clo + ceqa;
  const int ibits = nbits64(hi - lo);
  uint64_t a1 = 0, a2 = 0;
  if (w1 == 2 && w2 == 2) {
    lds_select(buf, (int)cmid, lo, ibits, k - base, even, hist, tot, st, a1, a2);
    v1 = a1;
    v2 = even ? a2 : a1;
    return true;
  }
  if (w1 == 2) lds_select(buf, (int)cmid, lo, ibits, k - base, false, hist, tot, st, a1, a1);
  v1 = w1 == 2 ? a1 : (w1 == 1 ? lo : hi);
  if (!even) {
    v2 = v1;
    return true;
  }
  if (w2 == 2) lds_select(buf, (int)cmid, lo, ibits, k + 1 - base, false, hist, tot, st, a2, a2);
  v2 = w2 == 2 ? a2 : (w2 == 1 ? lo : hi);
  return true;
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
  __shared__ int64_t xacc[RW * XL];
  __shared__ uint32_t xbad;
  __shared__ uint64_t st2[4 + RW];
  __shared__ uint32_t s2cnt;
  extern __shared__ uint64_t s2buf[];  // S2_LDS_BYTES, launched with MAD only
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  int64_t *xw = xacc + (tid >> 6) * XL;
  // exact sum over the active ranks of f(r), rounded once (FP64 stage)
  auto exact_sum = [&](auto f) {
    xsum_clear<RT>(xacc, &xbad);
    for (int64_t r0 = 0; r0 < R; r0 += RT) {
      const int64_t r = r0 + tid;
      const bool act = r < R && rank_active(it, I, r);
      xsum_add_wave(xw, act ? f(r) : 0.0, act, &xbad);
    }
    return xsum_block_result<RT>(xacc, &xbad, fb);
  };
  const double *vd = reinterpret_cast<const double *>(vals_t) + (int64_t)g * R;
  const int64_t *vi = reinterpret_cast<const int64_t *>(vals_t) + (int64_t)g * R;
  for (int k = tid; k < RW * 256; k += RT) (&hist[0][0])[k] = 0;

  int64_t n = 0;
  for (int64_t r = tid; r < R; r += RT) n += rank_active(it, I, r) ? 1 : 0;
  n = block_sum_i64<RT>(n, ib);
  // the middle order statistics: by bracket when the region is large enough,
  // else (or when the bracket misses) by radix passes over the region
  auto select = [&](auto keyf, uint64_t &a, uint64_t &b) {
    if (n >= S2_MIN_N &&
        bracket_select(R, it, I, n, keyf, s2buf, hist, tot, st2, ib, &s2cnt, a, b))
      return;
    block_select(R, it, I, n, keyf, hist, tot, sh_u64, a, b);
  };

  // Centre and scale.
  double med = 0.0, scale = 0.0;
  int64_t med2 = 0;
  int mode = 0;  // 1: MAD, 2: mean AD / plain std, 0: all z = 0
  if (n > 0) {
    if (MAD) {
      uint64_t a, b;
      if (F64) {
        select([&](int64_t r) { return key_f64(vd[r]); }, a, b);
        med = (n & 1) ? dec_f64(a) : 0.5 * (dec_f64(a) + dec_f64(b));
        select([&](int64_t r) { return key_f64(fabs(vd[r] - med)); }, a, b);
        const double mad = (n & 1) ? dec_f64(a) : 0.5 * (dec_f64(a) + dec_f64(b));
        if (mad > 0.0) {
          mode = 1;
          scale = 1.4826 * mad;
        } else {
          const double s = exact_sum([&](int64_t r) { return fabs(vd[r] - med); });
          const double mean_ad = s / (double)n;
          if (mean_ad > 0.0) {
            mode = 2;
            scale = 1.253314 * mean_ad;
          }
        }
      } else {
        select([&](int64_t r) { return (uint64_t)vi[r] ^ SIGN; }, a, b);
        med2 = (int64_t)(a ^ SIGN) + (int64_t)(b ^ SIGN);
        select(
            [&](int64_t r) {
              const int64_t d = 2 * vi[r] - med2;
              return (uint64_t)(d < 0 ? -d : d);
            },
            a, b);
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
        // mean = (exact sum, rounded) / n; std from the exact sum of the
        // rounded squared deviations (the same operations as the oracle)
        med = exact_sum([&](int64_t r) { return vd[r]; }) / (double)n;
        const double q = exact_sum([&](int64_t r) {
          const double d = vd[r] - med;
          return d * d;
        });
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

// Per-rank maximum |z| over regions as FP32 (ranks without iterations: 0).
__global__ __launch_bounds__(256) void rank_max_f32(const double *z_t, int64_t R, int G,
                                                    const int32_t *it, int I, float *score) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  double best = 0.0;
  if (rank_active(it, I, r))
    for (int g = 0; g < G; g++) {
      const double v = fabs(z_t[(int64_t)g * R + r]);
      if (v > best) best = v;
    }
  score[r] = (float)best;
}

struct OWs {
  int64_t *Tt;      // [IG][Rp] column-major copy of the tensor (FULL, short columns or z-score)
  int64_t *scr;     // row-major path: [IG][chunks][SCAP] bracket interiors per column and chunk;
                    // column-major bracket path: [min(IG, SEL_GRID_MAX)][sel_cap(R)]
  int64_t *smp;     // row-major path: [IG][MS] column samples
  int64_t *slots;   // row-major path: [min(IG, SEL_GRID_MAX)][Rp] gathered columns
  int32_t *cx;      // row-major path: [R][IG] the median pass's 32-bit copy of the tensor
  int32_t *esc;     // row-major path: [2] per column half, set when the copy does not serve
  int64_t *qa, *qb, *da, *db;  // row-major path: [IG] brackets
  RmPart rp;        // row-major path: [groups][IG] pass counts
  ColSel cs;
  ColMom cm;
  double *m_t;      // [G][R] doubles (FULL) -- also reused as z_t
  int64_t *S_t;     // [G][R] (TOTALS)
  double *z_t;      // [G][R]
  int64_t *part;    // [ceil(R/256)]
};

// The robust FULL scan over long columns runs on the row-major tensor.
inline bool row_major_path(int64_t R, int mode, int kind) {
  return mode == TA_SCAN_FULL && kind == TA_SCORE_MAD && pad_ranks(R) >= SEL_BRACKET_MIN_RP &&
         transpose_groups_of(R) <= SEG_MAX;
}

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
    if (row_major_path(R, mode, kind)) {
      const size_t ng = (size_t)transpose_groups_of(R);
      w.scr = (int64_t *)take(IG * ng * SCAP * 8);
      w.cx = (int32_t *)take((size_t)R * IG * 4);
      w.esc = (int32_t *)take(8);
      w.smp = (int64_t *)take(IG * MS * 8);
      w.slots = (int64_t *)take((size_t)std::min<size_t>(IG, SEL_GRID_MAX) * pad_ranks(R) * 8);
      w.qa = (int64_t *)take(IG * 8);
      w.qb = (int64_t *)take(IG * 8);
      w.da = (int64_t *)take(IG * 8);
      w.db = (int64_t *)take(IG * 8);
      w.rp.n = (int32_t *)take(ng * IG * 4);
      w.rp.cl = (int32_t *)take(ng * IG * 4);
      w.rp.cea = (int32_t *)take(ng * IG * 4);
      w.rp.ceb = (int32_t *)take(ng * IG * 4);
      w.rp.cm = (int32_t *)take(ng * IG * 4);
      w.rp.sd = (int64_t *)take(ng * IG * 8);
      w.cs.zc = (double *)take(IG * 8);
      w.cs.zd = (double *)take(IG * 8);
    } else {
      w.Tt = (int64_t *)take((size_t)pad_ranks(R) * IG * 8);
      if (kind == TA_SCORE_MAD && pad_ranks(R) >= SEL_BRACKET_MIN_RP)  // more than SEG_MAX chunks
        w.scr = (int64_t *)take((size_t)std::min<size_t>(IG, SEL_GRID_MAX) * sel_cap(R) * 8);
    }
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

// rm_pass over the columns [c_lo, c_hi) with CPL columns per lane (16-byte
// row loads for two columns when the row length and c_lo are even).
constexpr int RM_CPL_STATS = 1, RM_CPL_MAD = 2, RM_CPL_COUNT = 2;
template <bool MAD, bool STATS>
void launch_rm_pass(int ng, const OutArgs &a, int IG, int c_lo, int c_hi, RmBr br, const OWs &w,
                    int h, hipStream_t s) {
  constexpr int CPL = STATS ? RM_CPL_STATS : (MAD ? RM_CPL_MAD : RM_CPL_COUNT);
  const dim3 grid((unsigned)((c_hi - c_lo + 256 * CPL - 1) / (256 * CPL)), (unsigned)ng);
  const bool vec = CPL == 2 && (IG & 1) == 0 && (c_lo & 1) == 0;
  // the MAD pass in both forms (32-bit copy, int64 tensor): one returns at once
  for (int f = 0; f < (MAD ? 2 : 1); f++) {
    const bool s32 = MAD && f == 0;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, a.T, a.R, IG, a.G, a.it, c_lo, c_hi, br, w.scr, w.rp,
                         a.stats, w.cx, (const int64_t *)w.qa, w.esc + h);
    };
    if (vec && s32) go(rm_pass<MAD, STATS, true, CPL, MAD>);
    else if (vec) go(rm_pass<MAD, STATS, true, CPL, false>);
    else if (s32) go(rm_pass<MAD, STATS, false, CPL, MAD>);
    else go(rm_pass<MAD, STATS, false, CPL, false>);
  }
}

// The row-major robust FULL scan.  Serially: sample, brackets, median pass,
// median selection, MAD pass, MAD selection, row scores.  With a side stream
// the columns are split at iteration ih (halves A = [0, ih*G) and B =
// [ih*G, IG)): the passes stay in order on the launch stream and the
// latency-bound selections (and B's brackets) run on the side stream, each
// beside the next pass:
//   launch: sample | br A | pass med A | pass med B | pass MAD A | pass MAD B | score A | score B
//   side:                 | br B       | select A   | select B   | select A   | select B
// Every half reads and writes only its own columns' entries of the shared
// buffers (partials, interior slots, brackets, results); the selections are
// serialised on the side stream, so its gather slots are never shared.  The
// row scores run as two launches over the iterations of A and of B (the second
// continues the first's running sums), so score A overlaps B's MAD selection.
hipError_t scan_row_major(const OutArgs &a, const OWs &w, int IG, hipStream_t s) {
  const int ng = transpose_groups_of(a.R);
  const unsigned strips = (unsigned)((IG + TT - 1) / TT);
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int sel_max = std::min(SEL_GRID_MAX, SEL_WGS_PER_CU * cus);
  const RmBr bm{w.qa, w.qb, nullptr};
  const RmBr bd{w.da, w.db, w.cs.med2};
  const RmOut ro{w.da, w.db};
  auto brackets = [&](int lo, int hi, hipStream_t q) {
    hipLaunchKernelGGL(rm_brackets, dim3((unsigned)(hi - lo)), dim3(CS), 0, q, (const int64_t *)w.smp, lo,
                       w.qa, w.qb);
  };
  // h: the column half (0 or 1) whose copy flag a kernel sets or reads
  auto select = [&](bool mad, int lo, int hi, int h, hipStream_t q) {
    const int grid = std::min(hi - lo, sel_max);
    if (mad)
      hipLaunchKernelGGL(rm_select<true>, dim3(grid), dim3(CS), 0, q, a.T, a.R, IG, a.G, a.it,
                         (const int64_t *)w.smp, ng, lo, hi, w.rp, bd, (const int64_t *)w.scr, w.slots, ro,
                         w.cs, w.esc + h);
    else
      hipLaunchKernelGGL(rm_select<false>, dim3(grid), dim3(CS), 0, q, a.T, a.R, IG, a.G, a.it,
                         (const int64_t *)w.smp, ng, lo, hi, w.rp, bm, (const int64_t *)w.scr, w.slots, ro,
                         w.cs, w.esc + h);
  };
  auto med_pass = [&](int lo, int hi, int h) {
    if (a.stats.rc > 0)
      launch_rm_pass<false, true>(ng, a, IG, lo, hi, bm, w, h, s);
    else
      launch_rm_pass<false, false>(ng, a, IG, lo, hi, bm, w, h, s);
  };
  const int64_t waves = ((a.R + SRW - 1) / SRW) * ((a.G + 63) / 64);
  const dim3 sgrid((unsigned)((waves + 3) / 4));
  auto score = [&](int i_lo, int i_hi, int h) {
    hipLaunchKernelGGL(score_rows<true>, sgrid, dim3(256), 0, s, a.T, (const int32_t *)w.cx,
                       (const int64_t *)w.qa, (const int32_t *)(w.esc + h), a.R, a.I, a.G, a.it, i_lo, i_hi,
                       w.cs, w.m_t);
    hipLaunchKernelGGL(score_rows<false>, sgrid, dim3(256), 0, s, a.T, (const int32_t *)w.cx,
                       (const int64_t *)w.qa, (const int32_t *)(w.esc + h), a.R, a.I, a.G, a.it, i_lo, i_hi,
                       w.cs, w.m_t);
  };
  hipLaunchKernelGGL(rm_sample, dim3(MS / TT, strips), dim3(256), 0, s, a.T, a.R, IG, a.G, a.it, w.smp,
                     w.esc);
  // the split: even column counts on both sides when the rows are even, so
  // both halves keep the 16-byte loads
  int ih = a.I / 2;
  if ((IG & 1) == 0 && ((ih * a.G) & 1)) ih--;
  if (!a.side || ih <= 0) {
    brackets(0, IG, s);
    med_pass(0, IG, 0);
    if (a.stats.rc > 0 && a.stats_ready) (void)hipEventRecord(a.stats_ready, s);
    select(false, 0, IG, 0, s);
    launch_rm_pass<true, false>(ng, a, IG, 0, IG, bd, w, 0, s);
    select(true, 0, IG, 0, s);
    score(0, a.I, 0);
    return hipGetLastError();
  }
  const int cm = ih * a.G;
  hipStream_t q = a.side;
  const hipEvent_t *ev = a.ev;
  hipError_t e = hipSuccess;
  auto rec = [&](int k, hipStream_t on) {  // k < 0: the imbalance partials' event
    if (e == hipSuccess) e = hipEventRecord(k < 0 ? a.stats_ready : ev[k], on);
  };
  auto wait = [&](hipStream_t on, int k) {
    if (e == hipSuccess) e = hipStreamWaitEvent(on, ev[k], 0);
  };
  brackets(0, cm, s);
  rec(0, s);  // fork
  wait(q, 0);
  if (e != hipSuccess) return e;
  brackets(cm, IG, q);  // beside the median pass of A
  rec(1, q);
  med_pass(0, cm, 0);
  rec(2, s);
  wait(q, 2);
  select(false, 0, cm, 0, q);  // beside the median pass of B
  rec(3, q);
  wait(s, 1);
  med_pass(cm, IG, 1);
  if (a.stats.rc > 0 && a.stats_ready) rec(-1, s);
  rec(4, s);
  wait(q, 4);
  select(false, cm, IG, 1, q);  // beside the MAD pass of A
  rec(5, q);
  wait(s, 3);
  launch_rm_pass<true, false>(ng, a, IG, 0, cm, bd, w, 0, s);
  rec(6, s);
  wait(q, 6);
  select(true, 0, cm, 0, q);  // beside the MAD pass of B
  rec(7, q);
  wait(s, 5);
  launch_rm_pass<true, false>(ng, a, IG, cm, IG, bd, w, 1, s);
  rec(8, s);
  wait(q, 8);
  select(true, cm, IG, 1, q);  // beside score A
  rec(9, q);
  wait(s, 7);
  score(0, ih, 0);
  wait(s, 9);  // joins the side stream
  score(ih, a.I, 1);
  return e != hipSuccess ? e : hipGetLastError();
}

// sel_regions with the dynamic LDS its instantiation uses (the bracket buffer
// of the robust kind; the limit is raised by outliers_init).
template <bool F64, bool MAD>
void launch_sel_regions(const void *vals_t, int64_t R, int G, const int32_t *it, int I, double *z_t,
                        double *region_score, hipStream_t s) {
  hipLaunchKernelGGL((sel_regions<F64, MAD>), dim3(G), dim3(RT), MAD ? S2_LDS_BYTES : 0, s, vals_t, R,
                     G, it, I, z_t, region_score);
}

}  // namespace

void outliers_init() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&sel_regions<true, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)S2_LDS_BYTES);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&sel_regions<false, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)S2_LDS_BYTES);
}

namespace {
}  // namespace

size_t outliers_ws_bytes(int64_t R, int32_t I, int32_t G, int32_t mode, int32_t kind) {
  size_t used = 0;
  carve((void *)0x100, R, I, G, mode, kind, &used);
  return used + 256;
}

hipError_t launch_region_robust(const double *v_t, int64_t R, int G, const int32_t *it, int I,
                                double *z_t, float *score, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  launch_sel_regions<true, true>((const void *)v_t, R, G, it, I, z_t, (double *)nullptr, s);
  hipLaunchKernelGGL(rank_max_f32, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, z_t, R, G, it, I,
                     score);
  return hipGetLastError();
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
    if (row_major_path(a.R, a.mode, a.kind)) {
      if (IG > 0) {
        if (a.stats.rc > 0 && a.stats.rc != transpose_groups_of(a.R)) return hipErrorInvalidValue;
        const hipError_t e = scan_row_major(a, w, IG, s);
        if (e != hipSuccess) return e;
      } else {
        const int64_t waves = ((a.R + SRW - 1) / SRW) * ((a.G + 63) / 64);
        hipLaunchKernelGGL(score_rows<false>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a.T,
                           (const int32_t *)w.cx, (const int64_t *)w.qa, (const int32_t *)nullptr, a.R, a.I,
                           a.G, a.it, 0, a.I, w.cs, w.m_t);
      }
      launch_sel_regions<true, true>((const void *)w.m_t, a.R, a.G, a.it, a.I, w.z_t, a.region_score,
                                     s);
    } else if (a.mode == TA_SCAN_FULL) {
      if (IG > 0) {
        const dim3 tg((unsigned)transpose_groups_of(a.R), (IG + TT - 1) / TT);
        if (a.stats.rc > 0) {
          if (a.stats.rc != transpose_groups_of(a.R)) return hipErrorInvalidValue;
          hipLaunchKernelGGL(transpose_kernel<true>, tg, dim3(256), 0, s, a.T, a.R, IG, a.G, a.it, w.Tt,
                             a.stats);
          if (a.stats_ready) (void)hipEventRecord(a.stats_ready, s);
        } else {
          hipLaunchKernelGGL(transpose_kernel<false>, tg, dim3(256), 0, s, a.T, a.R, IG, a.G, a.it, w.Tt,
                             a.stats);
        }
        if (mad && pad_ranks(a.R) < SEL_BRACKET_MIN_RP) {
          hipLaunchKernelGGL(col_select_radix, dim3(IG), dim3(CS), 0, s, w.Tt, a.R, w.cs);
        } else if (mad) {
          int dev = 0, cus = 256;
          (void)hipGetDevice(&dev);
          (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
          const int grid = std::min(IG, std::min(SEL_GRID_MAX, SEL_WGS_PER_CU * cus));
          hipLaunchKernelGGL(col_select_bracket, dim3(grid), dim3(CS), 0, s, w.Tt, a.R, IG, w.scr,
                             sel_cap(a.R), w.cs);
        }
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
        launch_sel_regions<true, true>((const void *)w.m_t, a.R, a.G, a.it, a.I, w.z_t, a.region_score,
                                       s);
      else
        launch_sel_regions<true, false>((const void *)w.m_t, a.R, a.G, a.it, a.I, w.z_t,
                                         a.region_score, s);
    } else {
      hipLaunchKernelGGL(rank_totals_t, dim3(nb), dim3(256), 0, s, a.T, a.R, a.I, a.G, a.it, w.S_t);
      if (mad)
        launch_sel_regions<false, true>((const void *)w.S_t, a.R, a.G, a.it, a.I, w.z_t,
                                         a.region_score, s);
      else
        launch_sel_regions<false, false>((const void *)w.S_t, a.R, a.G, a.it, a.I, w.z_t,
                                         a.region_score, s);
    }
  }
  const unsigned nr = (unsigned)((a.R + 255) / 256);
  if (a.R > 0)
    hipLaunchKernelGGL(rank_final, dim3(nr), dim3(256), 0, s, w.z_t, a.R, a.G, a.it, a.I, a.tau,
                       a.rank_score, a.rank_flag, w.part);
  hipLaunchKernelGGL(count_final, dim3(1), dim3(256), 0, s, w.part, (int64_t)nr, a.n_flagged);
  return hipGetLastError();
}

int transpose_groups(int64_t R) { return transpose_groups_of(R); }

}  // namespace ta
