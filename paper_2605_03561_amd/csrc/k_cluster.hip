// k_cluster.hip -- clustering of ranks: K-Means (Lloyd), DBSCAN on one integer
// feature, and the compute nodes shared by clusters (Sec. VI-B clusters the
// ranks of one metric with DBSCAN, maps the groups to compute nodes, and tests
// K-Means with 2..5 groups by the compute nodes whose ranks fall in two groups).
//
// Every decision is taken in the same arithmetic as the definition: K-Means
// distances are FP64 sums over the features in ascending order with each
// product and sum rounded (the library is built without FP contraction);
// centroid sums are exact int64; DBSCAN works on int64 values only.
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int KT = 256;    // threads of the K-Means and grid kernels
constexpr int WG1 = 1024;  // threads of the single-workgroup kernels
constexpr uint64_t SIGN = 0x8000000000000000ull;

struct KmState {
  int32_t done;
  int32_t it;
};

// Workgroup partials go to one of KS slots (workgroup b to slot b mod KS):
// the integer sums do not depend on the order, and spreading them keeps the
// device-scope atomics on one address few.
constexpr int KS = 32;

// sum[KS][K*D], cnt[KS][K], chg[KS]
__global__ void km_init(const double *C0, double *C, int KD, int32_t *labels, int64_t R,
                        int64_t *sum, int64_t *cnt, uint64_t *chg, int K, KmState *st) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < KD; i += n) C[i] = C0[i];
  for (int64_t i = tid; i < (int64_t)KS * KD; i += n) sum[i] = 0;
  for (int64_t i = tid; i < (int64_t)KS * K; i += n) cnt[i] = 0;
  for (int64_t i = tid; i < KS; i += n) chg[i] = 0;
  for (int64_t r = tid; r < R; r += n) labels[r] = -1;
  if (tid == 0) {
    st->done = 0;
    st->it = 0;
  }
}

constexpr int KW = 256;  // threads of the K-Means assignment
// Copies of the workgroup's cluster sums in LDS for the register-resident
// row: lane l adds to copy l mod KNC, so the lanes of a wave that chose the
// same cluster hit KNC different addresses (in different banks: a copy is
// K*D + 1 words long) instead of one.
constexpr int KNC = 16;
__host__ __device__ inline int km_copies(bool reg) { return reg ? KNC : 1; }
constexpr int FB = 16;   // features loaded per batch
constexpr int DREG = 64; // features a row keeps in registers

// Xt[d][r] = X[r][d], once per call (64 x 64 tiles through LDS, both sides
// coalesced), so that the iterations read a feature of 64 consecutive rows
// with one contiguous 512-byte access.
__global__ __launch_bounds__(KT) void km_transpose(const int64_t *__restrict__ X, int64_t R, int D,
                                                  int64_t *__restrict__ Xt) {
  __shared__ int64_t tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int d0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int i = ty; i < 64; i += KT / 64) {
    const int64_t r = r0 + i;
    const int d = d0 + tx;
    tile[i][tx] = (r < R && d < D) ? X[r * D + d] : 0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += KT / 64) {
    const int d = d0 + i;
    const int64_t r = r0 + tx;
    if (d < D && r < R) Xt[(int64_t)d * R + r] = tile[tx][i];
  }
}

// Assignment: thread = row (grid-stride) over the transposed rows: feature d
// of 64 consecutive rows is one contiguous access.  With exactly DREG features
// (REG, a compile-time width) the whole row is loaded in one batch (one memory
// round trip: a batch of 100k rows is only a few waves per SIMD, so latency,
// not bandwidth, bounds this kernel) and stays in registers; otherwise it
// arrives FB features at a time and is read again for the sums.  The features are added, in ascending
// order, to the row's distances to all centroids, kept in registers: the same
// FP64 sums as the definition's; then to the workgroup's exact int64 cluster
// sums in LDS, flushed once per workgroup.
template <int KMAX, bool REG>
__global__ __launch_bounds__(KW) void km_assign(const int64_t *__restrict__ Xt, int64_t R, int D_,
                                               int K, const double *__restrict__ C,
                                               int32_t *__restrict__ labels, int64_t *sum,
                                               int64_t *cnt, uint64_t *chg, KmState *st) {
  if (st->done) return;
  const int D = REG ? DREG : D_;
  extern __shared__ uint64_t lds[];
  // centroids as [D][KMAX], so that feature d, centroid k sits at a fixed
  // offset from d's row (an immediate when d is unrolled)
  double *Cs = reinterpret_cast<double *>(lds);  // [D][KMAX]
  constexpr int NC = REG ? KNC : 1;
  const int KDP = K * D + 1, KP = K + 1;         // padded copy lengths
  uint64_t *Ss = lds + (size_t)D * KMAX;         // [NC][K*D + 1]
  uint64_t *Ns = Ss + (size_t)NC * KDP;          // [NC][K + 1]
  __shared__ uint32_t nchg;
  for (int i = threadIdx.x; i < D * KMAX; i += KW) {
    const int d = i / KMAX, k = i % KMAX;
    Cs[i] = k < K ? C[k * D + d] : 0.0;
  }
  for (int i = threadIdx.x; i < NC * KDP; i += KW) Ss[i] = 0;
  for (int i = threadIdx.x; i < NC * KP; i += KW) Ns[i] = 0;
  const int cp = (threadIdx.x & 63) % NC;
  uint64_t *Sc = Ss + (size_t)cp * KDP;
  uint64_t *Nc = Ns + (size_t)cp * KP;
  if (threadIdx.x == 0) nchg = 0;
  __syncthreads();
  uint32_t my_chg = 0;
  for (int64_t r = (int64_t)blockIdx.x * KW + threadIdx.x; r < R; r += (int64_t)gridDim.x * KW) {
    double dist[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; k++) dist[k] = 0.0;
    // all KMAX slots, without a branch per centroid (slots k >= K hold zeros
    // and never enter the choice below)
    auto add_feature = [&](int d, int64_t xv) {
      const double xd = (double)xv;
#pragma unroll
      for (int k = 0; k < KMAX; k++) {
        const double t = xd - Cs[d * KMAX + k];
        const double sq = t * t;
        dist[k] = dist[k] + sq;
      }
    };
    int64_t v[REG ? DREG : FB];
    if (REG) {
      const int64_t *p = Xt + r;
#pragma unroll
      for (int d = 0; d < DREG; d++) {
        v[d] = *p;
        p += R;
      }
#pragma unroll
      for (int d = 0; d < DREG; d++) add_feature(d, v[d]);
    } else {
      for (int d0 = 0; d0 < D; d0 += FB) {
#pragma unroll
        for (int u = 0; u < FB; u++) v[u] = d0 + u < D ? Xt[(int64_t)(d0 + u) * R + r] : 0;
#pragma unroll
        for (int u = 0; u < FB; u++)
          if (d0 + u < D) add_feature(d0 + u, v[u]);
      }
    }
    int best = 0;
    double bd = dist[0];
#pragma unroll
    for (int k = 1; k < KMAX; k++)
      if (k < K && dist[k] < bd) {
        best = k;
        bd = dist[k];
      }
    if (labels[r] != best) my_chg++;
    labels[r] = best;
    atomicAdd((unsigned long long *)&Nc[best], 1ull);
    if (REG) {
#pragma unroll
      for (int d = 0; d < DREG; d++)
        atomicAdd((unsigned long long *)&Sc[best * DREG + d], (unsigned long long)v[d]);
    } else {
      for (int d0 = 0; d0 < D; d0 += FB) {
#pragma unroll
        for (int u = 0; u < FB; u++) v[u] = d0 + u < D ? Xt[(int64_t)(d0 + u) * R + r] : 0;
#pragma unroll
        for (int u = 0; u < FB; u++)
          if (d0 + u < D) atomicAdd((unsigned long long *)&Sc[best * D + d0 + u], (unsigned long long)v[u]);
      }
    }
  }
  if (my_chg) atomicAdd(&nchg, my_chg);
  __syncthreads();
  const int slot = blockIdx.x % KS;
  int64_t *sum_s = sum + (size_t)slot * K * D;
  int64_t *cnt_s = cnt + (size_t)slot * K;
  for (int i = threadIdx.x; i < K * D; i += KW) {
    uint64_t t = 0;
#pragma unroll
    for (int c = 0; c < NC; c++) t += Ss[(size_t)c * KDP + i];
    if (t) atomicAdd((unsigned long long *)&sum_s[i], (unsigned long long)t);
  }
  for (int i = threadIdx.x; i < K; i += KW) {
    uint64_t t = 0;
#pragma unroll
    for (int c = 0; c < NC; c++) t += Ns[(size_t)c * KP + i];
    if (t) atomicAdd((unsigned long long *)&cnt_s[i], (unsigned long long)t);
  }
  if (threadIdx.x == 0 && nchg) atomicAdd((unsigned long long *)&chg[slot], (unsigned long long)nchg);
}

// Update (one workgroup, after the assignment kernel: the kernel boundary
// makes the sums visible): centroid = (double)(exact sum) / count, unchanged
// when the cluster is empty; clear the sums; stop after an iteration without
// change or after max_iter.
__global__ __launch_bounds__(KT) void km_update(int K, int D, int max_iter, double *C, int64_t *sum,
                                               int64_t *cnt, uint64_t *chg, int64_t *counts,
                                               int32_t *n_iter, KmState *st) {
  if (st->done) return;
  __shared__ int64_t n_k[32];
  __shared__ uint64_t changed;
  // the KS slots of one entry: all loads in flight, then the sum, then the
  // slots cleared for the next iteration
  auto take = [](uint64_t *p, size_t stride) {
    uint64_t v[KS];
#pragma unroll
    for (int s = 0; s < KS; s++) v[s] = p[(size_t)s * stride];
    uint64_t t = 0;
#pragma unroll
    for (int s = 0; s < KS; s++) t += v[s];
#pragma unroll
    for (int s = 0; s < KS; s++) p[(size_t)s * stride] = 0;
    return t;
  };
  for (int k = threadIdx.x; k < K; k += KT) {
    const int64_t n = (int64_t)take((uint64_t *)cnt + k, (size_t)K);
    n_k[k] = n;
    if (counts) counts[k] = n;
  }
  if (threadIdx.x == 0) changed = take(chg, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < K * D; i += KT) {
    const uint64_t sm = take((uint64_t *)sum + i, (size_t)K * D);
    const int64_t n = n_k[i / D];
    if (n > 0) C[i] = (double)(int64_t)sm / (double)n;
  }
  if (threadIdx.x == 0) {
    const int it = st->it + 1;
    st->it = it;
    if (n_iter) *n_iter = it;
    if (changed == 0 || it >= max_iter) st->done = 1;
  }
}

// ---- DBSCAN on one int64 feature --------------------------------------------
//
// Rows are sorted by value with a device-wide stable LSD radix sort (8-bit
// digits of the key minus the smallest key, only the digits that vary), in
// tiles of WG1 rows, one workgroup per tile:
//   db_keys     order-preserving keys x ^ SIGN, row ids, min and max key
//   per digit:  db_hist (the tile's digit counts, digit-major [256][tiles]),
//               db_xscan (exclusive sum over that array: each tile's start
//               for each digit), db_scatter (a row's place among the equal
//               digits of its tile from wave ballots and per-wave counts)
// then, on the sorted rows, core flags (two binary searches per row) and the
// labels from block scans with carries across tiles (db_xscan over the tiles'
// maxima, minima and start counts).  The number of passes is known only on the
// device, so all eight digit passes are queued and those past the last varying
// digit return at once; nothing waits on the host.

struct SortState {
  uint64_t kmin, kmax;
};

__device__ inline int sort_passes(const SortState *ss) {
  const uint64_t span = ss->kmax - ss->kmin;
  const int bits = span == 0 ? 0 : 64 - __clzll((long long)span);
  return (bits + 7) / 8;
}

__device__ inline uint64_t lane_lt_mask() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ inline int64_t key_value(uint64_t k) { return (int64_t)(k ^ SIGN); }

// Inclusive scan over the workgroup with a binary operation (wave shuffles,
// then the wave totals).  `wtot` holds NWV slots.
template <typename T, typename Op>
__device__ inline T block_incl_scan(T v, T *wtot, T ident, Op op) {
  constexpr int NWV = WG1 / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x = op(x, y);
  }
  if (lane == 63) wtot[w] = x;
  __syncthreads();
  T pre = ident;
  for (int i = 0; i < NWV; i++)
    if (i < w) pre = op(pre, wtot[i]);
  __syncthreads();
  return op(pre, x);
}

struct OpMax {
  __device__ int64_t operator()(int64_t a, int64_t b) const { return a > b ? a : b; }
};
struct OpMin {
  __device__ int64_t operator()(int64_t a, int64_t b) const { return a < b ? a : b; }
};
struct OpSum {
  __device__ int64_t operator()(int64_t a, int64_t b) const { return a + b; }
};

// The inclusive scan's value of the previous thread (ident for thread 0).
template <typename Op>
__device__ inline int64_t block_excl_scan(int64_t v, int64_t ident, Op op, int64_t *wtot,
                                          int64_t *shift, int64_t *total) {
  const int64_t incl = block_incl_scan<int64_t>(v, wtot, ident, op);
  shift[threadIdx.x] = incl;
  __syncthreads();
  const int64_t ex = threadIdx.x == 0 ? ident : shift[threadIdx.x - 1];
  if (total) *total = shift[WG1 - 1];
  __syncthreads();
  return ex;
}

__global__ void db_init(SortState *ss, int32_t *n_clusters, int64_t R) {
  ss->kmin = ~0ull;
  ss->kmax = 0;
  if (R == 0) *n_clusters = 0;
}

__global__ __launch_bounds__(WG1) void db_keys(const int64_t *__restrict__ x, int64_t R, uint64_t *kA,
                                              int32_t *iA, SortState *ss) {
  constexpr int NWV = WG1 / 64;
  __shared__ uint64_t rmin[NWV], rmax[NWV];
  const int64_t i = (int64_t)blockIdx.x * WG1 + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t mn = ~0ull, mx = 0;
  if (i < R) {
    const uint64_t k = (uint64_t)x[i] ^ SIGN;
    kA[i] = k;
    iA[i] = (int32_t)i;
    mn = mx = k;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    rmin[w] = mn;
    rmax[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < NWV; v++) {
      mn = rmin[v] < mn ? rmin[v] : mn;
      mx = rmax[v] > mx ? rmax[v] : mx;
    }
    atomicMin((unsigned long long *)&ss->kmin, (unsigned long long)mn);
    atomicMax((unsigned long long *)&ss->kmax, (unsigned long long)mx);
  }
}

// Digit pass p reads the keys from A when p is even, from B when odd.
__global__ __launch_bounds__(WG1) void db_hist(const uint64_t *kA, const uint64_t *kB, int64_t R,
                                              int p, const SortState *ss, int64_t *hist) {
  __shared__ uint32_t h[256];
  if (p >= sort_passes(ss)) return;
  const uint64_t *ks = (p & 1) ? kB : kA;
  const uint64_t kmin = ss->kmin;
  const int64_t tiles = gridDim.x;
  for (int d = threadIdx.x; d < 256; d += WG1) h[d] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * WG1 + threadIdx.x;
  if (i < R) atomicAdd(&h[(uint32_t)((ks[i] - kmin) >> (8 * p)) & 255u], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += WG1) hist[(int64_t)d * tiles + blockIdx.x] = h[d];
}

__global__ __launch_bounds__(WG1) void db_scatter(uint64_t *kA, int32_t *iA, uint64_t *kB, int32_t *iB,
                                                 int64_t R, int p, const SortState *ss,
                                                 const int64_t *__restrict__ start) {
  constexpr int NWV = WG1 / 64;
  __shared__ uint32_t wcnt[NWV][256];
  if (p >= sort_passes(ss)) return;
  const bool odd = p & 1;
  const uint64_t *ks = odd ? kB : kA;
  const int32_t *is = odd ? iB : iA;
  uint64_t *kd = odd ? kA : kB;
  int32_t *id = odd ? iA : iB;
  const uint64_t kmin = ss->kmin;
  const int64_t tiles = gridDim.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < NWV * 256; d += WG1) (&wcnt[0][0])[d] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * WG1 + threadIdx.x;
  const bool on = i < R;
  const uint64_t key = on ? ks[i] : 0;
  const int32_t val = on ? is[i] : 0;
  const uint32_t dg = (uint32_t)((key - kmin) >> (8 * p)) & 255u;
  // lanes of this wave with the same digit
  uint64_t peers = __ballot(on);
#pragma unroll
  for (int b = 0; b < 8; b++) {
    const uint64_t bb = __ballot((dg >> b) & 1u);
    peers &= ((dg >> b) & 1u) ? bb : ~bb;
  }
  const uint32_t rank = (uint32_t)__popcll(peers & lane_lt_mask());
  if (on && rank == 0) wcnt[w][dg] = (uint32_t)__popcll(peers);
  __syncthreads();
  // per digit: the tile's start, then the waves in order
  for (int d = threadIdx.x; d < 256; d += WG1) {
    uint32_t off = (uint32_t)start[(int64_t)d * tiles + blockIdx.x];
    for (int v = 0; v < NWV; v++) {
      const uint32_t c = wcnt[v][d];
      wcnt[v][d] = off;
      off += c;
    }
  }
  __syncthreads();
  if (on) {
    const uint32_t dst = wcnt[w][dg] + rank;
    kd[dst] = key;
    id[dst] = val;
  }
}

// Exclusive scan of n values in one workgroup, in chunks of XC values: each
// chunk is loaded coalesced into LDS, thread t scans its XP consecutive values
// there after the block's exclusive scan of the per-thread sums, and the chunk
// is stored coalesced; the running total carries to the next chunk.  `rev`
// scans from the last value down; in place allowed; total (optional) is the
// whole reduction.  With p >= 0 it belongs to digit pass p and returns when
// that pass does not run.
constexpr int XP = 4, XC = XP * WG1;
template <typename Op>
__global__ __launch_bounds__(WG1) void db_xscan(const int64_t *in, int64_t n, int rev, int64_t ident,
                                               int64_t *out, int32_t *total, int p,
                                               const SortState *ss) {
  __shared__ int64_t buf[XC];
  __shared__ int64_t wtot[WG1 / 64];
  __shared__ int64_t shift[WG1];
  __shared__ int64_t all;
  if (p >= 0 && p >= sort_passes(ss)) return;
  const Op op;
  const int t = threadIdx.x;
  auto at = [&](int64_t q) { return rev ? n - 1 - q : q; };
  int64_t carry = ident;
  for (int64_t c0 = 0; c0 < n; c0 += XC) {
#pragma unroll
    for (int u = 0; u < XP; u++) {
      const int64_t q = c0 + (int64_t)u * WG1 + t;
      buf[u * WG1 + t] = q < n ? in[at(q)] : ident;
    }
    __syncthreads();
    int64_t v[XP], acc = ident;
#pragma unroll
    for (int u = 0; u < XP; u++) {
      v[u] = buf[XP * t + u];
      acc = op(acc, v[u]);
    }
    int64_t run = op(carry, block_excl_scan(acc, ident, op, wtot, shift, &all));
#pragma unroll
    for (int u = 0; u < XP; u++) {
      buf[XP * t + u] = run;
      run = op(run, v[u]);
    }
    carry = op(carry, all);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < XP; u++) {
      const int64_t q = c0 + (int64_t)u * WG1 + t;
      if (q < n) out[at(q)] = buf[u * WG1 + t];
    }
    __syncthreads();
  }
  if (total && t == 0) *total = (int32_t)carry;
}

__device__ inline const uint64_t *sorted_keys(const uint64_t *kA, const uint64_t *kB,
                                              const SortState *ss) {
  return (sort_passes(ss) & 1) ? kB : kA;
}

// Core rows: the neighbours of sorted row j are the rows with values in
// [v_j - eps, v_j + eps], a contiguous range found by two binary searches.
// Per tile: the last and the first core row (-1 / INT64_MAX when none).
__global__ __launch_bounds__(WG1) void db_core(const uint64_t *kA, const uint64_t *kB, int64_t R,
                                              int64_t eps, int64_t min_pts, const SortState *ss,
                                              uint8_t *core_s, int64_t *tmax, int64_t *tmin) {
  __shared__ int64_t wtot[WG1 / 64];
  const uint64_t *k = sorted_keys(kA, kB, ss);
  const int64_t j = (int64_t)blockIdx.x * WG1 + threadIdx.x;
  bool c = false;
  if (j < R) {
    const int64_t v = key_value(k[j]);
    const int64_t lo_v = v < INT64_MIN + eps ? INT64_MIN : v - eps;
    const int64_t hi_v = v > INT64_MAX - eps ? INT64_MAX : v + eps;
    int64_t a = 0, b = j;  // first index with value >= lo_v (in [0, j])
    while (a < b) {
      const int64_t m = (a + b) >> 1;
      if (key_value(k[m]) < lo_v) a = m + 1;
      else b = m;
    }
    const int64_t lo = a;
    a = j + 1;
    b = R;  // first index with value > hi_v (in [j+1, R])
    while (a < b) {
      const int64_t m = (a + b) >> 1;
      if (key_value(k[m]) <= hi_v) a = m + 1;
      else b = m;
    }
    c = (a - lo) >= min_pts;
    core_s[j] = c ? 1 : 0;
  }
  const int64_t mx = block_incl_scan<int64_t>(c ? j : -1, wtot, (int64_t)-1, OpMax());
  const int64_t mn = block_incl_scan<int64_t>(c ? j : INT64_MAX, wtot, INT64_MAX, OpMin());
  if (threadIdx.x == WG1 - 1) {
    tmax[blockIdx.x] = mx;
    tmin[blockIdx.x] = mn;
  }
}

// Per sorted row: the last core row before it (prev_s), and for a core row
// whether it starts a new cluster (the previous core row is more than eps
// below it), written to cl_s; per tile the count of starts.
__global__ __launch_bounds__(WG1) void db_start(const uint64_t *kA, const uint64_t *kB, int64_t R,
                                               int64_t eps, const SortState *ss,
                                               const uint8_t *core_s, const int64_t *cprev,
                                               int32_t *prev_s, int32_t *cl_s, int64_t *tstart) {
  __shared__ int64_t wtot[WG1 / 64];
  __shared__ int64_t shift[WG1];
  __shared__ int64_t all;
  const uint64_t *k = sorted_keys(kA, kB, ss);
  const int64_t j = (int64_t)blockIdx.x * WG1 + threadIdx.x;
  const bool on = j < R;
  const bool c = on && core_s[j];
  const int64_t ex = block_excl_scan(c ? j : (int64_t)-1, (int64_t)-1, OpMax(), wtot, shift, nullptr);
  const int64_t cp = cprev[blockIdx.x];
  const int64_t prev = ex > cp ? ex : cp;
  int64_t st = 0;
  if (c) st = (prev < 0 || key_value(k[j]) - key_value(k[prev]) > eps) ? 1 : 0;
  if (on) {
    prev_s[j] = (int32_t)prev;
    cl_s[j] = (int32_t)st;
  }
  (void)block_excl_scan(st, (int64_t)0, OpSum(), wtot, shift, &all);
  if (threadIdx.x == 0) tstart[blockIdx.x] = all;
}

// Cluster numbers of the core rows: the starts up to and including the row,
// after the tile's base, minus one (-1 for the other rows).
__global__ __launch_bounds__(WG1) void db_number(int64_t R, const uint8_t *core_s, const int64_t *cbase,
                                                int32_t *cl_s) {
  __shared__ int64_t wtot[WG1 / 64];
  const int64_t j = (int64_t)blockIdx.x * WG1 + threadIdx.x;
  const bool on = j < R;
  const int64_t st = on ? cl_s[j] : 0;
  const int64_t incl = block_incl_scan<int64_t>(st, wtot, (int64_t)0, OpSum());
  if (on) cl_s[j] = core_s[j] ? (int32_t)(cbase[blockIdx.x] + incl - 1) : -1;
}

// Labels in row order: a border row joins the nearer of the previous and the
// next core row (the previous one on a tie) when it is within eps.  Thread t
// takes the tile's row WG1 - 1 - t, so a scan over threads runs from the
// tile's last row down and gives the first core row at or after each row.
__global__ __launch_bounds__(WG1) void db_out(const uint64_t *kA, const int32_t *iA, const uint64_t *kB,
                                             const int32_t *iB, int64_t R, int64_t eps,
                                             const SortState *ss, const uint8_t *core_s,
                                             const int64_t *cnext, const int32_t *prev_s,
                                             const int32_t *cl_s, int32_t *labels, uint8_t *core) {
  __shared__ int64_t wtot[WG1 / 64];
  const bool inB = sort_passes(ss) & 1;
  const uint64_t *k = inB ? kB : kA;
  const int32_t *perm = inB ? iB : iA;
  const int64_t j = (int64_t)blockIdx.x * WG1 + (WG1 - 1 - threadIdx.x);
  const bool on = j < R;
  const bool c = on && core_s[j];
  const int64_t sm = block_incl_scan<int64_t>(c ? j : INT64_MAX, wtot, INT64_MAX, OpMin());
  const int64_t cn = cnext[blockIdx.x];
  const int64_t next = sm < cn ? sm : cn;
  if (!on) return;
  int32_t lab = cl_s[j];
  if (!c) {
    const int64_t v = key_value(k[j]);
    const int64_t prev = prev_s[j];
    const int64_t dl = prev >= 0 ? v - key_value(k[prev]) : INT64_MAX;
    const int64_t dr = next != INT64_MAX ? key_value(k[next]) - v : INT64_MAX;
    if (dl <= eps && dl <= dr) lab = cl_s[prev];
    else if (dr <= eps) lab = cl_s[next];
    else lab = -1;
  }
  const int32_t r = perm[j];
  labels[r] = lab;
  if (core) core[r] = c ? 1 : 0;
}

// ---- compute nodes shared by clusters ---------------------------------------

__global__ void ni_clear(uint64_t *mask, int32_t n_nodes, int64_t *pair, int KK) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < n_nodes; i += n) mask[i] = 0;
  for (int64_t i = tid; i < KK; i += n) pair[i] = 0;
}

__global__ void ni_mark(const int32_t *labels, const int32_t *rank_node, int64_t R, int32_t n_nodes,
                        int K, uint64_t *mask, uint32_t *err) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t n = rank_node[r], l = labels[r];
    if (n < 0 || n >= n_nodes || l >= K || l < -1) {
      atomicOr(err, ERRBIT_OFFSETS);
      continue;
    }
    if (l >= 0) atomicOr((unsigned long long *)&mask[n], 1ull << l);
  }
}

__global__ void ni_count(const uint64_t *mask, int32_t n_nodes, int K, int64_t *pair,
                         int32_t *node_clusters) {
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t m = mask[n];
    if (node_clusters) node_clusters[n] = __popcll(m);
    if (__popcll(m) < 2) continue;
    for (int a = 0; a < K; a++)
      if ((m >> a) & 1)
        for (int b = 0; b < K; b++)
          if (b != a && ((m >> b) & 1)) atomicAdd((unsigned long long *)&pair[a * K + b], 1ull);
  }
}

int grid_of(int64_t n, int cus) {
  int64_t g = (n + KT - 1) / KT;
  const int64_t cap = (int64_t)cus * 8;
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

static size_t km_state_bytes(int K, int D) {
  return (((size_t)KS * K * D + (size_t)KS * K + KS) * sizeof(int64_t) + 64 + 255) / 256 * 256;
}

size_t kmeans_ws_bytes(int K, int D, int64_t R) {
  return km_state_bytes(K, D) + (size_t)R * D * sizeof(int64_t);
}

hipError_t launch_kmeans(const int64_t *X, int64_t R, int D, int K, const double *C0, int max_iter,
                         int32_t *labels, double *C, int64_t *counts, int32_t *n_iter, void *ws,
                         int cus, hipStream_t s) {
  int64_t *sum = (int64_t *)ws;
  int64_t *cnt = sum + (size_t)KS * K * D;
  uint64_t *chg = (uint64_t *)(cnt + (size_t)KS * K);
  KmState *st = (KmState *)(chg + KS);
  int64_t *Xt = (int64_t *)((char *)ws + km_state_bytes(K, D));
  km_init<<<grid_of(R > KS * K * D ? R : KS * K * D, cus), KT, 0, s>>>(C0, C, K * D, labels, R, sum,
                                                                       cnt, chg, K, st);
  if (R > 0) km_transpose<<<dim3((unsigned)((R + 63) / 64), (unsigned)((D + 63) / 64)), KT, 0, s>>>(X, R, D, Xt);
  // the register-resident row for the usual width (64 region totals, K <= 8)
  const bool reg = D == DREG && K <= 8;
  const size_t nc = (size_t)km_copies(reg);
  const size_t lds =
      ((size_t)D * (K <= 8 ? 8 : 32) + nc * ((size_t)K * D + 1) + nc * ((size_t)K + 1)) * sizeof(uint64_t);
  static bool attr = false;
  if (!attr) {
    const void *fns[] = {reinterpret_cast<const void *>(&km_assign<8, true>),
                         reinterpret_cast<const void *>(&km_assign<8, false>),
                         reinterpret_cast<const void *>(&km_assign<32, false>)};
    for (const void *f : fns)
      (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    attr = true;
  }
  // a row per thread; at most 8 workgroups per CU
  int64_t grid = (R + KW - 1) / KW;
  if (grid > (int64_t)cus * 8) grid = (int64_t)cus * 8;
  if (grid < 1) grid = 1;
  for (int it = 0; it < max_iter; it++) {
    if (reg)
      km_assign<8, true><<<(int)grid, KW, lds, s>>>(Xt, R, D, K, C, labels, sum, cnt, chg, st);
    else if (K <= 8)
      km_assign<8, false><<<(int)grid, KW, lds, s>>>(Xt, R, D, K, C, labels, sum, cnt, chg, st);
    else
      km_assign<32, false><<<(int)grid, KW, lds, s>>>(Xt, R, D, K, C, labels, sum, cnt, chg, st);
    km_update<<<1, KT, 0, s>>>(K, D, max_iter, C, sum, cnt, chg, counts, n_iter, st);
  }
  return hipGetLastError();
}

namespace {

struct DbWs {
  uint64_t *kA, *kB;
  int32_t *iA, *iB, *cl_s, *prev_s;
  uint8_t *core_s;
  SortState *ss;
  int64_t *hist;                // [256][tiles] digit counts, then each tile's start
  int64_t *tmax, *tmin, *tst;   // per tile: last / first core row, cluster starts
  int64_t *cprev, *cnext, *cbase;
};

DbWs db_carve(void *ws, int64_t R, size_t *used) {
  const size_t tiles = (size_t)((R + WG1 - 1) / WG1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = (char *)ws + off;
    off += (bytes + 255) & ~(size_t)255;
    return (void *)p;
  };
  DbWs w;
  w.kA = (uint64_t *)take((size_t)R * 8);
  w.kB = (uint64_t *)take((size_t)R * 8);
  w.iA = (int32_t *)take((size_t)R * 4);
  w.iB = (int32_t *)take((size_t)R * 4);
  w.cl_s = (int32_t *)take((size_t)R * 4);
  w.prev_s = (int32_t *)take((size_t)R * 4);
  w.core_s = (uint8_t *)take((size_t)R);
  w.ss = (SortState *)take(sizeof(SortState));
  w.hist = (int64_t *)take(256 * tiles * 8);
  w.tmax = (int64_t *)take(tiles * 8);
  w.tmin = (int64_t *)take(tiles * 8);
  w.tst = (int64_t *)take(tiles * 8);
  w.cprev = (int64_t *)take(tiles * 8);
  w.cnext = (int64_t *)take(tiles * 8);
  w.cbase = (int64_t *)take(tiles * 8);
  *used = off;
  return w;
}

}  // namespace

size_t dbscan_ws_bytes(int64_t R) {
  size_t used = 0;
  db_carve(nullptr, R, &used);
  return used;
}

hipError_t launch_dbscan1d(const int64_t *x, int64_t R, int64_t eps, int64_t min_pts,
                           int32_t *labels, int32_t *n_clusters, uint8_t *core, void *ws, int cus,
                           hipStream_t s) {
  (void)cus;
  size_t used = 0;
  const DbWs w = db_carve(ws, R, &used);
  db_init<<<1, 1, 0, s>>>(w.ss, n_clusters, R);
  if (R == 0) return hipGetLastError();
  const unsigned tiles = (unsigned)((R + WG1 - 1) / WG1);
  db_keys<<<tiles, WG1, 0, s>>>(x, R, w.kA, w.iA, w.ss);
  for (int p = 0; p < 8; p++) {  // passes past the last varying digit return at once
    db_hist<<<tiles, WG1, 0, s>>>(w.kA, w.kB, R, p, w.ss, w.hist);
    db_xscan<OpSum><<<1, WG1, 0, s>>>(w.hist, 256 * (int64_t)tiles, 0, 0, w.hist, nullptr, p, w.ss);
    db_scatter<<<tiles, WG1, 0, s>>>(w.kA, w.iA, w.kB, w.iB, R, p, w.ss, w.hist);
  }
  db_core<<<tiles, WG1, 0, s>>>(w.kA, w.kB, R, eps, min_pts, w.ss, w.core_s, w.tmax, w.tmin);
  db_xscan<OpMax><<<1, WG1, 0, s>>>(w.tmax, tiles, 0, -1, w.cprev, nullptr, -1, w.ss);
  db_xscan<OpMin><<<1, WG1, 0, s>>>(w.tmin, tiles, 1, INT64_MAX, w.cnext, nullptr, -1, w.ss);
  db_start<<<tiles, WG1, 0, s>>>(w.kA, w.kB, R, eps, w.ss, w.core_s, w.cprev, w.prev_s, w.cl_s, w.tst);
  db_xscan<OpSum><<<1, WG1, 0, s>>>(w.tst, tiles, 0, 0, w.cbase, n_clusters, -1, w.ss);
  db_number<<<tiles, WG1, 0, s>>>(R, w.core_s, w.cbase, w.cl_s);
  db_out<<<tiles, WG1, 0, s>>>(w.kA, w.iA, w.kB, w.iB, R, eps, w.ss, w.core_s, w.cnext, w.prev_s, w.cl_s,
                               labels, core);
  return hipGetLastError();
}

size_t node_intersections_ws_bytes(int32_t n_nodes) { return (size_t)n_nodes * 8 + 64; }

hipError_t launch_node_intersections(const int32_t *labels, const int32_t *rank_node, int64_t R,
                                     int32_t n_nodes, int K, int64_t *pair, int32_t *node_clusters,
                                     void *ws, uint32_t *err, int cus, hipStream_t s) {
  uint64_t *mask = (uint64_t *)ws;
  ni_clear<<<grid_of(n_nodes > K * K ? n_nodes : K * K, cus), KT, 0, s>>>(mask, n_nodes, pair, K * K);
  if (R > 0) ni_mark<<<grid_of(R, cus), KT, 0, s>>>(labels, rank_node, R, n_nodes, K, mask, err);
  ni_count<<<grid_of(n_nodes, cus), KT, 0, s>>>(mask, n_nodes, K, pair, node_clusters);
  return hipGetLastError();
}

}  // namespace ta
