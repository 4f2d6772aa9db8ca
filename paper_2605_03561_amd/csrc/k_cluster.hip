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
  uint64_t *Ss = lds + (size_t)D * KMAX;         // [K][D]
  uint64_t *Ns = Ss + (size_t)K * D;             // [K]
  __shared__ uint32_t nchg;
  for (int i = threadIdx.x; i < D * KMAX; i += KW) {
    const int d = i / KMAX, k = i % KMAX;
    Cs[i] = k < K ? C[k * D + d] : 0.0;
  }
  for (int i = threadIdx.x; i < K * D; i += KW) Ss[i] = 0;
  for (int i = threadIdx.x; i < K; i += KW) Ns[i] = 0;
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
    atomicAdd((unsigned long long *)&Ns[best], 1ull);
    if (REG) {
#pragma unroll
      for (int d = 0; d < DREG; d++)
        atomicAdd((unsigned long long *)&Ss[best * DREG + d], (unsigned long long)v[d]);
    } else {
      for (int d0 = 0; d0 < D; d0 += FB) {
#pragma unroll
        for (int u = 0; u < FB; u++) v[u] = d0 + u < D ? Xt[(int64_t)(d0 + u) * R + r] : 0;
#pragma unroll
        for (int u = 0; u < FB; u++)
          if (d0 + u < D) atomicAdd((unsigned long long *)&Ss[best * D + d0 + u], (unsigned long long)v[u]);
      }
    }
  }
  if (my_chg) atomicAdd(&nchg, my_chg);
  __syncthreads();
  const int slot = blockIdx.x % KS;
  int64_t *sum_s = sum + (size_t)slot * K * D;
  int64_t *cnt_s = cnt + (size_t)slot * K;
  for (int i = threadIdx.x; i < K * D; i += KW)
    if (Ss[i]) atomicAdd((unsigned long long *)&sum_s[i], (unsigned long long)Ss[i]);
  for (int i = threadIdx.x; i < K; i += KW)
    if (Ns[i]) atomicAdd((unsigned long long *)&cnt_s[i], (unsigned long long)Ns[i]);
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
  for (int k = threadIdx.x; k < K; k += KT) {
    int64_t n = 0;
    for (int s = 0; s < KS; s++) {
      n += cnt[(size_t)s * K + k];
      cnt[(size_t)s * K + k] = 0;
    }
    n_k[k] = n;
    if (counts) counts[k] = n;
  }
  if (threadIdx.x == 0) {
    uint64_t c = 0;
    for (int s = 0; s < KS; s++) {
      c += chg[s];
      chg[s] = 0;
    }
    changed = c;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < K * D; i += KT) {
    uint64_t sm = 0;
    for (int s = 0; s < KS; s++) {
      sm += (uint64_t)sum[(size_t)s * K * D + i];
      sum[(size_t)s * K * D + i] = 0;
    }
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

struct SortState {
  uint64_t kmin;
  int32_t which;  // buffer holding the sorted result (0 = A, 1 = B)
};

__device__ inline uint64_t lane_lt_mask() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Stable LSD radix sort of the keys x[r] ^ SIGN (order-preserving) with their
// row index, in one workgroup: the range [kmin, kmax] fixes how many 8-bit
// digits vary; each pass counts the digits, then scatters tiles of WG1 rows in
// order, a row's place among equal digits of its tile coming from wave ballots
// (lanes with the same digit) and the per-wave digit counts.
__global__ __launch_bounds__(WG1) void radix_sort_1wg(const int64_t *__restrict__ x, int64_t R,
                                                     uint64_t *kA, int32_t *iA, uint64_t *kB,
                                                     int32_t *iB, SortState *ss) {
  constexpr int NWV = WG1 / 64;
  __shared__ uint64_t red_min[NWV], red_max[NWV];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[NWV][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t mn = ~0ull, mx = 0;
  for (int64_t i = threadIdx.x; i < R; i += WG1) {
    const uint64_t k = (uint64_t)x[i] ^ SIGN;
    mn = k < mn ? k : mn;
    mx = k > mx ? k : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    red_min[w] = mn;
    red_max[w] = mx;
  }
  __syncthreads();
  mn = red_min[0];
  mx = red_max[0];
  for (int i = 1; i < NWV; i++) {
    mn = red_min[i] < mn ? red_min[i] : mn;
    mx = red_max[i] > mx ? red_max[i] : mx;
  }
  const uint64_t span = R > 0 ? mx - mn : 0;
  const int bits = span == 0 ? 0 : 64 - __clzll((long long)span);
  const int passes = (bits + 7) / 8;
  // keys relative to the minimum, in row order
  for (int64_t i = threadIdx.x; i < R; i += WG1) {
    kA[i] = ((uint64_t)x[i] ^ SIGN) - mn;
    iA[i] = (int32_t)i;
  }
  __syncthreads();
  uint64_t *ks = kA, *kd = kB;
  int32_t *is = iA, *id = iB;
  for (int p = 0; p < passes; p++) {
    const int sh = 8 * p;
    for (int i = threadIdx.x; i < 256; i += WG1) hist[i] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < R; i += WG1) atomicAdd(&hist[(ks[i] >> sh) & 255], 1u);
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive scan of 256 counts by one wave
      uint32_t c[4], s = 0;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        c[u] = hist[4 * lane + u];
        s += c[u];
      }
      uint32_t incl = s;
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
      }
      uint32_t acc = incl - s;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        base[4 * lane + u] = acc;
        acc += c[u];
      }
    }
    __syncthreads();
    for (int64_t t0 = 0; t0 < R; t0 += WG1) {
      for (int i = threadIdx.x; i < NWV * 256; i += WG1) (&wcnt[0][0])[i] = 0;
      __syncthreads();
      const int64_t i = t0 + threadIdx.x;
      const bool on = i < R;
      const uint64_t key = on ? ks[i] : 0;
      const int32_t val = on ? is[i] : 0;
      const uint32_t dg = (uint32_t)(key >> sh) & 255u;
      uint64_t peers = __ballot(on);
#pragma unroll
      for (int b = 0; b < 8; b++) {
        const uint64_t bb = __ballot((dg >> b) & 1u);
        peers &= ((dg >> b) & 1u) ? bb : ~bb;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lane_lt_mask());
      if (on && rank == 0) wcnt[w][dg] = (uint32_t)__popcll(peers);
      __syncthreads();
      for (int d = threadIdx.x; d < 256; d += WG1) {
        uint32_t off = base[d];
        for (int v = 0; v < NWV; v++) {
          const uint32_t c = wcnt[v][d];
          wcnt[v][d] = off;
          off += c;
        }
        base[d] = off;
      }
      __syncthreads();
      if (on) {
        const uint32_t dst = wcnt[w][dg] + rank;
        kd[dst] = key;
        id[dst] = val;
      }
      __syncthreads();
    }
    uint64_t *tk = ks;
    ks = kd;
    kd = tk;
    int32_t *ti = is;
    is = id;
    id = ti;
  }
  if (threadIdx.x == 0) {
    ss->kmin = mn;
    ss->which = (passes & 1) ? 1 : 0;
  }
}

__device__ inline int64_t sorted_value(const uint64_t *k, int64_t j, uint64_t kmin) {
  return (int64_t)((k[j] + kmin) ^ SIGN);
}

// Core rows: the neighbours of sorted row j are the rows with values in
// [v_j - eps, v_j + eps], a contiguous range found by two binary searches.
__global__ __launch_bounds__(KT) void db_core(const uint64_t *kA, const uint64_t *kB, int64_t R,
                                             int64_t eps, int64_t min_pts, const SortState *ss,
                                             uint8_t *core_s) {
  const uint64_t *k = ss->which ? kB : kA;
  const uint64_t kmin = ss->kmin;
  for (int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x; j < R; j += (int64_t)gridDim.x * KT) {
    const int64_t v = sorted_value(k, j, kmin);
    const int64_t lo_v = v < INT64_MIN + eps ? INT64_MIN : v - eps;
    const int64_t hi_v = v > INT64_MAX - eps ? INT64_MAX : v + eps;
    int64_t a = 0, b = j;  // first index with value >= lo_v (in [0, j])
    while (a < b) {
      const int64_t m = (a + b) >> 1;
      if (sorted_value(k, m, kmin) < lo_v) a = m + 1;
      else b = m;
    }
    const int64_t lo = a;
    a = j + 1;
    b = R;  // first index with value > hi_v (in [j+1, R])
    while (a < b) {
      const int64_t m = (a + b) >> 1;
      if (sorted_value(k, m, kmin) <= hi_v) a = m + 1;
      else b = m;
    }
    core_s[j] = (a - lo) >= min_pts ? 1 : 0;
  }
}

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

// Cluster numbers (one workgroup, chunks of WG1 sorted rows with carries):
// forward, a core row starts a new cluster when the previous core row is more
// than eps below it, and every row learns the previous core row; backward,
// every row learns the next core row; a border row joins the nearer of the two
// (the previous one on a tie) when it is within eps.  Labels and core flags go
// back to row order.
__global__ __launch_bounds__(WG1) void db_label(const uint64_t *kA, const int32_t *iA,
                                               const uint64_t *kB, const int32_t *iB, int64_t R,
                                               int64_t eps, const SortState *ss,
                                               const uint8_t *core_s, int32_t *cl_s,
                                               int32_t *prev_s, int32_t *labels, uint8_t *core,
                                               int32_t *n_clusters) {
  constexpr int NWV = WG1 / 64;
  __shared__ int64_t wt64[NWV];
  __shared__ int32_t wt32[NWV];
  __shared__ int64_t idx_lds[WG1];
  __shared__ int32_t num_last;
  const uint64_t *k = ss->which ? kB : kA;
  const int32_t *perm = ss->which ? iB : iA;
  const uint64_t kmin = ss->kmin;
  auto imax = [](int64_t a, int64_t b) { return a > b ? a : b; };
  auto imin = [](int64_t a, int64_t b) { return a < b ? a : b; };
  auto iadd = [](int32_t a, int32_t b) { return a + b; };
  int64_t last_core = -1;  // carry: last core row before the chunk
  int32_t clusters = 0;    // carry: clusters started before the chunk
  for (int64_t t0 = 0; t0 < R; t0 += WG1) {
    const int64_t j = t0 + threadIdx.x;
    const bool on = j < R;
    const bool c = on && core_s[j];
    const int64_t pc = imax(last_core, block_incl_scan<int64_t>(c ? j : -1, wt64, (int64_t)-1, imax));
    idx_lds[threadIdx.x] = pc;  // last core row at or before j
    __syncthreads();
    const int64_t prev = threadIdx.x == 0 ? last_core : idx_lds[threadIdx.x - 1];
    int32_t start = 0;
    if (c) start = (prev < 0 || sorted_value(k, j, kmin) - sorted_value(k, prev, kmin) > eps) ? 1 : 0;
    const int32_t num = clusters + block_incl_scan<int32_t>(start, wt32, 0, iadd);
    if (on) {
      cl_s[j] = c ? num - 1 : -1;
      prev_s[j] = (int32_t)prev;
    }
    if (threadIdx.x == WG1 - 1) num_last = num;
    __syncthreads();
    last_core = idx_lds[WG1 - 1];
    clusters = num_last;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_clusters = clusters;
  // backward: thread t takes row t0 + (WG1 - 1 - t), so a scan over threads
  // runs from the chunk's last row down
  int64_t next_core = INT64_MAX;  // carry: first core row after the chunk
  const int64_t n_chunks = (R + WG1 - 1) / WG1;
  for (int64_t ci = n_chunks - 1; ci >= 0; ci--) {
    const int64_t j = ci * WG1 + (WG1 - 1 - threadIdx.x);
    const bool on = j < R;
    const bool c = on && core_s[j];
    const int64_t nc =
        imin(next_core, block_incl_scan<int64_t>(c ? j : INT64_MAX, wt64, INT64_MAX, imin));
    idx_lds[threadIdx.x] = nc;  // first core row at or after j
    __syncthreads();
    const int64_t next = threadIdx.x == 0 ? next_core : idx_lds[threadIdx.x - 1];
    if (on) {
      int32_t lab = cl_s[j];
      if (!c) {
        const int64_t v = sorted_value(k, j, kmin);
        const int64_t prev = prev_s[j];
        const int64_t dl = prev >= 0 ? v - sorted_value(k, prev, kmin) : INT64_MAX;
        const int64_t dr = next != INT64_MAX ? sorted_value(k, next, kmin) - v : INT64_MAX;
        if (dl <= eps && dl <= dr) lab = cl_s[prev];
        else if (dr <= eps) lab = cl_s[next];
      }
      const int32_t r = perm[j];
      labels[r] = lab;
      if (core) core[r] = c ? 1 : 0;
    }
    __syncthreads();
    next_core = idx_lds[WG1 - 1];
    __syncthreads();
  }
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
  const size_t lds = ((size_t)D * (K <= 8 ? 8 : 32) + (size_t)K * D + K) * sizeof(uint64_t);
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
  // the register-resident row for the usual width (64 region totals, K <= 8)
  const bool reg = D == DREG && K <= 8;
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

size_t dbscan_ws_bytes(int64_t R) {
  return (size_t)R * (8 + 4) * 2 + (size_t)R * (1 + 4 + 4) + 256;
}

hipError_t launch_dbscan1d(const int64_t *x, int64_t R, int64_t eps, int64_t min_pts,
                           int32_t *labels, int32_t *n_clusters, uint8_t *core, void *ws, int cus,
                           hipStream_t s) {
  char *p = (char *)ws;
  uint64_t *kA = (uint64_t *)p;
  p += (size_t)R * 8;
  uint64_t *kB = (uint64_t *)p;
  p += (size_t)R * 8;
  int32_t *iA = (int32_t *)p;
  p += (size_t)R * 4;
  int32_t *iB = (int32_t *)p;
  p += (size_t)R * 4;
  int32_t *cl_s = (int32_t *)p;
  p += (size_t)R * 4;
  int32_t *prev_s = (int32_t *)p;
  p += (size_t)R * 4;
  SortState *ss = (SortState *)p;
  p += 64;
  uint8_t *core_s = (uint8_t *)p;
  radix_sort_1wg<<<1, WG1, 0, s>>>(x, R, kA, iA, kB, iB, ss);
  db_core<<<grid_of(R, cus), KT, 0, s>>>(kA, kB, R, eps, min_pts, ss, core_s);
  db_label<<<1, WG1, 0, s>>>(kA, iA, kB, iB, R, eps, ss, core_s, cl_s, prev_s, labels, core, n_clusters);
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
