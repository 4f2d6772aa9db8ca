// k_prune.hip -- summary profile, pruning, pruned per-rank profiles and the
// inclusive form of the rank x iteration x region tensor.
//
// Sec. II-A: a pruning strategy is evaluated once on the summary profile (the
// aggregate of all per-rank profiles) and the resulting node set is applied to
// every rank; Sec. VI-B prunes the nodes below 1% of the total runtime.
//
// Every subtree sum here is a range sum in depth-first preorder: the subtree
// of v occupies preorder positions [tin(v), tout(v)).  A row (one rank's
// profile, or the summary) is scattered into LDS at preorder positions and
// scanned once; a node's inclusive cost is then P[tout] - P[tin] with P the
// exclusive prefix.  Sums are taken modulo 2^64 (uint64), so every result is
// the exact int64 sum whenever that sum fits, independent of order.
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int ST = 256;   // threads of the row-scan and column-sum kernels
constexpr int PT = 1024;  // threads of the single-workgroup pruning kernel

// Exclusive scan over the workgroup (NT a multiple of 64); `wsum` holds NT/64
// slots.  Returns the prefix of thread tid; *total gets the sum of all.
template <int NT, typename T>
__device__ inline T block_excl_scan(T v, T *wsum, T *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  T base = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; i++) {
    const T s = wsum[i];
    base += (i < w) ? s : (T)0;
    all += s;
  }
  __syncthreads();
  *total = all;
  return base + x - v;
}

// In-place exclusive prefix of P[0..n) in LDS, P[n] = total.  Each thread owns
// a contiguous chunk.
template <int NT>
__device__ inline void lds_scan(uint64_t *P, int n, uint64_t *wsum) {
  const int per = (n + NT - 1) / NT;
  const int j0 = min(n, (int)threadIdx.x * per), j1 = min(n, j0 + per);
  uint64_t s = 0;
  for (int j = j0; j < j1; j++) s += P[j];
  uint64_t total;
  uint64_t acc = block_excl_scan<NT>(s, wsum, &total);
  for (int j = j0; j < j1; j++) {
    const uint64_t x = P[j];
    P[j] = acc;
    acc += x;
  }
  if (threadIdx.x == 0) P[n] = total;
  __syncthreads();
}

__global__ void fill_u64(uint64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Column sums of x[R][N]: workgroup (bx, by) sums columns [bx*ST, bx*ST+ST)
// over the rows r = by, by + gridDim.y, ... and adds its partials atomically
// (integer atomics: the result does not depend on their order).
__global__ __launch_bounds__(ST) void colsum_kernel(const int64_t *__restrict__ x, int64_t R, int N,
                                                    uint64_t *__restrict__ out) {
  const int c = blockIdx.x * ST + threadIdx.x;
  if (c >= N) return;
  const int64_t step = gridDim.y;
  uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t r = blockIdx.y;
  for (; r + 3 * step < R; r += 4 * step) {
    s0 += (uint64_t)x[r * N + c];
    s1 += (uint64_t)x[(r + step) * N + c];
    s2 += (uint64_t)x[(r + 2 * step) * N + c];
    s3 += (uint64_t)x[(r + 3 * step) * N + c];
  }
  for (; r < R; r += step) s0 += (uint64_t)x[r * N + c];
  const uint64_t s = (s0 + s1) + (s2 + s3);
  if (s != 0) atomicAdd((unsigned long long *)&out[c], (unsigned long long)s);
}

// Row pass: for each row of rows[n_rows][N] (caller node order) and each query
// k with preorder range q[k] = (tin, tout): incl = sum of the row over the
// range.  With a child list (the kept children of query k in the pruned tree,
// kchild[koff[k] .. koff[k+1])), excl = incl minus the children's incl: the
// row's cost on the nodes whose nearest query ancestor-or-self is k.
__global__ __launch_bounds__(ST) void subtree_rows(const int64_t *__restrict__ rows, int64_t n_rows,
                                                  int N, const int2 *__restrict__ tin_tout,
                                                  const int2 *__restrict__ q, int K,
                                                  const int32_t *__restrict__ koff,
                                                  const int32_t *__restrict__ kchild,
                                                  int64_t *__restrict__ out_excl,
                                                  int64_t *__restrict__ out_incl) {
  extern __shared__ uint64_t lds[];
  __shared__ uint64_t wsum[ST / 64];
  uint64_t *P = lds;          // [N + 1]
  uint64_t *Q = lds + N + 1;  // [K] when out_excl
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    const int64_t *row = rows + r * N;
    for (int v = threadIdx.x; v < N; v += ST) P[tin_tout[v].x] = (uint64_t)row[v];
    __syncthreads();
    lds_scan<ST>(P, N, wsum);
    if (out_excl) {
      for (int k = threadIdx.x; k < K; k += ST) {
        const int2 t = q[k];
        Q[k] = P[t.y] - P[t.x];
      }
      __syncthreads();
      for (int k = threadIdx.x; k < K; k += ST) {
        const uint64_t inc = Q[k];
        uint64_t ex = inc;
        for (int j = koff[k]; j < koff[k + 1]; j++) ex -= Q[kchild[j]];
        out_excl[r * K + k] = (int64_t)ex;
        if (out_incl) out_incl[r * K + k] = (int64_t)inc;
      }
    } else {
      for (int k = threadIdx.x; k < K; k += ST) {
        const int2 t = q[k];
        out_incl[r * K + k] = (int64_t)(P[t.y] - P[t.x]);
      }
    }
    __syncthreads();
  }
}

// Pruning on the summary: keep v iff (double)sum_incl[v] >= fraction * (double)
// total, total = sum of sum_excl; kept ids in ascending order.  One workgroup.
__global__ __launch_bounds__(PT) void prune_kernel(const int64_t *__restrict__ sum_excl,
                                                  const int64_t *__restrict__ sum_incl, int N,
                                                  double fraction, int32_t *__restrict__ kept,
                                                  int32_t *__restrict__ n_kept) {
  __shared__ uint64_t wsum[PT / 64];
  __shared__ int32_t wcnt[PT / 64];
  uint64_t s = 0;
  for (int v = threadIdx.x; v < N; v += PT) s += (uint64_t)sum_excl[v];
  uint64_t total;
  (void)block_excl_scan<PT>(s, wsum, &total);
  const double cut = fraction * (double)(int64_t)total;
  int base = 0;
  for (int c0 = 0; c0 < N; c0 += PT) {
    const int v = c0 + threadIdx.x;
    const int f = (v < N && (double)sum_incl[v] >= cut) ? 1 : 0;
    int cnt;
    const int pos = block_excl_scan<PT>(f, wcnt, &cnt);
    if (f) kept[base + pos] = v;
    base += cnt;
  }
  if (threadIdx.x == 0) *n_kept = base;
}

// Inclusive tensor, G <= 64: segments of GP lanes (GP = power of two >= G),
// 64 / GP rows per wave.  Lane j of a segment holds the value of the region at
// region-preorder position j; a segmented inclusive scan S gives the range sum
// over [j, end_j) as S[end_j - 1] - S[j] + v_j.
template <int GP>
__global__ __launch_bounds__(ST) void incl_tensor_narrow(const int64_t *__restrict__ T,
                                                        int64_t n_rows, int G,
                                                        const int4 *__restrict__ rt,
                                                        int64_t *__restrict__ out) {
  constexpr int RPW = 64 / GP;
  const int lane = threadIdx.x & 63;
  const int seg = lane / GP, j = lane % GP;
  const int64_t wave = ((int64_t)blockIdx.x * ST + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * ST) >> 6;
  const int4 t = (j < G) ? rt[j] : make_int4(0, 0, 0, 1);
  const int g = t.z, last = t.w - 1;  // region at position j; last position of its range
  for (int64_t r0 = wave * RPW; r0 < n_rows; r0 += n_waves * RPW) {
    const int64_t r = r0 + seg;
    const bool on = (j < G) && (r < n_rows);
    const uint64_t v = on ? (uint64_t)T[r * G + g] : 0;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < GP; d <<= 1) {
      const uint64_t y = __shfl_up(x, d, GP);
      if (j >= d) x += y;
    }
    const uint64_t e = __shfl(x, last, GP);
    if (on) out[r * G + g] = (int64_t)(e - x + v);
  }
}

// Inclusive tensor, 64 < G <= 256: one row per wave; each lane owns up to four
// consecutive region-preorder positions; the wave's prefix goes to LDS.
__global__ __launch_bounds__(ST) void incl_tensor_wide(const int64_t *__restrict__ T,
                                                      int64_t n_rows, int G,
                                                      const int4 *__restrict__ rt,
                                                      int64_t *__restrict__ out) {
  __shared__ uint64_t S[ST / 64][MAX_REGIONS + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t *P = S[w];
  const int64_t wave = ((int64_t)blockIdx.x * ST + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * ST) >> 6;
  for (int64_t r = wave; r < n_rows; r += n_waves) {
    const int64_t *row = T + r * G;
    // region g = lane + 64c goes to its preorder position rt[g].x
    for (int g = lane; g < G; g += 64) P[rt[g].x] = (uint64_t)row[g];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int j0 = lane * 4;
    uint64_t a[4], s = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      a[u] = (j0 + u < G) ? P[j0 + u] : 0;
      s += a[u];
    }
    uint64_t x = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    uint64_t acc = x - s;  // exclusive prefix of position j0
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if (j0 + u <= G) P[j0 + u] = acc;  // P[G] = total (lane owning position G)
      acc += a[u];
    }
    if (j0 + 4 == G) P[G] = acc;  // G = 256: no lane owns position G
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int g = lane; g < G; g += 64) {
      const int4 t = rt[g];
      out[r * G + g] = (int64_t)(P[t.y] - P[t.x]);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

int grid_for(int64_t waves_of_work, int device_cus_hint) {
  const int64_t cap = (int64_t)device_cus_hint * 16;
  int64_t g = (waves_of_work + (ST / 64) - 1) / (ST / 64);
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

size_t subtree_rows_lds_bytes(int N, int K, bool excl) {
  return ((size_t)N + 1 + (excl ? (size_t)K : 0)) * sizeof(uint64_t);
}

static void allow_big_lds() {
  static bool done = false;
  if (!done) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&subtree_rows),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    done = true;
  }
}

hipError_t launch_summary(const int64_t *excl, int64_t R, int N, const int2 *tin_tout,
                          int64_t *sum_excl, int64_t *sum_incl, int cus, hipStream_t s) {
  fill_u64<<<(N + ST - 1) / ST, ST, 0, s>>>((uint64_t *)sum_excl, N);
  if (R > 0) {
    const int gx = (N + ST - 1) / ST;
    int64_t gy = ((int64_t)cus * 8 + gx - 1) / gx;  // about 8 workgroups per CU
    const int64_t rows_min = 16;                     // at least 16 rows per workgroup
    if (gy > (R + rows_min - 1) / rows_min) gy = (R + rows_min - 1) / rows_min;
    if (gy < 1) gy = 1;
    if (gy > 65535) gy = 65535;
    colsum_kernel<<<dim3(gx, (unsigned)gy), ST, 0, s>>>(excl, R, N, (uint64_t *)sum_excl);
  }
  if (sum_incl) {
    allow_big_lds();
    const size_t lds = subtree_rows_lds_bytes(N, N, false);
    subtree_rows<<<1, ST, lds, s>>>(sum_excl, 1, N, tin_tout, tin_tout, N, nullptr, nullptr,
                                    nullptr, sum_incl);
  }
  return hipGetLastError();
}

hipError_t launch_prune(const int64_t *sum_excl, const int64_t *sum_incl, int N, double fraction,
                        int32_t *kept, int32_t *n_kept, hipStream_t s) {
  prune_kernel<<<1, PT, 0, s>>>(sum_excl, sum_incl, N, fraction, kept, n_kept);
  return hipGetLastError();
}

hipError_t launch_pruned_profiles(const int64_t *excl, int64_t R, int N, const int2 *tin_tout,
                                  const int2 *kq, int K, const int32_t *koff,
                                  const int32_t *kchild, int64_t *p_excl, int64_t *p_incl,
                                  int cus, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const bool ex = p_excl != nullptr;
  const size_t lds = subtree_rows_lds_bytes(N, K, ex);
  allow_big_lds();
  // LDS bounds the workgroups per CU; a grid of a few per CU streams the rows.
  int per_cu = (int)((160 * 1024) / (lds + 1024));
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > R) grid = R;
  subtree_rows<<<(unsigned)grid, ST, lds, s>>>(excl, R, N, tin_tout, kq, K, ex ? koff : nullptr,
                                               ex ? kchild : nullptr, p_excl, p_incl);
  return hipGetLastError();
}

hipError_t launch_tensor_inclusive(const int64_t *T, int64_t n_rows, int G, const int4 *rt,
                                   int64_t *out, int cus, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  if (G > 64) {
    incl_tensor_wide<<<grid_for(n_rows, cus), ST, 0, s>>>(T, n_rows, G, rt, out);
    return hipGetLastError();
  }
  int gp = 1;
  while (gp < G) gp <<= 1;
  const int64_t waves = (n_rows + (64 / gp) - 1) / (64 / gp);
  const int grid = grid_for(waves, cus);
  switch (gp) {
    case 1: incl_tensor_narrow<1><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
    case 2: incl_tensor_narrow<2><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
    case 4: incl_tensor_narrow<4><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
    case 8: incl_tensor_narrow<8><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
    case 16: incl_tensor_narrow<16><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
    case 32: incl_tensor_narrow<32><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
    default: incl_tensor_narrow<64><<<grid, ST, 0, s>>>(T, n_rows, G, rt, out); break;
  }
  return hipGetLastError();
}

}  // namespace ta
