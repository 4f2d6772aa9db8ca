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

constexpr int ST = 256;   // threads of the column-sum and tensor kernels
constexpr int SR = 512;   // threads of the row-scan kernel
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

// x from the lane selected by a DPP control word; lanes with no source (or
// outside `ROWS`) get 0.  64-bit values move as two 32-bit halves.
template <int CTRL, int ROWS>
__device__ inline uint64_t dpp_u64(uint64_t x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROWS, 0xf, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Inclusive scan over the 64 lanes of a wave, on the VALU: shifts by 1, 2, 4
// and 8 within each 16-lane row, then the last lane of row 0 (2) is added to
// row 1 (3), and lane 31 to rows 2 and 3.
__device__ inline uint64_t wave_incl_scan(uint64_t x) {
  x += dpp_u64<0x111, 0xf>(x);  // row_shr:1
  x += dpp_u64<0x112, 0xf>(x);  // row_shr:2
  x += dpp_u64<0x114, 0xf>(x);  // row_shr:4
  x += dpp_u64<0x118, 0xf>(x);  // row_shr:8
  x += dpp_u64<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_u64<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ inline uint64_t lane63(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// Exclusive prefix of P[0..n) in LDS, by wave segments: wave w scans positions
// [w*L, (w+1)*L) (L a multiple of 256; P is zero from n up to NW*L) in tiles of
// 256, lane l taking 4 consecutive positions (two 16-byte reads), and leaves
// the prefix within its segment at the positions below n; seg[w] gets the
// segment's total.  The full prefix of position x < n is then
// P[x] + (sum of seg[w'] for w' < x / L).
__device__ inline void lds_scan_segments(uint64_t *P, int n, int L, uint64_t *seg) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = w * L, e = min(n, b + L);
  uint64_t carry = 0;
  for (int t = b; t < e; t += 256) {
    const int j = t + 4 * lane;
    const u64x2 p0 = *reinterpret_cast<const u64x2 *>(&P[j]);
    const u64x2 p1 = *reinterpret_cast<const u64x2 *>(&P[j + 2]);
    const uint64_t a0 = p0.x, a1 = p0.y, a2 = p1.x, a3 = p1.y;
    const uint64_t sum = (a0 + a1) + (a2 + a3);
    const uint64_t inc = wave_incl_scan(sum);
    uint64_t acc = carry + inc - sum;
    if (j < e) P[j] = acc;
    acc += a0;
    if (j + 1 < e) P[j + 1] = acc;
    acc += a1;
    if (j + 2 < e) P[j + 2] = acc;
    acc += a2;
    if (j + 3 < e) P[j + 3] = acc;
    carry += lane63(inc);
  }
  if (lane == 0) seg[w] = carry;
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

// Positions per wave segment of the row scan: a multiple of 256 with
// (SR / 64) segments covering N.
__host__ __device__ inline int seg_len(int N) {
  const int per = (N + SR / 64 - 1) / (SR / 64);
  return ((per + 255) / 256) * 256 > 0 ? ((per + 255) / 256) * 256 : 256;
}

// Row pass: for each row of rows[n_rows][N] (caller node order) and each query
// k with preorder range q[k] = (tin, tout): incl = sum of the row over the
// range.  With kpar (kpar[k] = the query that is k's nearest query strict
// ancestor, or -1), excl[k] = incl[k] minus the incl of every query whose kpar
// is k: the row's cost on the nodes whose nearest query ancestor-or-self is k
// (exact: 64-bit LDS atomics on integers).
//
// Thread t owns nodes t + SR*u (u < B, B*SR >= N): their preorder positions
// stay in registers, a row arrives in one batch of loads, and the next row's
// loads are issued before the current row is scanned.  With KB > 0 (K <=
// KB*SR) the queries' ranges and parents also stay in registers, so nothing
// waits on the prefetch until the next row is scattered (vector memory
// counters retire in order).
template <int B, int KB>
__global__ __launch_bounds__(SR) void subtree_rows(const int64_t *__restrict__ rows, int64_t n_rows,
                                                  int N, const int2 *__restrict__ tin_tout,
                                                  const int2 *__restrict__ q, int K,
                                                  const int32_t *__restrict__ kpar,
                                                  int64_t *__restrict__ out_excl,
                                                  int64_t *__restrict__ out_incl) {
  constexpr int NW = SR / 64;
  constexpr int KR = KB > 0 ? KB : 1;
  extern __shared__ uint64_t lds[];
  __shared__ uint64_t seg[NW];
  const int L = seg_len(N);
  uint64_t *P = lds;           // [NW * L], zero from N on
  uint64_t *E = lds + NW * L;  // [K] when out_excl
  for (int j = N + threadIdx.x; j < NW * L; j += SR) P[j] = 0;
  int pos[B];
  uint64_t x[B];
#pragma unroll
  for (int u = 0; u < B; u++) {
    const int v = threadIdx.x + SR * u;
    pos[u] = v < N ? tin_tout[v].x : -1;
  }
  int2 qk[KR];
  int pk[KR];
#pragma unroll
  for (int i = 0; i < KR; i++) {
    const int k = threadIdx.x + SR * i;
    const bool on = KB > 0 && k < K;
    qk[i] = on ? q[k] : make_int2(0, 0);
    pk[i] = on && out_excl ? kpar[k] : -1;
  }
  auto load_row = [&](int64_t r) {
    const int64_t *row = rows + r * N;
#pragma unroll
    for (int u = 0; u < B; u++) x[u] = pos[u] >= 0 ? (uint64_t)row[threadIdx.x + SR * u] : 0;
  };
  int64_t r = blockIdx.x;
  if (r < n_rows) load_row(r);
  for (; r < n_rows; r += gridDim.x) {
#pragma unroll
    for (int u = 0; u < B; u++)
      if (pos[u] >= 0) P[pos[u]] = x[u];
    __syncthreads();
    if (r + gridDim.x < n_rows) load_row(r + gridDim.x);  // in flight during the scan
    lds_scan_segments(P, N, L, seg);
    __syncthreads();
    uint64_t off[NW + 1];
    off[0] = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) off[w + 1] = off[w] + seg[w];
    // full exclusive prefix at position p in [0, N]
    auto pref = [&](int p) -> uint64_t { return p >= N ? off[NW] : P[p] + off[p / L]; };
    if (KB > 0) {
      uint64_t inc[KR];
#pragma unroll
      for (int i = 0; i < KR; i++) {
        const int k = threadIdx.x + SR * i;
        inc[i] = k < K ? pref(qk[i].y) - pref(qk[i].x) : 0;
        if (out_excl && k < K) E[k] = inc[i];
      }
      if (out_excl) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < KR; i++)
          if (pk[i] >= 0) atomicAdd((unsigned long long *)&E[pk[i]], (unsigned long long)(0 - inc[i]));
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < KR; i++) {
        const int k = threadIdx.x + SR * i;
        if (k < K) {
          if (out_excl) out_excl[r * K + k] = (int64_t)E[k];
          if (out_incl) out_incl[r * K + k] = (int64_t)inc[i];
        }
      }
    } else {
      for (int k = threadIdx.x; k < K; k += SR) {
        const int2 t = q[k];
        const uint64_t inc = pref(t.y) - pref(t.x);
        if (out_excl) E[k] = inc;
        if (out_incl) out_incl[r * K + k] = (int64_t)inc;
      }
      if (out_excl) {
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += SR) {
          const int2 t = q[k];
          const int p = kpar[k];
          if (p >= 0) atomicAdd((unsigned long long *)&E[p], (unsigned long long)(0 - (pref(t.y) - pref(t.x))));
        }
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += SR) out_excl[r * K + k] = (int64_t)E[k];
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

// The inclusive-tensor kernels may run in place (out == T): a row is read
// whole by one wave before that wave writes it, and no other wave touches it.
//
// Inclusive tensor, G <= 64: segments of GP lanes (GP = power of two >= G),
// 64 / GP rows per wave.  Lane j of a segment holds the value of the region at
// region-preorder position j; a segmented inclusive scan S gives the range sum
// over [j, end_j) as S[end_j - 1] - S[j] + v_j.
template <int GP>
__global__ __launch_bounds__(ST) void incl_tensor_narrow(const int64_t *T, int64_t n_rows, int G,
                                                        const int4 *__restrict__ rt,
                                                        int64_t *out) {
  constexpr int RPW = 64 / GP;  // rows per wave-step
  constexpr int RB = 4;         // wave-steps whose loads are issued together
  const int lane = threadIdx.x & 63;
  const int seg = lane / GP, j = lane % GP;
  const int64_t wave = ((int64_t)blockIdx.x * ST + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * ST) >> 6;
  const int4 t = (j < G) ? rt[j] : make_int4(0, 0, 0, 1);
  const int g = t.z, last = t.w - 1;  // region at position j; last position of its range
  for (int64_t r0 = wave * RPW * RB; r0 < n_rows; r0 += n_waves * RPW * RB) {
    uint64_t v[RB];
#pragma unroll
    for (int b = 0; b < RB; b++) {
      const int64_t r = r0 + b * RPW + seg;
      v[b] = (j < G && r < n_rows) ? (uint64_t)T[r * G + g] : 0;
    }
#pragma unroll
    for (int b = 0; b < RB; b++) {
      const int64_t r = r0 + b * RPW + seg;
      uint64_t x = v[b];
#pragma unroll
      for (int d = 1; d < GP; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, GP);
        if (j >= d) x += y;
      }
      const uint64_t e = __shfl(x, last, GP);
      if (j < G && r < n_rows) out[r * G + g] = (int64_t)(e - x + v[b]);
    }
  }
}

// Inclusive tensor, 64 < G <= 256: one row per wave, RB rows whose loads are
// issued together.  Lane l loads and stores regions l + 64c (coalesced); the
// values go to LDS at their region-preorder positions, lane l scans positions
// 4l .. 4l+3 locally, one wave scan joins the lanes, and the exclusive prefix
// E (E[G] = row total) goes back to LDS: out[g] = E[end(g)] - E[pos(g)].
__global__ __launch_bounds__(ST) void incl_tensor_wide(const int64_t *T, int64_t n_rows, int G,
                                                      const int4 *__restrict__ rt,
                                                      int64_t *out) {
  constexpr int RB = 4;
  __shared__ uint64_t S[ST / 64][MAX_REGIONS + 4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t *P = S[w];
  const int64_t wave = ((int64_t)blockIdx.x * ST + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * ST) >> 6;
  int ps[4], pe[4];
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int g = lane + 64 * c;
    const int4 t = g < G ? rt[g] : make_int4(0, 0, 0, 0);
    ps[c] = t.x;
    pe[c] = t.y;
  }
  for (int64_t r0 = wave * RB; r0 < n_rows; r0 += n_waves * RB) {
    uint64_t v[RB][4];
#pragma unroll
    for (int b = 0; b < RB; b++)
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const int g = lane + 64 * c;
        v[b][c] = (g < G && r0 + b < n_rows) ? (uint64_t)T[(r0 + b) * G + g] : 0;
      }
#pragma unroll
    for (int b = 0; b < RB; b++) {
      if (r0 + b >= n_rows) break;
#pragma unroll
      for (int c = 0; c < 4; c++)
        if (lane + 64 * c < G) P[ps[c]] = v[b][c];
      __builtin_amdgcn_wave_barrier();
      uint64_t a[4], s = 0;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        a[u] = 4 * lane + u < G ? P[4 * lane + u] : 0;
        s += a[u];
      }
      uint64_t acc = wave_incl_scan(s) - s;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < 4; u++) {
        P[4 * lane + u] = acc;  // exclusive prefix; positions >= G hold the total
        acc += a[u];
      }
      if (lane == 63) P[4 * 64] = acc;  // the total, for G = 256
      __builtin_amdgcn_wave_barrier();
      int64_t *o = out + (r0 + b) * G;
#pragma unroll
      for (int c = 0; c < 4; c++)
        if (lane + 64 * c < G) o[lane + 64 * c] = (int64_t)(P[pe[c]] - P[ps[c]]);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

int grid_for(int64_t waves_of_work, int device_cus_hint) {
  const int64_t cap = (int64_t)device_cus_hint * 16;
  int64_t g = (waves_of_work + (ST / 64) - 1) / (ST / 64);
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

template <int B>
void allow_big_lds_b() {
  const void *fns[] = {reinterpret_cast<const void *>(&subtree_rows<B, 0>),
                       reinterpret_cast<const void *>(&subtree_rows<B, 1>),
                       reinterpret_cast<const void *>(&subtree_rows<B, 2>)};
  for (const void *f : fns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
}

void allow_big_lds() {
  static bool done = false;
  if (!done) {
    allow_big_lds_b<2>();
    allow_big_lds_b<4>();
    allow_big_lds_b<8>();
    allow_big_lds_b<12>();
    allow_big_lds_b<16>();
    done = true;
  }
}

// Registers per thread: B >= ceil(N / SR) row values, KB >= ceil(K / SR)
// queries (0: queries read from memory, any K).
template <int B>
void launch_rows_b(int grid, size_t lds, hipStream_t s, const int64_t *rows, int64_t n_rows,
                          int N, const int2 *tin_tout, const int2 *q, int K, const int32_t *kpar,
                          int64_t *out_excl, int64_t *out_incl) {
  const int kq = (K + SR - 1) / SR;
  if (kq <= 1)
    subtree_rows<B, 1><<<grid, SR, lds, s>>>(rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
  else if (kq <= 2)
    subtree_rows<B, 2><<<grid, SR, lds, s>>>(rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
  else
    subtree_rows<B, 0><<<grid, SR, lds, s>>>(rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
}

void launch_rows(int grid, size_t lds, hipStream_t s, const int64_t *rows, int64_t n_rows,
                        int N, const int2 *tin_tout, const int2 *q, int K, const int32_t *kpar,
                        int64_t *out_excl, int64_t *out_incl) {
  const int per = (N + SR - 1) / SR;
  if (per <= 2) launch_rows_b<2>(grid, lds, s, rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
  else if (per <= 4) launch_rows_b<4>(grid, lds, s, rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
  else if (per <= 8) launch_rows_b<8>(grid, lds, s, rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
  else if (per <= 12) launch_rows_b<12>(grid, lds, s, rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
  else launch_rows_b<16>(grid, lds, s, rows, n_rows, N, tin_tout, q, K, kpar, out_excl, out_incl);
}

}  // namespace

size_t subtree_rows_lds_bytes(int N, int K, bool excl) {
  return ((size_t)(SR / 64) * seg_len(N) + (excl ? (size_t)K : 0)) * sizeof(uint64_t);
}

// ---- subtree sums of one node vector, any tree size --------------------------
// N <= 8192: one workgroup scans the vector in LDS (subtree_rows).  Larger: the
// vector is scattered to preorder positions, scanned in blocks of SB positions
// (block-local prefixes + block totals), the block totals are scanned by one
// workgroup, and out[v] = P[tout(v)] - P[tin(v)] with P[x] = local[x] +
// total of the blocks before x.
constexpr int SBT = 1024;          // threads of the block-scan kernels
constexpr int SBE = 4;             // positions per thread
constexpr int SB = SBT * SBE;      // positions per block

__global__ void pre_scatter(const int64_t *__restrict__ vec, int N, const int2 *__restrict__ tin_tout,
                            uint64_t *__restrict__ P) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N;
       v += (int64_t)gridDim.x * blockDim.x)
    P[tin_tout[v].x] = (uint64_t)vec[v];
}

__global__ __launch_bounds__(SBT) void block_scan_local(uint64_t *__restrict__ P, int N,
                                                       uint64_t *__restrict__ bt) {
  __shared__ uint64_t wsum[SBT / 64];
  const int64_t base = (int64_t)blockIdx.x * SB + (int64_t)threadIdx.x * SBE;
  uint64_t a[SBE], s = 0;
#pragma unroll
  for (int u = 0; u < SBE; u++) {
    a[u] = base + u < N ? P[base + u] : 0;
    s += a[u];
  }
  uint64_t total;
  uint64_t acc = block_excl_scan<SBT>(s, wsum, &total);
#pragma unroll
  for (int u = 0; u < SBE; u++) {
    if (base + u < N) P[base + u] = acc;
    acc += a[u];
  }
  if (threadIdx.x == 0) bt[blockIdx.x] = total;
}

// Exclusive scan of the nb block totals in place (nb <= SBT * SBE); bt[nb] = total.
__global__ __launch_bounds__(SBT) void block_scan_totals(uint64_t *__restrict__ bt, int nb) {
  __shared__ uint64_t wsum[SBT / 64];
  const int base = threadIdx.x * SBE;
  uint64_t a[SBE], s = 0;
#pragma unroll
  for (int u = 0; u < SBE; u++) {
    a[u] = base + u < nb ? bt[base + u] : 0;
    s += a[u];
  }
  uint64_t total;
  uint64_t acc = block_excl_scan<SBT>(s, wsum, &total);
#pragma unroll
  for (int u = 0; u < SBE; u++) {
    if (base + u < nb) bt[base + u] = acc;
    acc += a[u];
  }
  if (threadIdx.x == 0) bt[nb] = total;
}

__global__ void subtree_from_prefix(const uint64_t *__restrict__ P, const uint64_t *__restrict__ bt,
                                    int N, int nb, const int2 *__restrict__ tin_tout,
                                    int64_t *__restrict__ out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int2 t = tin_tout[v];
    auto pref = [&](int x) -> uint64_t { return x >= N ? bt[nb] : P[x] + bt[x / SB]; };
    out[v] = (int64_t)(pref(t.y) - pref(t.x));
  }
}

hipError_t launch_summary(const int64_t *excl, int64_t R, int N, const int2 *tin_tout,
                          int64_t *sum_excl, int64_t *sum_incl, void *ws, int cus, hipStream_t s) {
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
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sum_incl) return e;
  return launch_subtree_sums(sum_excl, N, tin_tout, sum_incl, ws, cus, s);
}

hipError_t launch_prune(const int64_t *sum_excl, const int64_t *sum_incl, int N, double fraction,
                        int32_t *kept, int32_t *n_kept, hipStream_t s) {
  prune_kernel<<<1, PT, 0, s>>>(sum_excl, sum_incl, N, fraction, kept, n_kept);
  return hipGetLastError();
}

hipError_t launch_pruned_profiles(const int64_t *excl, int64_t R, int N, const int2 *tin_tout,
                                  const int2 *kq, int K, const int32_t *kpar, int64_t *p_excl,
                                  int64_t *p_incl, int cus, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const bool ex = p_excl != nullptr;
  const size_t lds = subtree_rows_lds_bytes(N, K, ex);
  allow_big_lds();
  // LDS bounds the workgroups per CU; a grid of a few per CU streams the rows.
  int per_cu = (int)((160 * 1024) / (lds + 1024));
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > R) grid = R;
  launch_rows((int)grid, lds, s, excl, R, N, tin_tout, kq, K, ex ? kpar : nullptr, p_excl,
              p_incl);
  return hipGetLastError();
}

hipError_t launch_tensor_inclusive(const int64_t *T, int64_t n_rows, int G, const int4 *rt,
                                   int64_t *out, int cus, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  if (G > 64) {
    incl_tensor_wide<<<grid_for((n_rows + 3) / 4, cus), ST, 0, s>>>(T, n_rows, G, rt, out);
    return hipGetLastError();
  }
  int gp = 1;
  while (gp < G) gp <<= 1;
  const int64_t per_wave = 4 * (64 / gp);  // rows per wave per iteration
  const int64_t waves = (n_rows + per_wave - 1) / per_wave;
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

size_t subtree_sums_ws_bytes(int N) {
  if (N <= MAX_NODES_ATTR) return 0;
  const int64_t nb = ((int64_t)N + SB - 1) / SB;
  return ((size_t)N + (size_t)nb + 1) * sizeof(uint64_t);
}

hipError_t launch_subtree_sums(const int64_t *vec, int N, const int2 *tin_tout, int64_t *out, void *ws,
                               int cus, hipStream_t s) {
  if (N <= MAX_NODES_ATTR) {
    allow_big_lds();
    const size_t lds = subtree_rows_lds_bytes(N, N, false);
    launch_rows(1, lds, s, vec, 1, N, tin_tout, tin_tout, N, nullptr, nullptr, out);
    return hipGetLastError();
  }
  const int nb = (int)(((int64_t)N + SB - 1) / SB);
  if (nb > SBT * SBE) return hipErrorInvalidValue;
  uint64_t *P = (uint64_t *)ws;
  uint64_t *bt = P + N;
  int g = (N + 255) / 256;
  if (g > cus * 8) g = cus * 8;
  pre_scatter<<<g, 256, 0, s>>>(vec, N, tin_tout, P);
  block_scan_local<<<nb, SBT, 0, s>>>(P, N, bt);
  block_scan_totals<<<1, SBT, 0, s>>>(bt, nb);
  subtree_from_prefix<<<g, 256, 0, s>>>(P, bt, N, nb, tin_tout, out);
  return hipGetLastError();
}

}  // namespace ta
