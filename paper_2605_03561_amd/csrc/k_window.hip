// k_window.hip -- profile of a time window for any subset of ranks (Sec. II:
// a calling context tree for a trace interval).  Each event's interval
// [t_k, t_{k+1}) (a rank's last event lasts 0) is clipped to [t0, t1) and added
// to its context node; inclusive costs are subtree sums of the result.
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int WT = 256;   // threads of the small kernels
constexpr int WWT = 512;  // threads of a window workgroup

typedef long long v2ll __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));

// Visits events k in [lo, hi) of a rank whose events end at e, four
// consecutive events per thread per step from a 4-aligned index (16-byte loads
// of timestamps and contexts; scalar loads within 4 events of the array's end
// E), DEPTH steps' loads in flight before any is visited.  f(k, t_k, t_{k+1}
// (t_k for the rank's last event), ctx_k).
struct EvQuad {
  int64_t t[5];
  int32_t c[4];
};

__device__ inline EvQuad load_quad(const int64_t *__restrict__ ts, const int32_t *__restrict__ ctx,
                                   int64_t E, int64_t k0, int64_t e) {
  EvQuad q;
  if (k0 + 4 <= E) {
    const v2ll a = *reinterpret_cast<const v2ll *>(ts + k0);
    const v2ll b = *reinterpret_cast<const v2ll *>(ts + k0 + 2);
    const v4i c = *reinterpret_cast<const v4i *>(ctx + k0);
    q.t[0] = a.x;
    q.t[1] = a.y;
    q.t[2] = b.x;
    q.t[3] = b.y;
    q.c[0] = c.x;
    q.c[1] = c.y;
    q.c[2] = c.z;
    q.c[3] = c.w;
  } else {
#pragma unroll
    for (int u = 0; u < 4; u++) {
      q.t[u] = k0 + u < E ? ts[k0 + u] : 0;
      q.c[u] = k0 + u < E ? ctx[k0 + u] : 0;
    }
  }
  q.t[4] = k0 + 4 < e ? ts[k0 + 4] : 0;
  return q;
}

template <int NT, int DEPTH, class F>
__device__ inline void visit_events(const int64_t *__restrict__ ts, const int32_t *__restrict__ ctx,
                                    int64_t E, int64_t lo, int64_t hi, int64_t e, F &&f) {
  auto visit = [&](const EvQuad &q, int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int64_t k = k0 + u;
      if (k < lo || k >= hi) continue;
      f(k, q.t[u], k + 1 < e ? q.t[u + 1] : q.t[u], q.c[u]);
    }
  };
  constexpr int64_t STEP = 4 * (int64_t)NT;
  for (int64_t k0 = (lo & ~(int64_t)3) + 4 * (int64_t)threadIdx.x; k0 < hi; k0 += DEPTH * STEP) {
    // every load is in bounds of the arrays (load_quad guards E); a later
    // step that starts at or past hi loads nothing (visit skips its events)
    EvQuad q[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH; d++) {
      q[d] = EvQuad{};
      if (d == 0 || k0 + d * STEP < hi) q[d] = load_quad(ts, ctx, E, k0 + d * STEP, e);
    }
#pragma unroll
    for (int d = 0; d < DEPTH; d++) visit(q[d], k0 + d * STEP);
  }
}

__global__ void zero_i64(int64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// First index in [a, z) whose timestamp satisfies a monotone predicate (false
// then true), or z: binary search by one thread.
template <class P>
__device__ inline int64_t first_true(const int64_t *__restrict__ ts, int64_t a, int64_t z, P pred) {
  while (a < z) {
    const int64_t m = a + ((z - a) >> 1);
    if (pred(ts[m])) z = m;
    else a = m + 1;
  }
  return a;
}

// The events of each selected rank that overlap the window, one thread per
// rank (so the searches' round trips overlap one another): before the event
// preceding the first timestamp above t0 every interval ends by t0; from the
// first timestamp at or above t1 every interval starts at or after t1.
// bounds[i] = {lo, hi, e (the rank's end), 0}; an invalid rank gets an empty
// range and sets the offsets error bit.
__global__ __launch_bounds__(WT) void window_bounds(const int64_t *__restrict__ off,
                                                   const int64_t *__restrict__ ts, int64_t R, int64_t E,
                                                   const int32_t *__restrict__ ids, int64_t n_sel,
                                                   int64_t t0, int64_t t1, v2ll *__restrict__ bounds,
                                                   uint32_t *err) {
  const int64_t i = (int64_t)blockIdx.x * WT + threadIdx.x;
  if (i >= n_sel) return;
  const int64_t r = ids ? (int64_t)ids[i] : i;
  int64_t lo = 0, hi = 0, e = 0;
  if (r < 0 || r >= R || off[r] < 0 || off[r + 1] < off[r] || off[r + 1] > E) {
    atomicOr(err, ERRBIT_OFFSETS);
  } else {
    const int64_t b = off[r];
    e = off[r + 1];
    const int64_t a = first_true(ts, b, e, [&](int64_t v) { return v > t0; });
    lo = a > b ? a - 1 : b;
    hi = first_true(ts, b, e, [&](int64_t v) { return v >= t1; });
  }
  bounds[2 * i] = v2ll{lo, hi};
  bounds[2 * i + 1] = v2ll{e, 0};
}

// One workgroup per selected rank (grid-stride over the selection) over the
// events window_bounds found.  LDSH: an LDS histogram over the N nodes
// (N <= 8192) flushed once; otherwise 64-bit atomics on the output.  Integer
// sums: the order of the atomics does not matter.
template <bool LDSH>
__global__ __launch_bounds__(WWT) void window_excl(const int64_t *__restrict__ ts,
                                                 const int32_t *__restrict__ ctx, int64_t E,
                                                 const v2ll *__restrict__ bounds, int64_t n_sel, int N,
                                                 int64_t t0, int64_t t1, int64_t *__restrict__ excl,
                                                 uint32_t *err) {
  extern __shared__ uint64_t hist[];  // [N] when LDSH
  if (LDSH) {
    for (int v = threadIdx.x; v < N; v += WWT) hist[v] = 0;
  }
  __syncthreads();
  for (int64_t i = blockIdx.x; i < n_sel; i += gridDim.x) {
    const v2ll b0 = bounds[2 * i], b1 = bounds[2 * i + 1];
    const int64_t lo = b0.x, hi = b0.y, e = b1.x;
    visit_events<WWT, 2>(ts, ctx, E, lo, hi, e, [&](int64_t, int64_t s, int64_t f, int32_t c) {
      if (f < s) atomicOr(err, ERRBIT_UNSORTED);
      const int64_t a = s > t0 ? s : t0;
      const int64_t z = f < t1 ? f : t1;
      if (z > a) {
        if (c < 0 || c >= N) {
          atomicOr(err, ERRBIT_CTX);
        } else if (LDSH) {
          atomicAdd((unsigned long long *)&hist[c], (unsigned long long)(z - a));
        } else {
          atomicAdd((unsigned long long *)&excl[c], (unsigned long long)(z - a));
        }
      }
    });
  }
  if (LDSH) {
    __syncthreads();
    for (int v = threadIdx.x; v < N; v += WWT)
      if (hist[v]) atomicAdd((unsigned long long *)&excl[v], (unsigned long long)hist[v]);
  }
}

// ---- sparse per-rank profiles --------------------------------------------------

constexpr int SPT = 1024;               // threads per rank workgroup
constexpr int SPC = 8192;               // node ids per chunk (64 KB LDS histogram)
constexpr int SPE = SPC / SPT;          // bins per thread in the compaction
constexpr int SPW = MAX_NODES / SPC / 32;  // words of the touched-chunk mask
constexpr int SPBW = 4096;              // node-mask words: trees of up to 131,072 nodes take one pass
constexpr int SPBT = SPBW / SPT;        // mask words per thread
constexpr int SPACC = 4096;             // distinct nodes a rank may reach on the one-pass path

// Exclusive scan of per-thread counts over the workgroup; *total = the sum.
__device__ inline int block_excl_scan_i32(int v, int *wsum, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int base = 0, all = 0;
#pragma unroll
  for (int i = 0; i < SPT / 64; i++) {
    const int s = wsum[i];
    base += i < w ? s : 0;
    all += s;
  }
  __syncthreads();
  *total = all;
  return base + x - v;
}

// One workgroup per rank (grid-stride).  Trees of more than SPC nodes and at
// most SPBW * 32: a pass over the events' contexts (4 bytes per event) marks
// the nodes they reach in an LDS bit mask; a workgroup scan of the mask's word
// counts gives each reached node an accumulator index (ascending id); a
// second pass adds the durations into the LDS accumulator at those indices
// (exact 64-bit atomics), and the nodes with a positive total are written in
// ascending id (a second scan of the per-thread counts of those).  Otherwise,
// or when a rank reaches more than SPACC nodes:
// for each chunk of SPC node ids that the events reach, an LDS histogram of
// the chunk, then its non-zero bins in ascending id, compacted by a workgroup
// scan and appended after the previous chunks'.  Output goes to the rank's own
// event range.
__global__ __launch_bounds__(SPT) void sparse_profiles_kernel(const int64_t *__restrict__ off,
                                                             const int64_t *__restrict__ ts,
                                                             const int32_t *__restrict__ ctx,
                                                             int64_t R, int64_t E, int N,
                                                             int64_t *__restrict__ counts,
                                                             int32_t *__restrict__ ids,
                                                             int64_t *__restrict__ vals,
                                                             uint32_t *err) {
  __shared__ uint64_t pool[SPC];  // chunk histogram, or mask | word prefixes | accumulator
  __shared__ uint32_t touched[SPW];
  __shared__ int wsum[SPT / 64];
  uint64_t *hist = pool;
  uint32_t *bm = reinterpret_cast<uint32_t *>(pool);
  uint32_t *pre = bm + SPBW;
  uint64_t *acc = pool + SPBW;
  const int n_chunks = (N + SPC - 1) / SPC;
  const bool one_pass = n_chunks > 1 && N <= SPBW * 32;
  const int nw = (N + 31) / 32;
  const int t = threadIdx.x;
  for (int64_t r = blockIdx.x; r < R; r += gridDim.x) {
    // a rank's range, clamped to [0, E] (inconsistent offsets are an error)
    const int64_t o0 = off[r], o1 = off[r + 1];
    const bool bad = o0 < 0 || o1 < o0 || o1 > E;
    const int64_t b = bad ? 0 : o0, e = bad ? 0 : o1;
    if (bad && t == 0) atomicOr(err, ERRBIT_OFFSETS);
    auto dur = [&](int64_t k) -> int64_t { return k + 1 < e ? ts[k + 1] - ts[k] : 0; };
    int64_t base = 0;
    bool done = false;
    if (one_pass) {
      for (int i = t; i < nw; i += SPT) bm[i] = 0;
      __syncthreads();
      // the nodes the rank's events reach, from the contexts alone (4 bytes
      // per event; the durations are read once, by the accumulating pass)
      for (int64_t k0 = (b & ~(int64_t)3) + 4 * (int64_t)t; k0 < e; k0 += 4 * (int64_t)SPT) {
        int32_t c4[4];
        if (k0 + 4 <= E) {
          const v4i q = *reinterpret_cast<const v4i *>(ctx + k0);
          c4[0] = q.x;
          c4[1] = q.y;
          c4[2] = q.z;
          c4[3] = q.w;
        } else {
#pragma unroll
          for (int u = 0; u < 4; u++) c4[u] = k0 + u < E ? ctx[k0 + u] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          if (k0 + u < b || k0 + u >= e) continue;
          const int32_t c = c4[u];
          if (c < 0 || c >= N) atomicOr(err, ERRBIT_CTX);
          else atomicOr(&bm[c >> 5], 1u << (c & 31));
        }
      }
      __syncthreads();
      uint32_t wv[SPBT];
      int own = 0;
#pragma unroll
      for (int u = 0; u < SPBT; u++) {
        const int w = t * SPBT + u;
        wv[u] = w < nw ? bm[w] : 0u;
        own += __popc(wv[u]);
      }
      int total;
      int pos = block_excl_scan_i32(own, wsum, &total);
#pragma unroll
      for (int u = 0; u < SPBT; u++) {
        const int w = t * SPBT + u;
        if (w < nw) pre[w] = (uint32_t)pos;
        pos += __popc(wv[u]);
      }
      if (total <= SPACC) {  // uniform
        for (int i = t; i < total; i += SPT) acc[i] = 0;
        __syncthreads();
        visit_events<SPT, 1>(ts, ctx, E, b, e, e, [&](int64_t, int64_t s, int64_t f, int32_t c) {
          const int64_t d = f - s;
          if (d < 0) atomicOr(err, ERRBIT_UNSORTED);
          if (c >= 0 && c < N && d > 0) {
            const int w = c >> 5;
            const int idx = (int)pre[w] + __popc(bm[w] & ((1u << (c & 31)) - 1u));
            atomicAdd((unsigned long long *)&acc[idx], (unsigned long long)d);
          }
        });
        __syncthreads();
        // the reached nodes with a positive total, in ascending id: a node
        // reached only by zero durations is marked but not written
        int nz = 0;
#pragma unroll
        for (int u = 0; u < SPBT; u++) {
          const int w = t * SPBT + u;
          if (w >= nw) continue;
          const int p0 = (int)pre[w];
          for (int q = 0; q < __popc(wv[u]); q++) nz += acc[p0 + q] != 0 ? 1 : 0;
        }
        int nz_total;
        int o = block_excl_scan_i32(nz, wsum, &nz_total);
#pragma unroll
        for (int u = 0; u < SPBT; u++) {
          const int w = t * SPBT + u;
          if (w >= nw) continue;
          uint32_t m = wv[u];
          int p = (int)pre[w];
          while (m) {
            const int j = __ffs(m) - 1;
            m &= m - 1u;
            if (acc[p] != 0) {
              ids[b + o] = w * 32 + j;
              vals[b + o] = (int64_t)acc[p];
              o++;
            }
            p++;
          }
        }
        base = nz_total;
        done = true;
      }
      __syncthreads();
    }
    if (!done) {
      if (n_chunks > 1) {
        for (int i = t; i < SPW; i += SPT) touched[i] = 0;
        __syncthreads();
        for (int64_t k = b + t; k < e; k += SPT) {
          const int32_t c = ctx[k];
          if (c >= 0 && c < N && dur(k) > 0) atomicOr(&touched[(c / SPC) >> 5], 1u << ((c / SPC) & 31));
        }
        __syncthreads();
      }
      for (int ch = 0; ch < n_chunks; ch++) {
        if (n_chunks > 1 && !((touched[ch >> 5] >> (ch & 31)) & 1u)) continue;  // uniform
        const int lo = ch * SPC;
        for (int i = t; i < SPC; i += SPT) hist[i] = 0;
        __syncthreads();
        visit_events<SPT, 1>(ts, ctx, E, b, e, e, [&](int64_t, int64_t s, int64_t f, int32_t c) {
          const int64_t d = f - s;
          if (d < 0) atomicOr(err, ERRBIT_UNSORTED);
          if (c < 0 || c >= N) {
            if (ch == 0) atomicOr(err, ERRBIT_CTX);
          } else if (c >= lo && c < lo + SPC && d != 0) {
            atomicAdd((unsigned long long *)&hist[c - lo], (unsigned long long)d);
          }
        });
        __syncthreads();
        uint64_t v[SPE];
        int nz = 0;
#pragma unroll
        for (int u = 0; u < SPE; u++) {
          v[u] = hist[t * SPE + u];
          nz += v[u] != 0 ? 1 : 0;
        }
        int total;
        int pos = block_excl_scan_i32(nz, wsum, &total);
#pragma unroll
        for (int u = 0; u < SPE; u++)
          if (v[u] != 0) {
            const int64_t o = b + base + pos++;
            ids[o] = lo + t * SPE + u;
            vals[o] = (int64_t)v[u];
          }
        base += total;
        __syncthreads();
      }
    }
    if (t == 0) counts[r] = base;
    __syncthreads();
  }
}

int grid_w(int64_t n, int cus, int per_cu) {
  int64_t g = n < (int64_t)cus * per_cu ? n : (int64_t)cus * per_cu;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

// The subtree-sum workspace, then 32 bytes of event bounds per selected rank.
size_t window_ws_bytes(int N, int64_t n_sel) {
  return ((subtree_sums_ws_bytes(N) + 255) & ~(size_t)255) + (size_t)(n_sel > 0 ? n_sel : 0) * 32;
}

hipError_t launch_window_profile(const int64_t *off, const int64_t *ts, const int32_t *ctx, int64_t R,
                                 int64_t E, const int32_t *ids, int64_t n_sel, int N, const int2 *tin_tout,
                                 int64_t t0, int64_t t1, int64_t *excl, int64_t *incl, void *ws,
                                 uint32_t *err, int cus, hipStream_t s) {
  zero_i64<<<grid_w((N + WT - 1) / WT, cus, 4), WT, 0, s>>>(excl, N);
  if (n_sel > 0) {
    v2ll *bounds = reinterpret_cast<v2ll *>(static_cast<char *>(ws) +
                                            ((subtree_sums_ws_bytes(N) + 255) & ~(size_t)255));
    window_bounds<<<(unsigned)((n_sel + WT - 1) / WT), WT, 0, s>>>(off, ts, R, E, ids, n_sel, t0, t1,
                                                                   bounds, err);
    if (N <= MAX_NODES_ATTR) {
      static bool attr = false;
      if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&window_excl<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
        attr = true;
      }
      window_excl<true><<<grid_w(n_sel, cus, 4), WWT, (size_t)N * 8, s>>>(ts, ctx, E, bounds, n_sel, N,
                                                                         t0, t1, excl, err);
    } else {
      window_excl<false><<<grid_w(n_sel, cus, 4), WWT, 0, s>>>(ts, ctx, E, bounds, n_sel, N, t0, t1,
                                                              excl, err);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !incl) return e;
  return launch_subtree_sums(excl, N, tin_tout, incl, ws, cus, s);
}

hipError_t launch_sparse_profiles(const int64_t *off, const int64_t *ts, const int32_t *ctx, int64_t R,
                                  int64_t E, int N, int64_t *counts, int32_t *ids, int64_t *vals, uint32_t *err,
                                  int cus, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  sparse_profiles_kernel<<<grid_w(R, cus, 2), SPT, 0, s>>>(off, ts, ctx, R, E, N, counts, ids, vals, err);
  return hipGetLastError();
}

}  // namespace ta
