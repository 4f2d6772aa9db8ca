// k_window.hip -- profile of a time window for any subset of ranks (Sec. II:
// a calling context tree for a trace interval).  Each event's interval
// [t_k, t_{k+1}) (a rank's last event lasts 0) is clipped to [t0, t1) and added
// to its context node; inclusive costs are subtree sums of the result.
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int WT = 256;

__global__ void zero_i64(int64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// One workgroup per selected rank (grid-stride over the selection).  Binary
// searches on the rank's sorted timestamps bound the events that overlap the
// window: before the event preceding the first timestamp above t0 every
// interval ends by t0; from the first timestamp at or above t1 every interval
// starts at or after t1.  LDSH: an LDS histogram over the N nodes (N <= 8192)
// flushed once; otherwise 64-bit atomics on the output.  Integer sums: the
// order of the atomics does not matter.
template <bool LDSH>
__global__ __launch_bounds__(WT) void window_excl(const int64_t *__restrict__ off,
                                                 const int64_t *__restrict__ ts,
                                                 const int32_t *__restrict__ ctx, int64_t R,
                                                 const int32_t *__restrict__ ids, int64_t n_sel,
                                                 int N, int64_t t0, int64_t t1,
                                                 int64_t *__restrict__ excl, uint32_t *err) {
  extern __shared__ uint64_t hist[];  // [N] when LDSH
  __shared__ int64_t range[3];
  if (LDSH) {
    for (int v = threadIdx.x; v < N; v += WT) hist[v] = 0;
  }
  __syncthreads();
  for (int64_t i = blockIdx.x; i < n_sel; i += gridDim.x) {
    if (threadIdx.x == 0) {
      const int64_t r = ids ? (int64_t)ids[i] : i;
      int64_t lo = 0, hi = 0, e = 0;
      if (r < 0 || r >= R || off[r + 1] < off[r]) {
        atomicOr(err, ERRBIT_OFFSETS);
      } else {
        const int64_t b = off[r];
        e = off[r + 1];
        int64_t a = b, z = e;  // first index with ts > t0
        while (a < z) {
          const int64_t m = (a + z) >> 1;
          if (ts[m] > t0) z = m;
          else a = m + 1;
        }
        lo = a > b ? a - 1 : b;
        a = b;
        z = e;  // first index with ts >= t1
        while (a < z) {
          const int64_t m = (a + z) >> 1;
          if (ts[m] >= t1) z = m;
          else a = m + 1;
        }
        hi = a;
      }
      range[0] = lo;
      range[1] = hi;
      range[2] = e;
    }
    __syncthreads();
    const int64_t lo = range[0], hi = range[1], e = range[2];
    for (int64_t k = lo + threadIdx.x; k < hi; k += WT) {
      const int64_t s = ts[k];
      const int64_t f = k + 1 < e ? ts[k + 1] : s;
      if (f < s) atomicOr(err, ERRBIT_UNSORTED);
      const int64_t a = s > t0 ? s : t0;
      const int64_t z = f < t1 ? f : t1;
      if (z > a) {
        const int32_t c = ctx[k];
        if (c < 0 || c >= N) {
          atomicOr(err, ERRBIT_CTX);
        } else if (LDSH) {
          atomicAdd((unsigned long long *)&hist[c], (unsigned long long)(z - a));
        } else {
          atomicAdd((unsigned long long *)&excl[c], (unsigned long long)(z - a));
        }
      }
    }
    __syncthreads();
  }
  if (LDSH) {
    for (int v = threadIdx.x; v < N; v += WT)
      if (hist[v]) atomicAdd((unsigned long long *)&excl[v], (unsigned long long)hist[v]);
  }
}

int grid_w(int64_t n, int cus, int per_cu) {
  int64_t g = n < (int64_t)cus * per_cu ? n : (int64_t)cus * per_cu;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

size_t window_ws_bytes(int N) { return subtree_sums_ws_bytes(N); }

hipError_t launch_window_profile(const int64_t *off, const int64_t *ts, const int32_t *ctx, int64_t R,
                                 const int32_t *ids, int64_t n_sel, int N, const int2 *tin_tout,
                                 int64_t t0, int64_t t1, int64_t *excl, int64_t *incl, void *ws,
                                 uint32_t *err, int cus, hipStream_t s) {
  zero_i64<<<grid_w((N + WT - 1) / WT, cus, 4), WT, 0, s>>>(excl, N);
  if (n_sel > 0) {
    if (N <= MAX_NODES_ATTR) {
      static bool attr = false;
      if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&window_excl<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
        attr = true;
      }
      window_excl<true><<<grid_w(n_sel, cus, 4), WT, (size_t)N * 8, s>>>(off, ts, ctx, R, ids, n_sel,
                                                                        N, t0, t1, excl, err);
    } else {
      window_excl<false><<<grid_w(n_sel, cus, 8), WT, 0, s>>>(off, ts, ctx, R, ids, n_sel, N, t0, t1,
                                                             excl, err);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !incl) return e;
  return launch_subtree_sums(excl, N, tin_tout, incl, ws, cus, s);
}

}  // namespace ta
