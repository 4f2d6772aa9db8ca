// gen_traces.hip -- GPU generator of synthetic iteration-structured traces.
// Input generation only (benchmark and test workloads); see ta_synth.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../../include/ta_synth.h"

namespace {

// SplitMix64 output mixing (Steele, Lea, Flood 2014) applied to a counter.
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline uint64_t draw(uint64_t seed, uint64_t r, uint64_t i, uint64_t j, uint64_t what) {
  uint64_t h = mix64(seed ^ mix64(r * 0x100000001B3ull + what));
  h = mix64(h ^ (i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull));
  return mix64(h ^ (j * 0xD1B54A32D192ED03ull + what));
}

// Uniform in (0, 1).
__device__ inline double u01(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

enum : uint64_t { W_GAMMA = 1, W_PERM = 2, W_FILL = 3, W_EXTRA = 4, W_PICK = 5, W_APICK = 6 };

// Stratified-jittered sample time j of n inside an iteration of length Ti.
__device__ inline int64_t extra_time(uint64_t seed, int64_t r, int i, int j, int n, int64_t Ti) {
  if (Ti <= 0) return 0;
  const double u = u01(draw(seed, (uint64_t)r, (uint64_t)i, (uint64_t)j, W_EXTRA));
  int64_t x = (int64_t)floor(((double)j + u) * ((double)Ti / (double)n));
  if (x >= Ti) x = Ti - 1;
  if (x < 0) x = 0;
  return x;
}

constexpr int GT = 128;  // threads per rank; one per segment (G + 1 <= 128)

__global__ __launch_bounds__(GT) void gen_kernel(tas_params p) {
  __shared__ int64_t start[GT + 2];
  __shared__ int kind[GT];
  __shared__ int64_t dur[GT];
  __shared__ uint64_t keys[GT];
  const int lane = threadIdx.x;
  const int64_t r = blockIdx.x;
  const int G = p.n_regions, I = p.n_iters;
  const uint64_t seed = p.seed;
  const int64_t off = p.offsets[r];
  const int b = p.events_per_iter[r];
  const bool anchored = b >= G + 2;
  const int n_extra = anchored ? b - G - 2 : b - 1;
  int64_t t = p.t0[r];
  for (int i = 0; i < I; i++) {
    if (lane < G) {
      double prod = 1.0;
      for (int q = 0; q < 4; q++) prod *= u01(draw(seed, r, i, (uint64_t)(4 * lane + q), W_GAMMA));
      const double d = p.scale[r * G + lane] * (p.mu[lane] * 0.25) * -log(prod);
      dur[lane] = (int64_t)llrint(d);
      keys[lane] = draw(seed, r, i, (uint64_t)lane, W_PERM);
    } else if (lane == G) {
      dur[G] = (int64_t)llrint(-p.filler_mean_ns * log(u01(draw(seed, r, i, 0, W_FILL))));
    }
    __syncthreads();
    // Random order of the regions: each region's position is the number of
    // smaller keys; the filler segment comes last.
    if (lane < G) {
      const uint64_t k = keys[lane];
      int pos = 0;
      for (int q = 0; q < G; q++) {
        const uint64_t kq = keys[q];
        pos += (kq < k) || (kq == k && q < lane);
      }
      kind[pos] = lane;
    } else if (lane == G) {
      kind[G] = G;
    }
    __syncthreads();
    if (lane == 0) {
      int64_t x = t;
      for (int s = 0; s <= G; s++) {
        start[s] = x;
        x += dur[kind[s]];
      }
      start[G + 1] = x;
    }
    __syncthreads();
    const int64_t Ti = start[G + 1] - t;

    const int64_t base = off + (int64_t)i * b;
    if (lane == 0) {
      p.ts[base] = t;
      p.ctx[base] = p.marker;
    }
    for (int j = lane; j < n_extra; j += GT) {
      const int64_t tj = t + extra_time(seed, r, i, j, n_extra, Ti);
      int lo = 0, hi = G;  // last segment whose start is <= tj
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= tj) lo = mid;
        else hi = mid - 1;
      }
      const int64_t pos = base + 1 + j + (anchored ? lo + 1 : 0);
      const int kk = kind[lo];
      const int32_t a0 = p.pool_off[kk], a1 = p.pool_off[kk + 1];
      p.ts[pos] = tj;
      p.ctx[pos] = p.pool[a0 + (int32_t)(draw(seed, r, i, (uint64_t)j, W_PICK) % (uint64_t)(a1 - a0))];
    }
    if (anchored && lane <= G) {
      const int64_t x = start[lane];
      int lo = 0, hi = n_extra;  // number of extras strictly before x
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t + extra_time(seed, r, i, mid, n_extra, Ti) < x) lo = mid + 1;
        else hi = mid;
      }
      const int64_t pos = base + 1 + lane + lo;
      const int kk = kind[lane];
      const int32_t a0 = p.pool_off[kk], a1 = p.pool_off[kk + 1];
      p.ts[pos] = x;
      p.ctx[pos] = p.pool[a0 + (int32_t)(draw(seed, r, i, (uint64_t)lane, W_APICK) % (uint64_t)(a1 - a0))];
    }
    t += Ti;
    __syncthreads();
  }
  if (lane == 0) {
    const int64_t pos = off + (int64_t)I * b;
    p.ts[pos] = t;
    p.ctx[pos] = p.root;
  }
}

}  // namespace

extern "C" int32_t tas_generate(const tas_params *p, void *stream) {
  if (!p || p->n_ranks < 0 || p->n_iters < 1 || p->n_regions < 1 || p->n_regions > 127) return 1;
  if (p->n_ranks == 0) return 0;
  if (!p->offsets || !p->events_per_iter || !p->t0 || !p->scale || !p->mu || !p->pool ||
      !p->pool_off || !p->ts || !p->ctx)
    return 1;
  hipLaunchKernelGGL(gen_kernel, dim3((unsigned)p->n_ranks), dim3(GT), 0, (hipStream_t)stream, *p);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}

namespace {

typedef long long v2ll __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void copy_kernel(v2ll *__restrict__ dst,
                                                   const v2ll *__restrict__ src, int64_t n) {
  constexpr int U = 4;
  const int64_t stride = (int64_t)gridDim.x * 256 * U;
  for (int64_t b = (int64_t)blockIdx.x * 256 * U + threadIdx.x; b < n; b += stride) {
    v2ll v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t k = b + (int64_t)u * 256;
      if (k < n) v[u] = src[k];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t k = b + (int64_t)u * 256;
      if (k < n) dst[k] = v[u];
    }
  }
}

}  // namespace

extern "C" int32_t tas_copy(void *dst, const void *src, int64_t n_bytes, int32_t workgroups_per_cu,
                            void *stream) {
  if (!dst || !src || n_bytes < 0 || (n_bytes & 15) || ((uintptr_t)dst & 15) ||
      ((uintptr_t)src & 15) || workgroups_per_cu < 0)
    return 1;
  if (n_bytes == 0) return 0;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  }
  const int64_t n = n_bytes / 16;
  int64_t grid = (int64_t)cus * (workgroups_per_cu ? workgroups_per_cu : 8);
  const int64_t need = (n + 1023) / 1024;
  if (grid > need) grid = need;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                     (v2ll *)dst, (const v2ll *)src, n);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}
