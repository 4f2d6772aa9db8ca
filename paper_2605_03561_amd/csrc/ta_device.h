// ta_device.h -- small device helpers shared by the statistics kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ta {

typedef __int128 i128;
typedef unsigned __int128 u128;

// Unsigned 64-bit -> double, correctly rounded: two exact 32-bit conversions
// and one rounding in the final addition.
__device__ inline double u64_to_f64(uint64_t x) {
  double hi = (double)(uint32_t)(x >> 32);
  double lo = (double)(uint32_t)x;
  return fma(hi, 4294967296.0, lo);
}

// Unsigned 128-bit -> double, correctly rounded (round to nearest even): keep
// the top 64 significant bits, fold every bit shifted out into the lowest
// kept bit (a sticky bit below the rounding position), convert, rescale.
__device__ inline double u128_to_f64(u128 x) {
  uint64_t hi = (uint64_t)(x >> 64);
  if (hi == 0) return u64_to_f64((uint64_t)x);
  int sh = 64 - __clzll((long long)hi);      // 1..64
  uint64_t top = (uint64_t)(x >> sh);
  u128 rest = x & (((u128)1 << sh) - 1);
  top |= (rest != 0) ? 1u : 0u;
  return ldexp(u64_to_f64(top), sh);
}

__device__ inline double i128_to_f64(i128 x) {
  return x < 0 ? -u128_to_f64((u128)(-x)) : u128_to_f64((u128)x);
}

__device__ inline double i64_to_f64(int64_t x) {
  return x < 0 ? -u64_to_f64((uint64_t)(-x)) : u64_to_f64((uint64_t)x);
}

// Deterministic block reductions (fixed tree over threads; NT a power of 2,
// `buf` has NT slots).  All threads get the result.
template <int NT>
__device__ inline double block_sum_f64(double v, double *buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] = buf[threadIdx.x] + buf[threadIdx.x + s];
    __syncthreads();
  }
  double r = buf[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ inline int64_t block_sum_i64(int64_t v, int64_t *buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] += buf[threadIdx.x + s];
    __syncthreads();
  }
  int64_t r = buf[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ inline int64_t block_max_i64(int64_t v, int64_t *buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      int64_t o = buf[threadIdx.x + s];
      if (o > buf[threadIdx.x]) buf[threadIdx.x] = o;
    }
    __syncthreads();
  }
  int64_t r = buf[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ inline double block_max_f64(double v, double *buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double o = buf[threadIdx.x + s];
      if (o > buf[threadIdx.x]) buf[threadIdx.x] = o;
    }
    __syncthreads();
  }
  double r = buf[0];
  __syncthreads();
  return r;
}

__device__ inline double nan_f64() { return __longlong_as_double(0x7ff8000000000000LL); }

}  // namespace ta
