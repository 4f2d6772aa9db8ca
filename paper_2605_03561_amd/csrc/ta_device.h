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

// ---- exact FP64 sums ------------------------------------------------------
// A finite double is m * 2^(s - 1074) with an integer 0 <= m < 2^53 and a shift
// 0 <= s <= 2045, so a sum of doubles is an integer count of 2^-1074 units.
// The accumulator keeps that integer as XL signed 64-bit limbs of 32-bit
// weight (limb k counts units of 2^(32k - 1074)): a value adds its three 32-bit
// pieces to three consecutive limbs.  Integer adds are exact and associative,
// so the total does not depend on which lane or wave adds what, or in which
// order.  One thread then carries the limbs into 32-bit digits and rounds the
// integer once to the nearest double (ties to even).  A limb takes pieces below
// 2^32 and so holds at least 2^31 terms; 68 limbs cover 2^31 maximal doubles.
constexpr int XL = 68;

// Adds v to this wave's limbs (LDS) when act; every lane of the wave calls it.
// A non-finite v sets *nonfinite (the sum is then NaN).  When the active lanes'
// values share their lowest limb (the usual case: values of one magnitude),
// the wave adds the pieces first and one lane does three LDS atomics.
__device__ inline void xsum_add_wave(int64_t *wl, double v, bool act, uint32_t *nonfinite) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int ex = (int)((b >> 52) & 0x7ff);
  if (act && ex == 0x7ff) {
    atomicOr(nonfinite, 1u);
    act = false;
  }
  uint64_t m = b & ((1ull << 52) - 1);
  if (ex) m |= 1ull << 52;
  act = act && m != 0;
  const int sft = ex ? ex - 1 : 0;   // v = m * 2^(sft - 1074)
  const int L = sft >> 5;
  const u128 w = (u128)m << (sft & 31);
  const bool neg = (b >> 63) != 0;
  int64_t p0 = (int64_t)((uint64_t)w & 0xffffffffull);
  int64_t p1 = (int64_t)((uint64_t)(w >> 32) & 0xffffffffull);
  int64_t p2 = (int64_t)(uint64_t)(w >> 64);
  if (neg) {
    p0 = -p0;
    p1 = -p1;
    p2 = -p2;
  }
  const uint64_t am = __ballot(act);
  if (!am) return;
  const int lane = (int)(threadIdx.x & 63);
  const int lead = __ffsll((long long)am) - 1;
  const int L0 = __shfl(L, lead, 64);
  if (__ballot(act && L == L0) == am) {
    int64_t s0 = act ? p0 : 0, s1 = act ? p1 : 0, s2 = act ? p2 : 0;
    for (int d = 32; d >= 1; d >>= 1) {
      s0 += __shfl_xor(s0, d, 64);
      s1 += __shfl_xor(s1, d, 64);
      s2 += __shfl_xor(s2, d, 64);
    }
    if (lane == lead) {
      atomicAdd((unsigned long long *)&wl[L0], (unsigned long long)s0);
      atomicAdd((unsigned long long *)&wl[L0 + 1], (unsigned long long)s1);
      atomicAdd((unsigned long long *)&wl[L0 + 2], (unsigned long long)s2);
    }
  } else if (act) {
    atomicAdd((unsigned long long *)&wl[L], (unsigned long long)p0);
    atomicAdd((unsigned long long *)&wl[L + 1], (unsigned long long)p1);
    atomicAdd((unsigned long long *)&wl[L + 2], (unsigned long long)p2);
  }
}

// The integer in x[0 .. XL) (limbs of 32-bit weight, any signs) rounded to the
// nearest double, ties to even; x is overwritten.  One thread.
__device__ inline double xsum_round(int64_t *x) {
  int64_t c = 0;
  for (int i = 0; i < XL; i++) {
    const int64_t t = x[i] + c;
    x[i] = t & 0xffffffffll;
    c = t >> 32;  // arithmetic shift: floor(t / 2^32)
  }
  // c is the sign extension: 0 (value >= 0) or -1 (value < 0)
  const bool neg = c < 0;
  if (neg) {
    int64_t k = 1;
    for (int i = 0; i < XL; i++) {
      const int64_t t = ((~x[i]) & 0xffffffffll) + k;
      x[i] = t & 0xffffffffll;
      k = t >> 32;
    }
  }
  int top = XL - 1;
  while (top >= 0 && x[top] == 0) top--;
  if (top < 0) return 0.0;
  const int hb = 31 - __clz((int)(uint32_t)x[top]);
  const int P = 32 * top + hb;   // position of the leading bit, in 2^-1074 units
  double mag;
  if (P <= 52) {
    // below 2^53 units: exactly representable (subnormal or the first binade)
    const uint64_t mm = (uint64_t)x[0] | (top >= 1 ? ((uint64_t)x[1] << 32) : 0ull);
    mag = ldexp((double)mm, -1074);
  } else {
    const u128 w = ((u128)(uint64_t)x[top] << 64) |
                   ((u128)(uint64_t)(top >= 1 ? x[top - 1] : 0) << 32) |
                   (u128)(uint64_t)(top >= 2 ? x[top - 2] : 0);
    const int sh = hb + 11;  // the leading bit is bit hb + 64 of w: keep 54 bits
    const uint64_t keep = (uint64_t)(w >> sh);
    bool sticky = (w & (((u128)1 << sh) - 1)) != 0;
    for (int i = top - 3; i >= 0 && !sticky; i--) sticky = x[i] != 0;
    uint64_t mant = keep >> 1;
    if ((keep & 1) && (sticky || (mant & 1))) mant++;
    mag = ldexp((double)mant, P - 52 - 1074);
  }
  return neg ? -mag : mag;
}

// Block-wide exact sum.  acc[(NT/64) * XL] and *nonfinite are LDS, cleared by
// xsum_clear before the adds; every thread calls xsum_add_wave on
// acc + (threadIdx.x / 64) * XL, then every thread calls xsum_block_result,
// which returns the rounded total to all threads (acc is left dirty).
template <int NT>
__device__ inline void xsum_clear(int64_t *acc, uint32_t *nonfinite) {
  for (int k = threadIdx.x; k < (NT / 64) * XL; k += NT) acc[k] = 0;
  if (threadIdx.x == 0) *nonfinite = 0;
  __syncthreads();
}

template <int NT>
__device__ inline double xsum_block_result(int64_t *acc, uint32_t *nonfinite, double *bcast) {
  __syncthreads();
  for (int k = threadIdx.x; k < XL; k += NT) {
    int64_t s = 0;
    for (int w = 0; w < NT / 64; w++) s += acc[w * XL + k];
    acc[k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) bcast[0] = *nonfinite ? nan_f64() : xsum_round(acc);
  __syncthreads();
  const double r = bcast[0];
  __syncthreads();
  return r;
}

}  // namespace ta
