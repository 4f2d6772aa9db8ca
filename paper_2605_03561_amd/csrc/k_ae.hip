// k_ae.hip -- learned pre-screen: autoencoder training and scoring kernels.
//
// Dense layers run on the matrix cores (v_mfma_f32_16x16x16_bf16): operands
// are bfloat16 (round to nearest even), accumulation is FP32.  A workgroup
// (4 waves) processes row tiles of 16 profile rows; every wave owns a fixed set
// of 16x16 output tiles per layer, so weight-gradient tiles stay in the MFMA
// accumulators across all row tiles of a training step and are written once
// per workgroup.  Partials are summed in workgroup order by the Adam kernel, so
// a step is deterministic.
#include "ta_ae.h"
#include "ta_device.h"
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int AT = 256;       // threads per workgroup
constexpr int TR = 16;        // rows per tile

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// One 16x16 tile of D += A * B over K (a multiple of 16).  A(m, k) is
// A[m*sam + k*sak], B(k, n) is B[k*sbk + n*sbn] (bfloat16 in LDS).  Operand
// lane layout: lane l supplies row/column (l & 15) and k = 4*(l >> 4) + 0..3;
// the result holds rows 4*(l >> 4) + 0..3 of column (l & 15).
__device__ inline f4 mma_tile(const uint16_t *A, int sam, int sak, const uint16_t *B, int sbk,
                              int sbn, int m0, int n0, int K, f4 acc) {
  const int lane = threadIdx.x & 63;
  const int mi = m0 + (lane & 15), ni = n0 + (lane & 15), kq = 4 * (lane >> 4);
  for (int k0 = 0; k0 < K; k0 += 16) {
    s4 a, b;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int k = k0 + kq + j;
      a[j] = (short)A[mi * sam + k * sak];
      b[j] = (short)B[k * sbk + ni * sbn];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ inline int out_row(int j) { return 4 * ((threadIdx.x & 63) >> 4) + j; }
__device__ inline int out_col() { return threadIdx.x & 15; }

// Sum of a value over the four lane groups that hold the same column.
__device__ inline float col_sum(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

__device__ inline double col_sum(double v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

struct AeLds {
  uint16_t W[AE_NW];          // bf16 weights
  float b[AE_NP - AE_NW];     // biases
  float X[TR * AE_IN];        // targets (FP32)
  uint16_t Xb[TR * AE_IN];
  uint16_t H1[TR * AE_H1], H2[TR * AE_H2], H3[TR * AE_H3];
  uint16_t D4[TR * AE_IN], D3[TR * AE_H3], D2[TR * AE_H2], D1[TR * AE_H1];
  float red[AT];
  double redd[AT];
  int valid[TR];
};

// The bf16 weights (16-byte loads, all of a thread's loads issued before its
// first LDS store: one round trip, not one per word) and the FP32 biases.
__device__ void stage_weights(AeLds &L, const uint16_t *wb, const float *w) {
  constexpr int NV = AE_NW * 2 / 16;     // 16-byte words of bf16 weights
  constexpr int PER = NV / AT;
  constexpr int NB = AE_NP - AE_NW;      // biases
  constexpr int PB = (NB + AT - 1) / AT;
  static_assert(NV % AT == 0, "the weights are staged in whole steps of the workgroup");
  const int t = threadIdx.x;
  const uint4 *src = reinterpret_cast<const uint4 *>(wb);
  uint4 *dst = reinterpret_cast<uint4 *>(L.W);
  uint4 v[PER];
  float bv[PB];
#pragma unroll
  for (int u = 0; u < PER; u++) v[u] = src[u * AT + t];
#pragma unroll
  for (int u = 0; u < PB; u++) bv[u] = u * AT + t < NB ? w[AE_NW + u * AT + t] : 0.f;
#pragma unroll
  for (int u = 0; u < PER; u++) dst[u * AT + t] = v[u];
#pragma unroll
  for (int u = 0; u < PB; u++)
    if (u * AT + t < NB) L.b[u * AT + t] = bv[u];
}

// Forward through the four layers for the tile in L.Xb.  Hidden activations
// are stored as bf16 after ReLU; the output pre-activation tile of wave w
// (columns 16w..16w+15) is returned in `y` (bias added).
__device__ inline void forward(AeLds &L, f4 &y) {
  const int wid = threadIdx.x >> 6;
  const f4 z0 = {0.f, 0.f, 0.f, 0.f};
  // L1: [16 x 64] * W1^T -> [16 x 128]
  for (int t = wid; t < AE_H1 / 16; t += 4) {
    f4 a = mma_tile(L.Xb, AE_IN, 1, L.W + AE_W1, 1, AE_IN, 0, 16 * t, AE_IN, z0);
    const int c = 16 * t + out_col();
#pragma unroll
    for (int j = 0; j < 4; j++) L.H1[out_row(j) * AE_H1 + c] = f2bf(fmaxf(a[j] + L.b[c], 0.f));
  }
  __syncthreads();
  // L2: [16 x 128] * W2^T -> [16 x 32]
  for (int t = wid; t < AE_H2 / 16; t += 4) {
    f4 a = mma_tile(L.H1, AE_H1, 1, L.W + AE_W2, 1, AE_H1, 0, 16 * t, AE_H1, z0);
    const int c = 16 * t + out_col();
#pragma unroll
    for (int j = 0; j < 4; j++)
      L.H2[out_row(j) * AE_H2 + c] = f2bf(fmaxf(a[j] + L.b[AE_B2 - AE_B1 + c], 0.f));
  }
  __syncthreads();
  // L3: [16 x 32] * W3^T -> [16 x 128]
  for (int t = wid; t < AE_H3 / 16; t += 4) {
    f4 a = mma_tile(L.H2, AE_H2, 1, L.W + AE_W3, 1, AE_H2, 0, 16 * t, AE_H2, z0);
    const int c = 16 * t + out_col();
#pragma unroll
    for (int j = 0; j < 4; j++)
      L.H3[out_row(j) * AE_H3 + c] = f2bf(fmaxf(a[j] + L.b[AE_B3 - AE_B1 + c], 0.f));
  }
  __syncthreads();
  // L4: [16 x 128] * W4^T -> [16 x 64]; wave w owns columns 16w..16w+15
  y = mma_tile(L.H3, AE_H3, 1, L.W + AE_W4, 1, AE_H3, 0, 16 * wid, AE_H3, z0);
  const int c = 16 * wid + out_col();
#pragma unroll
  for (int j = 0; j < 4; j++) y[j] += L.b[AE_B4 - AE_B1 + c];
}

// SplitMix64 finaliser (Steele, Lea & Flood 2014), used as a counter-based
// generator: draw = mix64(key + counter * golden gamma).
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Standard normal draw for (key, row, feature): two 24-bit uniforms from
// SplitMix64 counter draws, then Box-Muller (Box & Muller 1958),
// sqrt(-2 ln u1) cos(2 pi u2), with u1 in (0, 1).
__device__ inline float gauss_draw(uint64_t key, uint64_t row, int c) {
  const uint64_t base = mix64(key ^ mix64(row * (uint64_t)AE_IN + (uint64_t)c));
  const uint64_t z1 = mix64(base), z2 = mix64(base ^ 0xD1B54A32D192ED03ull);
  const float u1 = ((float)(z1 >> 40) + 0.5f) * (1.0f / 16777216.0f);
  const float u2 = (float)(z2 >> 40) * (1.0f / 16777216.0f);
  return sqrtf(-2.0f * logf(u1)) * cosf(6.2831853071795864f * u2);
}

__device__ inline uint64_t perm_row(uint64_t k, uint64_t a, uint64_t c, uint64_t n) {
  return (a * k + c) % n;
}

// ---------------------------------------------------------------------------
// Training step: gradient partials of the mean squared error over the rows
// perm(k), k in [k0, k_end), written per workgroup to part[wg][AE_NP + 1].
// With noise_sd > 0 the network sees x + noise_sd * N(0, 1) (drawn for the
// row's index and the feature under noise_key) and is scored against x
// (denoising training).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(AT) void ae_fwdbwd(const float *__restrict__ rows, int64_t n,
                                                 int64_t k0, int64_t k_end, uint64_t pa,
                                                 uint64_t pc, float scale, float noise_sd,
                                                 uint64_t noise_key,
                                                 const uint16_t *__restrict__ wb,
                                                 const float *__restrict__ w, float *part) {
  extern __shared__ __align__(16) unsigned char smem[];
  AeLds &L = *reinterpret_cast<AeLds *>(smem);
  const int tid = threadIdx.x, wid = tid >> 6;
  stage_weights(L, wb, w);
  const int64_t tiles = (k_end - k0 + TR - 1) / TR;
  const int64_t t_lo = tiles * blockIdx.x / gridDim.x, t_hi = tiles * (blockIdx.x + 1) / gridDim.x;

  const f4 z0 = {0.f, 0.f, 0.f, 0.f};
  f4 gW1[8], gW4[8], gW2[4], gW3[4];
#pragma unroll
  for (int q = 0; q < 8; q++) gW1[q] = gW4[q] = z0;
#pragma unroll
  for (int q = 0; q < 4; q++) gW2[q] = gW3[q] = z0;
  float gb1[2] = {0.f, 0.f}, gb3[2] = {0.f, 0.f}, gb2 = 0.f, gb4 = 0.f, loss = 0.f;

  for (int64_t t = t_lo; t < t_hi; t++) {
    __syncthreads();
    {  // load 16 rows (4 floats per thread)
      const int r = tid >> 4, c4 = (tid & 15) * 4;
      const int64_t k = k0 + t * TR + r;
      const bool ok = k < k_end;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      const uint64_t row = ok ? perm_row((uint64_t)k, pa, pc, (uint64_t)n) : 0;
      if (ok) v = *reinterpret_cast<const float4 *>(rows + row * AE_IN + c4);
      L.X[r * AE_IN + c4 + 0] = v.x;
      L.X[r * AE_IN + c4 + 1] = v.y;
      L.X[r * AE_IN + c4 + 2] = v.z;
      L.X[r * AE_IN + c4 + 3] = v.w;
      float4 xin = v;
      if (ok && noise_sd > 0.f) {
        xin.x += noise_sd * gauss_draw(noise_key, row, c4 + 0);
        xin.y += noise_sd * gauss_draw(noise_key, row, c4 + 1);
        xin.z += noise_sd * gauss_draw(noise_key, row, c4 + 2);
        xin.w += noise_sd * gauss_draw(noise_key, row, c4 + 3);
      }
      L.Xb[r * AE_IN + c4 + 0] = f2bf(xin.x);
      L.Xb[r * AE_IN + c4 + 1] = f2bf(xin.y);
      L.Xb[r * AE_IN + c4 + 2] = f2bf(xin.z);
      L.Xb[r * AE_IN + c4 + 3] = f2bf(xin.w);
      if ((tid & 15) == 0) L.valid[r] = ok;
    }
    __syncthreads();
    f4 y;
    forward(L, y);
    {  // output error -> D4 (dL/dy), loss, db4
      const int c = 16 * wid + out_col();
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int r = out_row(j);
        float d = 0.f;
        if (L.valid[r]) {
          const float e = y[j] - L.X[r * AE_IN + c];
          loss += e * e;
          d = scale * e;
        }
        gb4 += d;
        L.D4[r * AE_IN + c] = f2bf(d);
      }
    }
    __syncthreads();
    // dW4 [64 x 128] += D4^T H3 ; 32 tiles, 8 per wave
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const int tt = wid * 8 + q, mt = tt >> 3, nt = tt & 7;
      gW4[q] = mma_tile(L.D4, 1, AE_IN, L.H3, AE_H3, 1, 16 * mt, 16 * nt, TR, gW4[q]);
    }
    // dH3 [16 x 128] = D4 W4 ; mask by H3 > 0 -> D3
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int nt = wid + 4 * q;
      f4 a = mma_tile(L.D4, AE_IN, 1, L.W + AE_W4, AE_H3, 1, 0, 16 * nt, AE_IN, z0);
      const int c = 16 * nt + out_col();
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int r = out_row(j);
        const float d = (int16_t)L.H3[r * AE_H3 + c] > 0 ? a[j] : 0.f;  // ReLU was active
        gb3[q] += d;
        L.D3[r * AE_H3 + c] = f2bf(d);
      }
    }
    __syncthreads();
    // dW3 [128 x 32] += D3^T H2 ; 16 tiles, 4 per wave
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int tt = wid * 4 + q, mt = tt >> 1, nt = tt & 1;
      gW3[q] = mma_tile(L.D3, 1, AE_H3, L.H2, AE_H2, 1, 16 * mt, 16 * nt, TR, gW3[q]);
    }
    // dH2 [16 x 32] = D3 W3 -> D2
    if (wid < 2) {
      f4 a = mma_tile(L.D3, AE_H3, 1, L.W + AE_W3, AE_H2, 1, 0, 16 * wid, AE_H3, z0);
      const int c = 16 * wid + out_col();
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int r = out_row(j);
        const float d = (int16_t)L.H2[r * AE_H2 + c] > 0 ? a[j] : 0.f;
        gb2 += d;
        L.D2[r * AE_H2 + c] = f2bf(d);
      }
    }
    __syncthreads();
    // dW2 [32 x 128] += D2^T H1 ; 16 tiles, 4 per wave
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int tt = wid * 4 + q, mt = tt >> 3, nt = tt & 7;
      gW2[q] = mma_tile(L.D2, 1, AE_H2, L.H1, AE_H1, 1, 16 * mt, 16 * nt, TR, gW2[q]);
    }
    // dH1 [16 x 128] = D2 W2 -> D1
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int nt = wid + 4 * q;
      f4 a = mma_tile(L.D2, AE_H2, 1, L.W + AE_W2, AE_H1, 1, 0, 16 * nt, AE_H2, z0);
      const int c = 16 * nt + out_col();
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int r = out_row(j);
        const float d = (int16_t)L.H1[r * AE_H1 + c] > 0 ? a[j] : 0.f;
        gb1[q] += d;
        L.D1[r * AE_H1 + c] = f2bf(d);
      }
    }
    __syncthreads();
    // dW1 [128 x 64] += D1^T Xb ; 32 tiles, 8 per wave
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const int tt = wid * 8 + q, mt = tt >> 2, nt = tt & 3;
      gW1[q] = mma_tile(L.D1, 1, AE_H1, L.Xb, AE_IN, 1, 16 * mt, 16 * nt, TR, gW1[q]);
    }
  }

  // Write this workgroup's partials (every element exactly once).
  float *P = part + (int64_t)blockIdx.x * (AE_NP + 1);
  const int cc = out_col();
#pragma unroll
  for (int q = 0; q < 8; q++) {
    {
      const int tt = wid * 8 + q, mt = tt >> 2, nt = tt & 3;
#pragma unroll
      for (int j = 0; j < 4; j++) P[AE_W1 + (16 * mt + out_row(j)) * AE_IN + 16 * nt + cc] = gW1[q][j];
    }
    {
      const int tt = wid * 8 + q, mt = tt >> 3, nt = tt & 7;
#pragma unroll
      for (int j = 0; j < 4; j++) P[AE_W4 + (16 * mt + out_row(j)) * AE_H3 + 16 * nt + cc] = gW4[q][j];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    {
      const int tt = wid * 4 + q, mt = tt >> 3, nt = tt & 7;
#pragma unroll
      for (int j = 0; j < 4; j++) P[AE_W2 + (16 * mt + out_row(j)) * AE_H1 + 16 * nt + cc] = gW2[q][j];
    }
    {
      const int tt = wid * 4 + q, mt = tt >> 1, nt = tt & 1;
#pragma unroll
      for (int j = 0; j < 4; j++) P[AE_W3 + (16 * mt + out_row(j)) * AE_H2 + 16 * nt + cc] = gW3[q][j];
    }
  }
  const int lane = tid & 63;
  const float b4s = col_sum(gb4);
  const float b3s0 = col_sum(gb3[0]), b3s1 = col_sum(gb3[1]);
  const float b1s0 = col_sum(gb1[0]), b1s1 = col_sum(gb1[1]);
  const float b2s = col_sum(gb2);
  if (lane < 16) {
    P[AE_B4 + 16 * wid + lane] = b4s;
    P[AE_B3 + 16 * wid + lane] = b3s0;
    P[AE_B3 + 16 * (wid + 4) + lane] = b3s1;
    P[AE_B1 + 16 * wid + lane] = b1s0;
    P[AE_B1 + 16 * (wid + 4) + lane] = b1s1;
    if (wid < 2) P[AE_B2 + 16 * wid + lane] = b2s;
  }
  const double ls = block_sum_f64<AT>((double)loss, L.redd);
  if (tid == 0) P[AE_NP] = (float)ls;
}

// ---------------------------------------------------------------------------
// FP32 debug gradient: the same network, loss and input noise with every
// operation in FP32 (no bfloat16 operand rounding), for checking the gradient
// code against an FP64 reference.  A workgroup takes rows blockIdx.x,
// blockIdx.x + gridDim.x, ...; each layer's outputs are dot products in
// ascending k by single threads; thread t owns the partial entries p = t mod
// 256 (so the read-modify-writes of a row need no atomics).  Not a fast path.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ae_grad_f32_kernel(const float *__restrict__ rows, int64_t n,
                                                          float scale, float noise_sd,
                                                          uint64_t noise_key,
                                                          const float *__restrict__ w, float *part) {
  __shared__ float x[AE_IN], xin[AE_IN], h1[AE_H1], h2[AE_H2], h3[AE_H3];
  __shared__ float d4[AE_IN], d3[AE_H3], d2[AE_H2], d1[AE_H1];
  __shared__ double red[256];
  const int t = threadIdx.x;
  float *P = part + (int64_t)blockIdx.x * (AE_NP + 1);
  for (int p = t; p < AE_NP; p += 256) P[p] = 0.f;
  double loss = 0.0;
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
    if (t < AE_IN) {
      x[t] = rows[r * AE_IN + t];
      xin[t] = noise_sd > 0.f ? x[t] + noise_sd * gauss_draw(noise_key, (uint64_t)r, t) : x[t];
    }
    __syncthreads();
    if (t < AE_H1) {
      float a = w[AE_B1 + t];
      for (int k = 0; k < AE_IN; k++) a = fmaf(w[AE_W1 + t * AE_IN + k], xin[k], a);
      h1[t] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (t < AE_H2) {
      float a = w[AE_B2 + t];
      for (int k = 0; k < AE_H1; k++) a = fmaf(w[AE_W2 + t * AE_H1 + k], h1[k], a);
      h2[t] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (t < AE_H3) {
      float a = w[AE_B3 + t];
      for (int k = 0; k < AE_H2; k++) a = fmaf(w[AE_W3 + t * AE_H2 + k], h2[k], a);
      h3[t] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (t < AE_IN) {
      float a = w[AE_B4 + t];
      for (int k = 0; k < AE_H3; k++) a = fmaf(w[AE_W4 + t * AE_H3 + k], h3[k], a);
      const float e = a - x[t];
      loss += (double)e * e;
      d4[t] = scale * e;
    }
    __syncthreads();
    if (t < AE_H3) {
      float a = 0.f;
      for (int o = 0; o < AE_IN; o++) a = fmaf(w[AE_W4 + o * AE_H3 + t], d4[o], a);
      d3[t] = h3[t] > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (t < AE_H2) {
      float a = 0.f;
      for (int o = 0; o < AE_H3; o++) a = fmaf(w[AE_W3 + o * AE_H2 + t], d3[o], a);
      d2[t] = h2[t] > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (t < AE_H1) {
      float a = 0.f;
      for (int o = 0; o < AE_H2; o++) a = fmaf(w[AE_W2 + o * AE_H1 + t], d2[o], a);
      d1[t] = h1[t] > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int p = t; p < AE_NP; p += 256) {
      float g;
      if (p < AE_W2) g = d1[p / AE_IN] * xin[p % AE_IN];
      else if (p < AE_W3) g = d2[(p - AE_W2) / AE_H1] * h1[(p - AE_W2) % AE_H1];
      else if (p < AE_W4) g = d3[(p - AE_W3) / AE_H2] * h2[(p - AE_W3) % AE_H2];
      else if (p < AE_NW) g = d4[(p - AE_W4) / AE_H3] * h3[(p - AE_W4) % AE_H3];
      else if (p < AE_B2) g = d1[p - AE_B1];
      else if (p < AE_B3) g = d2[p - AE_B2];
      else if (p < AE_B4) g = d3[p - AE_B3];
      else g = d4[p - AE_B4];
      P[p] += g;
    }
    __syncthreads();
  }
  const double ls = block_sum_f64<256>(loss, red);
  if (t == 0) P[AE_NP] = (float)ls;
}

// Entry p of the workgroup partials summed in workgroup order; the loads go
// out 16 at a time (one round trip per 16 partials instead of one each), the
// additions stay in order.
__device__ inline float sum_partials(const float *part, int nwg, int p) {
  constexpr int U = 16;
  float g = 0.f;
  for (int k0 = 0; k0 < nwg; k0 += U) {
    float pv[U];
#pragma unroll
    for (int u = 0; u < U; u++) pv[u] = k0 + u < nwg ? part[(int64_t)(k0 + u) * (AE_NP + 1) + p] : 0.f;
#pragma unroll
    for (int u = 0; u < U; u++)
      if (k0 + u < nwg) g += pv[u];
  }
  return g;
}

// Parameter p: the sum of the workgroup partials in workgroup order, then
// optionally one Adam step.
__device__ inline void adam_param(int p, const float *part, int nwg, float *w, uint16_t *wb, float *m,
                                  float *v, float lr, float bc1, float bc2, int update,
                                  float *grad_out) {
  const float g = sum_partials(part, nwg, p);
  if (grad_out) grad_out[p] = g;
  if (update) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float wn = w[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    w[p] = wn;
    if (p < AE_NW) wb[p] = f2bf(wn);
  }
}

__device__ inline float loss_sum(const float *part, int nwg) { return sum_partials(part, nwg, AE_NP); }

// Sum the workgroup partials in workgroup order; optionally take one Adam step.
// With epoch_loss, also epoch_loss[0] += loss * lfrac (the step's share of the
// epoch's rows), in the kernel rather than a launch of its own.
__global__ __launch_bounds__(256) void ae_adam(const float *part, int nwg, float *w, uint16_t *wb,
                                               float *m, float *v, float lr, float bc1, float bc2,
                                               int update, float *grad_out, float *loss_out,
                                               float loss_scale, float *epoch_loss, float lfrac) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < AE_NP) adam_param(p, part, nwg, w, wb, m, v, lr, bc1, bc2, update, grad_out);
  if (p == 0 && loss_out) {
    loss_out[0] = loss_sum(part, nwg) * loss_scale;
    if (epoch_loss) epoch_loss[0] += loss_out[0] * lfrac;
  }
}


// ---------------------------------------------------------------------------
// Initialisation: Xavier-uniform weights from SplitMix64 counter draws.
// ---------------------------------------------------------------------------

__global__ void ae_init_kernel(uint64_t seed, float *w, uint16_t *wb, float *m, float *v) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= AE_NP) return;
  float val = 0.f;
  if (p < AE_NW) {
    int l, base, fin, fout;
    if (p < AE_W2) { l = 0; base = AE_W1; fin = AE_IN; fout = AE_H1; }
    else if (p < AE_W3) { l = 1; base = AE_W2; fin = AE_H1; fout = AE_H2; }
    else if (p < AE_W4) { l = 2; base = AE_W3; fin = AE_H2; fout = AE_H3; }
    else { l = 3; base = AE_W4; fin = AE_H3; fout = AE_IN; }
    const uint64_t s = mix64(seed);
    const uint64_t key = s ^ mix64((uint64_t)(l + 1));
    const uint64_t idx = (uint64_t)(p - base);
    const uint64_t z = mix64(key + idx * 0x9E3779B97F4A7C15ull);
    const double u = ((double)(z >> 11) + 0.5) / 9007199254740992.0;
    const double a = sqrt(6.0 / (double)(fin + fout));
    val = (float)((2.0 * u - 1.0) * a);
    wb[p] = f2bf(val);
  }
  w[p] = val;
  m[p] = 0.f;
  v[p] = 0.f;
}

// ---------------------------------------------------------------------------
// Normalisation fit: exact per-region sums over the valid cells.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ae_norm_partial(const int64_t *__restrict__ T, int64_t R,
                                                       int I, const int32_t *it, int64_t rpb,
                                                       int64_t *ps, uint64_t *pq, int64_t *pc) {
  const int g = threadIdx.x & 63, rs = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = r0 + rpb < R ? r0 + rpb : R;
  int64_t s = 0, cnt = 0;
  u128 q = 0;
  for (int64_t r = r0 + rs; r < r1; r += 4) {
    int ni = it ? it[r] : I;
    if (ni > I) ni = I;
    if (ni < 0) ni = 0;
    const int64_t *row = T + r * (int64_t)I * AE_IN + g;
    for (int i = 0; i < ni; i++) {
      const int64_t x = row[(int64_t)i * AE_IN];
      s += x;
      q += (u128)((i128)x * x);
    }
    cnt += ni;
  }
  __shared__ int64_t ss[256], sc[256];
  __shared__ uint64_t sl[256], sh[256];
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = cnt;
  sl[threadIdx.x] = (uint64_t)q;
  sh[threadIdx.x] = (uint64_t)(q >> 64);
  __syncthreads();
  if (threadIdx.x < 64) {
    int64_t a = 0, c = 0;
    u128 b = 0;
    for (int k = 0; k < 4; k++) {
      const int t = k * 64 + threadIdx.x;
      a += ss[t];
      c += sc[t];
      b += ((u128)sh[t] << 64) | sl[t];
    }
    ps[(int64_t)blockIdx.x * 64 + g] = a;
    pq[((int64_t)blockIdx.x * 64 + g) * 2] = (uint64_t)b;
    pq[((int64_t)blockIdx.x * 64 + g) * 2 + 1] = (uint64_t)(b >> 64);
    if (g == 0) pc[blockIdx.x] = c;
  }
}

__global__ void ae_norm_final(int nb, const int64_t *ps, const uint64_t *pq, const int64_t *pc,
                              int reset, int64_t *nsum, uint64_t *nsq, int64_t *ncnt, float *mu,
                              float *isd) {
  const int g = threadIdx.x;
  if (g >= 64) return;
  int64_t s = reset ? 0 : nsum[g];
  u128 q = reset ? 0 : (((u128)nsq[2 * g + 1] << 64) | nsq[2 * g]);
  int64_t n = reset ? 0 : ncnt[0];
  int64_t add = 0;
  for (int b = 0; b < nb; b++) {
    s += ps[(int64_t)b * 64 + g];
    q += ((u128)pq[((int64_t)b * 64 + g) * 2 + 1] << 64) | pq[((int64_t)b * 64 + g) * 2];
    add += pc[b];
  }
  n += add;
  nsum[g] = s;
  nsq[2 * g] = (uint64_t)q;
  nsq[2 * g + 1] = (uint64_t)(q >> 64);
  if (g == 0) ncnt[0] = n;
  double m = 0.0, sd = 1.0;
  if (n > 0) {
    m = i64_to_f64(s) / (double)n;
    const i128 num = (i128)((u128)n * q) - (i128)s * s;
    sd = sqrt(i128_to_f64(num) / ((double)n * (double)n));
    if (!(sd > 0.0)) sd = 1.0;
  }
  const float sd32 = (float)sd;
  mu[g] = (float)m;
  isd[g] = 1.0f / sd32;
}

// ---------------------------------------------------------------------------
// Training rows: normalised profile rows of every valid (rank, iteration).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void ae_rows_scan(const int32_t *it, int64_t R, int I,
                                                     int64_t *off) {
  __shared__ int64_t buf[1024];
  const int t = threadIdx.x;
  const int64_t per = (R + 1023) / 1024;
  const int64_t a = t * per, b = a + per < R ? a + per : R;
  int64_t s = 0;
  for (int64_t r = a; r < b; r++) {
    int ni = it ? it[r] : I;
    s += ni > I ? I : (ni < 0 ? 0 : ni);
  }
  buf[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
    const int64_t x = t >= d ? buf[t - d] : 0;
    __syncthreads();
    buf[t] += x;
    __syncthreads();
  }
  int64_t run = buf[t] - s;
  for (int64_t r = a; r < b; r++) {
    off[r] = run;
    int ni = it ? it[r] : I;
    run += ni > I ? I : (ni < 0 ? 0 : ni);
  }
  if (t == 1023) off[R] = buf[1023];
}

__global__ __launch_bounds__(256) void ae_rows_fill(const int64_t *__restrict__ T, int64_t R, int I,
                                                    const int64_t *off, const float *mu,
                                                    const float *isd, float *rows) {
  const int64_t r = blockIdx.x;
  const int64_t o = off[r], n = off[r + 1] - o;
  const int g = threadIdx.x & 63;
  const float m = mu[g], s = isd[g];
  const int64_t *src = T + r * (int64_t)I * AE_IN;
  for (int64_t k = threadIdx.x; k < n * AE_IN; k += 256)
    rows[(o + k / AE_IN) * AE_IN + (k % AE_IN)] = ((float)src[k] - m) * s;
}

// ---------------------------------------------------------------------------
// Scoring.  One wave per rank (8 waves per workgroup share the weights in
// LDS).  The rank's profile rows go through the network 32 at a time, as two
// 16-row tiles of v_mfma_f32_16x16x32_bf16: every weight fragment read from
// LDS feeds both tiles, and each layer's input fragments are read once and kept
// in registers across its output tiles.  The FP32 input tile and the hidden
// tile share one LDS buffer (the inputs the residual needs are held in
// registers in the output layout), and the next 32 rows are loaded from HBM
// into registers while the current ones are in the network.  No workgroup
// barrier after the weights are staged.
//   kind 0: score = max_g mean_i (y - x)^2     kind 1: max_g |mean_i (y - x)|
// ---------------------------------------------------------------------------
constexpr int SW = 8;                  // waves per workgroup
constexpr int SR = 32;                 // rows per wave step (two MFMA tiles)
constexpr int P_W1 = 72, P_W2 = 136, P_W3 = 40, P_W4 = 136;   // padded row strides (bf16)
constexpr int P_X = 68;                // FP32 row stride of the input tile
constexpr int P_H = 136, P_H2 = 40;    // bf16 row strides of the hidden tiles

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

struct ScoreLds {
  uint16_t W1[AE_H1 * P_W1], W2[AE_H2 * P_W2], W3[AE_H3 * P_W3], W4[AE_IN * P_W4];
  float b[AE_NP - AE_NW];
  float mu[AE_IN], isd[AE_IN];
  struct Wave {
    union {
      float X[SR * P_X];       // normalised inputs (FP32)
      uint16_t H[SR * P_H];    // first, then third hidden layer (bf16)
    } u;
    uint16_t H2[SR * P_H2];
  } wv[SW];
};
static_assert(SR * P_X * 4 == SR * P_H * 2, "input and hidden tiles share a buffer");

__device__ inline bf8 ld_bf8(const uint16_t *p) {
  return __builtin_bit_cast(bf8, *reinterpret_cast<const u4v *>(p));
}

__device__ inline bf8 ld_bf8_from_f32(const float *p) {
  const float4 a = *reinterpret_cast<const float4 *>(p);
  const float4 b = *reinterpret_cast<const float4 *>(p + 4);
  u4v u;
  u[0] = (uint32_t)f2bf(a.x) | ((uint32_t)f2bf(a.y) << 16);
  u[1] = (uint32_t)f2bf(a.z) | ((uint32_t)f2bf(a.w) << 16);
  u[2] = (uint32_t)f2bf(b.x) | ((uint32_t)f2bf(b.y) << 16);
  u[3] = (uint32_t)f2bf(b.z) | ((uint32_t)f2bf(b.w) << 16);
  return __builtin_bit_cast(bf8, u);
}

// Orders this wave's LDS accesses: every earlier LDS read and write of the
// wave has completed before any later one is issued.
__device__ inline void lds_wave_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

__device__ inline f4 mfma32(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(SW * 64) void ae_score_kernel(const int64_t *__restrict__ T, int64_t R,
                                                           int I, const int32_t *it,
                                                           const uint16_t *__restrict__ wb,
                                                           const float *__restrict__ w,
                                                           const float *mu, const float *isd,
                                                           int kind, float *score, float *v_t) {
  extern __shared__ __align__(16) unsigned char smem[];
  ScoreLds &L = *reinterpret_cast<ScoreLds *>(smem);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int k = tid; k < AE_NW; k += SW * 64) {
    uint16_t v = wb[k];
    if (k < AE_W2) L.W1[(k / AE_IN) * P_W1 + k % AE_IN] = v;
    else if (k < AE_W3) L.W2[((k - AE_W2) / AE_H1) * P_W2 + (k - AE_W2) % AE_H1] = v;
    else if (k < AE_W4) L.W3[((k - AE_W3) / AE_H2) * P_W3 + (k - AE_W3) % AE_H2] = v;
    else L.W4[((k - AE_W4) / AE_H3) * P_W4 + (k - AE_W4) % AE_H3] = v;
  }
  for (int k = tid; k < AE_NP - AE_NW; k += SW * 64) L.b[k] = w[AE_NW + k];
  for (int k = tid; k < AE_IN; k += SW * 64) {
    L.mu[k] = mu[k];
    L.isd[k] = isd[k];
  }
  __syncthreads();
  auto &V = L.wv[wid];
  float *X = V.u.X;
  uint16_t *H = V.u.H;
  // MFMA operand layout: A/B lane -> row lane & 15, k = 8 * (lane >> 4) + 0..7;
  // D lane -> rows 4 * (lane >> 4) + 0..3, column lane & 15.
  const int row = lane & 15, kq = 8 * (lane >> 4), col = lane & 15, rq = 4 * (lane >> 4);
  // Loader: load h of a step reads rows 2h, 2h+1 (1 KB contiguous); lane ->
  // row 2h + lane / 32, columns lc, lc + 1.
  const int lh = lane >> 5, lc = 2 * (lane & 31);
  const float m0 = L.mu[lc], m1 = L.mu[lc + 1], s0 = L.isd[lc], s1 = L.isd[lc + 1];
  const float *bias = L.b;
  const int64_t nw = (int64_t)gridDim.x * SW;
  for (int64_t r = (int64_t)blockIdx.x * SW + wid; r < R; r += nw) {
    int n = it ? it[r] : I;
    if (n > I) n = I;
    if (n < 0) n = 0;
    const int64_t *src = T + r * (int64_t)I * AE_IN;
    // FP64 sums of the FP32 residuals: rows with equal residuals give exactly
    // equal means whatever the number of iterations (the robust z of kind 2
    // must see exact ties); squared errors are summed in FP32.
    float e2[4] = {0.f, 0.f, 0.f, 0.f};
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    u4v buf[16];
    // Rows past the rank's last one are clamped to it (loaded, then ignored),
    // so every load is in bounds and unconditional.
    auto load = [&](int i0) {
#pragma unroll
      for (int h = 0; h < 16; h++) {
        int i = i0 + 2 * h + lh;
        i = i < n ? i : n - 1;
        buf[h] = __builtin_nontemporal_load(reinterpret_cast<const u4v *>(src + (int64_t)i * AE_IN + lc));
      }
    };
    if (n > 0) load(0);
    for (int i0 = 0; i0 < n; i0 += SR) {
      // int64 -> FP32 (correctly rounded): cells in [0, 2^32) take one
      // unsigned conversion; a lane holding any wider cell converts all 32 in full.
      float cv[32];
      uint32_t wide = 0;
#pragma unroll
      for (int h = 0; h < 16; h++) {
        wide |= buf[h][1] | buf[h][3];
        cv[2 * h] = (float)buf[h][0];
        cv[2 * h + 1] = (float)buf[h][2];
      }
      if (wide) {
#pragma unroll
        for (int h = 0; h < 16; h++) {
          cv[2 * h] = (float)(int64_t)(((uint64_t)buf[h][1] << 32) | buf[h][0]);
          cv[2 * h + 1] = (float)(int64_t)(((uint64_t)buf[h][3] << 32) | buf[h][2]);
        }
      }
#pragma unroll
      for (int h = 0; h < 16; h++) {  // normalised inputs of this step (rows past n are zero)
        const int i = 2 * h + lh;
        const bool ok = i0 + i < n;
        float2 x;
        x.x = ok ? (cv[2 * h] - m0) * s0 : 0.f;
        x.y = ok ? (cv[2 * h + 1] - m1) * s1 : 0.f;
        *reinterpret_cast<float2 *>(&X[i * P_X + lc]) = x;
      }
      if (i0 + SR < n) load(i0 + SR);  // next step's rows, in flight during the network
      lds_wave_sync();
      bf8 a1[2][2];
      float xr[2][4][4];
#pragma unroll
      for (int t = 0; t < 2; t++) {
#pragma unroll
        for (int k = 0; k < 2; k++) a1[t][k] = ld_bf8_from_f32(&X[(16 * t + row) * P_X + 32 * k + kq]);
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
          for (int j = 0; j < 4; j++) xr[t][nt][j] = X[(16 * t + rq + j) * P_X + 16 * nt + col];
      }
      lds_wave_sync();
      // L1: [32 x 64] -> [32 x 128]
#pragma unroll
      for (int nt = 0; nt < AE_H1 / 16; nt++) {
        const bf8 b0 = ld_bf8(&L.W1[(16 * nt + row) * P_W1 + kq]);
        const bf8 b1 = ld_bf8(&L.W1[(16 * nt + row) * P_W1 + 32 + kq]);
        const int c = 16 * nt + col;
        const float bc = bias[c];
#pragma unroll
        for (int t = 0; t < 2; t++) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
          acc = mfma32(a1[t][0], b0, acc);
          acc = mfma32(a1[t][1], b1, acc);
#pragma unroll
          for (int j = 0; j < 4; j++) H[(16 * t + rq + j) * P_H + c] = f2bf(fmaxf(acc[j] + bc, 0.f));
        }
      }
      lds_wave_sync();
      // L2: [32 x 128] -> [32 x 32]
      {
        bf8 a2[2][4];
#pragma unroll
        for (int t = 0; t < 2; t++)
#pragma unroll
          for (int k = 0; k < 4; k++) a2[t][k] = ld_bf8(&H[(16 * t + row) * P_H + 32 * k + kq]);
#pragma unroll
        for (int nt = 0; nt < AE_H2 / 16; nt++) {
          bf8 bw[4];
#pragma unroll
          for (int k = 0; k < 4; k++) bw[k] = ld_bf8(&L.W2[(16 * nt + row) * P_W2 + 32 * k + kq]);
          const int c = 16 * nt + col;
          const float bc = bias[AE_B2 - AE_B1 + c];
#pragma unroll
          for (int t = 0; t < 2; t++) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 4; k++) acc = mfma32(a2[t][k], bw[k], acc);
#pragma unroll
            for (int j = 0; j < 4; j++) V.H2[(16 * t + rq + j) * P_H2 + c] = f2bf(fmaxf(acc[j] + bc, 0.f));
          }
        }
      }
      lds_wave_sync();
      // L3: [32 x 32] -> [32 x 128]
      {
        bf8 a3[2];
#pragma unroll
        for (int t = 0; t < 2; t++) a3[t] = ld_bf8(&V.H2[(16 * t + row) * P_H2 + kq]);
#pragma unroll
        for (int nt = 0; nt < AE_H3 / 16; nt++) {
          const bf8 bw = ld_bf8(&L.W3[(16 * nt + row) * P_W3 + kq]);
          const int c = 16 * nt + col;
          const float bc = bias[AE_B3 - AE_B1 + c];
#pragma unroll
          for (int t = 0; t < 2; t++) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma32(a3[t], bw, acc);
#pragma unroll
            for (int j = 0; j < 4; j++) H[(16 * t + rq + j) * P_H + c] = f2bf(fmaxf(acc[j] + bc, 0.f));
          }
        }
      }
      lds_wave_sync();
      // L4: [32 x 128] -> [32 x 64], residuals of the valid rows
      {
        bf8 a4[2][4];
#pragma unroll
        for (int t = 0; t < 2; t++)
#pragma unroll
          for (int k = 0; k < 4; k++) a4[t][k] = ld_bf8(&H[(16 * t + row) * P_H + 32 * k + kq]);
#pragma unroll
        for (int nt = 0; nt < AE_IN / 16; nt++) {
          bf8 bw[4];
#pragma unroll
          for (int k = 0; k < 4; k++) bw[k] = ld_bf8(&L.W4[(16 * nt + row) * P_W4 + 32 * k + kq]);
          const float bc = bias[AE_B4 - AE_B1 + 16 * nt + col];
#pragma unroll
          for (int t = 0; t < 2; t++) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 4; k++) acc = mfma32(a4[t][k], bw[k], acc);
#pragma unroll
            for (int j = 0; j < 4; j++) {
              const float r0 = acc[j] + bc - xr[t][nt][j];
              const float res = (i0 + 16 * t + rq + j < n) ? r0 : 0.f;  // rows past n add 0
              e2[nt] += res * res;
              rs[nt] += (double)res;
            }
          }
        }
      }
      lds_wave_sync();  // the next step's inputs overwrite H
    }
    float best = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const float a = col_sum(e2[nt]);
      const double b = col_sum(rs[nt]);
      if (kind == 2) {
        if (lane < 16) v_t[(int64_t)(16 * nt + col) * R + r] = n > 0 ? (float)(b / (double)n) : 0.f;
      } else {
        const float v = n > 0 ? (kind == 0 ? a / (float)n : (float)(fabs(b) / (double)n)) : 0.f;
        best = fmaxf(best, v);
      }
    }
    for (int d = 32; d >= 1; d >>= 1) best = fmaxf(best, __shfl_xor(best, d, 64));
    if (kind != 2 && lane == 0) score[r] = best;
  }
}

// ---------------------------------------------------------------------------
// Second stage of score kind 2, in FP32: per region g over the ranks with
// iterations, med = median of m(., g), MAD = median of |m - med|, z = (m - med)
// / (1.4826 MAD); when MAD is 0, 1.253314 * mean |m - med| (summed in FP64)
// replaces 1.4826 MAD; when that is 0 too, z = 0.  Medians of an even count
// are (a + b) * 0.5.  Every step is one IEEE FP32 operation in this order.
// Exact selection: radix select with 11-bit digits on order-preserving keys.
// ---------------------------------------------------------------------------
constexpr int RS = 1024;            // threads per region workgroup
constexpr int RSW = RS / 64;
constexpr int RNB = 2048;           // bins of an 11-bit digit
constexpr int RBPT = RNB / RS;

__device__ inline uint32_t fkey(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float fdec(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

struct RegLds {
  uint32_t hist[RNB];
  int64_t wtot[RSW];
  uint32_t wmin[RSW];
  double wsum[RSW];
  uint32_t state[4];
};

__device__ inline bool region_active(const int32_t *it, int I, int64_t r) {
  return it ? it[r] > 0 : I > 0;
}

// k-th smallest of keyf(r) over active ranks (32-bit keys), and with
// want_next the (k+1)-th.
template <class KeyF>
__device__ void select32(int64_t R, const int32_t *it, int I, KeyF keyf, int64_t k, bool want_next,
                         RegLds &L, uint32_t &v1, uint32_t &v2) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  uint32_t pref = 0;
  v1 = v2 = 0;
  for (int hi = 32; hi > 0;) {
    const int w = hi >= 11 ? 11 : hi;
    const int lo = hi - w;
    const bool last = lo == 0;
    uint32_t mgt = 0xffffffffu;
    for (int64_t r = t; r < R; r += RS) {
      if (!region_active(it, I, r)) continue;
      const uint32_t key = keyf(r);
      const uint32_t top = hi >= 32 ? 0u : key >> hi;
      if (top == pref) atomicAdd(&L.hist[(key >> lo) & ((1u << w) - 1)], 1u);
      else if (last && top > pref && key < mgt) mgt = key;
    }
    for (int d = 32; d >= 1; d >>= 1) {
      const uint32_t o = __shfl_xor(mgt, d, 64);
      mgt = o < mgt ? o : mgt;
    }
    if (lane == 0) L.wmin[wid] = mgt;
    __syncthreads();
    uint32_t cnt[RBPT];
    int64_t own = 0;
#pragma unroll
    for (int j = 0; j < RBPT; j++) {
      cnt[j] = L.hist[t * RBPT + j];
      own += cnt[j];
    }
    int64_t incl = own;
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(incl, d, 64);
      if (lane >= d) incl += o;
    }
    if (lane == 63) L.wtot[wid] = incl;
    __syncthreads();
    int64_t excl = incl - own;
    for (int q = 0; q < wid; q++) excl += L.wtot[q];
    uint32_t mg = L.wmin[0];
    for (int q = 1; q < RSW; q++) mg = L.wmin[q] < mg ? L.wmin[q] : mg;
    __syncthreads();  // all histogram reads are done
    for (int j = t; j < RNB; j += RS) L.hist[j] = 0;
    if (excl <= k && k < excl + own) {
      int64_t cum = excl;
      int j = 0;
      for (; j < RBPT; j++) {
        if (cum + (int64_t)cnt[j] > k) break;
        cum += cnt[j];
      }
      L.state[0] = (pref << w) | (uint32_t)(t * RBPT + j);
      L.state[1] = (uint32_t)(k - cum);
      L.state[2] = (k - cum + 1 < (int64_t)cnt[j]) ? 1u : 0u;
      // next non-empty bin above the selected one (only meaningful on the last digit)
      uint32_t nb = 0xffffffffu;
      for (int jj = j + 1; jj < RBPT && nb == 0xffffffffu; jj++)
        if (cnt[jj]) nb = (uint32_t)(t * RBPT + jj);
      L.state[3] = nb;
    }
    __syncthreads();
    const uint32_t np = L.state[0];
    const int64_t kk = (int64_t)L.state[1];
    if (last && want_next && L.state[2] == 0 && L.state[3] == 0xffffffffu) {
      // the next non-empty bin lies in a later thread's range: scan the merged
      // counts again (read before the clear by the owners, kept in cnt)
      uint32_t nb = 0xffffffffu;
      const uint32_t bsel = np & ((1u << w) - 1);
#pragma unroll
      for (int j = RBPT - 1; j >= 0; j--)
        if ((uint32_t)(t * RBPT + j) > bsel && cnt[j]) nb = (uint32_t)(t * RBPT + j);
      for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(nb, d, 64);
        nb = o < nb ? o : nb;
      }
      if (lane == 0) L.wmin[wid] = nb;
      __syncthreads();
      nb = L.wmin[0];
      for (int q = 1; q < RSW; q++) nb = L.wmin[q] < nb ? L.wmin[q] : nb;
      __syncthreads();
      if (t == 0) L.state[3] = nb;
      __syncthreads();
    }
    if (last) {
      v1 = np;
      if (!want_next || L.state[2]) v2 = np;
      else if (L.state[3] != 0xffffffffu) v2 = (pref << w) | L.state[3];
      else v2 = mg;
    }
    __syncthreads();
    pref = np;
    k = kk;
    hi = lo;
  }
  if (!want_next) v2 = v1;
}

__global__ __launch_bounds__(RS) void region_robust_f32(const float *__restrict__ v_t, int64_t R,
                                                        const int32_t *it, int I, float *z_t) {
  __shared__ RegLds L;
  const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const float *v = v_t + (int64_t)g * R;
  float *z = z_t + (int64_t)g * R;
  for (int j = t; j < RNB; j += RS) L.hist[j] = 0;
  int64_t nl = 0;
  for (int64_t r = t; r < R; r += RS) nl += region_active(it, I, r) ? 1 : 0;
  for (int d = 32; d >= 1; d >>= 1) nl += __shfl_xor(nl, d, 64);
  if (lane == 0) L.wtot[wid] = nl;
  __syncthreads();
  int64_t n = 0;
  for (int q = 0; q < RSW; q++) n += L.wtot[q];
  __syncthreads();
  float med = 0.f, scale = 0.f;
  if (n > 0) {
    const int64_t k = (n - 1) / 2;
    const bool even = (n & 1) == 0;
    uint32_t a, b;
    select32(R, it, I, [&](int64_t r) { return fkey(v[r]); }, k, even, L, a, b);
    med = even ? (fdec(a) + fdec(b)) * 0.5f : fdec(a);
    // |m - med| >= 0: its bit pattern orders like the value
    select32(R, it, I, [&](int64_t r) { return __float_as_uint(fabsf(v[r] - med)); }, k, even, L, a,
             b);
    const float mad = even ? (__uint_as_float(a) + __uint_as_float(b)) * 0.5f : __uint_as_float(a);
    if (mad > 0.f) {
      scale = 1.4826f * mad;
    } else {
      double sl = 0.0;
      for (int64_t r = t; r < R; r += RS)
        if (region_active(it, I, r)) sl += (double)fabsf(v[r] - med);
      for (int d = 32; d >= 1; d >>= 1) sl += __shfl_xor(sl, d, 64);
      if (lane == 0) L.wsum[wid] = sl;
      __syncthreads();
      double s = 0.0;
      for (int q = 0; q < RSW; q++) s += L.wsum[q];
      const double mean_ad = s / (double)n;
      if (mean_ad > 0.0) scale = (float)(1.253314 * mean_ad);
    }
  }
  for (int64_t r = t; r < R; r += RS)
    z[r] = (scale > 0.f && region_active(it, I, r)) ? (v[r] - med) / scale : 0.f;
}

// score[r] = max_g |z(r, g)| (0 for ranks without iterations).
__global__ __launch_bounds__(256) void rank_max_z32(const float *z_t, int64_t R, int G, float *score) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  float best = 0.f;
  for (int g = 0; g < G; g++) best = fmaxf(best, fabsf(z_t[(int64_t)g * R + r]));
  score[r] = best;
}

// ---------------------------------------------------------------------------
// Top-k: the k largest scores (ties toward the lower rank id), listed in
// ascending rank id; also counts scores above a threshold.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void topk_kernel(const float *score, int64_t R, int64_t k,
                                                    int32_t *idx, int32_t *n_above, float thr) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sh[4];
  __shared__ int64_t sc[1024];
  const int t = threadIdx.x;
  // Threshold key K*: the (R-k)-th smallest key (0-based); keys > K* all
  // selected, keys == K* taken in rank order until k are chosen.
  uint32_t pref = 0;
  int64_t want = R - k;  // rank of K* among ascending keys
  for (int sh_ = 24; sh_ >= 0; sh_ -= 8) {
    for (int b = t; b < 256; b += 1024) hist[b] = 0;
    __syncthreads();
    for (int64_t r = t; r < R; r += 1024) {
      const uint32_t key = fkey(score[r]);
      if (sh_ == 24 || (key >> (sh_ + 8)) == pref) atomicAdd(&hist[(key >> sh_) & 255], 1u);
    }
    __syncthreads();
    if (t == 0) {
      int64_t cum = 0;
      int b = 0;
      for (; b < 256; b++) {
        if (cum + (int64_t)hist[b] > want) break;
        cum += hist[b];
      }
      sh[0] = (pref << 8) | (uint32_t)b;
      sh[1] = (uint32_t)(want - cum);
    }
    __syncthreads();
    pref = sh[0];
    want = sh[1];
    __syncthreads();
  }
  const uint32_t kstar = pref;
  // count keys strictly greater than K*
  int64_t gt = 0, above = 0;
  for (int64_t r = t; r < R; r += 1024) {
    gt += fkey(score[r]) > kstar;
    above += score[r] > thr;
  }
  sc[t] = gt;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) sc[t] += sc[t + s];
    __syncthreads();
  }
  const int64_t n_gt = sc[0];
  __syncthreads();
  sc[t] = above;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) sc[t] += sc[t + s];
    __syncthreads();
  }
  if (t == 0 && n_above) n_above[0] = (int32_t)sc[0];
  __syncthreads();
  const int64_t ties = k - n_gt;  // how many keys equal to K* to take
  // Ordered compaction in chunks of 1024 ranks.
  int64_t base_gt = 0, base_tie = 0;
  for (int64_t c0 = 0; c0 < R; c0 += 1024) {
    const int64_t r = c0 + t;
    const uint32_t key = r < R ? fkey(score[r]) : 0u;
    const int is_gt = r < R && key > kstar;
    const int is_eq = r < R && key == kstar;
    sc[t] = ((int64_t)is_eq << 32) | is_gt;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int64_t x = t >= d ? sc[t - d] : 0;
      __syncthreads();
      sc[t] += x;
      __syncthreads();
    }
    const int64_t incl = sc[t];
    const int64_t gt_before = base_gt + (incl & 0xffffffffll) - is_gt;
    const int64_t tie_before = base_tie + (incl >> 32) - is_eq;
    if (is_gt || (is_eq && tie_before < ties))
      idx[gt_before + (tie_before < ties ? tie_before : ties)] = (int32_t)r;
    const int64_t tot = sc[1023];
    __syncthreads();
    base_gt += tot & 0xffffffffll;
    base_tie += tot >> 32;
  }
}

}  // namespace

hipError_t ae_alloc(AeState &s) {
  hipError_t e = hipSuccess;
  auto A = [&](void **p, size_t b) {
    if (e == hipSuccess) e = hipMalloc(p, b);
  };
  A((void **)&s.w, AE_NP * 4);
  A((void **)&s.wb, AE_NW * 2);
  A((void **)&s.m, AE_NP * 4);
  A((void **)&s.v, AE_NP * 4);
  A((void **)&s.mu, 64 * 4);
  A((void **)&s.isd, 64 * 4);
  A((void **)&s.nsum, 64 * 8);
  A((void **)&s.nsq, 128 * 8);
  A((void **)&s.ncnt, 8 * 8);
  A((void **)&s.part, (size_t)AE_WG * (AE_NP + 1) * 4);
  A((void **)&s.loss, 16);
  return e;
}

void ae_free(AeState &s) {
  void *ps[] = {s.w, s.wb, s.m, s.v, s.mu, s.isd, s.nsum, s.nsq, s.ncnt, s.part, s.loss};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  s = AeState{};
}

hipError_t launch_ae_init(AeState &s, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(ae_init_kernel, dim3((AE_NP + 255) / 256), dim3(256), 0, st, seed, s.w, s.wb,
                     s.m, s.v);
  s.step = 0;
  return hipGetLastError();
}

size_t ae_norm_ws_bytes(int64_t R) {
  const int64_t nb = (R + 63) / 64 < 1024 ? (R + 63) / 64 + 1 : 1025;
  return (size_t)nb * (64 * 8 + 128 * 8 + 8) + 1024;
}

hipError_t launch_ae_norm(AeState &s, const int64_t *T, int64_t R, int I, const int32_t *it,
                          bool reset, void *ws, size_t ws_bytes, hipStream_t st) {
  int64_t nb = (R + 63) / 64;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  const int64_t rpb = (R + nb - 1) / nb;
  char *p = (char *)ws;
  int64_t *ps = (int64_t *)p;
  uint64_t *pq = (uint64_t *)(p + nb * 64 * 8);
  int64_t *pc = (int64_t *)(p + nb * 64 * 8 + nb * 128 * 8);
  if ((size_t)(nb * (64 * 8 + 128 * 8 + 8)) > ws_bytes) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ae_norm_partial, dim3((unsigned)nb), dim3(256), 0, st, T, R, I, it, rpb, ps, pq, pc);
  hipLaunchKernelGGL(ae_norm_final, dim3(1), dim3(64), 0, st, (int)nb, ps, pq, pc, reset ? 1 : 0,
                     s.nsum, s.nsq, s.ncnt, s.mu, s.isd);
  return hipGetLastError();
}

size_t ae_rows_ws_bytes(int64_t R) { return (size_t)(R + 1) * 8 + 256; }

hipError_t launch_ae_rows(const AeState &s, const int64_t *T, int64_t R, int I, const int32_t *it,
                          float *rows, int64_t *n_rows, void *ws, size_t ws_bytes, hipStream_t st) {
  if ((size_t)(R + 1) * 8 > ws_bytes) return hipErrorInvalidValue;
  int64_t *off = (int64_t *)ws;
  hipLaunchKernelGGL(ae_rows_scan, dim3(1), dim3(1024), 0, st, it, R, I, off);
  if (rows && R > 0)
    hipLaunchKernelGGL(ae_rows_fill, dim3((unsigned)R), dim3(256), 0, st, T, R, I, off, s.mu, s.isd, rows);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && n_rows) e = hipMemcpyAsync(n_rows, off + R, 8, hipMemcpyDeviceToHost, st);
  return e;
}

template <class K>
void allow_lds(K k) {
  static bool done = false;
  if (!done) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)sizeof(AeLds));
    done = true;
  }
}

hipError_t launch_ae_step(AeState &s, const float *rows, int64_t n, int64_t k0, int batch,
                          uint64_t a, uint64_t c, float lr, bool update, float noise_sd,
                          uint64_t noise_key, hipStream_t st, float *grad_out, float *loss_out,
                          float *epoch_loss, float lfrac) {
  const int64_t k_end = k0 + batch < n ? k0 + batch : n;
  const int64_t bv = k_end - k0;
  if (bv <= 0) return hipErrorInvalidValue;
  const float scale = 2.0f / (float)(bv * AE_IN);
  allow_lds(&ae_fwdbwd);
  hipLaunchKernelGGL(ae_fwdbwd, dim3(AE_WG), dim3(AT), sizeof(AeLds), st, rows, n, k0, k_end, a, c,
                     scale, noise_sd, noise_key, s.wb, s.w, s.part);
  float bc1 = 1.f, bc2 = 1.f;
  if (update) {
    s.step++;
    bc1 = (float)(1.0 - pow(0.9, (double)s.step));
    bc2 = (float)(1.0 - pow(0.999, (double)s.step));
  }
  hipLaunchKernelGGL(ae_adam, dim3((AE_NP + 255) / 256), dim3(256), 0, st, s.part, AE_WG, s.w, s.wb,
                     s.m, s.v, lr, bc1, bc2, update ? 1 : 0, grad_out, loss_out ? loss_out : s.loss,
                     1.0f / (float)(bv * AE_IN), epoch_loss, lfrac);
  return hipGetLastError();
}

hipError_t launch_ae_grad_f32(AeState &s, const float *rows, int64_t n, float noise_sd,
                              uint64_t noise_key, hipStream_t st, float *grad_out, float *loss_out) {
  if (n <= 0) return hipErrorInvalidValue;
  const float scale = 2.0f / (float)(n * AE_IN);
  hipLaunchKernelGGL(ae_grad_f32_kernel, dim3(AE_WG), dim3(256), 0, st, rows, n, scale, noise_sd,
                     noise_key, s.w, s.part);
  hipLaunchKernelGGL(ae_adam, dim3((AE_NP + 255) / 256), dim3(256), 0, st, s.part, AE_WG, s.w, s.wb,
                     s.m, s.v, 0.f, 1.f, 1.f, 0, grad_out, loss_out ? loss_out : s.loss,
                     1.0f / (float)(n * AE_IN), (float *)nullptr, 0.f);
  return hipGetLastError();
}

size_t ae_score_ws_bytes(int64_t R) { return 2 * (((size_t)R * AE_IN * 4 + 255) & ~(size_t)255); }

hipError_t launch_ae_score(const AeState &s, const int64_t *T, int64_t R, int I, const int32_t *it,
                           float *score, void *ws, size_t ws_bytes, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&ae_score_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(ScoreLds));
    attr = true;
  }
  if (R <= 0) return hipSuccess;
  const bool stage2 = s.score_kind == 2;
  const size_t half = ae_score_ws_bytes(R) / 2;
  if (stage2 && (ws == nullptr || ws_bytes < 2 * half)) return hipErrorInvalidValue;
  float *v_t = stage2 ? (float *)ws : nullptr;
  float *z_t = stage2 ? (float *)((char *)ws + half) : nullptr;
  int cus = 256, dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int64_t grid = (R + SW - 1) / SW;
  if (grid > cus) grid = cus;
  hipLaunchKernelGGL(ae_score_kernel, dim3((unsigned)grid), dim3(SW * 64), sizeof(ScoreLds), st, T, R,
                     I, it, s.wb, s.w, s.mu, s.isd, s.score_kind, score, v_t);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && stage2) {
    hipLaunchKernelGGL(region_robust_f32, dim3(AE_IN), dim3(RS), 0, st, v_t, R, it, I, z_t);
    hipLaunchKernelGGL(rank_max_z32, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, z_t, R, AE_IN,
                       score);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_topk(const float *score, int64_t R, int64_t k, int32_t *idx, int32_t *n_above,
                       float thr, hipStream_t st) {
  hipLaunchKernelGGL(topk_kernel, dim3(1), dim3(1024), 0, st, score, R, k, idx, n_above, thr);
  return hipGetLastError();
}

}  // namespace ta
