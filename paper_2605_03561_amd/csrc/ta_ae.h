// ta_ae.h -- autoencoder (learned pre-screen) state and launchers.
//
// Network 64 -> 128 -> 32 -> 128 -> 64, ReLU after the hidden layers, linear
// output; FP32 master weights and Adam moments, bfloat16 copies of the weights
// for the matrix cores, FP32 accumulation.  Parameter vector layout (FP32):
//   W1[128][64] W2[32][128] W3[128][32] W4[64][128] b1[128] b2[32] b3[128] b4[64]
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ta {

constexpr int AE_IN = 64;
constexpr int AE_H1 = 128;
constexpr int AE_H2 = 32;
constexpr int AE_H3 = 128;
constexpr int AE_W1 = 0;
constexpr int AE_W2 = AE_W1 + AE_H1 * AE_IN;   // 8192
constexpr int AE_W3 = AE_W2 + AE_H2 * AE_H1;   // 12288
constexpr int AE_W4 = AE_W3 + AE_H3 * AE_H2;   // 16384
constexpr int AE_NW = AE_W4 + AE_IN * AE_H3;   // 24576 weights
constexpr int AE_B1 = AE_NW;
constexpr int AE_B2 = AE_B1 + AE_H1;
constexpr int AE_B3 = AE_B2 + AE_H2;
constexpr int AE_B4 = AE_B3 + AE_H3;
constexpr int AE_NP = AE_B4 + AE_IN;           // 24928 parameters

struct AeState {
  float *w = nullptr;        // [AE_NP] FP32 master parameters
  uint16_t *wb = nullptr;    // [AE_NW] bfloat16 copy of the weights
  float *m = nullptr;        // [AE_NP] Adam first moment
  float *v = nullptr;        // [AE_NP] Adam second moment
  float *mu = nullptr;       // [64] region mean
  float *isd = nullptr;      // [64] 1 / region standard deviation
  int64_t *nsum = nullptr;   // [64] running sum of cell values   (normalisation fit)
  uint64_t *nsq = nullptr;   // [64][2] running 128-bit sum of squares
  int64_t *ncnt = nullptr;   // [1] running cell count per region
  float *part = nullptr;     // [AE_WG][AE_NP + 1] per-workgroup gradient partials (+ loss)
  float *loss = nullptr;     // [1] loss of the last step / batch
  int64_t step = 0;          // Adam step counter
  bool ready = false;        // weights initialised
  bool normed = false;       // normalisation fitted
  float threshold = -1.f;    // calibrated score threshold (fallback rule); < 0: none
  int score_kind = 0;        // 0: max mean squared error, 1: max |mean residual|,
                             // 2: max robust z over ranks of the mean residual
};

constexpr int AE_WG = 256;  // workgroups per training step (gradient partials): one
                            // 16-row tile each at the default batch of 4,096 rows

hipError_t ae_alloc(AeState &s);
void ae_free(AeState &s);
hipError_t launch_ae_init(AeState &s, uint64_t seed, hipStream_t st);
hipError_t launch_ae_norm(AeState &s, const int64_t *T, int64_t R, int I, const int32_t *it,
                          bool reset, void *ws, size_t ws_bytes, hipStream_t st);
size_t ae_norm_ws_bytes(int64_t R);
hipError_t launch_ae_rows(const AeState &s, const int64_t *T, int64_t R, int I, const int32_t *it,
                          float *rows, int64_t *n_rows, void *ws, size_t ws_bytes, hipStream_t st);
size_t ae_rows_ws_bytes(int64_t R);
// One optimiser step on rows perm(k), k in [k0, k0 + batch), perm(k) = (a*k + c) mod n;
// noise_sd > 0: denoising step (inputs x + noise_sd * N(0,1) drawn under noise_key).
// With epoch_loss, also epoch_loss[0] += (the step's loss) * lfrac.
hipError_t launch_ae_step(AeState &s, const float *rows, int64_t n, int64_t k0, int batch,
                          uint64_t a, uint64_t c, float lr, bool update, float noise_sd,
                          uint64_t noise_key, hipStream_t st, float *grad_out, float *loss_out,
                          float *epoch_loss = nullptr, float lfrac = 0.f);
// The same gradient and mean loss over rows[0..n) in FP32 throughout (a debug
// reference for the matrix-core path; no update).
hipError_t launch_ae_grad_f32(AeState &s, const float *rows, int64_t n, float noise_sd,
                              uint64_t noise_key, hipStream_t st, float *grad_out, float *loss_out);
// Workspace of launch_ae_score (score kind 2 keeps per-region residual means
// and their z-scores, [64][R] FP64 each).
size_t ae_score_ws_bytes(int64_t R);
hipError_t launch_ae_score(const AeState &s, const int64_t *T, int64_t R, int I, const int32_t *it,
                           float *score, void *ws, size_t ws_bytes, hipStream_t st);
hipError_t launch_topk(const float *score, int64_t R, int64_t k, int32_t *idx, int32_t *count_gt_thr,
                       float thr, hipStream_t st);

}  // namespace ta
