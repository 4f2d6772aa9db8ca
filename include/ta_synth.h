/*
 * ta_synth.h -- GPU generator of synthetic execution traces (benchmark and
 * test inputs only; it computes nothing of the analysis method).
 *
 * The traces follow the iteration-structured recipe of the library's seeded
 * workload generator: per rank and iteration, region durations
 * D = round(scale[r,g] * Gamma(4, mu[g]/4)) ns laid out as
 * [marker][regions in a random per-iteration order][filler ~ Exp(filler_mean)],
 * with b = events_per_iter[r] events per iteration: when b >= G + 2 one event
 * at every segment start plus b - G - 2 events at stratified-jittered times
 * (so the segmented tensor equals D exactly), otherwise the marker plus b - 1
 * stratified-jittered samples.  A final root event closes each trace.  The
 * shapes mimic the paper's workloads (Sec. VI: iterative applications, many
 * ranks); the values are random draws from SplitMix64 (Steele, Lea, Flood,
 * OOPSLA 2014) on per-(seed, rank, iteration, slot) counters.
 *
 * All array pointers are DEVICE pointers owned by the caller.
 */
#ifndef TA_SYNTH_H_
#define TA_SYNTH_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t n_ranks;
  int32_t n_iters;
  int32_t n_regions;        /* G <= 127 */
  int32_t marker;           /* node id of the iteration marker */
  int32_t root;             /* node id used for the closing event */
  uint64_t seed;
  double filler_mean_ns;
  const int64_t *offsets;   /* [R+1]; offsets[r+1]-offsets[r] = n_iters*b_r + 1 */
  const int32_t *events_per_iter; /* [R] b_r >= 1 */
  const int64_t *t0;        /* [R] first timestamp */
  const double *scale;      /* [R*G] duration multiplier per rank and region */
  const double *mu;         /* [G] mean region duration (ns) */
  const int32_t *pool;      /* node ids: region 0 members, ..., region G-1, filler */
  const int32_t *pool_off;  /* [G+2] offsets into pool */
  int64_t *ts;              /* [E] out */
  int32_t *ctx;             /* [E] out */
} tas_params;

/* Fills ts/ctx for every rank; asynchronous on `stream`.  Returns 0, or 1 for
 * an invalid argument, or 8 for a HIP launch error. */
int32_t tas_generate(const tas_params *p, void *stream);

/* A plain device-to-device copy of n_bytes (a multiple of 16, both pointers
 * 16-byte aligned): the reference kernel whose measured rate calibrates the
 * HBM figures (what a streaming read + write reaches on this GPU).  Each
 * thread moves four 16-byte vectors per step, loads issued before stores;
 * grid = workgroups_per_cu x the device's compute units (0: 8).  Asynchronous
 * on `stream`; returns 0, 1 for an invalid argument, 8 for a launch error. */
int32_t tas_copy(void *dst, const void *src, int64_t n_bytes, int32_t workgroups_per_cu,
                 void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TA_SYNTH_H_ */
