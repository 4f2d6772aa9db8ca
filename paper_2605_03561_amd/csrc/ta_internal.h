// ta_internal.h -- shared declarations of the HIP trace-analysis library.
// Device code is written for gfx950 (CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ta.h"

namespace ta {

// Sticky device error bits (one per data-error kind).
enum : uint32_t {
  ERRBIT_CTX = 1u,
  ERRBIT_UNSORTED = 2u,
  ERRBIT_OVERFLOW = 4u,
  ERRBIT_OFFSETS = 8u,
};

// Packed per-node word used by the trace kernels (indexed by caller node id):
//   bits 0..8   region index + 1 (0 = the node is in no region)
//   bit  9      node lies in the marker's subtree
//   bits 10..31 preorder index of the node
constexpr int INFO_REGION_BITS = 9;
constexpr uint32_t INFO_REGION_MASK = (1u << INFO_REGION_BITS) - 1u;
constexpr uint32_t INFO_MARKER_BIT = 1u << INFO_REGION_BITS;
constexpr int INFO_TIN_SHIFT = 10;

constexpr int MAX_NODES_ATTR = 8192;      // LDS histogram limit for attribution
constexpr int MAX_NODES = 1 << 22;        // preorder index field width
constexpr int MAX_REGIONS = 256;

// One request of a mixed batch: its traces, iteration count and outputs.
struct SegReq {
  const int64_t *off;
  const int64_t *ts;
  const int32_t *ctx;
  int64_t E;
  int32_t I;
  int64_t *tensor;
  int32_t *iters_found;
  int64_t *outside;
  int64_t *span;
  int64_t *rank_sum;
  uint64_t *rank_sumsq;
  int64_t *excl;
  int64_t *incl;
};

struct SegArgs {
  const int64_t *off;
  const int64_t *ts;
  const int32_t *ctx;
  int64_t R;
  int64_t E;
  const uint32_t *info;   // [N]
  const int2 *tin_tout;   // [N] preorder index and subtree end, by caller id
  const int32_t *order;   // rank visiting order (NULL = identity)
  int32_t N, G, I, W, log2W;
  int64_t *tensor;
  int32_t *iters_found;
  int64_t *outside;
  int64_t *span;
  int64_t *rank_sum;
  uint64_t *rank_sumsq;
  int64_t *excl;
  int64_t *incl;
  uint32_t *err;
  // Mixed batch (reqs != NULL): R tasks; tasks[k] = (request << 32) | rank, and the
  // per-request fields come from reqs[request] instead of the ones above.
  const SegReq *reqs;
  const int64_t *tasks;
};

// Launch shape of the fused pass (chosen by the batch autotuner).
struct SegShape {
  int threads = 256;        // workgroup size: 256, or 512 (fused pass, ept 2 or 4)
  int ept = 4;              // events per thread per tile: 2, 4, 8 or 16
  bool nontemporal = false; // streaming loads/stores that bypass cache retention
  int wgs_per_cu = 0;       // 0: one workgroup per rank; k > 0: persistent, k per CU
};

// Launchers (defined in the kernel translation units).
hipError_t launch_segment(const SegArgs &a, bool attr, bool seg, const SegShape &sh, int grid,
                          size_t lds_bytes, hipStream_t s);
size_t segment_lds_bytes(int N, int G, bool attr, bool seg, int *W, int *log2W);

struct ImbArgs {
  const int64_t *T;
  int64_t R;
  int32_t I, G;
  const int32_t *it;
  const int64_t *rank_sum;
  const uint64_t *rank_sumsq;
  const int64_t *span;
  int32_t ddof;
  double t_app;
  ta_imbalance_out o;
};
// Per-column partial statistics over chunks of ranks, [rc][I*G] each: valid
// cell count, int64 sum, unsigned 128-bit sum of squares (lo, hi), min, max.
// Integer partials: how the ranks are split into chunks does not change the
// combined result.
struct ColPartials {
  int64_t *n, *s1, *mn, *mx;
  uint64_t *lo, *hi;
  int rc;  // 0: none
};
// rc_ext > 0: the partials ([rc_ext] chunks, in the workspace as
// imbalance_partials() places them) were written by another kernel (the FULL
// outlier scan's transpose), so the column pass over the tensor is skipped.
hipError_t launch_imbalance(const ImbArgs &a, void *ws, size_t ws_bytes, hipStream_t s,
                            int rc_ext = 0);
size_t imbalance_ws_bytes(int64_t R, int32_t I, int32_t G, bool need_rank_stats, int rc_ext = 0);
ColPartials imbalance_partials(void *ws, int64_t R, int32_t I, int32_t G, bool need_rank_stats,
                               int rc_ext);

struct OutArgs {
  const int64_t *T;
  int64_t R;
  int32_t I, G;
  const int32_t *it;
  int32_t mode, kind;
  double tau;
  double *rank_score;
  uint8_t *rank_flag;
  int64_t *n_flagged;
  double *region_score;
  // FULL scan: the transpose also writes the imbalance column partials here
  // (stats.rc must be transpose_groups(R)).
  ColPartials stats;
  // When set (with stats), recorded on the stream right after the pass that
  // writes the imbalance partials, so a consumer on another stream can start.
  hipEvent_t stats_ready = nullptr;
  // When set, the row-major robust FULL scan runs as two column halves
  // (iterations [0, I/2) and [I/2, I)) in a pipeline: the streaming passes on
  // the launch stream, each half's per-column selection on `side` beside the
  // other half's pass; ev[] are the fork and join events (all ten distinct).
  // `side` is joined back into the launch stream before the call returns.
  hipStream_t side = nullptr;
  hipEvent_t ev[10] = {};
};
// Rank chunks of the FULL scan's transpose (TG tiles of 64 ranks each).
int transpose_groups(int64_t R);
// Robust z over active ranks of per-rank region values v_t[G][R] (median and
// MAD per region, the exact scan's second stage), z_t[G][R], and FP32
// score[r] = max_g |z|.
hipError_t launch_region_robust(const double *v_t, int64_t R, int G, const int32_t *it, int I,
                                double *z_t, float *score, hipStream_t s);
// Raises the dynamic LDS limit of the outlier kernels that use more than
// 64 KB; called once per handle, before any launch or capture.
void outliers_init();
hipError_t launch_outliers(const OutArgs &a, void *ws, size_t ws_bytes, hipStream_t s);
size_t outliers_ws_bytes(int64_t R, int32_t I, int32_t G, int32_t mode, int32_t kind);

// Summary profile, pruning, pruned per-rank profiles and the inclusive
// tensor (k_prune.hip).  tin_tout[v] = (preorder index, subtree end).
size_t subtree_rows_lds_bytes(int N, int K, bool excl);
hipError_t launch_summary(const int64_t *excl, int64_t R, int N, const int2 *tin_tout,
                          int64_t *sum_excl, int64_t *sum_incl, void *ws, int cus, hipStream_t s);
// out[v] = sum of vec over the subtree of v, any N up to MAX_NODES (workspace
// subtree_sums_ws_bytes(N), none for N <= 8192).
size_t subtree_sums_ws_bytes(int N);
hipError_t launch_subtree_sums(const int64_t *vec, int N, const int2 *tin_tout, int64_t *out, void *ws,
                               int cus, hipStream_t s);
// Sparse per-rank profiles (k_window.hip): rank r's non-zero exclusive costs
// in ascending node id at [off[r], off[r] + counts[r]).
hipError_t launch_sparse_profiles(const int64_t *off, const int64_t *ts, const int32_t *ctx, int64_t R,
                                  int64_t E, int N, int64_t *counts, int32_t *ids, int64_t *vals, uint32_t *err,
                                  int cus, hipStream_t s);
// Time-window profile (k_window.hip).
size_t window_ws_bytes(int N, int64_t n_sel);
hipError_t launch_window_profile(const int64_t *off, const int64_t *ts, const int32_t *ctx, int64_t R,
                                 int64_t E, const int32_t *ids, int64_t n_sel, int N, const int2 *tin_tout,
                                 int64_t t0, int64_t t1, int64_t *excl, int64_t *incl, void *ws,
                                 uint32_t *err, int cus, hipStream_t s);
hipError_t launch_prune(const int64_t *sum_excl, const int64_t *sum_incl, int N, double fraction,
                        int32_t *kept, int32_t *n_kept, hipStream_t s);
hipError_t launch_pruned_profiles(const int64_t *excl, int64_t R, int N, const int2 *tin_tout,
                                  const int2 *kq, int K, const int32_t *kpar, int64_t *p_excl,
                                  int64_t *p_incl, int cus, hipStream_t s);
hipError_t launch_tensor_inclusive(const int64_t *T, int64_t n_rows, int G, const int4 *rt,
                                   int64_t *out, int cus, hipStream_t s);

// Sparse node x rank x iteration model (k_nodemodel.hip).  ptab[p] for the
// preorder position p: (caller id, parent position or -1, subtree end, 0).
struct NodeModelArgs {
  const int64_t *off, *ts;
  const int32_t *ctx;
  int64_t R, E;
  int I, N;
  const uint32_t *info;
  const int4 *ptab;
  int64_t *row_start;     // count: written; fill: read
  int32_t *iters_found;   // count: written; fill: read
  int64_t *row_off_x, *row_off_i;  // count: written ([R*I + 1]); fill: read
  int32_t *node_x, *node_i;
  int64_t *val_x, *val_i;
  uint32_t *err;
};
size_t node_model_ws_bytes(int64_t R, int I, int64_t E, int N, int cus);
hipError_t launch_node_model(const NodeModelArgs &m, bool fill, void *ws, int cus, hipStream_t s);

// Clustering of ranks (k_cluster.hip).
size_t kmeans_ws_bytes(int K, int D, int64_t R);
hipError_t launch_kmeans(const int64_t *X, int64_t R, int D, int K, const double *C0, int max_iter,
                         int32_t *labels, double *C, int64_t *counts, int32_t *n_iter, void *ws,
                         int cus, hipStream_t s);
size_t dbscan_ws_bytes(int64_t R);
hipError_t launch_dbscan1d(const int64_t *x, int64_t R, int64_t eps, int64_t min_pts,
                           int32_t *labels, int32_t *n_clusters, uint8_t *core, void *ws, int cus,
                           hipStream_t s);
size_t node_intersections_ws_bytes(int32_t n_nodes);
hipError_t launch_node_intersections(const int32_t *labels, const int32_t *rank_node, int64_t R,
                                     int32_t n_nodes, int K, int64_t *pair, int32_t *node_clusters,
                                     void *ws, uint32_t *err, int cus, hipStream_t s);

struct TopoArgs {
  const double *score;
  const uint8_t *flag;
  int64_t R;
  const int32_t *rank_node, *node_rack, *node_chassis;
  int32_t n_nodes, n_racks, n_chassis;
  int64_t *fl_rack;
  double *mx_rack, *mn_rack;
  int64_t *fl_ch;
  double *mx_ch, *mn_ch;
  uint32_t *err;
};
hipError_t launch_topology(const TopoArgs &a, hipStream_t s);

}  // namespace ta
