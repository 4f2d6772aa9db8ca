/*
 * ta.h -- C ABI of the MI355X (gfx950) trace-analysis library.
 *
 * The library reduces a batch of per-rank execution traces (timestamped
 * calling-context-tree node events) to a rank x iteration x region time tensor
 * and computes cross-rank imbalance and outlier statistics on it.
 *
 * Paper: "Enhancing Performance Insight at Scale: A Heterogeneous Framework for
 * Exascale Diagnostics" (arXiv 2605.03561).  Sec. II defines an execution
 * trace as a series of timed CCT-node events per rank; Sec. V re-materialises
 * per-iteration profiles from traces (iteration boundaries found by a scan)
 * into a node x trace x iteration model; Sec. VI-A derives per-iteration
 * groupby statistics, the global balance ratio, coefficients of variation and
 * the potential savings (Tables IV and V); Sec. VI-B maps ranks to compute
 * nodes and to physical rack / chassis coordinates.
 *
 * Conventions (all calls):
 *   - Bulk arrays are DEVICE pointers owned by the caller; the library never
 *     frees or keeps them past the call.  Small descriptors (the parent array,
 *     the region list, host offsets for planning) are HOST pointers, copied
 *     during the call.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  Outputs are valid once the stream has reached the call.
 *   - Argument errors are detected on the host before anything is launched
 *     and returned as a status; nothing is written then.
 *   - Data errors (context id out of range, decreasing timestamps, more
 *     iterations than the tensor holds, inconsistent offsets) are detected on
 *     the device and recorded in a sticky per-handle word; the outputs of the
 *     call that met them are unspecified.  ta_sync_status() waits for the
 *     stream, returns the error (or TA_OK) and clears it.
 *   - Row-major layouts: tensor[(r*I + i)*G + g], excl[r*N + v].
 *   - Alignment: every device array must be 16-byte aligned (torch's default
 *     allocations are); otherwise TA_ERR_INVALID_ARG.
 *   - A handle may be used from one host thread at a time.  Calls on one
 *     handle share its workspace: calls issued on different streams of the
 *     same handle must not overlap in time.
 *   - No C++ exception crosses this interface.
 */
#ifndef TA_H_
#define TA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ta_status;
enum {
  TA_OK = 0,
  TA_ERR_INVALID_ARG = 1,    /* bad argument, or (device) inconsistent offsets */
  TA_ERR_BAD_TREE = 2,       /* parent array has a cycle or an out-of-range id */
  TA_ERR_CTX_RANGE = 3,      /* (device) a context id outside [0, N)           */
  TA_ERR_UNSORTED = 4,       /* (device) timestamps decrease within a rank     */
  TA_ERR_ITER_OVERFLOW = 5,  /* (device) a rank has more than n_iters iterations */
  TA_ERR_SIZE_OVERFLOW = 6,  /* a size exceeds what a kernel supports          */
  TA_ERR_OOM = 7,            /* workspace allocation failed                    */
  TA_ERR_HIP = 8,            /* a HIP runtime call failed                      */
  TA_ERR_STATE = 9           /* a required earlier call is missing             */
};

typedef struct ta_handle_s *ta_handle;

/* Handle life cycle.  `device` is the HIP device ordinal the handle's
 * workspace and kernels use.  The handle owns its workspace and the call-path
 * tables.  ta_destroy waits for the device; it returns TA_ERR_STATE (and
 * keeps the handle) while batch plans made on the handle still exist. */
ta_status ta_create(ta_handle *out, int device);
ta_status ta_destroy(ta_handle h);
const char *ta_status_string(ta_status s);
/* Human-readable detail of the last failure on this handle (never NULL). */
const char *ta_last_error(ta_handle h);
/* Blocks until `stream` is idle; returns and clears the sticky device error.
 * When several kinds were met, the first of CTX_RANGE, UNSORTED,
 * ITER_OVERFLOW, INVALID_ARG is returned. */
ta_status ta_sync_status(ta_handle h, void *stream);

/* Calling-context tree (Sec. II; Sec. VI-B walks it bottom-up from a leaf).
 * parent_host[v] is the parent of node v, -1 for a root; a forest is allowed.
 * Any numbering is accepted: the library renumbers nodes in depth-first
 * preorder internally.  A cycle or an id outside [-1, N) -> TA_ERR_BAD_TREE.
 * N must be at most 8192 for attribution (exclusive/inclusive cost) and at
 * most 4194304 otherwise.  Resets the regions.  Waits for the device before
 * replacing the previous tables; TA_ERR_STATE while batch plans exist. */
ta_status ta_set_tree(ta_handle h, int32_t n_nodes, const int32_t *parent_host);

/* Iteration marker and regions (Sec. V: iterations are found by scanning the
 * traces; Sec. VI-A: the regions are the kernels under study).  An event opens
 * a new iteration when its context lies in the marker's subtree and the
 * previous event of the same rank does not.  An event belongs to region g when
 * region_nodes_host[g] is the nearest ancestor-or-self of its context among
 * the region nodes.  1 <= n_regions <= 256, distinct nodes.  Waits for the
 * device before replacing the tables; TA_ERR_STATE while batch plans exist. */
ta_status ta_set_regions(ta_handle h, int32_t marker_node, int32_t n_regions,
                         const int32_t *region_nodes_host);

/* A batch of traces in CSR form (device pointers):
 *   offsets[n_ranks + 1] (int64, offsets[0] = 0, non-decreasing,
 *   offsets[n_ranks] = n_events), ts[n_events] (int64 ns, non-decreasing within
 *   a rank), ctx[n_events] (int32 node ids).  The duration of an event is the
 *   next timestamp of the same rank minus its own; a rank's last event lasts 0. */
typedef struct {
  int64_t n_ranks;
  int64_t n_events;
  const int64_t *offsets;
  const int64_t *ts;
  const int32_t *ctx;
} ta_traces;

/* Outputs of the segmentation / attribution pass (device pointers; any may be
 * NULL unless stated):
 *   tensor[R*I*G]   int64 time per (rank, iteration, region) -- required for
 *                   segmentation; rows i >= iters_found[r] are zero
 *   iters_found[R]  int32 number of iterations (boundaries) found -- required
 *                   for segmentation
 *   outside[R]      int64 time in no region or before the first boundary
 *   span[R]         int64 last minus first timestamp
 *   rank_sum[R*G]   int64 sum over the rank's iterations of its cells
 *   rank_sumsq[R*G*2] unsigned 128-bit sum of squares of the same cells, as
 *                   (low, high) uint64 pairs
 *   excl[R*N], incl[R*N]  int64 exclusive / inclusive time per CCT node, in
 *                   the caller's node numbering */
typedef struct {
  int64_t *tensor;
  int32_t *iters_found;
  int64_t *outside;
  int64_t *span;
  int64_t *rank_sum;
  uint64_t *rank_sumsq;
  int64_t *excl;
  int64_t *incl;
} ta_seg_out;

/* Exclusive and inclusive cost per CCT node and rank (Sec. VI-B: profiles
 * carry inclusive and exclusive costs per calling context; Sec. II: trace
 * samples are timed CCT-node events).  excl[r][v] = total duration of rank
 * r's events whose context is v; incl[r][v] = sum of excl[r][u] over the
 * subtree of v.  Needs ta_set_tree(). */
ta_status ta_attribute(ta_handle h, const ta_traces *t, int64_t *excl, int64_t *incl,
                       void *stream);

/* Iteration segmentation into the rank x iteration x region tensor (Sec. V,
 * Fig. 2: one re-materialised profile per iteration interval, indexed by
 * trace and iteration).  Events before the first boundary and events in no
 * region go to `outside`.  Needs ta_set_tree() and ta_set_regions(). */
ta_status ta_segment(ta_handle h, const ta_traces *t, int32_t n_iters, int64_t *tensor,
                     int32_t *iters_found, int64_t *outside, void *stream);

/* Fused single pass over the traces producing everything in `out` that is
 * non-NULL (attribution needs excl and/or incl; segmentation needs tensor and
 * iters_found).  This is the measured hot path. */
ta_status ta_attribute_segment(ta_handle h, const ta_traces *t, int32_t n_iters,
                               const ta_seg_out *out, void *stream);

/* Imbalance statistics (Sec. VI-A: the groupby listing's mean / min / max /
 * std per iteration across ranks with pandas' ddof; global balance ratio =
 * mean over ranks / max over ranks of the run totals; coefficients of
 * variation across and within ranks, Table IV; potential savings = average
 * max - average mean per iteration, total = savings x iterations, speedup =
 * total / application time, Table V).
 * Per cell (i,g) over the ranks valid in iteration i (i < iters_found[r];
 * all ranks when iters_found is NULL):
 *   mean = s1/n, std = sqrt((n*s2 - s1^2)/(n*(n-ddof))), max_minus_mean =
 *   (n*max - s1)/n, min, max   -- from exact int64 / int128 sums.
 * Per region g over the iterations with at least one valid rank (I'):
 *   avg_mean, avg_max, savings_per_iter = mean over I' of max_minus_mean,
 *   total_savings = savings_per_iter * |I'|, balance_ratio = (sum_r S/R) /
 *   max_r S with S the rank's total, cv_across = mean over I' (mean > 0,
 *   n > ddof) of std/mean, cv_within = mean over ranks (n_r > ddof, S > 0) of
 *   the rank's std over its iterations / its mean, share = region total /
 *   all regions' total.  potential_speedup = sum_g total_savings / t_app_ns;
 *   t_app_ns <= 0 uses max_r span[r] (NaN if span is NULL).
 * rank_sum / rank_sumsq (as produced by ta_attribute_segment) may be NULL;
 * the library then computes them with an extra pass over the tensor.
 * Every output pointer in `o` is a device pointer and may be NULL. */
typedef struct {
  double *mean, *std, *max_minus_mean; /* [I*G] */
  int64_t *min, *max;                  /* [I*G] */
  double *avg_mean, *avg_max, *savings_per_iter, *total_savings, *balance_ratio,
      *cv_across, *cv_within, *share;  /* [G] */
  double *potential_speedup;           /* [1] */
} ta_imbalance_out;

ta_status ta_imbalance(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                       int32_t n_regions, const int32_t *iters_found, const int64_t *rank_sum,
                       const uint64_t *rank_sumsq, const int64_t *span, int32_t ddof,
                       double t_app_ns, const ta_imbalance_out *o, void *stream);

/* Allocation-free variant of ta_imbalance, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, outputs, results and error
 * behaviour as ta_imbalance; it calls no allocating routine.  Its workspace is
 * a static device array of TA_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, which
 * the library holds from the first ta_create on that GPU until the process
 * ends; nothing in it needs to start at zero.  A call whose workspace would
 * exceed it (per-column partials of about 48 B x n_iters x n_regions x rank
 * chunks, plus 24 B x n_ranks x n_regions when rank_sum or rank_sumsq is
 * NULL) returns TA_ERR_SIZE_OVERFLOW before anything is launched.  Every call
 * on one GPU shares that array: calls that overlap in time on one GPU (on
 * different streams, handles or host threads) race and give undefined
 * results; calls ordered on one stream do not. */
#define TA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ta_status ta_imbalance_noalloc(ta_handle h, const int64_t *tensor, int64_t n_ranks,
                               int32_t n_iters, int32_t n_regions, const int32_t *iters_found,
                               const int64_t *rank_sum, const uint64_t *rank_sumsq,
                               const int64_t *span, int32_t ddof, double t_app_ns,
                               const ta_imbalance_out *o, void *stream);

/* Exact outlier scan (not in the paper, which clusters ranks, Sec. VI-B; this
 * is the textbook modified z-score).  Ranks with no iteration take no part and
 * score 0.
 *   TA_SCAN_FULL: per cell (i,g) a score over the ranks valid in i; m(r,g) =
 *     mean over the rank's iterations of its cell scores (summed in ascending
 *     i); then per region a second score over ranks of m(r,g).
 *   TA_SCAN_TOTALS: per region one score over ranks of the rank totals.
 *   TA_SCORE_MAD: robust z = (x - median) / (1.4826 * MAD); when MAD is 0,
 *     1.253314 * mean absolute deviation replaces 1.4826 * MAD; when that is
 *     0 too, z = 0.  Medians of an even count average the two middle values.
 *   TA_SCORE_Z: (x - mean) / std with ddof = 1 (0 when std is 0).
 * rank_score[r] = max_g |z2(r,g)|; rank_flag[r] = rank_score > tau;
 * n_flagged[0] = number of flags; region_score[r*G+g] = z2(r,g) (signed, may
 * be NULL).  All outputs are device pointers.
 * Cell values must lie in (-2^61, 2^61); n_iters * n_regions <= 4,194,240
 * (TA_ERR_SIZE_OVERFLOW otherwise).  The FULL scan's workspace is about as
 * large as the tensor: for the robust kind over columns of at least 32,768
 * padded ranks it holds a 32-bit copy of the tensor (half its size) and a
 * slot of 256 cells per column and chunk of 1,024 ranks for the bracket
 * interiors (a quarter of the tensor), plus the column samples and one
 * gathered column per selection workgroup; otherwise a column-major copy of
 * the tensor. */
enum { TA_SCAN_FULL = 0, TA_SCAN_TOTALS = 1 };
enum { TA_SCORE_MAD = 0, TA_SCORE_Z = 1 };
ta_status ta_outliers(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                      int32_t n_regions, const int32_t *iters_found, int32_t mode, int32_t kind,
                      double tau, double *rank_score, uint8_t *rank_flag, int64_t *n_flagged,
                      double *region_score, void *stream);

/* Sparse node x rank x iteration model (Sec. V: one profile per iteration,
 * indexed by calling-context node, trace and iteration; Thicket keeps
 * inclusive and exclusive costs per node).  Row q = r * n_iters + i is
 * iteration i of rank r, iterations as in ta_segment (entry into the subtree
 * of the marker given to ta_set_regions opens one; events before the first
 * boundary belong to no row).  Its entries:
 *   exclusive: (v, excl) for every node v with excl(r,i,v) != 0, where
 *     excl(r,i,v) = sum of d_k over rank r's events k of iteration i with
 *     context v (d_k = t_{k+1} - t_k, 0 for a rank's last event);
 *   inclusive: (v, incl) for every node with incl(r,i,v) != 0, where incl is
 *     the sum of excl over the subtree of v;
 * each list in the tree's preorder (a node before its descendants, children
 * and roots in ascending id).  Rows i >= iters_found[r] are empty.  Any tree
 * size up to 2^22 nodes.  Two calls on the same traces, n_iters and tables:
 * ta_node_model_count writes row_start[R * n_iters] (index in ts/ctx of the
 * event that opens row q, written for i < iters_found[r]), iters_found[R],
 * and row_off_x, row_off_i [R * n_iters + 1]: the number of exclusive
 * (inclusive) entries of the rows before q, so [R * n_iters] holds the
 * total.  The caller reads the totals to size the entry arrays, then
 * ta_node_model_fill writes row q's entries at [row_off_x[q], row_off_x[q+1])
 * of node_x (caller ids) / val_x, and at [row_off_i[q], row_off_i[q+1]) of
 * node_i / val_i; either pair may be NULL to skip that list.  All arrays are
 * device pointers.  Sticky device errors: context out of range, a timestamp
 * decreasing inside a row, inconsistent offsets, more than n_iters
 * boundaries in a rank (TA_ERR_ITER_OVERFLOW; iters_found is then n_iters).  TA_ERR_STATE without
 * ta_set_tree and ta_set_regions. */
ta_status ta_node_model_count(ta_handle h, const ta_traces *t, int32_t n_iters,
                              int64_t *row_start, int32_t *iters_found, int64_t *row_off_x,
                              int64_t *row_off_i, void *stream);
ta_status ta_node_model_fill(ta_handle h, const ta_traces *t, int32_t n_iters,
                             const int64_t *row_start, const int32_t *iters_found,
                             const int64_t *row_off_x, int32_t *node_x, int64_t *val_x,
                             const int64_t *row_off_i, int32_t *node_i, int64_t *val_i,
                             void *stream);

/* Node-level and physical localisation (Sec. VI-B: ranks are joined with their
 * compute node, nodes are mapped to rack and chassis coordinates).  For each
 * rack and each chassis: the number of flagged ranks placed there, their max
 * score and mean score (NaN where no rank is placed).  rank_node[R] indexes
 * node_rack[n_nodes] and node_chassis[n_nodes] (chassis numbered globally).
 * Device pointers; any of the six outputs may be NULL. */
ta_status ta_topology_aggregate(ta_handle h, const double *rank_score, const uint8_t *rank_flag,
                                int64_t n_ranks, const int32_t *rank_node,
                                const int32_t *node_rack, const int32_t *node_chassis,
                                int32_t n_nodes, int32_t n_racks, int32_t n_chassis,
                                int64_t *flagged_per_rack, double *max_per_rack,
                                double *mean_per_rack, int64_t *flagged_per_chassis,
                                double *max_per_chassis, double *mean_per_chassis,
                                void *stream);

/* Return a call-path: walks from `leaf` to its root over the tree given to
 * ta_set_tree (Sec. VI-B reconstructs the call chain of a leaf id bottom-up).
 * Writes up to `cap` node ids (leaf first) into path_host and the full length
 * into *len.  Host-only, synchronous. */
ta_status ta_callpath(ta_handle h, int32_t leaf, int32_t *path_host, int32_t cap, int32_t *len);

/* Summary profile (Sec. II-A: the aggregate of all per-rank profiles).
 * excl[n_ranks][N] holds per-rank exclusive costs in the caller's node
 * numbering (as written by ta_attribute).  sum_excl[v] = sum over ranks of
 * excl[r][v] (required); sum_incl[v] = sum of sum_excl over the subtree of v
 * in the tree given to ta_set_tree (optional, NULL to skip), which equals
 * the sum over ranks of the inclusive costs.  Exact int64 sums.  Any tree
 * size (N up to 4,194,304).  Device pointers. */
ta_status ta_summary(ta_handle h, const int64_t *excl, int64_t n_ranks, int64_t *sum_excl,
                     int64_t *sum_incl, void *stream);

/* Pruning (Sec. II-A: a strategy evaluated once on the summary profile and
 * applied to every rank; Sec. VI-B drops the nodes below 1% of the total
 * runtime).  Keeps node v iff (double)sum_incl[v] >= fraction * (double)total,
 * total = sum over v of sum_excl[v] (FP64, round to nearest).  Writes the kept
 * ids in ascending order to kept[0 .. *n_kept) (kept has room for N entries)
 * and their count to *n_kept (a DEVICE int32).  With non-negative costs the
 * inclusive cost never grows from a node to its child, so the kept set holds
 * the parent of each kept non-root node.  fraction >= 0 (NaN ->
 * TA_ERR_INVALID_ARG); fraction 0 keeps every node. */
ta_status ta_prune(ta_handle h, const int64_t *sum_excl, const int64_t *sum_incl, double fraction,
                   int32_t *kept, int32_t *n_kept, void *stream);

/* Installs a pruned tree: the kept node ids (HOST array, any order, distinct,
 * in [0, N)), copied during the call.  Needs ta_set_tree(); ta_set_tree()
 * drops it.  Waits for the device to go idle before replacing the previous
 * kept set. */
ta_status ta_set_pruned(ta_handle h, int32_t n_kept, const int32_t *kept_host);

/* Per-rank profiles on the pruned tree (Sec. II-A: the kept set is propagated
 * across the per-rank profiles).  For rank r and kept index k (the order given
 * to ta_set_pruned):
 *   p_excl[r][k] = sum of excl[r][u] over the nodes u whose nearest kept
 *                  ancestor-or-self is kept[k] (pruned descendants fold into
 *                  their nearest kept ancestor; nodes with no kept ancestor are
 *                  dropped),
 *   p_incl[r][k] = sum of excl[r][u] over the subtree of kept[k].
 * Either output may be NULL (not both, unless n_ranks is 0).  N at most 8192.
 * Device pointers. */
ta_status ta_pruned_profiles(ta_handle h, const int64_t *excl, int64_t n_ranks, int64_t *p_excl,
                             int64_t *p_incl, void *stream);

/* Inclusive form of a rank x iteration x region tensor (Sec. V: the node x
 * trace x iteration model; with the regions set to the kept nodes of a pruned
 * tree, ta_segment gives its exclusive form).  out[r][i][g] = sum of
 * tensor[r][i][h] over the regions h whose node lies in the subtree of region
 * g's node (region g included), for the regions of the last ta_set_regions().
 * tensor and out are [n_ranks][n_iters][G] device arrays; out may be tensor
 * itself (in place: each row is read whole before it is written) but must not
 * otherwise overlap it. */
ta_status ta_tensor_inclusive(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                              int64_t *out, void *stream);

/* Profile of a time window for any subset of ranks (Sec. II: a calling context
 * tree for a trace interval).  For the ranks rank_ids[0 .. n_sel) (DEVICE
 * int32; NULL = all t->n_ranks ranks in order; a rank listed twice counts
 * twice), every event's interval [t_k, t_{k+1}) (a rank's last event lasts 0)
 * is clipped to [t0, t1) and added to its context node: excl[N] (required);
 * incl[N] (optional) = the sum of excl over the subtree of each node.  The
 * nodes with a non-zero inclusive cost form the calling context tree of the
 * window.  Binary searches on each rank's timestamps bound the events read,
 * so a narrow window costs little.  Any tree size (N up to 4,194,304).  Data
 * errors (rank id out of range, decreasing timestamps, context out of range)
 * are detected for the events the window touches and reported by
 * ta_sync_status.  Needs ta_set_tree().  t1 >= t0.  Device pointers. */
ta_status ta_window_profile(ta_handle h, const ta_traces *t, const int32_t *rank_ids, int64_t n_sel,
                            int64_t t0, int64_t t1, int64_t *excl, int64_t *incl, void *stream);

/* Sparse per-rank profiles (Sec. I: stored densely, GPU profiles can be over
 * 1000x larger than sparsely; Sec. VI-B: 97,833 calling contexts).  For each
 * rank r, the nodes with a non-zero exclusive time (the sum of the durations
 * of r's events in that context) in ascending node id, at node_ids[off[r] + j]
 * and excl[off[r] + j] for j < counts[r]; counts[r] <= the rank's event count,
 * so each rank's entries fit in its own event range (entries after them are
 * left unwritten).  Any tree size (N up to 4,194,304): node ids are taken in
 * chunks of 8,192 (an LDS histogram each), one pass over a rank's events per
 * chunk its events reach.  counts[n_ranks], node_ids[n_events],
 * excl[n_events]: device pointers.  Needs ta_set_tree(). */
ta_status ta_sparse_profiles(ta_handle h, const ta_traces *t, int64_t *counts, int32_t *node_ids,
                             int64_t *excl, void *stream);

/* Clustering of ranks (Sec. VI-B: the ranks of one metric are clustered with
 * DBSCAN and the groups mapped to compute nodes; K-Means with 2..5 groups is
 * tested by the compute nodes whose ranks fall in two groups).
 *
 * K-Means (Lloyd) on integer feature rows X[n_rows][n_features] (e.g. the
 * per-rank region totals), from the centroids init[k][n_features] (FP64,
 * chosen by the caller).  An iteration assigns each row to the centroid with
 * the smallest squared distance, summed over the features in ascending order
 * with each product and sum rounded to FP64 (no fused multiply-add), ties to
 * the smaller index; each centroid then becomes (double)(exact int64 sum of
 * its rows) / count, and keeps its value when no row chose it.  Iterations stop
 * after the first one in which no row changes cluster, or after max_iter.
 * Outputs: labels[n_rows], centroids[k][n_features], counts[k] (optional),
 * *n_iter (optional, device int32: iterations run).  Feature sums must fit in
 * int64.  k <= 32, n_features <= 256, k * n_features <= 5632.  Device pointers;
 * the host queues max_iter iterations without waiting (the ones after the stop
 * return at once). */
ta_status ta_kmeans(ta_handle h, const int64_t *X, int64_t n_rows, int32_t n_features, int32_t k,
                    const double *init, int32_t max_iter, int32_t *labels, double *centroids,
                    int64_t *counts, int32_t *n_iter, void *stream);

/* DBSCAN on one integer feature per row (the metric's value per rank).  The
 * neighbours of row i are the rows j with |x[j] - x[i]| <= eps (i included); i
 * is a core row with at least min_pts neighbours.  Clusters are the connected
 * components of the core rows under the neighbour relation, numbered 0, 1, ...
 * by increasing value; a non-core row with a core neighbour joins the cluster
 * of its nearest core neighbour (the smaller number on a tie); other rows are
 * noise (-1).  Outputs labels[n_rows], *n_clusters (device int32), core[n_rows]
 * (optional, 1 for core rows).  Values and eps must keep x +- eps and the
 * differences of values inside int64.  Device pointers. */
ta_status ta_dbscan1d(ta_handle h, const int64_t *x, int64_t n_rows, int64_t eps, int64_t min_pts,
                      int32_t *labels, int32_t *n_clusters, uint8_t *core, void *stream);

/* Compute nodes shared by clusters: pair[a][b] (k x k, symmetric, zero
 * diagonal) = the number of compute nodes holding ranks of both cluster a and
 * cluster b; node_clusters[n] (optional) = the number of distinct clusters
 * among node n's ranks.  labels[n_ranks] in [-1, k) (-1 ignored),
 * rank_node[n_ranks] in [0, n_nodes); other values are a sticky device error
 * (TA_ERR_INVALID_ARG from ta_sync_status).  k <= 64.  Device pointers. */
ta_status ta_node_intersections(ta_handle h, const int32_t *labels, const int32_t *rank_node,
                                int64_t n_ranks, int32_t n_nodes, int32_t k, int64_t *pair,
                                int32_t *node_clusters, void *stream);

/* Batch plan: the whole batch in one HIP graph launch.
 * ta_plan_create orders the ranks longest first (so the longest traces start
 * first and the tail is short), picks the launch shape of the fused pass
 * (threads per workgroup, events per thread per tile, streaming loads, one
 * workgroup per rank or a persistent grid) and captures the fused pass --
 * optionally followed by the imbalance and outlier stages -- into a graph
 * over the buffers given here.
 *   autotune 0: the default shape (fused pass: 512 threads x 4 events per
 *   thread, one workgroup per rank; the eager calls use it too); 1: time
 *   every candidate shape on this
 *   batch (each produces identical results) and keep the fastest; 2: as 1, but
 *   reuse the choice stored in the JSON file named by the TA_AUTOTUNE_CACHE
 *   environment variable when it holds this batch shape (and store new ones).
 * offsets_host is a host copy of t->offsets.  The plan keeps its own
 * workspace; the traces and every output buffer must stay allocated while
 * the plan is used.  The graph also uses the handle's call-path and region
 * tables, so while any plan of the handle exists ta_set_tree,
 * ta_set_regions and ta_destroy return TA_ERR_STATE and change nothing:
 * destroy the plans first. */
typedef struct ta_plan_s *ta_plan;
typedef struct {
  int32_t n_iters;
  ta_seg_out seg;            /* outputs of the fused pass */
  int32_t with_imbalance;    /* nonzero: add ta_imbalance on seg's outputs */
  ta_imbalance_out imb;
  int32_t ddof;
  double t_app_ns;
  int32_t with_outliers;     /* nonzero: add ta_outliers on seg's tensor */
  int32_t outlier_mode, outlier_kind;
  double tau;
  double *rank_score;
  uint8_t *rank_flag;
  int64_t *n_flagged;
  double *region_score;
  int32_t autotune;
} ta_batch_desc;

ta_status ta_plan_create(ta_handle h, const ta_traces *t, const int64_t *offsets_host,
                         const ta_batch_desc *d, ta_plan *out, void *stream);
/* Replays the captured graph on `stream`. */
ta_status ta_plan_launch(ta_plan p, void *stream);
/* Replays the graph like ta_plan_launch, with the event record nodes that
 * sit right before and right after the fused pass in the graph pointed at
 * the plan's event pair number `slot` (0 <= slot < 4096; pairs are created on
 * first use), so each replay of a timed loop keeps its own pair and no host
 * synchronisation is needed between replays.  TA_ERR_STATE if the graph has
 * no timing nodes.  For the measurement of the fused pass inside the whole
 * step (what a one-kernel graph would not show). */
ta_status ta_plan_launch_timed(ta_plan p, int32_t slot, void *stream);
/* Milliseconds between the two events of `slot` (the fused pass of the
 * replay that used it, plus the record nodes' own latency); waits for that
 * replay to reach the second event. */
ta_status ta_plan_segment_ms(ta_plan p, int32_t slot, float *ms);
/* The chosen launch shape (threads per workgroup, events per thread per tile,
 * streaming loads, workgroups per CU of a persistent grid or 0) and its
 * measured time (ms; 0 when not tuned).  Any pointer may be NULL. */
ta_status ta_plan_info(ta_plan p, int32_t *threads, int32_t *events_per_thread,
                       int32_t *nontemporal, int32_t *wgs_per_cu, float *tuned_ms);
ta_status ta_plan_destroy(ta_plan p);

/* Mixed batch: many trace-analysis requests over one call-path tree and one
 * region list (the handle's), each with its own ranks, events and iteration
 * count, reduced by ONE persistent fused pass (a task per rank of every
 * request, longest first) followed by each request's exact FULL robust outlier
 * scan (modified z, Sec. VI-B stand-in as for ta_outliers), all captured in one
 * graph.  Per request: traces and a host copy of its offsets; seg.tensor and
 * seg.iters_found are required, the other seg outputs may be NULL; rank_score
 * and rank_flag (both or neither) ask for the outlier scan of that request
 * (n_flagged may be NULL).  Device data errors of any request set the handle's
 * sticky error word.  Launch, query and destroy with ta_plan_launch /
 * ta_plan_info / ta_plan_destroy; autotune as for ta_plan_create. */
typedef struct {
  ta_traces traces;
  const int64_t *offsets_host;
  int32_t n_iters;
  ta_seg_out seg;
  double *rank_score;
  uint8_t *rank_flag;
  int64_t *n_flagged;
} ta_request;

ta_status ta_batch_create(ta_handle h, int32_t n_requests, const ta_request *requests, double tau,
                          int32_t autotune, ta_plan *out, void *stream);

/* ---- Learned pre-screen -------------------------------------------------
 * Not part of the paper's method: a small autoencoder over per-rank iteration
 * profiles, 64 -> 128 -> 32 -> 128 -> 64 (ReLU on the hidden layers, linear
 * output, mean squared error, Adam with bias correction), bfloat16 weights and
 * activations on the matrix cores with FP32 accumulation and FP32 master
 * weights.  A profile row is x[r,i,g] = (T[r,i,g] - mu_g) / sigma_g over a
 * rank's valid iterations; mu, sigma are fitted on training tensors.  The rank
 * score is chosen by ta_ae_set_score_kind.  All need n_regions == 64.  The
 * state lives in the handle. */

/* Xavier-uniform weights from SplitMix64 draws of `seed`, zero biases and
 * optimiser moments, step 0. */
ta_status ta_ae_init(ta_handle h, uint64_t seed, void *stream);
/* Adds the valid cells of `tensor` to the running per-region sums (reset != 0
 * starts over) and refreshes mu and sigma (population standard deviation). */
ta_status ta_ae_fit_norm(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                         int32_t n_regions, const int32_t *iters_found, int32_t reset,
                         void *stream);
/* Writes the normalised profile rows of every valid (rank, iteration), rank by
 * rank, to rows[n][64] (device; may be NULL to count) and their number to
 * *n_rows_host.  Synchronises the stream. */
ta_status ta_ae_rows(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                     int32_t n_regions, const int32_t *iters_found, float *rows,
                     int64_t *n_rows_host, void *stream);
/* Gradient (grad[24928], layout W1 W2 W3 W4 b1 b2 b3 b4, row-major [out][in])
 * and mean loss (loss[1]) over rows[0..n_rows) without updating anything.
 * input_noise > 0 gives the denoising gradient: the network sees
 * x[j][c] + input_noise * N_key(j, c) and is scored against x[j][c], where
 * N_key(j, c) is the standard normal draw for row j and feature c under
 * noise_key: base = M(key ^ M(64 j + c)), z1 = M(base),
 * z2 = M(base ^ 0xD1B54A32D192ED03), u1 = ((z1 >> 40) + 1/2) / 2^24,
 * u2 = (z2 >> 40) / 2^24, N = sqrt(-2 ln u1) cos(2 pi u2) (FP32), with M the
 * SplitMix64 finaliser of the initialiser. */
ta_status ta_ae_grad(ta_handle h, const float *rows, int64_t n_rows, float input_noise,
                     uint64_t noise_key, float *grad, float *loss, void *stream);
/* The same gradient and loss as ta_ae_grad with every operation in FP32 (no
 * bfloat16 rounding of the matrix-product operands): a debug reference for
 * the matrix-core training path (single threads per dot product; slow). */
ta_status ta_ae_grad_f32(ta_handle h, const float *rows, int64_t n_rows, float input_noise,
                         uint64_t noise_key, float *grad, float *loss, void *stream);
/* `epochs` passes over the rows in batches of `batch` (a fresh permutation of
 * the rows per epoch, drawn from shuffle_seed), one Adam step (learning rate
 * lr) per batch; with input_noise > 0 every step is a denoising step with its
 * own noise key (drawn from shuffle_seed); epoch_loss[e] (device, may be NULL)
 * is the row-weighted mean batch loss of epoch e. */
ta_status ta_ae_train(ta_handle h, const float *rows, int64_t n_rows, int32_t epochs, int32_t batch,
                      float lr, float input_noise, uint64_t shuffle_seed, float *epoch_loss,
                      void *stream);
/* Score used by ta_ae_score / ta_prescreen: TA_AE_SCORE_ERROR (default) =
 * max_g mean_i (y - x)^2, the reconstruction error; TA_AE_SCORE_RESIDUAL =
 * max_g |mean_i (y - x)|, a region's persistent residual over the rank's
 * iterations; TA_AE_SCORE_RESIDUAL_Z = max_g |z(r,g)| where z is the robust
 * z-score over ranks (median, 1.4826 * MAD, mean-absolute-deviation fallback:
 * the exact scan's second stage) of m(r,g) = mean_i (y - x) -- the network's
 * residual takes the place of the exact scan's per-cell first stage.  Saved
 * with the network state. */
enum { TA_AE_SCORE_ERROR = 0, TA_AE_SCORE_RESIDUAL = 1, TA_AE_SCORE_RESIDUAL_Z = 2 };
ta_status ta_ae_set_score_kind(ta_handle h, int32_t kind);
/* The score kind in use (host int32). */
ta_status ta_ae_get_score_kind(ta_handle h, int32_t *kind_host);
/* rank_score[r] (device FP32) for every rank; ranks without iterations score 0. */
ta_status ta_ae_score(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                      int32_t n_regions, const int32_t *iters_found, float *rank_score,
                      void *stream);
/* Sets the fallback threshold to the given quantile of rank_score (device);
 * synchronises. */
ta_status ta_ae_calibrate(ta_handle h, const float *rank_score, int64_t n_ranks, double quantile,
                          void *stream);
/* The fallback threshold in use (host float; negative when none is set). */
ta_status ta_ae_get_threshold(ta_handle h, float *threshold_host);
/* Pre-screen: topk_ranks[k] (device) = the k ranks with the largest scores
 * (ties toward the lower rank id), in ascending rank id.  Fallback to the exact
 * scan (TA_SCAN_FULL, TA_SCORE_MAD) -- the k ranks with the largest exact
 * scores -- when the network is not initialised or fitted, or when more than k
 * ranks exceed the calibrated threshold; *used_fallback_host says which ran.
 * rank_score (device FP32, may be NULL) receives the network's scores.
 * Synchronises the stream once (to decide on the fallback). */
ta_status ta_prescreen(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                       int32_t n_regions, const int32_t *iters_found, int64_t k,
                       int32_t *topk_ranks, float *rank_score, int32_t *used_fallback_host,
                       void *stream);
/* Checkpoint of the network (weights, optimiser moments and step,
 * normalisation, threshold) to / from a host buffer of ta_ae_state_bytes(). */
size_t ta_ae_state_bytes(void);
ta_status ta_ae_get_state(ta_handle h, void *buf_host, size_t bytes);
ta_status ta_ae_set_state(ta_handle h, const void *buf_host, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* TA_H_ */
