// k_nodemodel.hip -- the sparse node x rank x iteration model (Sec. V: one
// profile per iteration, indexed by calling-context node, trace and iteration,
// with exclusive and inclusive costs per node).
//
// Row q = r * I + i is iteration i of rank r.  Its exclusive entries are the
// nodes whose events of that iteration add up to a non-zero time; its
// inclusive entries are those nodes and all their ancestors (with non-negative
// durations a node has a non-zero inclusive cost exactly when some node of its
// subtree has a non-zero exclusive cost).  Both lists are in preorder.
//
// Pass 1 (`nm_rows`): one wave per rank finds the boundary events (entry into
//   the marker's subtree) and writes the first event of every row.
// Pass 2 (`nm_short<FILL, ...>`): one wave per row of at most SHORT_CAP events
//   (one kernel for rows of up to 64 events with the tree and the position map
//   staged in LDS, one for 65..SHORT_CAP events with the LDS radix sort and
//   the tree read through L2); all of a row's events are loaded at once.  The
//   events with a positive duration are sorted by the preorder position of
//   their node (a 64-lane bitonic network in registers up to 64 events, else an
//   LSD radix sort with 8-bit digits in the wave's LDS), equal positions are
//   merged into (position, exclusive cost) with a running sum Q of the sorted
//   durations, so a node's cost is a difference of Q.  Inclusive entries: for
//   unique nodes u_0 < u_1 < ... (preorder), the ancestors of u_j that are not
//   ancestors of u_{j-1} lie strictly between u_{j-1} and u_j in preorder, so
//   lane j walks up from u_j until it reaches an ancestor of u_{j-1}; the walks
//   cover every inclusive node once, already in preorder after a prefix sum of
//   their lengths; the inclusive cost of a visited node a is Q over the unique
//   nodes inside [a, tout(a)), whose first one is u_j itself.
// Pass 3 (`nm_long<FILL>`): one workgroup per longer row (listed by pass 2):
//   a dense histogram over preorder positions plus bit masks of the touched
//   positions; each touched node adds its cost to all its ancestors; the masks
//   are enumerated in position order by a scan of their population counts.
//   Histograms in LDS up to LONG_LDS_NODES nodes, else in the workspace.
// The count run writes the entry counts, which an exclusive scan turns into
// row offsets; the fill run writes the entries.  Integer sums throughout, so
// the result does not depend on the order of any atomic.
#include <mutex>

#include "ta_internal.h"

namespace ta {
namespace {

constexpr int NMT = 256;            // threads per workgroup of the wave kernels
constexpr int NMW = NMT / 64;       // waves per workgroup
constexpr int SHORT_CAP = 512;      // events per row handled by one wave
constexpr int SLOT_BITS = 9;        // log2(SHORT_CAP): sort keys are pos << 9 | slot
constexpr int LONG_T = 512;         // threads per workgroup of the long-row kernel
constexpr int LONG_LDS_NODES = 4096;
constexpr int SMALL_TAB_NODES = 8192; // the <= 64-event row kernel keeps the tree in LDS up to here
constexpr int SCAN_T = 1024;
constexpr int SCAN_EPT = 8;
constexpr int SCAN_B = SCAN_T * SCAN_EPT;

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

__device__ inline int wave_excl_scan_i32(int v, int *total) {
  const int lane = lane_id();
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(x, d, 64);
    if (lane >= d) x += t;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

__device__ inline int64_t wave_incl_scan_i64(int64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ inline uint64_t lanemask_lt() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// A rank's event range, clamped to [0, E]; inconsistent offsets are an error
// and the rank is then taken as empty.
__device__ inline void rank_range(const int64_t *off, int64_t r, int64_t E, int64_t *b,
                                  int64_t *e, uint32_t *err) {
  const int64_t o0 = off[r], o1 = off[r + 1];
  const bool bad = o0 < 0 || o1 < o0 || o1 > E;
  if (bad && lane_id() == 0) atomicOr(err, ERRBIT_OFFSETS);
  *b = bad ? 0 : o0;
  *e = bad ? 0 : o1;
}

// ---- pass 1: row boundaries ---------------------------------------------------

// One wave per rank; each lane takes 4 consecutive events per step (16-byte
// context loads from 4-aligned indices), 4 steps in flight.  An event opens a
// row when its node lies in the marker's subtree and the rank's previous event
// does not (the rank's first event counts as following an event outside).
__global__ __launch_bounds__(NMT) void nm_rows(const int64_t *__restrict__ off,
                                               const int32_t *__restrict__ ctx, int64_t R,
                                               int64_t E, int I, const uint32_t *__restrict__ info,
                                               int N, int64_t *__restrict__ row_start,
                                               int32_t *__restrict__ iters_found, uint32_t *err) {
  constexpr int U = 4;
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * NMW;
  uint32_t errb = 0;
  for (int64_t r = (int64_t)blockIdx.x * NMW + (threadIdx.x >> 6); r < R; r += nwaves) {
    int64_t b, e;
    rank_range(off, r, E, &b, &e, err);
    int64_t found = 0;   // boundaries seen so far
    int carry = 0;       // previous event lies in the marker subtree
    for (int64_t k0 = b & ~(int64_t)3; k0 < e; k0 += 256 * U) {
      int32_t c[U][4];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int64_t kb = k0 + 256 * u + 4 * lane;
        if (kb + 4 <= E && kb < e) {
          const v4i q = *reinterpret_cast<const v4i *>(ctx + kb);
          c[u][0] = q.x;
          c[u][1] = q.y;
          c[u][2] = q.z;
          c[u][3] = q.w;
        } else {
#pragma unroll
          for (int j = 0; j < 4; j++) c[u][j] = (kb + j < e && kb + j < E) ? ctx[kb + j] : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int64_t kb = k0 + 256 * u + 4 * lane;
        uint32_t inm = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int64_t k = kb + j;
          if (k >= b && k < e) {
            const int32_t cc = c[u][j];
            if ((uint32_t)cc < (uint32_t)N) inm |= ((info[cc] & INFO_MARKER_BIT) ? 1u : 0u) << j;
            else errb |= ERRBIT_CTX;
          }
        }
        // membership of the event before my first one
        int pin = __shfl_up((int)(inm >> 3), 1, 64);
        if (lane == 0) pin = carry;
        const uint32_t prev = ((inm << 1) | (uint32_t)pin) & 0xfu;
        const uint32_t bnd = inm & ~prev;
        int tot;
        const int before = wave_excl_scan_i32(__popc(bnd), &tot);
        int64_t idx = found + before;
#pragma unroll
        for (int j = 0; j < 4; j++)
          if ((bnd >> j) & 1u) {
            if (idx < I) row_start[r * (int64_t)I + idx] = kb + j;
            else errb |= ERRBIT_OVERFLOW;
            idx++;
          }
        found += tot;
        carry = __shfl((int)(inm >> 3), 63, 64);
      }
    }
    if (lane == 0) iters_found[r] = (int32_t)(found < I ? found : I);
  }
  if (errb) atomicOr(err, errb);
}

// ---- pass 2: one wave per short row ---------------------------------------------

struct NmArgs {
  const int64_t *off, *ts;
  const int32_t *ctx;
  int64_t R, E;
  int I, N;
  int pos_bits;               // bits of the largest preorder position
  const uint32_t *info;       // [N] packed node word (preorder position in bits 10..)
  const int4 *ptab;           // [N] by position: caller id, parent position, subtree end
  const int64_t *row_start;   // [R*I]
  const int32_t *iters_found; // [R]
  int64_t *cnt_x, *cnt_i;     // count run: [R*I] entry counts
  const int64_t *off_x, *off_i;  // fill run: [R*I + 1] row offsets
  int32_t *node_x, *node_i;
  int64_t *val_x, *val_i;
  int64_t *long_rows;         // rows of more than SHORT_CAP events
  int64_t *n_long;            // [1]
  int64_t long_cap;
  int64_t *long_ws;           // long kernel: per-workgroup histograms (large trees)
  uint32_t *err;
};

// Row q's event range [s, e) and the end of its rank (for the last duration);
// false for an empty row (iteration past the rank's count).
__device__ inline bool row_range(const NmArgs &a, int64_t q, int64_t *s, int64_t *e,
                                 int64_t *re) {
  const int64_t r = q / a.I;
  const int i = (int)(q - r * a.I);
  int nit = a.iters_found[r];
  nit = nit < a.I ? nit : a.I;
  if (i >= nit) return false;
  const int64_t o0 = a.off[r], o1 = a.off[r + 1];
  if (o0 < 0 || o1 < o0 || o1 > a.E) return false;  // reported by the rows pass
  int64_t s0 = a.row_start[q];
  int64_t e0 = i + 1 < nit ? a.row_start[q + 1] : o1;
  s0 = s0 < o0 ? o0 : (s0 > o1 ? o1 : s0);
  e0 = e0 < s0 ? s0 : (e0 > o1 ? o1 : e0);
  *s = s0;
  *e = e0;
  *re = o1;
  return true;
}

template <int CAP>
struct WaveLds {
  uint32_t ka[CAP];      // sort keys (pos << SLOT_BITS | slot), then positions of the unique nodes
  uint32_t kb[CAP];
  int64_t d[CAP];        // duration by slot
  int64_t q[CAP + 1];    // running sum of the sorted durations before each unique node
  uint32_t hist[CAP > 64 ? 256 : 1];
};

// The tree by preorder position for the walks: (parent position + 1, subtree
// end) from an LDS copy (small trees) or from the global table.
template <bool LDS_TAB>
struct TreeTab {
  const uint2 *lds;
  const int4 *glb;
  __device__ __forceinline__ void at(int32_t x, int32_t &parent, int32_t &tout) const {
    if (LDS_TAB) {
      const uint2 t = lds[x];
      parent = (int32_t)t.x - 1;
      tout = (int32_t)t.y;
    } else {
      const int4 t = glb[x];
      parent = t.y;
      tout = t.z;
    }
  }
};

// Sorts keys[0 .. n) (distinct) ascending by bits [SLOT_BITS, SLOT_BITS + nbits)
// with LSD passes of 8-bit digits; returns the buffer that holds the result.
__device__ inline uint32_t *wave_radix_sort(uint32_t *src, uint32_t *dst, uint32_t *hist, int n,
                                            int nbits) {
  const int lane = lane_id();
  for (int sh = SLOT_BITS; sh < SLOT_BITS + nbits; sh += 8) {
    const int w = SLOT_BITS + nbits - sh < 8 ? SLOT_BITS + nbits - sh : 8;
    const uint32_t dm = (1u << w) - 1u;
    for (int j = lane; j < 256; j += 64) hist[j] = 0;
    __builtin_amdgcn_wave_barrier();
    // digit counts; the lowest lane of each group of equal digits adds the group
    for (int c0 = 0; c0 < n; c0 += 64) {
      const bool act = c0 + lane < n;
      const uint32_t dg = act ? (src[c0 + lane] >> sh) & dm : 0u;
      uint64_t peers = __ballot(act);
      for (int bit = 0; bit < w; bit++) {
        const uint64_t m = __ballot(act && ((dg >> bit) & 1u));
        peers &= ((dg >> bit) & 1u) ? m : ~m;
      }
      if (act && (peers & lanemask_lt()) == 0) hist[dg] += (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    // exclusive scan of the 256 counts, 4 per lane
    uint32_t h[4];
    uint32_t own = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      h[u] = hist[4 * lane + u];
      own += h[u];
    }
    int tot;
    uint32_t run = (uint32_t)wave_excl_scan_i32((int)own, &tot);
#pragma unroll
    for (int u = 0; u < 4; u++) {
      hist[4 * lane + u] = run;
      run += h[u];
    }
    __builtin_amdgcn_wave_barrier();
    // stable scatter
    for (int c0 = 0; c0 < n; c0 += 64) {
      const bool act = c0 + lane < n;
      const uint32_t key = act ? src[c0 + lane] : 0u;
      const uint32_t dg = (key >> sh) & dm;
      uint64_t peers = __ballot(act);
      for (int bit = 0; bit < w; bit++) {
        const uint64_t m = __ballot(act && ((dg >> bit) & 1u));
        peers &= ((dg >> bit) & 1u) ? m : ~m;
      }
      const uint32_t base = act ? hist[dg] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (act) dst[base + (uint32_t)__popcll(peers & lanemask_lt())] = key;
      if (act && (peers & lanemask_lt()) == 0) hist[dg] = base + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    uint32_t *t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// 64 keys, one per lane, sorted ascending across the wave (bitonic network).
__device__ inline uint32_t wave_bitonic_sort(uint32_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t other = (uint32_t)__shfl_xor((int)key, j, 64);
      const bool up = (lane & k) == 0;
      const bool low = (lane & j) == 0;
      const uint32_t mn = key < other ? key : other;
      const uint32_t mx = key < other ? other : key;
      key = (low == up) ? mn : mx;
    }
  }
  return key;
}

// Smallest index j in [lo, hi) with pos[j] >= x, or hi.
__device__ inline int lower_bound_u32(const uint32_t *pos, int lo, int hi, uint32_t x) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pos[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One wave per row of LO < n <= CAP events (n = the row's event count); with
// CAP = SHORT_CAP the rows above it are listed for the long-row kernel, and
// with LO = 0 the empty rows' counts are written.  NT threads per workgroup;
// LDS_TAB: the walks read the tree from an LDS copy (dynamic LDS, 8 B a node).
template <bool FILL, int CAP, int LO, int NT, bool LDS_TAB, bool POS_LDS>
__global__ __launch_bounds__(NT) void nm_short(NmArgs a) {
  constexpr int NW = NT / 64;
  __shared__ WaveLds<CAP> lds_all[NW];
  extern __shared__ uint2 tab_lds[];
  WaveLds<CAP> &L = lds_all[threadIdx.x >> 6];
  TreeTab<LDS_TAB> tree{tab_lds, a.ptab};
  // POS_LDS: the preorder position of every caller id, after the tree table
  uint32_t *pos_lds = reinterpret_cast<uint32_t *>(tab_lds + (LDS_TAB ? a.N : 0));
  if (LDS_TAB) {
    for (int p = threadIdx.x; p < a.N; p += NT) {
      const int4 t = a.ptab[p];
      tab_lds[p] = make_uint2((uint32_t)(t.y + 1), (uint32_t)t.z);
    }
  }
  if (POS_LDS)
    for (int v = threadIdx.x; v < a.N; v += NT) pos_lds[v] = a.info[v] >> INFO_TIN_SHIFT;
  if (LDS_TAB || POS_LDS) __syncthreads();
  const int lane = lane_id();
  const int64_t rows = a.R * (int64_t)a.I;
  const int64_t nwaves = (int64_t)gridDim.x * NW;
  uint32_t errb = 0;
  for (int64_t q = (int64_t)blockIdx.x * NW + (threadIdx.x >> 6); q < rows; q += nwaves) {
    int64_t s = 0, e = 0, re = 0;
    if (!row_range(a, q, &s, &e, &re)) {
      if (LO == 0 && !FILL && lane == 0) {
        a.cnt_x[q] = 0;
        a.cnt_i[q] = 0;
      }
      continue;
    }
    const int64_t n = e - s;
    if (n <= LO) continue;
    if (n > CAP) {
      if (CAP == SHORT_CAP && lane == 0) {
        const int64_t j = (int64_t)atomicAdd((unsigned long long *)a.n_long, 1ull);
        if (j < a.long_cap) a.long_rows[j] = q;
      }
      continue;
    }
    // events with a positive duration -> (key, duration by slot).  All of the
    // row's timestamps and contexts are loaded first (CAP / 64 chunks, one
    // event per lane each); an event's next timestamp comes from the next
    // lane (or chunk), the row's last event takes the next row's first
    // timestamp, and a rank's last event lasts 0.
    constexpr int NCH = CAP / 64;
    int64_t tv[NCH];
    int32_t cv[NCH];
#pragma unroll
    for (int j = 0; j < NCH; j++) {
      const bool in = 64 * j + lane < n;
      tv[j] = in ? a.ts[s + 64 * j + lane] : 0;
      cv[j] = in ? a.ctx[s + 64 * j + lane] : 0;
    }
    const int64_t tail = e < re ? a.ts[e] : 0;
    int m = 0;
#pragma unroll
    for (int j = 0; j < NCH; j++) {
      if (64 * j >= n) break;
      const int i = 64 * j + lane;
      int64_t nx = __shfl_down(tv[j], 1, 64);
      const int64_t nc = j + 1 < NCH ? __shfl(tv[j + 1 < NCH ? j + 1 : j], 0, 64) : 0;
      if (lane == 63) nx = nc;
      bool keep = false;
      uint32_t pos = 0;
      int64_t d = 0;
      if (i < n) {
        d = i + 1 < n ? nx - tv[j] : (e < re ? tail - tv[j] : 0);
        if (d < 0) errb |= ERRBIT_UNSORTED;
        const int32_t c = cv[j];
        if ((uint32_t)c < (uint32_t)a.N) {
          pos = POS_LDS ? pos_lds[c] : a.info[c] >> INFO_TIN_SHIFT;
          keep = d > 0;
        } else {
          errb |= ERRBIT_CTX;
        }
      }
      const uint64_t km = __ballot(keep);
      const int slot = m + __popcll(km & lanemask_lt());
      if (keep) {
        const uint32_t key = (pos << SLOT_BITS) | (uint32_t)slot;
        L.ka[slot] = key;
        L.d[slot] = d;
      }
      m += __popcll(km);
    }
    int nu = 0;          // unique nodes
    const uint32_t *ups = L.kb;  // their positions
    if (m <= 64) {
      // the compacted keys, one per lane: sort in registers, merge equal
      // positions by ballot
      __builtin_amdgcn_wave_barrier();
      const uint32_t key = wave_bitonic_sort(lane < m ? L.ka[lane] : 0xffffffffu);
      const bool act = lane < m;
      const uint32_t pos = key >> SLOT_BITS;
      const int64_t d = act ? L.d[key & ((1u << SLOT_BITS) - 1)] : 0;
      const int64_t run = wave_incl_scan_i64(d);
      const uint32_t ppos = (uint32_t)__shfl_up((int)pos, 1, 64);
      const bool head = act && (lane == 0 || ppos != pos);
      const uint64_t hm = __ballot(head);
      const int u = __popcll(hm & lanemask_lt());
      __builtin_amdgcn_wave_barrier();
      if (head) {
        L.kb[u] = pos;
        L.q[u] = run - d;
      }
      nu = __popcll(hm);
      const int64_t total = __shfl(run, 63, 64);
      if (lane == 0) L.q[nu] = total;
      ups = L.kb;
    } else if constexpr (CAP > 64) {
      uint32_t *sorted = wave_radix_sort(L.ka, L.kb, L.hist, m, a.pos_bits);
      uint32_t *upos = sorted == L.ka ? L.kb : L.ka;
      int64_t carry = 0;
      uint32_t cpos = 0xffffffffu;
      for (int c0 = 0; c0 < m; c0 += 64) {
        const bool act = c0 + lane < m;
        const uint32_t key = act ? sorted[c0 + lane] : 0xffffffffu;
        const uint32_t pos = key >> SLOT_BITS;
        const int64_t d = act ? L.d[key & ((1u << SLOT_BITS) - 1)] : 0;
        const int64_t run = carry + wave_incl_scan_i64(d);
        uint32_t ppos = (uint32_t)__shfl_up((int)pos, 1, 64);
        if (lane == 0) ppos = cpos;
        const bool head = act && ppos != pos;
        const uint64_t hm = __ballot(head);
        const int u = nu + __popcll(hm & lanemask_lt());
        if (head) {
          upos[u] = pos;
          L.q[u] = run - d;
        }
        nu += __popcll(hm);
        carry = __shfl(run, 63, 64);
        cpos = (uint32_t)__shfl((int)pos, 63, 64);
      }
      if (lane == 0) L.q[nu] = carry;
      ups = upos;
    }
    __builtin_amdgcn_wave_barrier();
    // exclusive entries and the walks up the tree
    const int64_t ox = FILL ? a.off_x[q] : 0;
    const int64_t oi = FILL ? a.off_i[q] : 0;
    int64_t n_incl = 0;
    for (int c0 = 0; c0 < nu; c0 += 64) {
      const int u = c0 + lane;
      const bool act = u < nu;
      int len = 0;
      int32_t pu = -1;
      if (act) {
        pu = (int32_t)ups[u];
        const int32_t prev = u > 0 ? (int32_t)ups[u - 1] : -1;
        int32_t x = pu;
        while (x >= 0) {
          int32_t par, tz;
          tree.at(x, par, tz);
          if (prev >= 0 && x <= prev && prev < tz) break;  // x is an ancestor of prev
          len++;
          x = par;
        }
      }
      int tot;
      const int before = wave_excl_scan_i32(len, &tot);
      if (FILL && act) {
        const int64_t qu = L.q[u];
        if (a.node_x) {
          a.node_x[ox + u] = a.ptab[pu].x;
          a.val_x[ox + u] = L.q[u + 1] - qu;
        }
        if (a.node_i) {
          int32_t x = pu;
          for (int t = 0; t < len; t++) {
            int32_t par, tz;
            tree.at(x, par, tz);
            const int j = lower_bound_u32(ups, u, nu, (uint32_t)tz);
            const int64_t at = oi + n_incl + before + (len - 1 - t);
            a.node_i[at] = a.ptab[x].x;
            a.val_i[at] = L.q[j] - qu;
            x = par;
          }
        }
      }
      n_incl += tot;
    }
    if (!FILL && lane == 0) {
      a.cnt_x[q] = nu;
      a.cnt_i[q] = n_incl;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (errb) atomicOr(a.err, errb);
}

// ---- pass 3: one workgroup per long row -------------------------------------------

__device__ inline int block_excl_scan(int v, int *wsum, int *total) {
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  int t;
  const int ex = wave_excl_scan_i32(v, &t);
  if (lane == 63) wsum[wid] = ex + v;
  __syncthreads();
  int base = 0, all = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
    const int sw = wsum[w];
    base += w < wid ? sw : 0;
    all += sw;
  }
  __syncthreads();
  *total = all;
  return base + ex;
}

// Histograms hx (exclusive) and hi (inclusive) over positions, masks mx and mi
// of the positions touched; all zero between rows.
template <bool FILL>
__device__ inline void long_row(const NmArgs &a, int64_t q, int64_t *hx, int64_t *hi, uint32_t *mx,
                                uint32_t *mi, int *wsum, uint32_t &errb) {
  int64_t s = 0, e = 0, re = 0;
  row_range(a, q, &s, &e, &re);
  const int tid = threadIdx.x;
  for (int64_t k = s + tid; k < e; k += LONG_T) {
    const int64_t t0 = a.ts[k];
    const int64_t t1 = k + 1 < re ? a.ts[k + 1] : t0;
    const int64_t d = t1 - t0;
    if (d < 0) errb |= ERRBIT_UNSORTED;
    const int32_t c = a.ctx[k];
    if ((uint32_t)c >= (uint32_t)a.N) {
      errb |= ERRBIT_CTX;
    } else if (d > 0) {
      const uint32_t p = a.info[c] >> INFO_TIN_SHIFT;
      atomicAdd((unsigned long long *)&hx[p], (unsigned long long)d);
      atomicOr(&mx[p >> 5], 1u << (p & 31));
    }
  }
  __threadfence_block();
  __syncthreads();
  const int nw = (a.N + 31) >> 5;
  // every touched node adds its exclusive cost to itself and all its ancestors
  for (int w = tid; w < nw; w += LONG_T) {
    uint32_t bits = __hip_atomic_load(&mx[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (bits) {
      const int p = 32 * w + (__ffs(bits) - 1);
      bits &= bits - 1;
      const int64_t v = __hip_atomic_load(&hx[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int32_t x = p; x >= 0; x = a.ptab[x].y) {
        atomicAdd((unsigned long long *)&hi[x], (unsigned long long)v);
        atomicOr(&mi[x >> 5], 1u << (x & 31));
      }
    }
  }
  __threadfence_block();
  __syncthreads();
  // enumerate both masks in position order: thread t owns words [t*wpt, (t+1)*wpt)
  const int wpt = (nw + LONG_T - 1) / LONG_T;
  int own_x = 0, own_i = 0;
  for (int u = 0; u < wpt; u++) {
    const int w = tid * wpt + u;
    if (w < nw) {
      own_x += __popc(__hip_atomic_load(&mx[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      own_i += __popc(__hip_atomic_load(&mi[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
  }
  int tot_x, tot_i;
  int at_x = block_excl_scan(own_x, wsum, &tot_x);
  int at_i = block_excl_scan(own_i, wsum, &tot_i);
  const int64_t ox = FILL ? a.off_x[q] : 0;
  const int64_t oi = FILL ? a.off_i[q] : 0;
  for (int u = 0; u < wpt; u++) {
    const int w = tid * wpt + u;
    if (w >= nw) break;
    uint32_t bx = __hip_atomic_load(&mx[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t bi = __hip_atomic_load(&mi[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&mx[w], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&mi[w], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (bx) {
      const int p = 32 * w + (__ffs(bx) - 1);
      bx &= bx - 1;
      if (FILL && a.node_x) {
        a.node_x[ox + at_x] = a.ptab[p].x;
        a.val_x[ox + at_x] = __hip_atomic_load(&hx[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_store(&hx[p], (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      at_x++;
    }
    while (bi) {
      const int p = 32 * w + (__ffs(bi) - 1);
      bi &= bi - 1;
      if (FILL && a.node_i) {
        a.node_i[oi + at_i] = a.ptab[p].x;
        a.val_i[oi + at_i] = __hip_atomic_load(&hi[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_store(&hi[p], (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      at_i++;
    }
  }
  if (!FILL && tid == 0) {
    a.cnt_x[q] = tot_x;
    a.cnt_i[q] = tot_i;
  }
  __threadfence_block();
  __syncthreads();
}

template <bool FILL, bool IN_LDS>
__global__ __launch_bounds__(LONG_T) void nm_long(NmArgs a) {
  __shared__ int wsum[LONG_T / 64];
  extern __shared__ int64_t dyn[];
  const int nw = (a.N + 31) >> 5;
  int64_t *hx, *hi;
  uint32_t *mx, *mi;
  if (IN_LDS) {
    hx = dyn;
    hi = dyn + a.N;
    mx = reinterpret_cast<uint32_t *>(dyn + 2 * (int64_t)a.N);
    mi = mx + nw;
    for (int j = threadIdx.x; j < a.N; j += LONG_T) {
      hx[j] = 0;
      hi[j] = 0;
    }
    for (int j = threadIdx.x; j < nw; j += LONG_T) {
      mx[j] = 0;
      mi[j] = 0;
    }
    __syncthreads();
  } else {
    // this workgroup's slice of the workspace (zeroed before the launch and
    // left zero by every row)
    const int64_t per = 2 * (int64_t)a.N + nw + 1;
    hx = a.long_ws + (int64_t)blockIdx.x * per;
    hi = hx + a.N;
    mx = reinterpret_cast<uint32_t *>(hi + a.N);
    mi = mx + nw;
  }
  int64_t nl = *a.n_long;
  nl = nl < a.long_cap ? nl : a.long_cap;
  uint32_t errb = 0;
  for (int64_t j = blockIdx.x; j < nl; j += gridDim.x)
    long_row<FILL>(a, a.long_rows[j], hx, hi, mx, mi, wsum, errb);
  if (errb) atomicOr(a.err, errb);
}

__global__ void nm_zero(int64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---- exclusive scan of the entry counts -----------------------------------------

// Block sums of SCAN_B consecutive counts.
__global__ __launch_bounds__(SCAN_T) void scan_sums(const int64_t *__restrict__ x, int64_t n,
                                                    int64_t *__restrict__ bs) {
  __shared__ int64_t buf[SCAN_T / 64];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_B;
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < SCAN_EPT; u++) {
    const int64_t k = b0 + (int64_t)u * SCAN_T + threadIdx.x;
    s += k < n ? x[k] : 0;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane_id() == 0) buf[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < SCAN_T / 64; w++) t += buf[w];
    bs[blockIdx.x] = t;
  }
}

// Exclusive scan of the block sums in place (one workgroup); bs[nb] = total.
__global__ __launch_bounds__(SCAN_T) void scan_top(int64_t *bs, int64_t nb) {
  __shared__ int64_t wsum[SCAN_T / 64];
  int64_t carry = 0;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < nb; c0 += SCAN_T) {
    const int64_t k = c0 + threadIdx.x;
    const int64_t v = k < nb ? bs[k] : 0;
    const int64_t inc = wave_incl_scan_i64(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int64_t base = 0, all = 0;
    for (int w = 0; w < SCAN_T / 64; w++) {
      base += w < wid ? wsum[w] : 0;
      all += wsum[w];
    }
    if (k < nb) bs[k] = carry + base + inc - v;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) bs[nb] = carry;
}

// out[k] = bs[block] + exclusive prefix of x within the block (out may be x);
// the thread after the last element writes the grand total.
__global__ __launch_bounds__(SCAN_T) void scan_apply(const int64_t *x, int64_t n,
                                                     const int64_t *__restrict__ bs, int64_t nb,
                                                     int64_t *out) {
  __shared__ int64_t wsum[SCAN_T / 64];
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_EPT;
  int64_t v[SCAN_EPT];
  int64_t own = 0;
#pragma unroll
  for (int u = 0; u < SCAN_EPT; u++) {
    v[u] = b0 + u < n ? x[b0 + u] : 0;
    own += v[u];
  }
  const int64_t inc = wave_incl_scan_i64(own);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t base = bs[blockIdx.x];
  for (int w = 0; w < wid; w++) base += wsum[w];
  int64_t run = base + inc - own;
#pragma unroll
  for (int u = 0; u < SCAN_EPT; u++) {
    if (b0 + u < n) out[b0 + u] = run;
    run += v[u];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bs[nb];
}

// Raises a kernel's dynamic LDS limit to what the CU holds beside its static
// LDS (needed above 64 KB).
template <class K>
void allow_dynamic_lds(K k, size_t static_bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(160 * 1024 - static_bytes));
}

int grid_for(int64_t units, int cus, int per_cu) {
  int64_t g = units < (int64_t)cus * per_cu ? units : (int64_t)cus * per_cu;
  return g < 1 ? 1 : (int)g;
}

struct NmWs {
  int64_t *bs_x, *bs_i, *long_rows, *n_long, *long_ws;
  int64_t nb, long_cap;
  int long_grid;
  bool long_in_lds;
};

NmWs carve_nm(void *ws, int64_t rows, int64_t E, int N, int cus, size_t *used) {
  NmWs w{};
  char *p = (char *)ws;
  size_t u = 0;
  auto take = [&](size_t n) {
    int64_t *r = reinterpret_cast<int64_t *>(p + u);
    u += ((n * 8) + 255) & ~(size_t)255;
    return r;
  };
  w.nb = (rows + SCAN_B - 1) / SCAN_B;
  w.bs_x = take(w.nb + 1);
  w.bs_i = take(w.nb + 1);
  const int64_t by_events = E / (SHORT_CAP + 1) + 1;
  w.long_cap = rows < by_events ? rows : by_events;
  w.long_rows = take(w.long_cap > 0 ? w.long_cap : 1);
  w.n_long = take(1);
  w.long_in_lds = N <= LONG_LDS_NODES;
  w.long_grid = grid_for(w.long_cap, cus, w.long_in_lds ? 2 : 1);
  if (!w.long_in_lds) {
    const int64_t per = 2 * (int64_t)N + (N + 31) / 32 + 1;
    w.long_ws = take((size_t)per * w.long_grid);
  }
  *used = u;
  return w;
}

}  // namespace

int node_model_pos_bits(int N) {
  int b = 1;
  while ((1 << b) < N) b++;
  return b;
}

size_t node_model_ws_bytes(int64_t R, int I, int64_t E, int N, int cus) {
  size_t used = 0;
  carve_nm((void *)0x100, R * (int64_t)I, E, N, cus, &used);
  return used + 256;
}

hipError_t launch_node_model(const NodeModelArgs &m, bool fill, void *ws, int cus, hipStream_t s) {
  const int64_t rows = m.R * (int64_t)m.I;
  size_t used = 0;
  NmWs w = carve_nm(ws, rows, m.E, m.N, cus, &used);
  NmArgs a{};
  a.off = m.off;
  a.ts = m.ts;
  a.ctx = m.ctx;
  a.R = m.R;
  a.E = m.E;
  a.I = m.I;
  a.N = m.N;
  a.pos_bits = node_model_pos_bits(m.N);
  a.info = m.info;
  a.ptab = m.ptab;
  a.row_start = m.row_start;
  a.iters_found = m.iters_found;
  a.err = m.err;
  a.long_rows = w.long_rows;
  a.n_long = w.n_long;
  a.long_cap = w.long_cap;
  a.long_ws = w.long_ws;
  if (!fill) {
    if (m.R > 0)
      hipLaunchKernelGGL(nm_rows, dim3(grid_for((m.R + NMW - 1) / NMW, cus, 8)), dim3(NMT), 0, s,
                         m.off, m.ctx, m.R, m.E, m.I, m.info, m.N, m.row_start, m.iters_found,
                         m.err);
    // counts go to the offset arrays, then scanned in place
    a.cnt_x = m.row_off_x;
    a.cnt_i = m.row_off_i;
  } else {
    a.off_x = m.row_off_x;
    a.off_i = m.row_off_i;
    a.node_x = m.node_x;
    a.val_x = m.val_x;
    a.node_i = m.node_i;
    a.val_i = m.val_i;
  }
  hipLaunchKernelGGL(nm_zero, dim3(1), dim3(64), 0, s, w.n_long, (int64_t)1);
  if (!w.long_in_lds)
    hipLaunchKernelGGL(nm_zero, dim3(grid_for(1 << 20, cus, 4)), dim3(256), 0, s, w.long_ws,
                       (int64_t)(2 * (int64_t)m.N + (m.N + 31) / 32 + 1) * w.long_grid);
  if (rows > 0) {
    // rows of up to 64 events: small per-wave buffers, the tree and the
    // position map in LDS when they fit (two workgroups of eight waves per CU);
    // 65..SHORT_CAP events: the LDS radix sort, the tree from L2 (three
    // workgroups of four waves per CU: more waves in flight beat LDS walks)
    static std::once_flag lds_once;
    std::call_once(lds_once, [] {
      allow_dynamic_lds(&nm_short<true, 64, 0, 512, true, true>, 8 * sizeof(WaveLds<64>));
      allow_dynamic_lds(&nm_short<false, 64, 0, 512, true, true>, 8 * sizeof(WaveLds<64>));
      allow_dynamic_lds(&nm_long<true, true>, 64);
      allow_dynamic_lds(&nm_long<false, true>, 64);
    });
    const bool tab1 = m.N <= SMALL_TAB_NODES;
    const size_t lds1 = tab1 ? (size_t)m.N * (sizeof(uint2) + sizeof(uint32_t)) : 0;
    const int g1 = grid_for((rows + 7) / 8, cus, 2);
    if (fill) {
      if (tab1) hipLaunchKernelGGL((nm_short<true, 64, 0, 512, true, true>), dim3(g1), dim3(512), lds1, s, a);
      else hipLaunchKernelGGL((nm_short<true, 64, 0, 512, false, false>), dim3(g1), dim3(512), 0, s, a);
    } else {
      if (tab1) hipLaunchKernelGGL((nm_short<false, 64, 0, 512, true, true>), dim3(g1), dim3(512), lds1, s, a);
      else hipLaunchKernelGGL((nm_short<false, 64, 0, 512, false, false>), dim3(g1), dim3(512), 0, s, a);
    }
    const int g2 = grid_for((rows + NMW - 1) / NMW, cus, 3);
    if (fill) hipLaunchKernelGGL((nm_short<true, SHORT_CAP, 64, NMT, false, false>), dim3(g2), dim3(NMT), 0, s, a);
    else hipLaunchKernelGGL((nm_short<false, SHORT_CAP, 64, NMT, false, false>), dim3(g2), dim3(NMT), 0, s, a);
    const size_t lds = w.long_in_lds ? (size_t)(2 * m.N) * 8 + (size_t)((m.N + 31) / 32) * 8 : 0;
    if (w.long_in_lds) {
      if (fill) hipLaunchKernelGGL((nm_long<true, true>), dim3(w.long_grid), dim3(LONG_T), lds, s, a);
      else hipLaunchKernelGGL((nm_long<false, true>), dim3(w.long_grid), dim3(LONG_T), lds, s, a);
    } else {
      if (fill) hipLaunchKernelGGL((nm_long<true, false>), dim3(w.long_grid), dim3(LONG_T), 0, s, a);
      else hipLaunchKernelGGL((nm_long<false, false>), dim3(w.long_grid), dim3(LONG_T), 0, s, a);
    }
  }
  if (!fill) {
    for (int which = 0; which < 2; which++) {
      int64_t *x = which ? m.row_off_i : m.row_off_x;
      int64_t *bs = which ? w.bs_i : w.bs_x;
      if (w.nb > 0) hipLaunchKernelGGL(scan_sums, dim3((unsigned)w.nb), dim3(SCAN_T), 0, s, x, rows, bs);
      hipLaunchKernelGGL(scan_top, dim3(1), dim3(SCAN_T), 0, s, bs, w.nb);
      hipLaunchKernelGGL(scan_apply, dim3((unsigned)(w.nb > 0 ? w.nb : 1)), dim3(SCAN_T), 0, s, x,
                         rows, bs, w.nb, x);
    }
  }
  return hipGetLastError();
}

}  // namespace ta
