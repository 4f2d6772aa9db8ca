// k_segment.hip -- fused attribution + iteration segmentation over CSR traces.
//
// One workgroup owns one rank at a time (grid-stride over a rank order, so the
// same kernel serves one-workgroup-per-rank launches and persistent plans).
// Per rank it streams the rank's events in tiles of NT*EPT, each thread holding
// EPT consecutive events loaded with 16-byte vector loads from tile-aligned
// global indices:
//   duration  d_k = t_{k+1} - t_k (last event 0)                  [Sec. II]
//   excl      LDS histogram keyed by preorder index (ds_add_u64)  [Sec. VI-B]
//   boundary  entry into the marker subtree; iteration index by a
//             workgroup scan of per-thread boundary counts        [Sec. V]
//   tensor    LDS ring of W iteration rows x G regions; completed rows are
//             written once, whole and coalesced, then cleared     [Sec. V]
//   incl      one exclusive scan of the histogram in preorder:
//             incl[v] = P[tout(v)] - P[tin(v)]
// Everything is integer, so the result does not depend on the order of the
// LDS atomics.  No global atomics except the sticky error word (errors only).
#include "ta_internal.h"

namespace ta {
namespace {

constexpr int NT_MAX = 512;  // largest workgroup (LDS reductions are sized for it)

// The events of one tile held by one thread, plus the two halo values the
// wave edges need (the timestamp after lane 63's last event and the context
// before lane 0's first event).
template <int EPT>
struct Tile {
  int64_t ts[EPT];
  int32_t cv[EPT];
  int64_t halo_ts;
  int32_t halo_ctx;
};

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

template <bool NTMP, class T>
__device__ inline T ld(const T *p) {
  if constexpr (NTMP) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NTMP, class T>
__device__ inline void st(T *p, T v) {
  if constexpr (NTMP) __builtin_nontemporal_store(v, p);
  else *p = v;
}

__device__ inline int64_t join64(int lo, int hi) {
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Load the EPT events starting at global index c0 (a multiple of EPT, so the
// vector loads are aligned) if any of them belongs to the rank [b, e).
template <int EPT, bool NTMP>
__device__ inline void load_tile(Tile<EPT> &t, const int64_t *__restrict__ ts,
                                 const int32_t *__restrict__ ctx, int64_t E, int64_t c0,
                                 int64_t b, int64_t e, int lane) {
#pragma unroll
  for (int j = 0; j < EPT; j++) {
    t.ts[j] = 0;
    t.cv[j] = 0;
  }
  if ((c0 + EPT > b) && (c0 < e)) {
    if (c0 + EPT <= E) {
      const v4i *pt = reinterpret_cast<const v4i *>(ts + c0);
#pragma unroll
      for (int q = 0; q < EPT / 2; q++) {
        const v4i x = ld<NTMP>(pt + q);
        t.ts[2 * q] = join64(x.x, x.y);
        t.ts[2 * q + 1] = join64(x.z, x.w);
      }
      if constexpr (EPT == 2) {
        const v2i y = ld<NTMP>(reinterpret_cast<const v2i *>(ctx + c0));
        t.cv[0] = y.x;
        t.cv[1] = y.y;
      } else {
        const v4i *pc = reinterpret_cast<const v4i *>(ctx + c0);
#pragma unroll
        for (int q = 0; q < EPT / 4; q++) {
          const v4i y = ld<NTMP>(pc + q);
          t.cv[4 * q] = y.x;
          t.cv[4 * q + 1] = y.y;
          t.cv[4 * q + 2] = y.z;
          t.cv[4 * q + 3] = y.w;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < EPT; j++)
        if (c0 + j < E) {
          t.ts[j] = ts[c0 + j];
          t.cv[j] = ctx[c0 + j];
        }
    }
  }
  t.halo_ts = 0;
  t.halo_ctx = -1;
  if (lane == 63 && c0 + EPT < e) t.halo_ts = ts[c0 + EPT];
  if (lane == 0 && c0 - 1 >= b && c0 - 1 < e) t.halo_ctx = ctx[c0 - 1];
}

__device__ inline int wave_incl_scan_i32(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ inline int64_t wave_incl_scan_i64(int64_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// 64x64 -> 128-bit unsigned square accumulated into (lo, hi).
__device__ inline void acc_sq(uint64_t &lo, uint64_t &hi, int64_t v) {
  unsigned __int128 p = (unsigned __int128)(__int128)v * (unsigned __int128)(__int128)v;
  unsigned __int128 s = ((unsigned __int128)hi << 64 | lo) + p;
  lo = (uint64_t)s;
  hi = (uint64_t)(s >> 64);
}

// NT threads per workgroup (256 or 512); a 512-thread workgroup is limited to
// 128 VGPRs so that two fit on a CU beside each other (the LDS allows two).
template <bool ATTR, bool SEG, int EPT, bool NTMP, int NT, bool MULTI>
__global__ __launch_bounds__(NT, NT == 512 ? 4 : 1) void seg_kernel(SegArgs a) {
  constexpr int NWAVE = NT / 64;
  constexpr int TILE = NT * EPT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.N, G = a.G, W = a.W;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  // ---- LDS layout ------------------------------------------------------
  size_t o = 0;
  int64_t *hist = reinterpret_cast<int64_t *>(smem + o);            // [N+1]
  if (ATTR) o += ((size_t)(N + 1) * 8 + 15) & ~(size_t)15;
  int64_t *ring = reinterpret_cast<int64_t *>(smem + o);            // [W*G]
  size_t ring_bytes = SEG ? (size_t)W * G * 8 : 0;
  size_t ring_area = ring_bytes > (size_t)NT * 24 ? ring_bytes : (size_t)NT * 24;
  o += ring_area;
  uint32_t *info = reinterpret_cast<uint32_t *>(smem + o);          // [N]
  o += ((size_t)N * 4 + 15) & ~(size_t)15;
  int *wsum = reinterpret_cast<int *>(smem + o);                    // [2][NWAVE]
  int64_t *wsum64 = reinterpret_cast<int64_t *>(smem + o + 2 * NWAVE * sizeof(int));
  // Rank-end reductions alias the ring area (the ring is cleared after).
  int64_t *redS = ring;                                             // [NT]
  uint64_t *redQ = reinterpret_cast<uint64_t *>(ring + NT);         // [NT][2]

  // ---- stage the call-path table, clear histogram and ring -------------
  for (int v = tid; v < N; v += NT) info[v] = a.info[v];
  if (ATTR)
    for (int v = tid; v <= N; v += NT) hist[v] = 0;
  for (size_t v = tid; v < ring_area / 8; v += NT) ring[v] = 0;
  __syncthreads();

  // Region-row flush mapping: thread -> (row offset, region) with a fixed
  // region per thread, so rank totals accumulate in registers.
  const int rows_pp = SEG ? NT / G : 1;
  const int gme = SEG ? tid % G : 0;
  const int rsub = SEG ? tid / G : 0;
  const bool fl_active = SEG && tid < rows_pp * G;

  // A rank task: the rank id, its event range [b, e) (an invalid range is
  // recorded and treated as empty) and its request's traces.  Outputs are read
  // from the request (mixed batch) or the arguments where they are written.
  struct Task {
    int64_t r, b, e;
    uint32_t err;
    const int64_t *ts;
    const int32_t *ctx;
    int64_t E;
    int I;
    const SegReq *q;  // MULTI only
  };
  auto task_at = [&](int64_t rr) {
    Task k;
    const int64_t *off;
    if constexpr (MULTI) {
      const int64_t tv = a.tasks[rr];
      k.q = a.reqs + (tv >> 32);
      k.r = tv & 0xffffffffll;
      off = k.q->off;
      k.ts = k.q->ts;
      k.ctx = k.q->ctx;
      k.E = k.q->E;
      k.I = k.q->I;
    } else {
      k.q = nullptr;
      k.r = a.order ? (int64_t)a.order[rr] : rr;
      off = a.off;
      k.ts = a.ts;
      k.ctx = a.ctx;
      k.E = a.E;
      k.I = a.I;
    }
    k.b = off[k.r];
    k.e = off[k.r + 1];
    k.err = 0;
    if (k.b < 0 || k.e < k.b || k.e > k.E) {
      k.err = ERRBIT_OFFSETS;
      k.b = k.e = 0;
    }
    return k;
  };
#define TA_OUT(f) (MULTI ? T.q->f : a.f)

  // First tile of task n into `dst`.
  auto prefetch_first = [&](const Task &n, Tile<EPT> &dst) {
    const int64_t t0n = n.b & ~(int64_t)(TILE - 1);
    if (t0n < n.e) load_tile<EPT, NTMP>(dst, n.ts, n.ctx, n.E, t0n + (int64_t)tid * EPT, n.b, n.e, lane);
  };

  int parity = 0;
  Tile<EPT> cur, nxt_tile;
  Task nt{};
  if ((int64_t)blockIdx.x < a.R) {
    nt = task_at(blockIdx.x);
    prefetch_first(nt, cur);
  }
  for (int64_t rr = blockIdx.x; rr < a.R; rr += gridDim.x) {
    const Task T = nt;
    const int64_t r = T.r;
    const int64_t b = T.b, e = T.e;
    const int I = T.I;
    uint32_t errb = T.err;
    int carry = -1;      // iteration index in effect after the processed events
    int flushed = 0;     // tensor rows [0, flushed) are written
    int64_t out_acc = 0; // time outside every region / before the first boundary
    int64_t S = 0;
    uint64_t Qlo = 0, Qhi = 0;
    int64_t *trow = SEG ? TA_OUT(tensor) + r * (int64_t)I * G : nullptr;

    auto flush = [&](int row_lo, int row_hi) {  // rows inclusive, all in the ring
      if (!fl_active) return;
      for (int row = row_lo + rsub; row <= row_hi; row += rows_pp) {
        int slot = (row & (W - 1)) * G + gme;
        int64_t v = ring[slot];
        ring[slot] = 0;
        st<NTMP>(&trow[(int64_t)row * G + gme], v);
        S += v;
        acc_sq(Qlo, Qhi, v);
      }
    };

    // The first tile of this rank is already in `cur` (loaded before the
    // previous rank's epilogue, or before the loop).
    int64_t t0 = b & ~(int64_t)(TILE - 1);
    for (; t0 < e; t0 += TILE) {
      const int64_t c0 = t0 + (int64_t)tid * EPT;
      // Issue the next tile's loads now; they complete while this tile is
      // processed (barriers wait only for LDS traffic).
      if (t0 + TILE < e)
        load_tile<EPT, NTMP>(nxt_tile, T.ts, T.ctx, T.E, c0 + TILE, b, e, lane);
      const int64_t *tsv = cur.ts;
      const int32_t *cv = cur.cv;
      // Timestamp after my last event (lane + 1's first, or the halo at the
      // wave edge) and context before my first event.
      int64_t nxt = __shfl_down(tsv[0], 1, 64);
      if (lane == 63) nxt = cur.halo_ts;
      int32_t pc = __shfl_up(cv[EPT - 1], 1, 64);
      if (lane == 0) pc = cur.halo_ctx;
      int prev_in = 0;
      if (c0 - 1 >= b && c0 - 1 < e && (uint32_t)pc < (uint32_t)N)
        prev_in = (info[pc] & INFO_MARKER_BIT) ? 1 : 0;

      int64_t d[EPT];
      uint32_t inf[EPT];
      uint32_t inr = 0, bmask = 0;
      int bcount = 0;
#pragma unroll
      for (int j = 0; j < EPT; j++) {
        const int64_t k = c0 + j;
        const bool in_r = (k >= b) && (k < e);
        const int64_t tn = (j < EPT - 1) ? tsv[j + 1] : nxt;
        int64_t dj = (in_r && k + 1 < e) ? tn - tsv[j] : 0;
        if (dj < 0) errb |= ERRBIT_UNSORTED;
        uint32_t w = 0;
        if (in_r) {
          if ((uint32_t)cv[j] < (uint32_t)N) w = info[cv[j]];
          else errb |= ERRBIT_CTX;
        }
        const int inm = (w & INFO_MARKER_BIT) ? 1 : 0;
        const int bnd = inm & (prev_in ^ 1);
        prev_in = inm;
        bmask |= (uint32_t)bnd << j;
        inr |= (uint32_t)in_r << j;
        bcount += bnd;
        d[j] = dj;
        inf[j] = w;
      }

      // Workgroup scan of boundary counts -> iteration index of each event.
      const int inc = wave_incl_scan_i32(bcount, lane);
      int *ws = wsum + parity * NWAVE;
      parity ^= 1;
      if (lane == 63) ws[wid] = inc;
      __syncthreads();
      int wbase = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < NWAVE; w++) {
        int s = ws[w];
        wbase += (w < wid) ? s : 0;
        tot += s;
      }
      const int it_first = carry;
      const int it_last = carry + tot;
      int itj[EPT];
      int run = carry + wbase + inc - bcount;
#pragma unroll
      for (int j = 0; j < EPT; j++) {
        run += (bmask >> j) & 1;
        itj[j] = run;
      }

      if (ATTR) {
#pragma unroll
        for (int j = 0; j < EPT; j++)
          if (d[j] != 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&hist[inf[j] >> INFO_TIN_SHIFT]),
                      (unsigned long long)d[j]);
      }

      if (SEG) {
#pragma unroll
        for (int j = 0; j < EPT; j++) {
          const int gj = (int)(inf[j] & INFO_REGION_MASK) - 1;
          if (((inr >> j) & 1) && (itj[j] < 0 || gj < 0)) out_acc += d[j];
          if (((inr >> j) & 1) && itj[j] >= I) errb |= ERRBIT_OVERFLOW;
        }
        int lo = it_first > 0 ? it_first : 0;
        while (true) {
          const int hi = lo + W - 1;
          int64_t pend = 0;
          int pslot = -1;
#pragma unroll
          for (int j = 0; j < EPT; j++) {
            const int gj = (int)(inf[j] & INFO_REGION_MASK) - 1;
            const int it = itj[j];
            if (((inr >> j) & 1) && gj >= 0 && it >= lo && it <= hi && it < I) {
              const int slot = (it & (W - 1)) * G + gj;
              if (slot == pslot) {
                pend += d[j];
              } else {
                if (pslot >= 0 && pend != 0)
                  atomicAdd(reinterpret_cast<unsigned long long *>(&ring[pslot]),
                            (unsigned long long)pend);
                pslot = slot;
                pend = d[j];
              }
            }
          }
          if (pslot >= 0 && pend != 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&ring[pslot]), (unsigned long long)pend);
          __syncthreads();
          int fl_hi = hi < it_last - 1 ? hi : it_last - 1;
          if (fl_hi > I - 1) fl_hi = I - 1;
          if (fl_hi >= flushed) {
            flush(flushed, fl_hi);
            flushed = fl_hi + 1;
          }
          __syncthreads();
          if (hi >= it_last) break;
          lo = hi + 1;
        }
      }
      carry = it_last;
      cur = nxt_tile;
    }

    // Next rank's first tile: its loads are in flight during this epilogue.
    if (rr + gridDim.x < a.R) {
      nt = task_at(rr + gridDim.x);
      prefetch_first(nt, cur);
    }

    // ---- rank epilogue --------------------------------------------------
    if (SEG) {
      const int last_data = carry < I - 1 ? carry : I - 1;
      if (fl_active) {
        for (int row = flushed + rsub; row < I; row += rows_pp) {
          int64_t v = 0;
          if (row <= last_data) {
            int slot = (row & (W - 1)) * G + gme;
            v = ring[slot];
            ring[slot] = 0;
          }
          st<NTMP>(&trow[(int64_t)row * G + gme], v);
          S += v;
          acc_sq(Qlo, Qhi, v);
        }
      }
      // outside: workgroup sum
      int64_t os = wave_sum_i64(out_acc);
      __syncthreads();
      if (lane == 0) wsum64[wid] = os;
      redS[tid] = S;
      redQ[2 * tid] = Qlo;
      redQ[2 * tid + 1] = Qhi;
      __syncthreads();
      if (tid < G) {
        int64_t s = 0;
        unsigned __int128 q = 0;
        for (int k = 0; k < rows_pp; k++) {
          int idx = k * G + tid;
          s += redS[idx];
          q += ((unsigned __int128)redQ[2 * idx + 1] << 64) | redQ[2 * idx];
        }
        if (TA_OUT(rank_sum)) TA_OUT(rank_sum)[r * G + tid] = s;
        if (TA_OUT(rank_sumsq)) {
          TA_OUT(rank_sumsq)[2 * (r * G + tid)] = (uint64_t)q;
          TA_OUT(rank_sumsq)[2 * (r * G + tid) + 1] = (uint64_t)(q >> 64);
        }
      }
      if (tid == 0) {
        int64_t s = 0;
        for (int w = 0; w < NWAVE; w++) s += wsum64[w];
        if (TA_OUT(outside)) TA_OUT(outside)[r] = s;
        if (TA_OUT(iters_found)) TA_OUT(iters_found)[r] = carry + 1;
      }
      __syncthreads();
      for (int v = tid; v < 3 * NT; v += NT) ring[v] = 0;  // redS + redQ area
    }
    if (tid == 0 && TA_OUT(span)) TA_OUT(span)[r] = (e > b) ? T.ts[e - 1] - T.ts[b] : 0;

    if (ATTR) {
      __syncthreads();
      // Exclusive scan of the histogram in preorder: P[j] = sum_{j' < j} h[j'].
      const int n1 = N + 1;
      const int L = (n1 + NT - 1) / NT;
      const int k0 = tid * L;
      const int k1 = (k0 + L < n1) ? k0 + L : n1;
      int64_t s = 0;
      for (int k = k0; k < k1; k++) s += (k < N) ? hist[k] : 0;
      const int64_t incs = wave_incl_scan_i64(s, lane);
      if (lane == 63) wsum64[wid] = incs;
      __syncthreads();
      int64_t runp = incs - s;
      for (int w = 0; w < wid; w++) runp += wsum64[w];
      for (int k = k0; k < k1; k++) {
        int64_t h = (k < N) ? hist[k] : 0;
        hist[k] = runp;
        runp += h;
      }
      __syncthreads();
      for (int v = tid; v < N; v += NT) {
        const int2 tt = a.tin_tout[v];
        const int64_t pa = hist[tt.x];
        if (TA_OUT(excl)) st<NTMP>(&TA_OUT(excl)[r * N + v], hist[tt.x + 1] - pa);
        if (TA_OUT(incl)) st<NTMP>(&TA_OUT(incl)[r * N + v], hist[tt.y] - pa);
      }
      __syncthreads();
      for (int v = tid; v <= N; v += NT) hist[v] = 0;
    }
    if (errb) atomicOr(a.err, errb);
    __syncthreads();
  }
#undef TA_OUT
}

}  // namespace

size_t segment_lds_bytes(int N, int G, bool attr, bool seg, int *W, int *log2W) {
  size_t fixed = 0;
  if (attr) fixed += ((size_t)(N + 1) * 8 + 15) & ~(size_t)15;
  fixed += ((size_t)N * 4 + 15) & ~(size_t)15;
  fixed += 2 * (NT_MAX / 64) * sizeof(int) + (NT_MAX / 64) * sizeof(int64_t);
  int w = 2, lw = 1;
  if (seg) {
    // Largest power-of-two ring within 16 KiB, and within what leaves room for
    // two workgroups per CU when the tables allow it.
    size_t budget = 16384;
    if (fixed + budget > 80 * 1024 && fixed + 8192 <= 80 * 1024) budget = 8192;
    while ((size_t)(w * 2) * G * 8 <= budget && w < 1024) {
      w *= 2;
      lw++;
    }
  }
  *W = w;
  *log2W = lw;
  size_t ring = seg ? (size_t)w * G * 8 : 0;
  if (ring < (size_t)NT_MAX * 24) ring = (size_t)NT_MAX * 24;
  return fixed + ring;
}

namespace {

template <bool A, bool S, int EPT, bool NTMP, int NT, bool MULTI>
hipError_t launch_one(const SegArgs &a, int grid, size_t lds, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&seg_kernel<A, S, EPT, NTMP, NT, MULTI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL((seg_kernel<A, S, EPT, NTMP, NT, MULTI>), dim3(grid), dim3(NT), lds, s, a);
  return hipGetLastError();
}

// Mixed batches use the fused pass only.
template <bool A, bool S, int EPT, bool NTMP, int NT>
hipError_t launch_variant(const SegArgs &a, int grid, size_t lds, hipStream_t s) {
  if (a.reqs) {
    if constexpr (A && S) return launch_one<A, S, EPT, NTMP, NT, true>(a, grid, lds, s);
    return hipErrorInvalidValue;
  }
  return launch_one<A, S, EPT, NTMP, NT, false>(a, grid, lds, s);
}

template <bool A, bool S>
hipError_t launch_ept(const SegArgs &a, const SegShape &sh, int grid, size_t lds, hipStream_t s) {
  if (sh.threads == 512) {
    // 512-thread workgroups: the fused pass only, 2 or 4 events per thread.
    if constexpr (A && S) {
      switch (sh.ept * 2 + (sh.nontemporal ? 1 : 0)) {
        case 4: return launch_variant<A, S, 2, false, 512>(a, grid, lds, s);
        case 5: return launch_variant<A, S, 2, true, 512>(a, grid, lds, s);
        case 8: return launch_variant<A, S, 4, false, 512>(a, grid, lds, s);
        case 9: return launch_variant<A, S, 4, true, 512>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
      }
    }
    return hipErrorInvalidValue;
  }
  if (sh.threads != 256) return hipErrorInvalidValue;
  switch (sh.ept * 2 + (sh.nontemporal ? 1 : 0)) {
    case 4: return launch_variant<A, S, 2, false, 256>(a, grid, lds, s);
    case 5: return launch_variant<A, S, 2, true, 256>(a, grid, lds, s);
    case 8: return launch_variant<A, S, 4, false, 256>(a, grid, lds, s);
    case 9: return launch_variant<A, S, 4, true, 256>(a, grid, lds, s);
    case 16: return launch_variant<A, S, 8, false, 256>(a, grid, lds, s);
    case 17: return launch_variant<A, S, 8, true, 256>(a, grid, lds, s);
    case 32: return launch_variant<A, S, 16, false, 256>(a, grid, lds, s);
    case 33: return launch_variant<A, S, 16, true, 256>(a, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_segment(const SegArgs &a, bool attr, bool seg, const SegShape &sh, int grid,
                          size_t lds, hipStream_t s) {
  if (attr && seg) return launch_ept<true, true>(a, sh, grid, lds, s);
  if (attr) return launch_ept<true, false>(a, sh, grid, lds, s);
  return launch_ept<false, true>(a, sh, grid, lds, s);
}

}  // namespace ta
