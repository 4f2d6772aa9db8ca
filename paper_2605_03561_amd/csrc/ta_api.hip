// ta_api.hip -- host side of the C ABI: handle, call-path tables, argument
// validation, workspace and kernel launches.  No exception crosses the ABI.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "ta_ae.h"
#include "ta_internal.h"

struct ta_handle_s {
  int device = 0;
  std::string last_error;
  // call-path tree (caller numbering) and derived tables
  int32_t N = 0;
  std::vector<int32_t> parent, tin, tout;
  // regions
  int32_t marker = -1, G = 0;
  std::vector<int32_t> regions;
  uint32_t *d_info = nullptr;
  int2 *d_tin_tout = nullptr;
  int4 *d_rt = nullptr;  // regions in preorder: see region_table()
  // by preorder position: caller id, parent position (-1 at a root), subtree end
  int4 *d_ptab = nullptr;
  // pruned tree (ta_set_pruned): kept nodes' preorder ranges and, for each, the
  // index of its nearest kept strict ancestor (-1 if none)
  int32_t K = 0;
  int2 *d_kq = nullptr;
  int32_t *d_kpar = nullptr;
  uint32_t *d_err = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int32_t *pin = nullptr;  // pinned host word (pre-screen fallback count)
  ta::AeState ae;
  // Batch plans alive on this handle: their graphs hold the call-path tables'
  // device addresses, so the tables cannot be replaced while any exists.
  int32_t live_plans = 0;
};

namespace {

ta_status fail(ta_handle h, ta_status s, const std::string &msg) {
  if (h) h->last_error = msg;
  return s;
}

ta_status hipfail(ta_handle h, hipError_t e, const char *what) {
  return fail(h, TA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define TA_HIP(h, call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hipfail((h), e_, #call); \
  } while (0)

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Workspace of ta_imbalance_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory, so it is never passed to a kernel or a copy:
// its device address is looked up once per device (ta_create, with that
// device current) and that address is used instead.
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[TA_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
hipError_t g_scratch_err[SCRATCH_MAX_DEVICES] = {};
bool g_scratch_done[SCRATCH_MAX_DEVICES] = {};

// Called with `device` current.
void scratch_setup(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
  g_scratch_done[device] = true;
}

ta_status scratch_address(ta_handle h, void **out) {
  const int d = h->device;
  if (d < 0 || d >= SCRATCH_MAX_DEVICES)
    return fail(h, TA_ERR_INVALID_ARG, "device index above the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[d] || !g_scratch_ptr[d])
    return fail(h, TA_ERR_HIP,
                std::string("device address of the static scratch array unavailable: ") +
                    hipGetErrorString(g_scratch_done[d] ? g_scratch_err[d] : hipErrorNotReady));
  *out = g_scratch_ptr[d];
  return TA_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int d) {
    if (hipGetDevice(&prev) == hipSuccess && prev != d) hipSetDevice(d);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

ta_status ensure_ws(ta_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return TA_OK;
  if (h->ws) {
    // Kernels already queued may still use the old workspace.
    TA_HIP(h, hipDeviceSynchronize());
    TA_HIP(h, hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4;
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    h->ws = nullptr;
    return fail(h, TA_ERR_OOM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  h->ws_bytes = want;
  return TA_OK;
}

// Validate a parent array; fill preorder index and subtree end.
ta_status build_tree(ta_handle h, int32_t N, const int32_t *parent, std::vector<int32_t> &tin,
                     std::vector<int32_t> &tout) {
  std::vector<int32_t> head(N, -1), next(N, -1);
  std::vector<int32_t> roots;
  for (int32_t v = N - 1; v >= 0; v--) {  // children lists in increasing id order
    const int32_t p = parent[v];
    if (p < -1 || p >= N) return fail(h, TA_ERR_BAD_TREE, "parent id out of range at node " + std::to_string(v));
    if (p == v) return fail(h, TA_ERR_BAD_TREE, "node is its own parent: " + std::to_string(v));
    if (p >= 0) {
      next[v] = head[p];
      head[p] = v;
    }
  }
  for (int32_t v = 0; v < N; v++)
    if (parent[v] == -1) roots.push_back(v);
  tin.assign(N, -1);
  tout.assign(N, -1);
  int32_t clock = 0;
  std::vector<int32_t> stack;
  for (int32_t root : roots) {
    stack.push_back(root);
    tin[root] = clock++;
    while (!stack.empty()) {
      const int32_t v = stack.back();
      const int32_t c = head[v];
      if (c >= 0) {
        head[v] = next[c];  // consume the child
        tin[c] = clock++;
        stack.push_back(c);
      } else {
        tout[v] = clock;
        stack.pop_back();
      }
    }
  }
  if (clock != N) return fail(h, TA_ERR_BAD_TREE, "parent array has a cycle");
  return TA_OK;
}

// Regions in preorder of their nodes: the regions inside region g's subtree
// then occupy consecutive positions [pos(g), end(g)).  Entry i holds
// (pos(i), end(i)) of region i and (region at position i, end of that region).
std::vector<int4> region_table(ta_handle h) {
  const int32_t G = h->G;
  std::vector<int32_t> perm(G), pos(G), end(G);
  for (int32_t g = 0; g < G; g++) perm[g] = g;
  std::sort(perm.begin(), perm.end(),
            [&](int32_t a, int32_t b) { return h->tin[h->regions[a]] < h->tin[h->regions[b]]; });
  for (int32_t j = 0; j < G; j++) pos[perm[j]] = j;
  for (int32_t g = 0; g < G; g++) {
    const int32_t tout = h->tout[h->regions[g]];
    int32_t e = pos[g] + 1;
    while (e < G && h->tin[h->regions[perm[e]]] < tout) e++;
    end[g] = e;
  }
  std::vector<int4> rt(G);
  for (int32_t i = 0; i < G; i++) rt[i] = make_int4(pos[i], end[i], perm[i], end[perm[i]]);
  return rt;
}

void free_pruned(ta_handle h) {
  if (h->d_kq) hipFree(h->d_kq);
  if (h->d_kpar) hipFree(h->d_kpar);
  h->d_kq = nullptr;
  h->d_kpar = nullptr;
  h->K = 0;
}

ta_status upload_tables(ta_handle h) {
  const int32_t N = h->N;
  std::vector<uint32_t> info(N);
  std::vector<int32_t> reg(N, -1);
  std::vector<int32_t> is_region(N, -1);
  for (int32_t g = 0; g < h->G; g++) is_region[h->regions[g]] = g;
  // Visit in preorder so a parent's region is known before its children's.
  std::vector<int32_t> order(N);
  for (int32_t v = 0; v < N; v++) order[h->tin[v]] = v;
  for (int32_t j = 0; j < N; j++) {
    const int32_t v = order[j];
    if (is_region[v] >= 0) reg[v] = is_region[v];
    else if (h->parent[v] >= 0) reg[v] = reg[h->parent[v]];
  }
  const int32_t m = h->marker;
  for (int32_t v = 0; v < N; v++) {
    uint32_t w = (uint32_t)h->tin[v] << ta::INFO_TIN_SHIFT;
    if (m >= 0 && h->tin[v] >= h->tin[m] && h->tin[v] < h->tout[m]) w |= ta::INFO_MARKER_BIT;
    w |= (uint32_t)(reg[v] + 1);
    info[v] = w;
  }
  std::vector<int2> tt(N);
  for (int32_t v = 0; v < N; v++) tt[v] = make_int2(h->tin[v], h->tout[v]);
  std::vector<int4> pt(N);
  for (int32_t v = 0; v < N; v++)
    pt[h->tin[v]] = make_int4(v, h->parent[v] >= 0 ? h->tin[h->parent[v]] : -1, h->tout[v], 0);
  // Kernels still queued may read the previous tables.
  if (h->d_info || h->d_tin_tout || h->d_rt || h->d_ptab) TA_HIP(h, hipDeviceSynchronize());
  if (h->d_info) hipFree(h->d_info);
  if (h->d_tin_tout) hipFree(h->d_tin_tout);
  if (h->d_rt) hipFree(h->d_rt);
  if (h->d_ptab) hipFree(h->d_ptab);
  h->d_info = nullptr;
  h->d_tin_tout = nullptr;
  h->d_rt = nullptr;
  h->d_ptab = nullptr;
  TA_HIP(h, hipMalloc(&h->d_info, (size_t)N * sizeof(uint32_t)));
  TA_HIP(h, hipMalloc(&h->d_tin_tout, (size_t)N * sizeof(int2)));
  TA_HIP(h, hipMalloc(&h->d_ptab, (size_t)N * sizeof(int4)));
  TA_HIP(h, hipMemcpy(h->d_info, info.data(), (size_t)N * sizeof(uint32_t), hipMemcpyHostToDevice));
  TA_HIP(h, hipMemcpy(h->d_tin_tout, tt.data(), (size_t)N * sizeof(int2), hipMemcpyHostToDevice));
  TA_HIP(h, hipMemcpy(h->d_ptab, pt.data(), (size_t)N * sizeof(int4), hipMemcpyHostToDevice));
  if (h->G > 0) {
    const std::vector<int4> rt = region_table(h);
    TA_HIP(h, hipMalloc(&h->d_rt, rt.size() * sizeof(int4)));
    TA_HIP(h, hipMemcpy(h->d_rt, rt.data(), rt.size() * sizeof(int4), hipMemcpyHostToDevice));
  }
  return TA_OK;
}

// Kept nodes of a pruned tree: preorder range of each and the index of its
// nearest kept strict ancestor (its parent in the pruned tree), found with a
// stack over the kept nodes in preorder.
ta_status upload_pruned(ta_handle h, const std::vector<int32_t> &kept) {
  const int32_t K = (int32_t)kept.size();
  std::vector<int32_t> by_tin(K);
  for (int32_t k = 0; k < K; k++) by_tin[k] = k;
  std::sort(by_tin.begin(), by_tin.end(),
            [&](int32_t a, int32_t b) { return h->tin[kept[a]] < h->tin[kept[b]]; });
  std::vector<int32_t> up(K, -1), stack;
  for (int32_t k : by_tin) {
    const int32_t t = h->tin[kept[k]];
    while (!stack.empty() && h->tout[kept[stack.back()]] <= t) stack.pop_back();
    up[k] = stack.empty() ? -1 : stack.back();
    stack.push_back(k);
  }
  std::vector<int2> kq(K);
  for (int32_t k = 0; k < K; k++) kq[k] = make_int2(h->tin[kept[k]], h->tout[kept[k]]);
  free_pruned(h);
  TA_HIP(h, hipMalloc(&h->d_kq, (size_t)K * sizeof(int2)));
  TA_HIP(h, hipMalloc(&h->d_kpar, (size_t)K * sizeof(int32_t)));
  TA_HIP(h, hipMemcpy(h->d_kq, kq.data(), (size_t)K * sizeof(int2), hipMemcpyHostToDevice));
  TA_HIP(h, hipMemcpy(h->d_kpar, up.data(), (size_t)K * sizeof(int32_t), hipMemcpyHostToDevice));
  h->K = K;
  return TA_OK;
}

ta_status check_traces(ta_handle h, const ta_traces *t) {
  if (!t) return fail(h, TA_ERR_INVALID_ARG, "traces is NULL");
  if (t->n_ranks < 0 || t->n_events < 0) return fail(h, TA_ERR_INVALID_ARG, "negative size");
  if (t->n_ranks >= (int64_t)1 << 31) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many ranks");
  if (!t->offsets || !aligned16(t->offsets)) return fail(h, TA_ERR_INVALID_ARG, "offsets NULL or not 16-byte aligned");
  if (t->n_events > 0 && (!t->ts || !t->ctx))
    return fail(h, TA_ERR_INVALID_ARG, "ts/ctx NULL");
  if ((t->ts && !aligned16(t->ts)) || (t->ctx && !aligned16(t->ctx)))
    return fail(h, TA_ERR_INVALID_ARG, "ts/ctx not 16-byte aligned");
  return TA_OK;
}

struct SegLaunch {
  ta::SegArgs a{};
  size_t lds = 0;
  bool attr = false, seg = false;
};

// Validate a fused-pass request and fill the kernel arguments (no launch).
ta_status prepare_segment(ta_handle h, const ta_traces *t, int32_t n_iters, const ta_seg_out *o,
                          bool want_attr, bool want_seg, SegLaunch *L) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta_status st = check_traces(h, t);
  if (st) return st;
  if (!o) return fail(h, TA_ERR_INVALID_ARG, "outputs NULL");
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  const bool attr = want_attr && (o->excl || o->incl);
  const bool seg = want_seg && (o->tensor || o->iters_found);
  if (!attr && !seg) return fail(h, TA_ERR_INVALID_ARG, "no output requested");
  if (seg) {
    if (h->G <= 0) return fail(h, TA_ERR_STATE, "ta_set_regions has not been called");
    if (!o->tensor || !o->iters_found)
      return fail(h, TA_ERR_INVALID_ARG, "segmentation needs tensor and iters_found");
    if (n_iters < 1) return fail(h, TA_ERR_INVALID_ARG, "n_iters must be >= 1");
    const double cells = (double)t->n_ranks * (double)n_iters * (double)h->G;
    if (cells > 4e18 || (double)n_iters * h->G > 2e9) return fail(h, TA_ERR_SIZE_OVERFLOW, "tensor too large");
  }
  if (attr && h->N > ta::MAX_NODES_ATTR)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "attribution supports at most 8192 CCT nodes");
  const void *ptrs[] = {o->tensor, o->iters_found, o->outside, o->span, o->rank_sum, o->rank_sumsq,
                        o->excl, o->incl};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "output not 16-byte aligned");
  int W = 2, lw = 1;
  L->lds = ta::segment_lds_bytes(h->N, seg ? h->G : 1, attr, seg, &W, &lw);
  if (L->lds > 160 * 1024) return fail(h, TA_ERR_SIZE_OVERFLOW, "call-path tables exceed LDS");
  ta::SegArgs &a = L->a;
  a.off = t->offsets;
  a.ts = t->ts;
  a.ctx = t->ctx;
  a.R = t->n_ranks;
  a.E = t->n_events;
  a.info = h->d_info;
  a.tin_tout = h->d_tin_tout;
  a.order = nullptr;
  a.N = h->N;
  a.G = seg ? h->G : 1;
  a.I = seg ? n_iters : 0;
  a.W = W;
  a.log2W = lw;
  a.tensor = seg ? o->tensor : nullptr;
  a.iters_found = seg ? o->iters_found : nullptr;
  a.outside = seg ? o->outside : nullptr;
  a.span = o->span;
  a.rank_sum = seg ? o->rank_sum : nullptr;
  a.rank_sumsq = seg ? o->rank_sumsq : nullptr;
  a.excl = attr ? o->excl : nullptr;
  a.incl = attr ? o->incl : nullptr;
  a.err = h->d_err;
  L->attr = attr;
  L->seg = seg;
  return TA_OK;
}

int device_cus(int device) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0)
    n = 256;
  return n;
}

// Launch shape of eager calls and of untuned plans: the fused pass with 512
// threads x 4 events per thread, one workgroup per rank (the tuned choice on
// the 100k-rank batch); the separate passes with 256 x 4.
ta::SegShape default_shape(const SegLaunch &L) {
  ta::SegShape sh{};
  if (L.attr && L.seg) {
    sh.threads = 512;
    sh.ept = 4;
  }
  return sh;
}

int grid_for(const SegLaunch &L, const ta::SegShape &sh, int cus) {
  const int64_t R = L.a.R;
  if (sh.wgs_per_cu <= 0) return (int)std::min<int64_t>(R, (int64_t)1 << 30);
  return (int)std::min<int64_t>(R, (int64_t)sh.wgs_per_cu * cus);
}

ta_status run_segment(ta_handle h, const ta_traces *t, int32_t n_iters, const ta_seg_out *o,
                      void *stream, bool want_attr, bool want_seg) {
  SegLaunch L;
  ta_status st = prepare_segment(h, t, n_iters, o, want_attr, want_seg, &L);
  if (st) return st;
  if (t->n_ranks == 0) return TA_OK;
  DeviceGuard dg(h->device);
  const ta::SegShape sh = default_shape(L);
  hipError_t e = ta::launch_segment(L.a, L.attr, L.seg, sh, grid_for(L, sh, device_cus(h->device)),
                                    L.lds, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "segment kernel launch");
  return TA_OK;
}

}  // namespace

struct ta_plan_s {
  ta_handle h = nullptr;
  int32_t *d_order = nullptr;
  ta::SegReq *d_reqs = nullptr;  // mixed batch: request descriptors
  int64_t *d_tasks = nullptr;    // mixed batch: (request << 32) | rank, longest first
  void *ws = nullptr;
  hipStream_t cap = nullptr;
  hipStream_t cap2 = nullptr;      // a second capture stream (imbalance epilogue beside the scan)
  hipEvent_t ev_stats = nullptr, ev_join = nullptr;
  hipStream_t cap3 = nullptr;      // the exact scan's selections beside its passes
  hipEvent_t ev_scan[10] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ta::SegShape shape;
  float tuned_ms = 0.f;
  // Event record nodes just before and just after the fused pass in the graph
  // (null when they could not be added), and the event pairs they are pointed
  // at by ta_plan_launch_timed, one pair per slot.
  hipGraphNode_t rec[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> slots;
};

namespace {

void plan_free(ta_plan p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->cap) hipStreamDestroy(p->cap);
  if (p->cap2) hipStreamDestroy(p->cap2);
  if (p->ev_stats) hipEventDestroy(p->ev_stats);
  if (p->ev_join) hipEventDestroy(p->ev_join);
  if (p->cap3) hipStreamDestroy(p->cap3);
  for (hipEvent_t ev : p->ev_scan)
    if (ev) hipEventDestroy(ev);
  for (hipEvent_t ev : p->slots)
    if (ev) hipEventDestroy(ev);
  if (p->d_order) hipFree(p->d_order);
  if (p->d_reqs) hipFree(p->d_reqs);
  if (p->d_tasks) hipFree(p->d_tasks);
  if (p->ws) hipFree(p->ws);
  delete p;
}

// --- autotune cache: a flat JSON object
// {"<key>": {"threads": t, "ept": e, "nt": n, "wgs": w, "ms": m}, ...}
// (entries without "threads" are read as 256-thread shapes).
struct CacheEntry {
  std::string key;
  int ept, nt, wgs;
  double ms;
  int threads;
};

std::vector<CacheEntry> cache_read(const char *path) {
  std::vector<CacheEntry> out;
  FILE *f = path ? fopen(path, "r") : nullptr;
  if (!f) return out;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  size_t pos = 0;
  while (true) {
    size_t q0 = txt.find('"', pos);
    if (q0 == std::string::npos) break;
    size_t q1 = txt.find('"', q0 + 1);
    size_t br = txt.find('{', q1);
    size_t be = txt.find('}', br);
    if (q1 == std::string::npos || br == std::string::npos || be == std::string::npos) break;
    CacheEntry c{txt.substr(q0 + 1, q1 - q0 - 1), 0, 0, 0, 0.0, 256};
    std::string body = txt.substr(br, be - br + 1);
    if (sscanf(body.c_str(), "{\"threads\": %d, \"ept\": %d, \"nt\": %d, \"wgs\": %d, \"ms\": %lf}",
               &c.threads, &c.ept, &c.nt, &c.wgs, &c.ms) == 5 ||
        sscanf(body.c_str(), "{\"ept\": %d, \"nt\": %d, \"wgs\": %d, \"ms\": %lf}", &c.ept, &c.nt,
               &c.wgs, &c.ms) == 4)
      out.push_back(c);
    pos = be + 1;
  }
  return out;
}

void cache_write(const char *path, const std::vector<CacheEntry> &es) {
  if (!path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  for (size_t i = 0; i < es.size(); i++)
    fprintf(f, "  \"%s\": {\"threads\": %d, \"ept\": %d, \"nt\": %d, \"wgs\": %d, \"ms\": %.4f}%s\n",
            es[i].key.c_str(), es[i].threads, es[i].ept, es[i].nt, es[i].wgs, es[i].ms,
            i + 1 < es.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

std::string plan_key(ta_handle h, const SegLaunch &L) {
  hipDeviceProp_t prop{};
  hipGetDeviceProperties(&prop, h->device);
  char k[512];
  snprintf(k, sizeof k, "%s/cu%d/R%lld/E%lld/N%d/G%d/I%d/a%d/s%d", prop.gcnArchName,
           prop.multiProcessorCount, (long long)L.a.R, (long long)L.a.E, L.a.N, L.a.G, L.a.I,
           (int)L.attr, (int)L.seg);
  for (char *c = k; *c; c++)
    if (*c == '"' || *c == '\\') *c = '_';
  return k;
}

ta_status time_shape(ta_handle h, const SegLaunch &L, const ta::SegShape &sh, int cus,
                     hipStream_t s, float *ms) {
  const int grid = grid_for(L, sh, cus);
  hipEvent_t e0, e1;
  TA_HIP(h, hipEventCreate(&e0));
  TA_HIP(h, hipEventCreate(&e1));
  hipError_t e = ta::launch_segment(L.a, L.attr, L.seg, sh, grid, L.lds, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int k = 0; k < 2 && e == hipSuccess; k++)
    e = ta::launch_segment(L.a, L.attr, L.seg, sh, grid, L.lds, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return hipfail(h, e, "autotune launch");
  *ms = t / 2.f;
  return TA_OK;
}

// Launch shape of a fused pass: the default, a cached choice (autotune 2) or
// the fastest candidate measured on this batch (every candidate produces
// identical outputs).
ta_status choose_shape(ta_handle h, const SegLaunch &L, int autotune, hipStream_t s,
                       ta::SegShape *best_out, float *best_ms_out) {
  const int cus = device_cus(h->device);
  const int occ = std::max(1, (int)((160 * 1024) / std::max<size_t>(L.lds, 1)));
  ta::SegShape best = default_shape(L);
  float best_ms = 0.f;
  const char *cpath = getenv("TA_AUTOTUNE_CACHE");
  const std::string key = plan_key(h, L);
  std::vector<CacheEntry> cache = autotune == 2 ? cache_read(cpath) : std::vector<CacheEntry>{};
  bool found = false;
  for (const CacheEntry &c : cache)
    if (c.key == key) {
      best.threads = c.threads;
      best.ept = c.ept;
      best.nontemporal = c.nt != 0;
      best.wgs_per_cu = c.wgs;
      best_ms = (float)c.ms;
      found = true;
    }
  if (autotune && !found) {
    bool have = false;
    struct TE {
      int threads, ept;
    };
    std::vector<TE> tes = {{256, 2}, {256, 4}, {256, 8}, {256, 16}};
    if (L.attr && L.seg) {
      tes.push_back({512, 2});
      tes.push_back({512, 4});
    }
    for (const TE &te : tes)
      for (int nt : {0, 1})
        for (int wgs : {0, occ}) {
          ta::SegShape sh;
          sh.threads = te.threads;
          sh.ept = te.ept;
          sh.nontemporal = nt != 0;
          sh.wgs_per_cu = wgs;
          float ms = 0.f;
          ta_status st = time_shape(h, L, sh, cus, s, &ms);
          if (st) return st;
          if (!have || ms < best_ms) {
            best = sh;
            best_ms = ms;
            have = true;
          }
        }
    if (autotune == 2 && cpath) {
      cache.push_back({key, best.ept, best.nontemporal ? 1 : 0, best.wgs_per_cu, best_ms, best.threads});
      cache_write(cpath, cache);
    }
  }
  *best_out = best;
  *best_ms_out = best_ms;
  return TA_OK;
}

}  // namespace

extern "C" {

const char *ta_status_string(ta_status s) {
  switch (s) {
    case TA_OK: return "ok";
    case TA_ERR_INVALID_ARG: return "invalid argument";
    case TA_ERR_BAD_TREE: return "bad call-path tree";
    case TA_ERR_CTX_RANGE: return "context id out of range";
    case TA_ERR_UNSORTED: return "timestamps decrease within a rank";
    case TA_ERR_ITER_OVERFLOW: return "more iterations than the tensor holds";
    case TA_ERR_SIZE_OVERFLOW: return "size exceeds a kernel limit";
    case TA_ERR_OOM: return "out of device memory";
    case TA_ERR_HIP: return "HIP runtime error";
    case TA_ERR_STATE: return "missing set-up call";
    default: return "unknown status";
  }
}

ta_status ta_create(ta_handle *out, int device) {
  if (!out) return TA_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TA_ERR_INVALID_ARG;
  ta_handle h = new (std::nothrow) ta_handle_s();
  if (!h) return TA_ERR_OOM;
  h->device = device;
  DeviceGuard dg(device);
  if (hipMalloc(&h->d_err, 256) != hipSuccess || hipMemset(h->d_err, 0, 256) != hipSuccess) {
    delete h;
    return TA_ERR_HIP;
  }
  scratch_setup(device);
  ta::outliers_init();
  *out = h;
  return TA_OK;
}

ta_status ta_destroy(ta_handle h) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->live_plans > 0) return fail(h, TA_ERR_STATE, "destroy the handle's batch plans first");
  DeviceGuard dg(h->device);
  hipDeviceSynchronize();
  if (h->d_info) hipFree(h->d_info);
  if (h->d_tin_tout) hipFree(h->d_tin_tout);
  if (h->d_rt) hipFree(h->d_rt);
  if (h->d_ptab) hipFree(h->d_ptab);
  free_pruned(h);
  if (h->d_err) hipFree(h->d_err);
  if (h->ws) hipFree(h->ws);
  if (h->pin) hipHostFree(h->pin);
  ta::ae_free(h->ae);
  delete h;
  return TA_OK;
}

const char *ta_last_error(ta_handle h) { return h ? h->last_error.c_str() : "NULL handle"; }

ta_status ta_sync_status(ta_handle h, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  DeviceGuard dg(h->device);
  TA_HIP(h, hipStreamSynchronize((hipStream_t)stream));
  uint32_t bits = 0;
  TA_HIP(h, hipMemcpy(&bits, h->d_err, sizeof(bits), hipMemcpyDeviceToHost));
  TA_HIP(h, hipMemset(h->d_err, 0, sizeof(bits)));
  if (bits & ta::ERRBIT_CTX) return fail(h, TA_ERR_CTX_RANGE, "a context id is outside [0, N)");
  if (bits & ta::ERRBIT_UNSORTED) return fail(h, TA_ERR_UNSORTED, "timestamps decrease within a rank");
  if (bits & ta::ERRBIT_OVERFLOW) return fail(h, TA_ERR_ITER_OVERFLOW, "a rank has more iterations than n_iters");
  if (bits & ta::ERRBIT_OFFSETS) return fail(h, TA_ERR_INVALID_ARG, "inconsistent offsets or placement ids");
  return TA_OK;
}

ta_status ta_set_tree(ta_handle h, int32_t n_nodes, const int32_t *parent_host) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (n_nodes <= 0 || !parent_host) return fail(h, TA_ERR_INVALID_ARG, "empty tree");
  if (n_nodes > ta::MAX_NODES) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many CCT nodes");
  if (h->live_plans > 0)
    return fail(h, TA_ERR_STATE, "batch plans use the current tree: destroy them first");
  std::vector<int32_t> tin, tout;
  ta_status st = build_tree(h, n_nodes, parent_host, tin, tout);
  if (st) return st;
  DeviceGuard dg(h->device);
  h->N = n_nodes;
  h->parent.assign(parent_host, parent_host + n_nodes);
  h->tin = std::move(tin);
  h->tout = std::move(tout);
  h->marker = -1;
  h->G = 0;
  h->regions.clear();
  free_pruned(h);
  return upload_tables(h);
}

ta_status ta_set_regions(ta_handle h, int32_t marker_node, int32_t n_regions,
                         const int32_t *region_nodes_host) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (h->live_plans > 0)
    return fail(h, TA_ERR_STATE, "batch plans use the current regions: destroy them first");
  if (marker_node < 0 || marker_node >= h->N) return fail(h, TA_ERR_INVALID_ARG, "marker out of range");
  if (n_regions < 1 || n_regions > ta::MAX_REGIONS || !region_nodes_host)
    return fail(h, TA_ERR_INVALID_ARG, "n_regions must be in [1, 256]");
  std::vector<int32_t> regs(region_nodes_host, region_nodes_host + n_regions);
  std::vector<char> seen(h->N, 0);
  for (int32_t v : regs) {
    if (v < 0 || v >= h->N) return fail(h, TA_ERR_INVALID_ARG, "region node out of range");
    if (seen[v]) return fail(h, TA_ERR_INVALID_ARG, "duplicate region node");
    seen[v] = 1;
  }
  DeviceGuard dg(h->device);
  h->marker = marker_node;
  h->G = n_regions;
  h->regions = std::move(regs);
  return upload_tables(h);
}

ta_status ta_callpath(ta_handle h, int32_t leaf, int32_t *path_host, int32_t cap, int32_t *len) {
  if (!h || !len) return TA_ERR_INVALID_ARG;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (leaf < 0 || leaf >= h->N) return fail(h, TA_ERR_INVALID_ARG, "leaf out of range");
  if (cap > 0 && !path_host) return fail(h, TA_ERR_INVALID_ARG, "path NULL");
  int32_t n = 0;
  for (int32_t v = leaf; v != -1; v = h->parent[v]) {
    if (n < cap) path_host[n] = v;
    n++;
  }
  *len = n;
  return TA_OK;
}

ta_status ta_attribute(ta_handle h, const ta_traces *t, int64_t *excl, int64_t *incl, void *stream) {
  ta_seg_out o{};
  o.excl = excl;
  o.incl = incl;
  if (!excl && !incl) return fail(h, TA_ERR_INVALID_ARG, "excl and incl are both NULL");
  return run_segment(h, t, 0, &o, stream, true, false);
}

ta_status ta_segment(ta_handle h, const ta_traces *t, int32_t n_iters, int64_t *tensor,
                     int32_t *iters_found, int64_t *outside, void *stream) {
  ta_seg_out o{};
  o.tensor = tensor;
  o.iters_found = iters_found;
  o.outside = outside;
  if (!tensor || !iters_found) return fail(h, TA_ERR_INVALID_ARG, "tensor and iters_found are required");
  return run_segment(h, t, n_iters, &o, stream, false, true);
}

ta_status ta_attribute_segment(ta_handle h, const ta_traces *t, int32_t n_iters,
                               const ta_seg_out *out, void *stream) {
  return run_segment(h, t, n_iters, out, stream, true, true);
}

namespace {

// Argument checks shared by ta_imbalance and ta_imbalance_noalloc.
ta_status imbalance_args(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                         int32_t n_regions, const int32_t *iters_found, const int64_t *rank_sum,
                         const uint64_t *rank_sumsq, const int64_t *span, int32_t ddof,
                         const ta_imbalance_out *o) {
  if (!o) return fail(h, TA_ERR_INVALID_ARG, "outputs NULL");
  if (n_ranks < 0 || n_iters < 1 || n_regions < 1 || ddof < 0)
    return fail(h, TA_ERR_INVALID_ARG, "bad sizes or ddof");
  if (n_ranks > 0 && !tensor) return fail(h, TA_ERR_INVALID_ARG, "tensor NULL");
  if ((double)n_iters * n_regions > 2e9 || (double)n_ranks * n_iters * n_regions > 4e18)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "tensor too large");
  const void *ptrs[] = {tensor, iters_found, rank_sum, rank_sumsq, span, o->mean, o->std,
                        o->max_minus_mean, o->min, o->max, o->avg_mean, o->avg_max,
                        o->savings_per_iter, o->total_savings, o->balance_ratio, o->cv_across,
                        o->cv_within, o->share, o->potential_speedup};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  return TA_OK;
}

ta_status imbalance_launch(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                           int32_t n_regions, const int32_t *iters_found, const int64_t *rank_sum,
                           const uint64_t *rank_sumsq, const int64_t *span, int32_t ddof,
                           double t_app_ns, const ta_imbalance_out *o, void *ws, size_t ws_bytes,
                           void *stream) {
  const bool need_rs = !rank_sum || !rank_sumsq;
  ta::ImbArgs a{};
  a.T = tensor;
  a.R = n_ranks;
  a.I = n_iters;
  a.G = n_regions;
  a.it = iters_found;
  a.rank_sum = need_rs ? nullptr : rank_sum;
  a.rank_sumsq = need_rs ? nullptr : rank_sumsq;
  a.span = span;
  a.ddof = ddof;
  a.t_app = t_app_ns;
  a.o = *o;
  hipError_t e = ta::launch_imbalance(a, ws, ws_bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "imbalance launch");
  return TA_OK;
}

}  // namespace

ta_status ta_imbalance(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                       int32_t n_regions, const int32_t *iters_found, const int64_t *rank_sum,
                       const uint64_t *rank_sumsq, const int64_t *span, int32_t ddof,
                       double t_app_ns, const ta_imbalance_out *o, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta_status st = imbalance_args(h, tensor, n_ranks, n_iters, n_regions, iters_found, rank_sum,
                                rank_sumsq, span, ddof, o);
  if (st) return st;
  const bool need_rs = !rank_sum || !rank_sumsq;
  DeviceGuard dg(h->device);
  st = ensure_ws(h, ta::imbalance_ws_bytes(n_ranks, n_iters, n_regions, need_rs));
  if (st) return st;
  return imbalance_launch(h, tensor, n_ranks, n_iters, n_regions, iters_found, rank_sum,
                          rank_sumsq, span, ddof, t_app_ns, o, h->ws, h->ws_bytes, stream);
}

ta_status ta_imbalance_noalloc(ta_handle h, const int64_t *tensor, int64_t n_ranks,
                               int32_t n_iters, int32_t n_regions, const int32_t *iters_found,
                               const int64_t *rank_sum, const uint64_t *rank_sumsq,
                               const int64_t *span, int32_t ddof, double t_app_ns,
                               const ta_imbalance_out *o, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta_status st = imbalance_args(h, tensor, n_ranks, n_iters, n_regions, iters_found, rank_sum,
                                rank_sumsq, span, ddof, o);
  if (st) return st;
  const bool need_rs = !rank_sum || !rank_sumsq;
  const size_t need = ta::imbalance_ws_bytes(n_ranks, n_iters, n_regions, need_rs);
  if (need > (size_t)TA_NOALLOC_SCRATCH_BYTES)
    return fail(h, TA_ERR_SIZE_OVERFLOW,
                "ta_imbalance_noalloc needs " + std::to_string(need) +
                    " bytes of workspace, above its static scratch of " +
                    std::to_string((size_t)TA_NOALLOC_SCRATCH_BYTES) +
                    " bytes (pass rank_sum and rank_sumsq, or call ta_imbalance)");
  void *ws = nullptr;
  st = scratch_address(h, &ws);
  if (st) return st;
  DeviceGuard dg(h->device);
  return imbalance_launch(h, tensor, n_ranks, n_iters, n_regions, iters_found, rank_sum,
                          rank_sumsq, span, ddof, t_app_ns, o, ws,
                          (size_t)TA_NOALLOC_SCRATCH_BYTES, stream);
}

ta_status ta_outliers(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                      int32_t n_regions, const int32_t *iters_found, int32_t mode, int32_t kind,
                      double tau, double *rank_score, uint8_t *rank_flag, int64_t *n_flagged,
                      double *region_score, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (n_ranks < 0 || n_iters < 1 || n_regions < 1) return fail(h, TA_ERR_INVALID_ARG, "bad sizes");
  if ((mode != TA_SCAN_FULL && mode != TA_SCAN_TOTALS) || (kind != TA_SCORE_MAD && kind != TA_SCORE_Z))
    return fail(h, TA_ERR_INVALID_ARG, "bad mode or kind");
  if (!(tau >= 0.0)) return fail(h, TA_ERR_INVALID_ARG, "tau must be >= 0");
  if (n_ranks > 0 && (!tensor || !rank_score || !rank_flag))
    return fail(h, TA_ERR_INVALID_ARG, "tensor, rank_score and rank_flag are required");
  if ((double)n_iters * n_regions > 4194240.0 || (double)n_ranks * n_iters * n_regions > 4e18)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "n_iters * n_regions above 4,194,240 or tensor too large");
  const void *ptrs[] = {tensor, iters_found, rank_score, rank_flag, n_flagged, region_score};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  ta_status st = ensure_ws(h, ta::outliers_ws_bytes(n_ranks, n_iters, n_regions, mode, kind));
  if (st) return st;
  ta::OutArgs a{};
  a.T = tensor;
  a.R = n_ranks;
  a.I = n_iters;
  a.G = n_regions;
  a.it = iters_found;
  a.mode = mode;
  a.kind = kind;
  a.tau = tau;
  a.rank_score = rank_score;
  a.rank_flag = rank_flag;
  a.n_flagged = n_flagged;
  a.region_score = region_score;
  hipError_t e = ta::launch_outliers(a, h->ws, h->ws_bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "outliers launch");
  return TA_OK;
}

ta_status ta_topology_aggregate(ta_handle h, const double *rank_score, const uint8_t *rank_flag,
                                int64_t n_ranks, const int32_t *rank_node,
                                const int32_t *node_rack, const int32_t *node_chassis,
                                int32_t n_nodes, int32_t n_racks, int32_t n_chassis,
                                int64_t *flagged_per_rack, double *max_per_rack,
                                double *mean_per_rack, int64_t *flagged_per_chassis,
                                double *max_per_chassis, double *mean_per_chassis,
                                void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (n_ranks < 0 || n_nodes < 1 || n_racks < 1 || n_chassis < 1)
    return fail(h, TA_ERR_INVALID_ARG, "bad sizes");
  if (n_ranks > 0 && (!rank_score || !rank_flag || !rank_node))
    return fail(h, TA_ERR_INVALID_ARG, "rank arrays NULL");
  if (!node_rack || !node_chassis) return fail(h, TA_ERR_INVALID_ARG, "node maps NULL");
  const void *ptrs[] = {rank_score, rank_flag, rank_node, node_rack, node_chassis,
                        flagged_per_rack, max_per_rack, mean_per_rack, flagged_per_chassis,
                        max_per_chassis, mean_per_chassis};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  ta::TopoArgs a{};
  a.score = rank_score;
  a.flag = rank_flag;
  a.R = n_ranks;
  a.rank_node = rank_node;
  a.node_rack = node_rack;
  a.node_chassis = node_chassis;
  a.n_nodes = n_nodes;
  a.n_racks = n_racks;
  a.n_chassis = n_chassis;
  a.fl_rack = flagged_per_rack;
  a.mx_rack = max_per_rack;
  a.mn_rack = mean_per_rack;
  a.fl_ch = flagged_per_chassis;
  a.mx_ch = max_per_chassis;
  a.mn_ch = mean_per_chassis;
  a.err = h->d_err;
  hipError_t e = ta::launch_topology(a, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "topology launch");
  return TA_OK;
}

ta_status ta_summary(ta_handle h, const int64_t *excl, int64_t n_ranks, int64_t *sum_excl,
                     int64_t *sum_incl, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (n_ranks < 0) return fail(h, TA_ERR_INVALID_ARG, "negative n_ranks");
  if (!sum_excl) return fail(h, TA_ERR_INVALID_ARG, "sum_excl is required");
  if (n_ranks > 0 && !excl) return fail(h, TA_ERR_INVALID_ARG, "excl NULL");
  if ((double)n_ranks * h->N > 4e18) return fail(h, TA_ERR_SIZE_OVERFLOW, "profiles too large");
  const void *ptrs[] = {excl, sum_excl, sum_incl};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  ta_status st = ensure_ws(h, ta::subtree_sums_ws_bytes(h->N));
  if (st) return st;
  hipError_t e = ta::launch_summary(excl, n_ranks, h->N, h->d_tin_tout, sum_excl, sum_incl, h->ws,
                                    device_cus(h->device), (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "summary launch");
  return TA_OK;
}

ta_status ta_prune(ta_handle h, const int64_t *sum_excl, const int64_t *sum_incl, double fraction,
                   int32_t *kept, int32_t *n_kept, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (!sum_excl || !sum_incl || !kept || !n_kept)
    return fail(h, TA_ERR_INVALID_ARG, "sum_excl, sum_incl, kept and n_kept are required");
  if (!(fraction >= 0.0)) return fail(h, TA_ERR_INVALID_ARG, "fraction must be >= 0");
  const void *ptrs[] = {sum_excl, sum_incl, kept, n_kept};
  for (const void *p : ptrs)
    if (!aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  hipError_t e = ta::launch_prune(sum_excl, sum_incl, h->N, fraction, kept, n_kept,
                                  (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "prune launch");
  return TA_OK;
}

ta_status ta_set_pruned(ta_handle h, int32_t n_kept, const int32_t *kept_host) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (n_kept < 1 || n_kept > h->N || !kept_host)
    return fail(h, TA_ERR_INVALID_ARG, "n_kept must be in [1, N]");
  std::vector<int32_t> kept(kept_host, kept_host + n_kept);
  std::vector<char> seen(h->N, 0);
  for (int32_t v : kept) {
    if (v < 0 || v >= h->N) return fail(h, TA_ERR_INVALID_ARG, "kept node out of range");
    if (seen[v]) return fail(h, TA_ERR_INVALID_ARG, "duplicate kept node");
    seen[v] = 1;
  }
  DeviceGuard dg(h->device);
  // Kernels still queued may read the previous tables.
  TA_HIP(h, hipDeviceSynchronize());
  return upload_pruned(h, kept);
}

ta_status ta_pruned_profiles(ta_handle h, const int64_t *excl, int64_t n_ranks, int64_t *p_excl,
                             int64_t *p_incl, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->K <= 0) return fail(h, TA_ERR_STATE, "ta_set_pruned has not been called");
  if (h->N > ta::MAX_NODES_ATTR)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "pruned profiles support at most 8192 CCT nodes");
  if (n_ranks < 0) return fail(h, TA_ERR_INVALID_ARG, "negative n_ranks");
  if (n_ranks > 0 && !p_excl && !p_incl) return fail(h, TA_ERR_INVALID_ARG, "no output requested");
  if (n_ranks > 0 && !excl) return fail(h, TA_ERR_INVALID_ARG, "excl NULL");
  if ((double)n_ranks * h->N > 4e18) return fail(h, TA_ERR_SIZE_OVERFLOW, "profiles too large");
  const void *ptrs[] = {excl, p_excl, p_incl};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  hipError_t e = ta::launch_pruned_profiles(excl, n_ranks, h->N, h->d_tin_tout, h->d_kq, h->K,
                                            h->d_kpar, p_excl, p_incl, device_cus(h->device),
                                            (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "pruned profiles launch");
  return TA_OK;
}

ta_status ta_tensor_inclusive(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                              int64_t *out, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (h->G <= 0 || !h->d_rt) return fail(h, TA_ERR_STATE, "ta_set_regions has not been called");
  if (n_ranks < 0 || n_iters < 1) return fail(h, TA_ERR_INVALID_ARG, "bad sizes");
  if ((double)n_ranks * n_iters * h->G > 4e18)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "tensor too large");
  if (n_ranks > 0 && (!tensor || !out)) return fail(h, TA_ERR_INVALID_ARG, "tensor and out are required");
  if ((tensor && !aligned16(tensor)) || (out && !aligned16(out)))
    return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  if (n_ranks > 0 && tensor != out) {
    const uint64_t bytes = (uint64_t)n_ranks * (uint64_t)n_iters * (uint64_t)h->G * 8u;
    const uintptr_t a = (uintptr_t)tensor, b = (uintptr_t)out;
    if (a < b + bytes && b < a + bytes)
      return fail(h, TA_ERR_INVALID_ARG, "out overlaps tensor without being equal to it");
  }
  DeviceGuard dg(h->device);
  hipError_t e = ta::launch_tensor_inclusive(tensor, n_ranks * n_iters, h->G, h->d_rt, out,
                                             device_cus(h->device), (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "tensor inclusive launch");
  return TA_OK;
}

ta_status ta_window_profile(ta_handle h, const ta_traces *t, const int32_t *rank_ids, int64_t n_sel,
                            int64_t t0, int64_t t1, int64_t *excl, int64_t *incl, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta_status st = check_traces(h, t);
  if (st) return st;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (t1 < t0) return fail(h, TA_ERR_INVALID_ARG, "t1 must be >= t0");
  if (!excl) return fail(h, TA_ERR_INVALID_ARG, "excl is required");
  if (rank_ids && n_sel < 0) return fail(h, TA_ERR_INVALID_ARG, "negative n_sel");
  const void *ptrs[] = {rank_ids, excl, incl};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  const int64_t n = rank_ids ? n_sel : t->n_ranks;
  DeviceGuard dg(h->device);
  st = ensure_ws(h, ta::window_ws_bytes(h->N, n));
  if (st) return st;
  hipError_t e = ta::launch_window_profile(t->offsets, t->ts, t->ctx, t->n_ranks, t->n_events, rank_ids,
                                           n, h->N,
                                           h->d_tin_tout, t0, t1, excl, incl, h->ws, h->d_err,
                                           device_cus(h->device), (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "window profile launch");
  return TA_OK;
}

ta_status ta_sparse_profiles(ta_handle h, const ta_traces *t, int64_t *counts, int32_t *node_ids,
                             int64_t *excl, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta_status st = check_traces(h, t);
  if (st) return st;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (t->n_ranks > 0 && !counts) return fail(h, TA_ERR_INVALID_ARG, "counts is required");
  if (t->n_events > 0 && (!node_ids || !excl))
    return fail(h, TA_ERR_INVALID_ARG, "node_ids and excl are required");
  const void *ptrs[] = {counts, node_ids, excl};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  hipError_t e = ta::launch_sparse_profiles(t->offsets, t->ts, t->ctx, t->n_ranks, t->n_events, h->N,
                                            counts, node_ids,
                                            excl, h->d_err, device_cus(h->device), (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "sparse profiles launch");
  return TA_OK;
}

namespace {

ta_status node_model_args(ta_handle h, const ta_traces *t, int32_t n_iters, ta::NodeModelArgs *m) {
  ta_status st = check_traces(h, t);
  if (st) return st;
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (h->marker < 0) return fail(h, TA_ERR_STATE, "ta_set_regions (the marker) has not been called");
  if (n_iters < 1) return fail(h, TA_ERR_INVALID_ARG, "n_iters must be >= 1");
  if ((double)t->n_ranks * (double)n_iters > 4e18)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "n_ranks * n_iters too large");
  m->off = t->offsets;
  m->ts = t->ts;
  m->ctx = t->ctx;
  m->R = t->n_ranks;
  m->E = t->n_events;
  m->I = n_iters;
  m->N = h->N;
  m->info = h->d_info;
  m->ptab = h->d_ptab;
  m->err = h->d_err;
  return TA_OK;
}

}  // namespace

ta_status ta_node_model_count(ta_handle h, const ta_traces *t, int32_t n_iters, int64_t *row_start,
                              int32_t *iters_found, int64_t *row_off_x, int64_t *row_off_i,
                              void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta::NodeModelArgs m{};
  ta_status st = node_model_args(h, t, n_iters, &m);
  if (st) return st;
  if (!row_off_x || !row_off_i || (t->n_ranks > 0 && (!row_start || !iters_found)))
    return fail(h, TA_ERR_INVALID_ARG, "row_start, iters_found, row_off_x and row_off_i are required");
  const void *ptrs[] = {row_start, iters_found, row_off_x, row_off_i};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  m.row_start = row_start;
  m.iters_found = iters_found;
  m.row_off_x = row_off_x;
  m.row_off_i = row_off_i;
  DeviceGuard dg(h->device);
  const int cus = device_cus(h->device);
  st = ensure_ws(h, ta::node_model_ws_bytes(m.R, m.I, m.E, m.N, cus));
  if (st) return st;
  hipError_t e = ta::launch_node_model(m, false, h->ws, cus, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "node model count launch");
  return TA_OK;
}

ta_status ta_node_model_fill(ta_handle h, const ta_traces *t, int32_t n_iters,
                             const int64_t *row_start, const int32_t *iters_found,
                             const int64_t *row_off_x, int32_t *node_x, int64_t *val_x,
                             const int64_t *row_off_i, int32_t *node_i, int64_t *val_i,
                             void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  ta::NodeModelArgs m{};
  ta_status st = node_model_args(h, t, n_iters, &m);
  if (st) return st;
  if (t->n_ranks > 0 && (!row_start || !iters_found))
    return fail(h, TA_ERR_INVALID_ARG, "row_start and iters_found are required");
  if ((node_x || val_x) && (!node_x || !val_x || !row_off_x))
    return fail(h, TA_ERR_INVALID_ARG, "node_x, val_x and row_off_x go together");
  if ((node_i || val_i) && (!node_i || !val_i || !row_off_i))
    return fail(h, TA_ERR_INVALID_ARG, "node_i, val_i and row_off_i go together");
  if (!node_x && !node_i) return fail(h, TA_ERR_INVALID_ARG, "no output requested");
  const void *ptrs[] = {row_start, iters_found, row_off_x, node_x, val_x, row_off_i, node_i, val_i};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  m.row_start = const_cast<int64_t *>(row_start);
  m.iters_found = const_cast<int32_t *>(iters_found);
  m.row_off_x = const_cast<int64_t *>(row_off_x);
  m.row_off_i = const_cast<int64_t *>(row_off_i);
  m.node_x = node_x;
  m.val_x = val_x;
  m.node_i = node_i;
  m.val_i = val_i;
  DeviceGuard dg(h->device);
  const int cus = device_cus(h->device);
  st = ensure_ws(h, ta::node_model_ws_bytes(m.R, m.I, m.E, m.N, cus));
  if (st) return st;
  hipError_t e = ta::launch_node_model(m, true, h->ws, cus, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "node model fill launch");
  return TA_OK;
}

ta_status ta_kmeans(ta_handle h, const int64_t *X, int64_t n_rows, int32_t n_features, int32_t k,
                    const double *init, int32_t max_iter, int32_t *labels, double *centroids,
                    int64_t *counts, int32_t *n_iter, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (n_rows < 0 || n_features < 1 || k < 1 || max_iter < 1)
    return fail(h, TA_ERR_INVALID_ARG, "bad sizes or max_iter");
  if (k > 32 || n_features > 256 || k * n_features > 5632 || n_rows >= ((int64_t)1 << 31))
    return fail(h, TA_ERR_SIZE_OVERFLOW, "k <= 32, n_features <= 256, k * n_features <= 5632 and "
                                         "n_rows < 2^31 are supported");
  if (!init || !centroids || (n_rows > 0 && (!X || !labels)))
    return fail(h, TA_ERR_INVALID_ARG, "X, init, labels and centroids are required");
  const void *ptrs[] = {X, init, labels, centroids, counts, n_iter};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  ta_status st = ensure_ws(h, ta::kmeans_ws_bytes(k, n_features, n_rows));
  if (st) return st;
  hipError_t e = ta::launch_kmeans(X, n_rows, n_features, k, init, max_iter, labels, centroids,
                                   counts, n_iter, h->ws, device_cus(h->device), (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "kmeans launch");
  return TA_OK;
}

ta_status ta_dbscan1d(ta_handle h, const int64_t *x, int64_t n_rows, int64_t eps, int64_t min_pts,
                      int32_t *labels, int32_t *n_clusters, uint8_t *core, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (n_rows < 0 || eps < 0 || min_pts < 1)
    return fail(h, TA_ERR_INVALID_ARG, "n_rows >= 0, eps >= 0 and min_pts >= 1 are required");
  if (n_rows >= ((int64_t)1 << 31)) return fail(h, TA_ERR_SIZE_OVERFLOW, "n_rows < 2^31 is supported");
  if (!n_clusters || (n_rows > 0 && (!x || !labels)))
    return fail(h, TA_ERR_INVALID_ARG, "x, labels and n_clusters are required");
  const void *ptrs[] = {x, labels, n_clusters, core};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  ta_status st = ensure_ws(h, ta::dbscan_ws_bytes(n_rows));
  if (st) return st;
  hipError_t e = ta::launch_dbscan1d(x, n_rows, eps, min_pts, labels, n_clusters, core, h->ws,
                                     device_cus(h->device), (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "dbscan launch");
  return TA_OK;
}

ta_status ta_node_intersections(ta_handle h, const int32_t *labels, const int32_t *rank_node,
                                int64_t n_ranks, int32_t n_nodes, int32_t k, int64_t *pair,
                                int32_t *node_clusters, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (n_ranks < 0 || n_nodes < 1 || k < 1) return fail(h, TA_ERR_INVALID_ARG, "bad sizes");
  if (k > 64) return fail(h, TA_ERR_SIZE_OVERFLOW, "at most 64 clusters are supported");
  if (!pair || (n_ranks > 0 && (!labels || !rank_node)))
    return fail(h, TA_ERR_INVALID_ARG, "labels, rank_node and pair are required");
  const void *ptrs[] = {labels, rank_node, pair, node_clusters};
  for (const void *p : ptrs)
    if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  DeviceGuard dg(h->device);
  ta_status st = ensure_ws(h, ta::node_intersections_ws_bytes(n_nodes));
  if (st) return st;
  hipError_t e = ta::launch_node_intersections(labels, rank_node, n_ranks, n_nodes, k, pair,
                                               node_clusters, h->ws, h->d_err, device_cus(h->device),
                                               (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "node intersections launch");
  return TA_OK;
}

namespace {

// Places event record nodes right before and right after the fused pass (the
// graph's one root node): root -> fused -> record -> the fused pass's former
// dependents, so the graph stays one chain there.  Best effort: without them
// the plan still works and ta_plan_launch_timed reports an error.
void add_timing_nodes(ta_plan p) {
  size_t nr = 0;
  if (hipGraphGetRootNodes(p->graph, nullptr, &nr) != hipSuccess || nr != 1) return;
  hipGraphNode_t fused = nullptr;
  if (hipGraphGetRootNodes(p->graph, &fused, &nr) != hipSuccess) return;
  hipGraphNodeType ty;
  if (hipGraphNodeGetType(fused, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) return;
  size_t nd = 0;
  if (hipGraphNodeGetDependentNodes(fused, nullptr, &nd) != hipSuccess) return;
  std::vector<hipGraphNode_t> deps(nd);
  if (nd && hipGraphNodeGetDependentNodes(fused, deps.data(), &nd) != hipSuccess) return;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return;
  }
  p->slots.push_back(e0);
  p->slots.push_back(e1);
  hipGraphNode_t r0 = nullptr, r1 = nullptr;
  if (hipGraphAddEventRecordNode(&r1, p->graph, &fused, 1, e1) != hipSuccess) return;
  // every former dependent waits on the record node first, then drops the
  // direct edge, so no dependent ever loses its wait on the fused pass
  for (hipGraphNode_t d : deps) {
    if (hipGraphAddDependencies(p->graph, &r1, &d, 1) != hipSuccess) return;
    hipGraphRemoveDependencies(p->graph, &fused, &d, 1);
  }
  if (hipGraphAddEventRecordNode(&r0, p->graph, nullptr, 0, e0) != hipSuccess) return;
  if (hipGraphAddDependencies(p->graph, &r0, &fused, 1) != hipSuccess) return;
  p->rec[0] = r0;
  p->rec[1] = r1;
}

}  // namespace

ta_status ta_plan_create(ta_handle h, const ta_traces *t, const int64_t *offsets_host,
                         const ta_batch_desc *d, ta_plan *out, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!out || !d || !offsets_host) return fail(h, TA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  SegLaunch L;
  ta_status st = prepare_segment(h, t, d->n_iters, &d->seg, true, true, &L);
  if (st) return st;
  if (t->n_ranks == 0) return fail(h, TA_ERR_INVALID_ARG, "empty batch");
  if ((d->with_imbalance || d->with_outliers) && !L.seg)
    return fail(h, TA_ERR_INVALID_ARG, "statistics stages need the tensor");
  if (d->with_outliers) {
    if ((d->outlier_mode != TA_SCAN_FULL && d->outlier_mode != TA_SCAN_TOTALS) ||
        (d->outlier_kind != TA_SCORE_MAD && d->outlier_kind != TA_SCORE_Z) || !(d->tau >= 0.0))
      return fail(h, TA_ERR_INVALID_ARG, "bad outlier mode, kind or tau");
    if (!d->rank_score || !d->rank_flag) return fail(h, TA_ERR_INVALID_ARG, "rank_score/rank_flag NULL");
    const void *ptrs[] = {d->rank_score, d->rank_flag, d->n_flagged, d->region_score};
    for (const void *p : ptrs)
      if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  }
  if (d->with_imbalance) {
    if (d->ddof < 0) return fail(h, TA_ERR_INVALID_ARG, "ddof < 0");
    const void *ptrs[] = {d->imb.mean, d->imb.std, d->imb.max_minus_mean, d->imb.min, d->imb.max,
                          d->imb.avg_mean, d->imb.avg_max, d->imb.savings_per_iter,
                          d->imb.total_savings, d->imb.balance_ratio, d->imb.cv_across,
                          d->imb.cv_within, d->imb.share, d->imb.potential_speedup};
    for (const void *p : ptrs)
      if (p && !aligned16(p)) return fail(h, TA_ERR_INVALID_ARG, "array not 16-byte aligned");
  }
  const int64_t R = t->n_ranks;
  for (int64_t r = 0; r < R; r++)
    if (offsets_host[r + 1] < offsets_host[r]) return fail(h, TA_ERR_INVALID_ARG, "offsets_host decreasing");
  DeviceGuard dg(h->device);
  ta_plan p = new (std::nothrow) ta_plan_s();
  if (!p) return TA_ERR_OOM;
  p->h = h;
  // Longest ranks first; ties by rank id.
  std::vector<int32_t> order(R);
  for (int64_t r = 0; r < R; r++) order[r] = (int32_t)r;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return offsets_host[x + 1] - offsets_host[x] > offsets_host[y + 1] - offsets_host[y];
  });
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMalloc(&p->d_order, (size_t)R * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_order, order.data(), (size_t)R * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    return hipfail(h, e, "plan order upload");
  }
  L.a.order = p->d_order;
  const int I = d->n_iters, G = h->G;
  // With both the imbalance statistics and the FULL outlier scan, the scan's
  // transpose also writes the imbalance column partials (one read of the
  // tensor instead of two); the two workspaces then sit side by side.
  const bool need_rs = !d->seg.rank_sum || !d->seg.rank_sumsq;
  const bool fuse = d->with_imbalance && d->with_outliers && d->outlier_mode == TA_SCAN_FULL &&
                    R > 0 && (int64_t)I * G > 0;
  const int rc_t = fuse ? ta::transpose_groups(R) : 0;
  const size_t ws_out =
      d->with_outliers ? (ta::outliers_ws_bytes(R, I, G, d->outlier_mode, d->outlier_kind) + 255) / 256 * 256 : 0;
  const size_t ws_imb = d->with_imbalance ? ta::imbalance_ws_bytes(R, I, G, need_rs, rc_t) : 0;
  size_t ws = fuse ? ws_out + ws_imb : std::max(ws_out, ws_imb);
  if (ws && hipMalloc(&p->ws, ws) != hipSuccess) {
    p->ws = nullptr;
    plan_free(p);
    return fail(h, TA_ERR_OOM, "plan workspace allocation failed");
  }

  // Launch shape: default, cached, or measured on this batch.
  const int cus = device_cus(h->device);
  ta::SegShape best;
  float best_ms = 0.f;
  st = choose_shape(h, L, d->autotune, s, &best, &best_ms);
  if (st) {
    plan_free(p);
    return st;
  }
  p->shape = best;
  p->tuned_ms = best_ms;

  // One eager pass (sets kernel attributes outside capture), then capture.
  const int grid = grid_for(L, best, cus);
  e = ta::launch_segment(L.a, L.attr, L.seg, best, grid, L.lds, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess && fuse) e = hipStreamCreateWithFlags(&p->cap2, hipStreamNonBlocking);
  if (e == hipSuccess && fuse) e = hipEventCreateWithFlags(&p->ev_stats, hipEventDisableTiming);
  if (e == hipSuccess && fuse) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
  const bool split = d->with_outliers && d->outlier_mode == TA_SCAN_FULL && R > 0 && (int64_t)I * G > 0;
  if (e == hipSuccess && split) e = hipStreamCreateWithFlags(&p->cap3, hipStreamNonBlocking);
  for (int k = 0; k < 10 && split; k++)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_scan[k], hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    plan_free(p);
    return hipfail(h, e, "plan capture start");
  }
  hipError_t le = ta::launch_segment(L.a, L.attr, L.seg, best, grid, L.lds, p->cap);
  void *imb_ws = fuse ? (void *)((char *)p->ws + ws_out) : p->ws;
  if (le == hipSuccess && d->with_imbalance && !fuse) {
    ta::ImbArgs ia{};
    ia.T = d->seg.tensor;
    ia.R = R;
    ia.I = I;
    ia.G = G;
    ia.it = d->seg.iters_found;
    ia.rank_sum = (d->seg.rank_sum && d->seg.rank_sumsq) ? d->seg.rank_sum : nullptr;
    ia.rank_sumsq = (d->seg.rank_sum && d->seg.rank_sumsq) ? d->seg.rank_sumsq : nullptr;
    ia.span = d->seg.span;
    ia.ddof = d->ddof;
    ia.t_app = d->t_app_ns;
    ia.o = d->imb;
    le = ta::launch_imbalance(ia, imb_ws, fuse ? ws_imb : ws, p->cap, rc_t);
  }
  if (le == hipSuccess && d->with_outliers) {
    ta::OutArgs oa{};
    oa.T = d->seg.tensor;
    oa.R = R;
    oa.I = I;
    oa.G = G;
    oa.it = d->seg.iters_found;
    oa.mode = d->outlier_mode;
    oa.kind = d->outlier_kind;
    oa.tau = d->tau;
    oa.rank_score = d->rank_score;
    oa.rank_flag = d->rank_flag;
    oa.n_flagged = d->n_flagged;
    oa.region_score = d->region_score;
    if (fuse) {
      oa.stats = ta::imbalance_partials(imb_ws, R, I, G, need_rs, rc_t);
      oa.stats_ready = p->ev_stats;
    }
    if (split) {
      oa.side = p->cap3;
      for (int k = 0; k < 10; k++) oa.ev[k] = p->ev_scan[k];
    }
    le = ta::launch_outliers(oa, p->ws, fuse ? ws_out : ws, p->cap);
  }
  // The imbalance epilogue needs only the partials: on the second capture
  // stream it runs beside the rest of the scan, joined before the graph ends.
  if (le == hipSuccess && d->with_imbalance && fuse) le = hipStreamWaitEvent(p->cap2, p->ev_stats, 0);
  if (le == hipSuccess && d->with_imbalance && fuse) {
    ta::ImbArgs ia{};
    ia.T = d->seg.tensor;
    ia.R = R;
    ia.I = I;
    ia.G = G;
    ia.it = d->seg.iters_found;
    ia.rank_sum = (d->seg.rank_sum && d->seg.rank_sumsq) ? d->seg.rank_sum : nullptr;
    ia.rank_sumsq = (d->seg.rank_sum && d->seg.rank_sumsq) ? d->seg.rank_sumsq : nullptr;
    ia.span = d->seg.span;
    ia.ddof = d->ddof;
    ia.t_app = d->t_app_ns;
    ia.o = d->imb;
    le = ta::launch_imbalance(ia, imb_ws, ws_imb, p->cap2, rc_t);
    if (le == hipSuccess) le = hipEventRecord(p->ev_join, p->cap2);
    if (le == hipSuccess) le = hipStreamWaitEvent(p->cap, p->ev_join, 0);
  }
  e = hipStreamEndCapture(p->cap, &p->graph);
  if (le != hipSuccess || e != hipSuccess) {
    plan_free(p);
    return hipfail(h, le != hipSuccess ? le : e, "plan capture");
  }
  add_timing_nodes(p);
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_free(p);
    return hipfail(h, e, "graph instantiate");
  }
  *out = p;
  h->live_plans++;
  return TA_OK;
}

ta_status ta_batch_create(ta_handle h, int32_t n_requests, const ta_request *requests, double tau,
                          int32_t autotune, ta_plan *out, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!out || !requests || n_requests < 1) return fail(h, TA_ERR_INVALID_ARG, "no requests");
  *out = nullptr;
  if (n_requests > (1 << 20)) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many requests");
  if (!(tau >= 0.0)) return fail(h, TA_ERR_INVALID_ARG, "tau must be >= 0");
  if (autotune < 0 || autotune > 2) return fail(h, TA_ERR_INVALID_ARG, "autotune must be 0, 1 or 2");
  if (h->N <= 0) return fail(h, TA_ERR_STATE, "ta_set_tree has not been called");
  if (h->G <= 0) return fail(h, TA_ERR_STATE, "ta_set_regions has not been called");
  if (h->N > ta::MAX_NODES_ATTR)
    return fail(h, TA_ERR_SIZE_OVERFLOW, "attribution supports at most 8192 CCT nodes");
  const int G = h->G;
  std::vector<ta::SegReq> qs(n_requests);
  std::vector<int64_t> tasks, lens;
  int64_t E_total = 0;
  size_t ws = 0;
  for (int32_t q = 0; q < n_requests; q++) {
    const ta_request &rq = requests[q];
    ta_status st = check_traces(h, &rq.traces);
    if (st) return st;
    const int64_t R = rq.traces.n_ranks;
    if (R > 0 && !rq.offsets_host) return fail(h, TA_ERR_INVALID_ARG, "offsets_host NULL");
    if (rq.n_iters < 1) return fail(h, TA_ERR_INVALID_ARG, "n_iters must be >= 1");
    if ((double)R * rq.n_iters * G > 4e18 || (double)rq.n_iters * G > 4194240.0)
      return fail(h, TA_ERR_SIZE_OVERFLOW, "tensor too large");
    if (!rq.seg.tensor || !rq.seg.iters_found)
      return fail(h, TA_ERR_INVALID_ARG, "each request needs tensor and iters_found");
    const ta_seg_out &o = rq.seg;
    const void *ptrs[] = {o.tensor, o.iters_found, o.outside, o.span, o.rank_sum, o.rank_sumsq,
                          o.excl, o.incl, rq.rank_score, rq.rank_flag, rq.n_flagged};
    for (const void *ptr : ptrs)
      if (ptr && !aligned16(ptr)) return fail(h, TA_ERR_INVALID_ARG, "output not 16-byte aligned");
    if ((rq.rank_score == nullptr) != (rq.rank_flag == nullptr))
      return fail(h, TA_ERR_INVALID_ARG, "rank_score and rank_flag go together");
    for (int64_t r = 0; r < R; r++)
      if (rq.offsets_host[r + 1] < rq.offsets_host[r])
        return fail(h, TA_ERR_INVALID_ARG, "offsets_host decreasing");
    qs[q] = ta::SegReq{rq.traces.offsets, rq.traces.ts, rq.traces.ctx, rq.traces.n_events,
                       rq.n_iters, o.tensor, o.iters_found, o.outside, o.span, o.rank_sum,
                       o.rank_sumsq, o.excl, o.incl};
    for (int64_t r = 0; r < R; r++) {
      tasks.push_back(((int64_t)q << 32) | r);
      lens.push_back(rq.offsets_host[r + 1] - rq.offsets_host[r]);
    }
    E_total += rq.traces.n_events;
    if (rq.rank_score)
      ws = std::max(ws, ta::outliers_ws_bytes(R, rq.n_iters, G, TA_SCAN_FULL, TA_SCORE_MAD));
  }
  // Longest ranks of every request first; ties in request, then rank order.
  std::vector<int64_t> idx(tasks.size());
  for (size_t k = 0; k < idx.size(); k++) idx[k] = (int64_t)k;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return lens[x] > lens[y]; });
  std::vector<int64_t> sorted(tasks.size());
  for (size_t k = 0; k < idx.size(); k++) sorted[k] = tasks[idx[k]];

  DeviceGuard dg(h->device);
  ta_plan p = new (std::nothrow) ta_plan_s();
  if (!p) return TA_ERR_OOM;
  p->h = h;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMalloc(&p->d_reqs, qs.size() * sizeof(ta::SegReq));
  if (e == hipSuccess && !sorted.empty()) e = hipMalloc(&p->d_tasks, sorted.size() * sizeof(int64_t));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_reqs, qs.data(), qs.size() * sizeof(ta::SegReq), hipMemcpyHostToDevice);
  if (e == hipSuccess && !sorted.empty())
    e = hipMemcpy(p->d_tasks, sorted.data(), sorted.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && ws) e = hipMalloc(&p->ws, ws);
  if (e != hipSuccess) {
    plan_free(p);
    return hipfail(h, e, "batch upload");
  }
  SegLaunch L;
  int W = 2, lw = 1;
  L.lds = ta::segment_lds_bytes(h->N, G, true, true, &W, &lw);
  if (L.lds > 160 * 1024) {
    plan_free(p);
    return fail(h, TA_ERR_SIZE_OVERFLOW, "call-path tables exceed LDS");
  }
  ta::SegArgs &a = L.a;
  a.R = (int64_t)sorted.size();
  a.E = E_total;
  a.info = h->d_info;
  a.tin_tout = h->d_tin_tout;
  a.N = h->N;
  a.G = G;
  a.I = -n_requests;  // distinguishes mixed batches in the autotune cache key
  a.W = W;
  a.log2W = lw;
  a.err = h->d_err;
  a.reqs = p->d_reqs;
  a.tasks = p->d_tasks;
  L.attr = L.seg = true;

  ta::SegShape best = default_shape(L);
  float best_ms = 0.f;
  if (a.R > 0) {
    ta_status st = choose_shape(h, L, autotune, s, &best, &best_ms);
    if (st) {
      plan_free(p);
      return st;
    }
  }
  p->shape = best;
  p->tuned_ms = best_ms;
  const int cus = device_cus(h->device);
  const int grid = grid_for(L, best, cus);
  e = hipSuccess;
  if (a.R > 0) e = ta::launch_segment(a, true, true, best, grid, L.lds, s);  // kernel attributes
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    plan_free(p);
    return hipfail(h, e, "batch capture start");
  }
  hipError_t le = hipSuccess;
  if (a.R > 0) le = ta::launch_segment(a, true, true, best, grid, L.lds, p->cap);
  for (int32_t q = 0; q < n_requests && le == hipSuccess; q++) {
    const ta_request &rq = requests[q];
    if (!rq.rank_score) continue;
    ta::OutArgs oa{};
    oa.T = rq.seg.tensor;
    oa.R = rq.traces.n_ranks;
    oa.I = rq.n_iters;
    oa.G = G;
    oa.it = rq.seg.iters_found;
    oa.mode = TA_SCAN_FULL;
    oa.kind = TA_SCORE_MAD;
    oa.tau = tau;
    oa.rank_score = rq.rank_score;
    oa.rank_flag = rq.rank_flag;
    oa.n_flagged = rq.n_flagged;
    oa.region_score = nullptr;
    le = ta::launch_outliers(oa, p->ws, ws, p->cap);
  }
  e = hipStreamEndCapture(p->cap, &p->graph);
  if (le != hipSuccess || e != hipSuccess) {
    plan_free(p);
    return hipfail(h, le != hipSuccess ? le : e, "batch capture");
  }
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_free(p);
    return hipfail(h, e, "graph instantiate");
  }
  *out = p;
  h->live_plans++;
  return TA_OK;
}

ta_status ta_plan_launch(ta_plan p, void *stream) {
  if (!p || !p->exec) return TA_ERR_INVALID_ARG;
  DeviceGuard dg(p->h->device);
  hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(p->h, e, "graph launch");
  return TA_OK;
}

ta_status ta_plan_launch_timed(ta_plan p, int32_t slot, void *stream) {
  if (!p) return TA_ERR_INVALID_ARG;
  ta_handle h = p->h;
  if (slot < 0 || slot >= 4096) return fail(h, TA_ERR_INVALID_ARG, "slot must be in [0, 4096)");
  if (!p->rec[0] || !p->rec[1])
    return fail(h, TA_ERR_STATE, "this plan's graph has no timing nodes");
  DeviceGuard dg(h->device);
  while ((int64_t)p->slots.size() < 2 * ((int64_t)slot + 2)) {
    hipEvent_t ev = nullptr;
    TA_HIP(h, hipEventCreate(&ev));
    p->slots.push_back(ev);
  }
  // slot k uses events 2k + 2 and 2k + 3 (the first pair belongs to the capture)
  TA_HIP(h, hipGraphExecEventRecordNodeSetEvent(p->exec, p->rec[0], p->slots[2 * slot + 2]));
  TA_HIP(h, hipGraphExecEventRecordNodeSetEvent(p->exec, p->rec[1], p->slots[2 * slot + 3]));
  TA_HIP(h, hipGraphLaunch(p->exec, (hipStream_t)stream));
  return TA_OK;
}

ta_status ta_plan_segment_ms(ta_plan p, int32_t slot, float *ms) {
  if (!p || !ms) return TA_ERR_INVALID_ARG;
  ta_handle h = p->h;
  if (slot < 0 || 2 * ((int64_t)slot + 2) > (int64_t)p->slots.size())
    return fail(h, TA_ERR_INVALID_ARG, "slot was never launched");
  DeviceGuard dg(h->device);
  TA_HIP(h, hipEventSynchronize(p->slots[2 * slot + 3]));
  TA_HIP(h, hipEventElapsedTime(ms, p->slots[2 * slot + 2], p->slots[2 * slot + 3]));
  return TA_OK;
}

ta_status ta_plan_info(ta_plan p, int32_t *threads, int32_t *events_per_thread,
                       int32_t *nontemporal, int32_t *wgs_per_cu, float *tuned_ms) {
  if (!p) return TA_ERR_INVALID_ARG;
  if (threads) *threads = p->shape.threads;
  if (events_per_thread) *events_per_thread = p->shape.ept;
  if (nontemporal) *nontemporal = p->shape.nontemporal ? 1 : 0;
  if (wgs_per_cu) *wgs_per_cu = p->shape.wgs_per_cu;
  if (tuned_ms) *tuned_ms = p->tuned_ms;
  return TA_OK;
}

ta_status ta_plan_destroy(ta_plan p) {
  if (!p) return TA_ERR_INVALID_ARG;
  DeviceGuard dg(p->h->device);
  hipStreamSynchronize(p->cap);
  p->h->live_plans--;
  plan_free(p);
  return TA_OK;
}

}  // extern "C"

// ---- learned pre-screen ---------------------------------------------------

namespace {

ta_status ae_check(ta_handle h, const int64_t *tensor, int64_t R, int32_t I, int32_t G) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (G != ta::AE_IN) return fail(h, TA_ERR_INVALID_ARG, "the pre-screen needs n_regions == 64");
  if (R < 0 || I < 1 || (R > 0 && !tensor) || !aligned16(tensor))
    return fail(h, TA_ERR_INVALID_ARG, "bad tensor or sizes");
  if (R >= ((int64_t)1 << 31)) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many ranks");
  return TA_OK;
}

ta_status ae_ensure(ta_handle h) {
  if (h->ae.w) return TA_OK;
  hipError_t e = ta::ae_alloc(h->ae);
  if (e != hipSuccess) {
    ta::ae_free(h->ae);
    return fail(h, TA_ERR_OOM, "autoencoder state allocation failed");
  }
  return TA_OK;
}

uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

__global__ void fill_f32(float *p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void f64_to_f32(const double *a, float *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

constexpr uint32_t AE_MAGIC = 0x45414154u;  // "TAAE"
struct AeHeader {
  uint32_t magic, version;
  int64_t step;
  int32_t ready, normed;
  float threshold;
  int32_t pad;  // score kind
};

}  // namespace

extern "C" {

ta_status ta_ae_init(ta_handle h, uint64_t seed, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  DeviceGuard dg(h->device);
  ta_status st = ae_ensure(h);
  if (st) return st;
  hipError_t e = ta::launch_ae_init(h->ae, seed, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "ae init");
  h->ae.ready = true;
  return TA_OK;
}

ta_status ta_ae_fit_norm(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                         int32_t n_regions, const int32_t *iters_found, int32_t reset,
                         void *stream) {
  ta_status st = ae_check(h, tensor, n_ranks, n_iters, n_regions);
  if (st) return st;
  DeviceGuard dg(h->device);
  st = ae_ensure(h);
  if (!st) st = ensure_ws(h, ta::ae_norm_ws_bytes(n_ranks));
  if (st) return st;
  if (!h->ae.normed) reset = 1;
  hipError_t e = ta::launch_ae_norm(h->ae, tensor, n_ranks, n_iters, iters_found, reset != 0, h->ws,
                                    h->ws_bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "ae norm");
  h->ae.normed = true;
  return TA_OK;
}

ta_status ta_ae_rows(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                     int32_t n_regions, const int32_t *iters_found, float *rows,
                     int64_t *n_rows_host, void *stream) {
  ta_status st = ae_check(h, tensor, n_ranks, n_iters, n_regions);
  if (st) return st;
  if (!n_rows_host) return fail(h, TA_ERR_INVALID_ARG, "n_rows_host NULL");
  if (rows && !aligned16(rows)) return fail(h, TA_ERR_INVALID_ARG, "rows not 16-byte aligned");
  if (!h->ae.normed) return fail(h, TA_ERR_STATE, "ta_ae_fit_norm has not been called");
  DeviceGuard dg(h->device);
  st = ensure_ws(h, ta::ae_rows_ws_bytes(n_ranks));
  if (st) return st;
  int64_t n = 0;
  hipError_t e = ta::launch_ae_rows(h->ae, tensor, n_ranks, n_iters, iters_found, rows, &n, h->ws,
                                    h->ws_bytes, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "ae rows");
  *n_rows_host = n;
  return TA_OK;
}

ta_status ta_ae_grad(ta_handle h, const float *rows, int64_t n_rows, float input_noise,
                     uint64_t noise_key, float *grad, float *loss, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!rows || n_rows < 1 || !grad || !aligned16(rows) || !aligned16(grad) || !aligned16(loss))
    return fail(h, TA_ERR_INVALID_ARG, "bad rows or outputs");
  if (!(input_noise >= 0.f) || input_noise > 1e6f)
    return fail(h, TA_ERR_INVALID_ARG, "input_noise must be in [0, 1e6]");
  if (!h->ae.ready) return fail(h, TA_ERR_STATE, "ta_ae_init has not been called");
  if (n_rows > ((int64_t)1 << 31)) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many rows");
  DeviceGuard dg(h->device);
  hipError_t e = ta::launch_ae_step(h->ae, rows, n_rows, 0, (int)n_rows, 1, 0, 0.f, false,
                                    input_noise, noise_key, (hipStream_t)stream, grad, loss);
  if (e != hipSuccess) return hipfail(h, e, "ae grad");
  return TA_OK;
}

ta_status ta_ae_grad_f32(ta_handle h, const float *rows, int64_t n_rows, float input_noise,
                         uint64_t noise_key, float *grad, float *loss, void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!rows || n_rows < 1 || !grad || !aligned16(rows) || !aligned16(grad) || !aligned16(loss))
    return fail(h, TA_ERR_INVALID_ARG, "bad rows or outputs");
  if (!(input_noise >= 0.f) || input_noise > 1e6f)
    return fail(h, TA_ERR_INVALID_ARG, "input_noise must be in [0, 1e6]");
  if (!h->ae.ready) return fail(h, TA_ERR_STATE, "ta_ae_init has not been called");
  if (n_rows > ((int64_t)1 << 31)) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many rows");
  DeviceGuard dg(h->device);
  hipError_t e = ta::launch_ae_grad_f32(h->ae, rows, n_rows, input_noise, noise_key,
                                        (hipStream_t)stream, grad, loss);
  if (e != hipSuccess) return hipfail(h, e, "ae grad f32");
  return TA_OK;
}

ta_status ta_ae_train(ta_handle h, const float *rows, int64_t n_rows, int32_t epochs, int32_t batch,
                      float lr, float input_noise, uint64_t shuffle_seed, float *epoch_loss,
                      void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!rows || n_rows < 1 || epochs < 0 || batch < 1 || !(lr > 0.f) || !aligned16(rows) ||
      !aligned16(epoch_loss) || !(input_noise >= 0.f) || input_noise > 1e6f)
    return fail(h, TA_ERR_INVALID_ARG, "bad training arguments");
  if (!h->ae.ready) return fail(h, TA_ERR_STATE, "ta_ae_init has not been called");
  if (n_rows > ((int64_t)1 << 32)) return fail(h, TA_ERR_SIZE_OVERFLOW, "too many rows");
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)stream;
  uint64_t rs = shuffle_seed;
  uint64_t ns = shuffle_seed ^ 0x5851F42D4C957F2Dull;  // noise keys: a stream of their own
  if (epoch_loss && epochs > 0)
    hipLaunchKernelGGL(fill_f32, dim3((epochs + 255) / 256), dim3(256), 0, s, epoch_loss, epochs, 0.f);
  const uint64_t n = (uint64_t)n_rows;
  for (int32_t ep = 0; ep < epochs; ep++) {
    // Row order of the epoch: k -> (a*k + c) mod n with gcd(a, n) = 1.
    uint64_t a = 1, c = 0;
    if (n > 1) {
      do {
        a = 1 + splitmix(rs) % (n - 1);
      } while (gcd64(a, n) != 1);
      c = splitmix(rs) % n;
    }
    for (int64_t k0 = 0; k0 < n_rows; k0 += batch) {
      const uint64_t nkey = splitmix(ns);
      const int64_t bv = std::min<int64_t>(batch, n_rows - k0);
      // two launches per step: the gradient partials, then their sum, the
      // Adam step and the epoch-loss add
      hipError_t e = ta::launch_ae_step(h->ae, rows, n_rows, k0, batch, a, c, lr, true, input_noise,
                                        nkey, s, nullptr, nullptr, epoch_loss ? epoch_loss + ep : nullptr,
                                        (float)((double)bv / (double)n_rows));
      if (e != hipSuccess) return hipfail(h, e, "ae step");
    }
  }
  const hipError_t le = hipGetLastError();
  return le == hipSuccess ? TA_OK : hipfail(h, le, "ae train");
}

ta_status ta_ae_set_score_kind(ta_handle h, int32_t kind) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (kind != TA_AE_SCORE_ERROR && kind != TA_AE_SCORE_RESIDUAL && kind != TA_AE_SCORE_RESIDUAL_Z)
    return fail(h, TA_ERR_INVALID_ARG, "unknown score kind");
  h->ae.score_kind = kind;
  return TA_OK;
}

ta_status ta_ae_get_score_kind(ta_handle h, int32_t *kind_host) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!kind_host) return fail(h, TA_ERR_INVALID_ARG, "kind_host is NULL");
  *kind_host = h->ae.score_kind;
  return TA_OK;
}

ta_status ta_ae_score(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                      int32_t n_regions, const int32_t *iters_found, float *rank_score,
                      void *stream) {
  ta_status st = ae_check(h, tensor, n_ranks, n_iters, n_regions);
  if (st) return st;
  if (!rank_score || !aligned16(rank_score)) return fail(h, TA_ERR_INVALID_ARG, "rank_score");
  if (!h->ae.ready || !h->ae.normed) return fail(h, TA_ERR_STATE, "network not initialised and fitted");
  DeviceGuard dg(h->device);
  st = ensure_ws(h, ta::ae_score_ws_bytes(n_ranks));
  if (st) return st;
  hipError_t e = ta::launch_ae_score(h->ae, tensor, n_ranks, n_iters, iters_found, rank_score, h->ws,
                                     h->ws_bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(h, e, "ae score");
  return TA_OK;
}

ta_status ta_ae_calibrate(ta_handle h, const float *rank_score, int64_t n_ranks, double quantile,
                          void *stream) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!rank_score || n_ranks < 1 || !(quantile >= 0.0 && quantile <= 1.0))
    return fail(h, TA_ERR_INVALID_ARG, "bad calibration arguments");
  DeviceGuard dg(h->device);
  std::vector<float> v(n_ranks);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(v.data(), rank_score, (size_t)n_ranks * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hipfail(h, e, "calibrate");
  std::sort(v.begin(), v.end());
  const int64_t idx = std::min<int64_t>(n_ranks - 1, (int64_t)(quantile * (double)(n_ranks - 1) + 0.5));
  h->ae.threshold = v[idx];
  return TA_OK;
}

ta_status ta_ae_get_threshold(ta_handle h, float *threshold_host) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!threshold_host) return fail(h, TA_ERR_INVALID_ARG, "threshold_host is NULL");
  *threshold_host = h->ae.threshold;
  return TA_OK;
}

ta_status ta_prescreen(ta_handle h, const int64_t *tensor, int64_t n_ranks, int32_t n_iters,
                       int32_t n_regions, const int32_t *iters_found, int64_t k,
                       int32_t *topk_ranks, float *rank_score, int32_t *used_fallback_host,
                       void *stream) {
  ta_status st = ae_check(h, tensor, n_ranks, n_iters, n_regions);
  if (st) return st;
  if (k < 1 || k > n_ranks || !topk_ranks || !used_fallback_host || !aligned16(topk_ranks) ||
      !aligned16(rank_score))
    return fail(h, TA_ERR_INVALID_ARG, "bad k or outputs");
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t fl = ((size_t)n_ranks * 4 + 255) & ~(size_t)255;
  const size_t need = fl + 256 + std::max(ta::ae_score_ws_bytes(n_ranks),
                                          ta::outliers_ws_bytes(n_ranks, n_iters, n_regions,
                                                                TA_SCAN_FULL, TA_SCORE_MAD) +
                                              ((size_t)n_ranks * 9 + 1024));
  st = ensure_ws(h, need);
  if (st) return st;
  float *score = rank_score ? rank_score : (float *)h->ws;
  int32_t *above = (int32_t *)((char *)h->ws + fl);
  bool fallback = !(h->ae.ready && h->ae.normed);
  hipError_t e = hipSuccess;
  if (!fallback) {
    char *aws = (char *)h->ws + fl + 256;
    e = ta::launch_ae_score(h->ae, tensor, n_ranks, n_iters, iters_found, score, aws,
                            h->ws_bytes - (fl + 256), s);
    const float thr = h->ae.threshold >= 0.f ? h->ae.threshold : 3.4e38f;
    if (e == hipSuccess) e = ta::launch_topk(score, n_ranks, k, topk_ranks, above, thr, s);
    if (e == hipSuccess && !h->pin) e = hipHostMalloc((void **)&h->pin, sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemcpyAsync(h->pin, above, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hipfail(h, e, "prescreen");
    const int32_t n_above = *h->pin;
    fallback = h->ae.threshold >= 0.f && n_above > k;
  }
  *used_fallback_host = fallback ? 1 : 0;
  if (!fallback) return TA_OK;
  // Exact scan, then the k ranks with the largest exact scores.
  char *base = (char *)h->ws + fl + 256;
  double *xs = (double *)base;
  uint8_t *xf = (uint8_t *)(base + (((size_t)n_ranks * 8 + 255) & ~(size_t)255));
  char *ows = (char *)xf + (((size_t)n_ranks + 255) & ~(size_t)255);
  ta::OutArgs oa{};
  oa.T = tensor;
  oa.R = n_ranks;
  oa.I = n_iters;
  oa.G = n_regions;
  oa.it = iters_found;
  oa.mode = TA_SCAN_FULL;
  oa.kind = TA_SCORE_MAD;
  oa.tau = 3.5;
  oa.rank_score = xs;
  oa.rank_flag = xf;
  const size_t ows_bytes = h->ws_bytes - (size_t)(ows - (char *)h->ws);
  e = ta::launch_outliers(oa, ows, ows_bytes, s);
  float *xs32 = (float *)h->ws;
  if (e == hipSuccess)
    hipLaunchKernelGGL(f64_to_f32, dim3((unsigned)((n_ranks + 255) / 256)), dim3(256), 0, s, xs, xs32,
                       n_ranks);
  if (e == hipSuccess) e = ta::launch_topk(xs32, n_ranks, k, topk_ranks, above, 3.4e38f, s);
  if (e != hipSuccess) return hipfail(h, e, "prescreen fallback");
  return TA_OK;
}

size_t ta_ae_state_bytes(void) {
  return sizeof(AeHeader) + (size_t)ta::AE_NP * 4 * 3 + 64 * 4 * 2;
}

ta_status ta_ae_get_state(ta_handle h, void *buf_host, size_t bytes) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!buf_host || bytes < ta_ae_state_bytes()) return fail(h, TA_ERR_INVALID_ARG, "buffer too small");
  if (!h->ae.w) return fail(h, TA_ERR_STATE, "no network state");
  DeviceGuard dg(h->device);
  TA_HIP(h, hipDeviceSynchronize());
  char *p = (char *)buf_host;
  AeHeader hd{AE_MAGIC, 1u, h->ae.step, h->ae.ready, h->ae.normed, h->ae.threshold,
              h->ae.score_kind};
  memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  TA_HIP(h, hipMemcpy(p, h->ae.w, ta::AE_NP * 4, hipMemcpyDeviceToHost));
  p += ta::AE_NP * 4;
  TA_HIP(h, hipMemcpy(p, h->ae.m, ta::AE_NP * 4, hipMemcpyDeviceToHost));
  p += ta::AE_NP * 4;
  TA_HIP(h, hipMemcpy(p, h->ae.v, ta::AE_NP * 4, hipMemcpyDeviceToHost));
  p += ta::AE_NP * 4;
  TA_HIP(h, hipMemcpy(p, h->ae.mu, 64 * 4, hipMemcpyDeviceToHost));
  p += 64 * 4;
  TA_HIP(h, hipMemcpy(p, h->ae.isd, 64 * 4, hipMemcpyDeviceToHost));
  return TA_OK;
}

ta_status ta_ae_set_state(ta_handle h, const void *buf_host, size_t bytes) {
  if (!h) return TA_ERR_INVALID_ARG;
  if (!buf_host || bytes < ta_ae_state_bytes()) return fail(h, TA_ERR_INVALID_ARG, "buffer too small");
  AeHeader hd;
  memcpy(&hd, buf_host, sizeof hd);
  if (hd.magic != AE_MAGIC || hd.version != 1u) return fail(h, TA_ERR_INVALID_ARG, "not a network state");
  DeviceGuard dg(h->device);
  ta_status st = ae_ensure(h);
  if (st) return st;
  TA_HIP(h, hipDeviceSynchronize());
  const char *p = (const char *)buf_host + sizeof hd;
  std::vector<uint16_t> wb(ta::AE_NW);
  const float *wf = (const float *)p;
  for (int i = 0; i < ta::AE_NW; i++) {
    uint32_t u;
    memcpy(&u, wf + i, 4);
    wb[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
  TA_HIP(h, hipMemcpy(h->ae.w, p, ta::AE_NP * 4, hipMemcpyHostToDevice));
  TA_HIP(h, hipMemcpy(h->ae.wb, wb.data(), ta::AE_NW * 2, hipMemcpyHostToDevice));
  p += ta::AE_NP * 4;
  TA_HIP(h, hipMemcpy(h->ae.m, p, ta::AE_NP * 4, hipMemcpyHostToDevice));
  p += ta::AE_NP * 4;
  TA_HIP(h, hipMemcpy(h->ae.v, p, ta::AE_NP * 4, hipMemcpyHostToDevice));
  p += ta::AE_NP * 4;
  TA_HIP(h, hipMemcpy(h->ae.mu, p, 64 * 4, hipMemcpyHostToDevice));
  p += 64 * 4;
  TA_HIP(h, hipMemcpy(h->ae.isd, p, 64 * 4, hipMemcpyHostToDevice));
  h->ae.step = hd.step;
  h->ae.ready = hd.ready != 0;
  h->ae.normed = hd.normed != 0;
  h->ae.threshold = hd.threshold;
  h->ae.score_kind = (hd.pad == TA_AE_SCORE_RESIDUAL || hd.pad == TA_AE_SCORE_RESIDUAL_Z)
                         ? (int)hd.pad : TA_AE_SCORE_ERROR;
  return TA_OK;
}

}  // extern "C"
