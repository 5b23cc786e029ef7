// libsfkde host runtime: the C ABI declared in include/sfkde.h.
//
// Owns contexts (device, allocator, budget, streams, batch slots), trees
// (device-resident index built by build.hip), the batched evaluation
// pipeline (eval.hip), the in-box / MBE pipeline (mbe.hip), tickets and the
// serving loop. No exception crosses the ABI; every entry point validates
// its arguments before any device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sfk_internal.h"
#include "sfkde.h"

namespace sfk {
hipError_t launch_trilinear_mean(const float4* pts, int64_t n_b, const float* grid,
                                 const double* lo, const double* hi, const int32_t* res,
                                 double* pden, double* block_sums, double* ave, hipStream_t s);
}

namespace {

thread_local std::string g_tls_err;

constexpr int kNumSlots = 4;
constexpr int kStagingRing = 8;
constexpr int kDefaultChunkLeaves = 256;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

// Workspace of sfk_eval_roi_noalloc: one static array per device, held until
// the process ends. In host code `scratch` names a host-side stand-in, not
// device memory: host code uses only the address hipGetSymbolAddress gives
// for the current device (noalloc_scratch_of).
static __device__ __align__(256) unsigned char scratch[SFK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// The device address of this device's scratch array, taken once per device
// with that device current (nullptr if the runtime cannot give it).
unsigned char* noalloc_scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_scratch_dev[device] = (unsigned char*)p;
  }
  return g_scratch_dev[device];
}

}  // namespace

struct Workspace {
  // hdr_rois = [BatchHdr][RoiDev x capacity]: staged by one host-to-device copy
  DevBuf hdr_rois, coords, tile_cnt, tile_fit, tile_done, leaf_off, partial_off, chunk_off, leaves,
      item_tile, partials, claims, plan_tmp, roi_leaves, roi_nl, tile_slots;
  uint64_t gen = 0;  // bumped whenever a buffer is replaced (captured graphs go stale)
  void* claims_cleared = nullptr;  // the claims buffer whose error word is zeroed
  int64_t want_leaf_cap = 0;
  int64_t want_partial_cap = 0;
  // last enqueued use of the buffers: a buffer that must grow waits for it
  hipEvent_t last_use = nullptr;
  bool last_use_valid = false;
};

struct Staging {
  char* host = nullptr;  // pinned: per group [BatchHdr][RoiDev...]
  size_t cap = 0;        // bytes
  uint64_t gen = 0;      // bumped when `host` is replaced (captured copies go stale)
  BatchHdr* hdr_host = nullptr;  // pinned readback of the last group's header,
                                 // followed by the workspace's error word
  int32_t* err_host() const { return (int32_t*)((char*)hdr_host + sizeof(BatchHdr)); }
  hipEvent_t ev = nullptr;
  bool ev_valid = false;
  bool stats_pending = false;  // ev follows a header readback not yet absorbed
};

// A captured batch pipeline of one slot, replayed while its key and the
// workspace generation are unchanged and the batch fits its capacities.
struct GraphCache {
  bool valid = false;
  TileShape ts{0, 0, 0};
  int kk = 0, pp = 0, ch = 0, nm = 0;
  bool cnt = false;
  bool interleave = false;  // captured with one-wave-per-tile evaluation grids
  sfk_tree tree = nullptr;
  uint64_t gen = 0, st_gen = 0;
  int64_t tiles_cap = 0, rois_cap = 0, coords_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct Slot {
  GraphCache gc;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Workspace ws;
  Staging st;
  bool busy = false;
  int64_t ticket = -1;
  size_t batch_bytes = 0;  // grid bytes admitted for the running batch
};

struct Ticket {
  int state = 0;  // 0 pending, 1 running, 2 done, 3 cancelled, 4 failed
  int slot = -1;
  sfk_tree tree = nullptr;
  std::vector<sfk_roi> rois;
  sfk_status status = SFK_OK;
};

enum ProfKind { PK_TILE_COUNT = 0, PK_PLAN, PK_TILE_FILL, PK_EVAL, PK_BUILD, PK_KNN, PK_N };

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  BatchHdr* hdr_dev;  // eval records: header to read totals from (may be null)
};

struct sfk_ctx_s {
  int device = 0;
  bool prof_on = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[PK_N] = {0};
  int64_t prof_evals = 0, prof_builds = 0, prof_last_leaves = 0, prof_last_items = 0;
  sfk_allocator alloc{};
  bool use_alloc = false;
  size_t budget = 0;
  size_t ws_bytes = 0;    // workspace held (bounded by budget)
  size_t tree_bytes = 0;  // trees held
  std::string err;
  int n_cu = 256;
  sfk_eval_opts opts{};
  Slot slots[kNumSlots];
  std::map<int64_t, Ticket> tickets;
  std::deque<int64_t> pending;
  int64_t next_ticket = 1;
  // one-ROI stream-ordered path
  Workspace direct_ws;
  Staging direct_st[kStagingRing];
  int direct_next = 0;
  hipEvent_t direct_last = nullptr;
  bool direct_last_valid = false;
  hipStream_t direct_last_stream = nullptr;
  // autotuner table: key -> tile shape id, and the summed time of every
  // shape over the key's samples (ms; index = shape id, 0 unused)
  std::map<int, int> tune;
  std::map<int, std::vector<double>> tune_cost;
  std::string arch;  // gcnArchName of the device (the tuning table's key)
  // sfk_eval_roi_noalloc: this device's copy of the static scratch array
  // (nullptr if its address could not be taken), a pinned staging ring set
  // up at creation, and the stream order of consecutive calls
  int32_t debug_poison = 0;  // sfk_debug_poison: test-only bits staged in every batch header
  bool serve_interleave = false;  // sfk_serve: evaluation grids of one wave per tile
  unsigned char* na_scratch = nullptr;
  char* na_host[kStagingRing] = {};
  hipEvent_t na_ev[kStagingRing] = {};
  bool na_ev_valid[kStagingRing] = {};
  int na_next = 0;
  hipEvent_t na_last = nullptr;
  bool na_last_valid = false;
  hipStream_t na_last_stream = nullptr;
};

struct sfk_tree_s {
  sfk_ctx ctx = nullptr;
  int64_t n = 0;
  double bbox[6] = {0, 0, 0, 0, 0, 0};
  int32_t n_leaves = 0, n_levels = 0;
  int32_t level_off[SFK_MAX_LEVELS] = {0};
  int32_t level_cnt[SFK_MAX_LEVELS] = {0};
  DevBuf pts, perm, nodes, node_ih, h2;
  // host copy of the coarse box levels (the finest with at most
  // kHostLevelNodes boxes and those above it), for particle-count estimates
  std::vector<NodeBox> host_nodes;
  int32_t host_level = 0;   // finest level held on the host
  int32_t host_base = 0;    // device node index of host_nodes[0]
  // summed counts of the finest host level's boxes, each counted in the cell
  // of a kEstGrid^3 lattice over the bounding box that holds its centre:
  // est_sat[(i + (G+1) (j + (G+1) k))] = the count in cells below (i, j, k)
  std::vector<double> est_sat;
  int32_t pp_mode = PP_UNIFORM;  // PP_ISO when a per-point bandwidth exists
  int32_t knn_k = 0;
  size_t bytes = 0;
};

namespace {

void set_err(sfk_ctx c, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  g_tls_err = buf;
}

#define SFK_HIP(c, expr)                                                        \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      set_err((c), "%s failed: %s", #expr, hipGetErrorString(e_));              \
      return SFK_E_DEVICE;                                                      \
    }                                                                           \
  } while (0)

#define SFK_TRY(expr)                   \
  do {                                  \
    sfk_status s_ = (expr);             \
    if (s_ != SFK_OK) return s_;        \
  } while (0)

#define SFK_GUARD_BEGIN try {
#define SFK_GUARD_END(c)                                   \
  }                                                        \
  catch (const std::bad_alloc&) {                          \
    set_err((c), "host allocation failed");                \
    return SFK_E_NOMEM;                                    \
  }                                                        \
  catch (...) {                                            \
    set_err((c), "internal error");                        \
    return SFK_E_INTERNAL;                                 \
  }

// ---- profiling events ----

hipEvent_t prof_event(sfk_ctx c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a phase (no-op unless profiling).
struct ProfScope {
  sfk_ctx c;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr;
  BatchHdr* hdr;
  ProfScope(sfk_ctx cc, int k, hipStream_t ss, BatchHdr* h = nullptr) : c(cc), kind(k), s(ss), hdr(h) {
    if (c->prof_on) {
      a = prof_event(c);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->prof_pending.push_back(ProfRec{kind, a, b, hdr});
  }
};

// ---- device memory through the context's allocator ----

void raw_free(sfk_ctx c, void* p, size_t bytes) {
  if (!p) return;
  if (c->use_alloc)
    c->alloc.free(p, bytes, c->alloc.user);
  else
    (void)hipFree(p);
}

void* raw_alloc(sfk_ctx c, size_t bytes) {
  if (c->use_alloc) return c->alloc.alloc(bytes, c->alloc.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

size_t round_bytes(size_t b) { return (b + 255) & ~(size_t)255; }

// Grow-only workspace buffer; before replacing a buffer it waits for the
// workspace's last enqueued use.
sfk_status ws_reserve(sfk_ctx c, Workspace& ws, DevBuf& b, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return SFK_OK;
  if (ws.last_use_valid) SFK_HIP(c, hipEventSynchronize(ws.last_use));
  size_t nb = round_bytes(std::max(bytes, b.bytes + b.bytes / 4));
  if (c->budget && c->ws_bytes - b.bytes + nb > c->budget) {
    nb = round_bytes(bytes);
    if (c->ws_bytes - b.bytes + nb > c->budget) {
      set_err(c, "workspace for %s (%zu bytes) exceeds the device-memory budget", what, nb);
      return SFK_E_BUDGET;
    }
  }
  raw_free(c, b.p, b.bytes);
  c->ws_bytes -= b.bytes;
  b.p = nullptr;
  b.bytes = 0;
  ++ws.gen;
  void* p = raw_alloc(c, nb);
  if (!p) {
    set_err(c, "device allocation of %zu bytes for %s failed", nb, what);
    return SFK_E_NOMEM;
  }
  b.p = p;
  b.bytes = nb;
  c->ws_bytes += nb;
  return SFK_OK;
}

void ws_release(sfk_ctx c, DevBuf& b) {
  if (b.p) {
    raw_free(c, b.p, b.bytes);
    c->ws_bytes -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

sfk_status tree_alloc(sfk_ctx c, sfk_tree t, DevBuf& b, size_t bytes, const char* what) {
  bytes = round_bytes(std::max<size_t>(bytes, 256));
  void* p = raw_alloc(c, bytes);
  if (!p) {
    set_err(c, "device allocation of %zu bytes for %s failed", bytes, what);
    return SFK_E_NOMEM;
  }
  b.p = p;
  b.bytes = bytes;
  c->tree_bytes += bytes;
  t->bytes += bytes;
  return SFK_OK;
}

void tree_free(sfk_ctx c, sfk_tree t, DevBuf& b) {
  if (b.p) {
    raw_free(c, b.p, b.bytes);
    c->tree_bytes -= b.bytes;
    t->bytes -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// Temporary device buffer freed on scope exit (build-time scratch).
struct TmpBuf {
  sfk_ctx c;
  DevBuf b;
  explicit TmpBuf(sfk_ctx cc) : c(cc) {}
  ~TmpBuf() { raw_free(c, b.p, b.bytes); }
  sfk_status get(size_t bytes, const char* what) {
    bytes = round_bytes(std::max<size_t>(bytes, 256));
    b.p = raw_alloc(c, bytes);
    if (!b.p) {
      set_err(c, "device allocation of %zu bytes for %s failed", bytes, what);
      return SFK_E_NOMEM;
    }
    b.bytes = bytes;
    return SFK_OK;
  }
  template <typename T>
  T* as() const { return (T*)b.p; }
};

sfk_status staging_reserve(sfk_ctx c, Staging& st, size_t bytes) {
  if (!st.ev) SFK_HIP(c, hipEventCreateWithFlags(&st.ev, hipEventDisableTiming));
  if (!st.hdr_host) {
    SFK_HIP(c, hipHostMalloc((void**)&st.hdr_host, sizeof(BatchHdr) + 64));
    *st.err_host() = 0;
  }
  if (st.cap >= bytes) return SFK_OK;
  if (st.host) {
    if (st.ev_valid) SFK_HIP(c, hipEventSynchronize(st.ev));
    SFK_HIP(c, hipHostFree(st.host));
    st.host = nullptr;
  }
  const size_t cap = std::max<size_t>(bytes, sizeof(BatchHdr) + 64 * sizeof(RoiDev));
  SFK_HIP(c, hipHostMalloc((void**)&st.host, cap));
  st.cap = cap;
  ++st.gen;
  return SFK_OK;
}

// ---- constants of the kernels (closed forms) ----

double ck_epanechnikov() { return 15.0 / (8.0 * M_PI); }
double ck_gauss_trunc3() {
  // 1 / ((2 pi)^{3/2} P(chi^2_3 < 9)), P = erf(3/sqrt2) - sqrt(2/pi) 3 e^{-9/2}
  const double p = std::erf(3.0 / std::sqrt(2.0)) - std::sqrt(2.0 / M_PI) * 3.0 * std::exp(-4.5);
  return 1.0 / (std::pow(2.0 * M_PI, 1.5) * p);
}

constexpr int kHostLevelNodes = 32768;  // boxes of the finest level kept on the host
constexpr int kNumShapes = SFK_NUM_TILE_SHAPES;  // tile shapes 1..7 of sfk_eval_opts.tile_shape
static_assert(SFK_NUM_TILE_SHAPES == 7, "tile shape table");
constexpr int kBrickShape = 6;  // bricks of kBrick^3 nodes, scatter evaluation
constexpr int kSweepShape = 7;  // particle sweep over the hierarchy's boxes

TileShape shape_of(int id) {
  switch (id) {
    case 2: return TileShape{4, 4, 2};
    case 3: return TileShape{4, 2, 2};
    case 4: return TileShape{2, 2, 2};
    case 5: return TileShape{1, 1, 1};
    case 6: return TileShape{kBrick, kBrick, kBrick};
    case 7: return TileShape{kSweep, kSweep, kSweep};
    default: return TileShape{4, 4, 4};
  }
}

// Bricks evaluate uniform bandwidths only (fixed or ROI-scaled)
bool uniform_bw(const sfk_roi* r) { return r->bw == SFK_BW_FIXED || r->bw == SFK_BW_ROI_SCALED; }

TreeView view_of(sfk_tree t) {
  TreeView tv{};
  tv.pts = (const float4*)t->pts.p;
  tv.pparam = nullptr;
  tv.nodes = (const NodeBox*)t->nodes.p;
  tv.node_ih = (const float4*)t->node_ih.p;
  for (int l = 0; l < SFK_MAX_LEVELS; ++l) {
    tv.level_off[l] = t->level_off[l];
    tv.level_cnt[l] = t->level_cnt[l];
  }
  tv.n_levels = t->n_levels;
  tv.n_leaves = t->n_leaves;
  tv.n = t->n;
  tv.pp_mode = t->pp_mode;
  return tv;
}

void level_layout(int32_t n_leaves, int32_t* off, int32_t* cnt, int32_t* n_levels,
                  int32_t* total) {
  int lv = 0, o = 0;
  if (n_leaves > 0) {
    int c = n_leaves;
    while (true) {
      off[lv] = o;
      cnt[lv] = c;
      o += c;
      ++lv;
      if (c <= SFK_FANOUT) break;
      c = (c + SFK_FANOUT - 1) / SFK_FANOUT;
    }
  }
  for (int l = lv; l < SFK_MAX_LEVELS; ++l) {
    off[l] = o;
    cnt[l] = 0;
  }
  *n_levels = lv;
  *total = o;
}

// Leaf boxes and the box hierarchy of a leaf layout.
// only_if: nullptr, or a device flag that leaves the boxes as they are while 0
// leaves_done: the leaf level is already written (the gather writes it)
sfk_status build_boxes(sfk_ctx c, const float4* pts, int64_t n, int32_t n_leaves,
                       NodeBox* nodes, const int32_t* off, const int32_t* cnt, int n_levels,
                       hipStream_t s, const int32_t* only_if = nullptr,
                       bool leaves_done = false) {
  if (n_levels <= 0) return SFK_OK;
  if (!leaves_done)
    SFK_HIP(c, sfk::launch_leaf_boxes(pts, n, n_leaves, nodes + off[0], only_if, s));
  for (int l = 1; l < n_levels; ++l)
    SFK_HIP(c, sfk::launch_level_boxes(nodes + off[l - 1], cnt[l - 1], nodes + off[l], cnt[l],
                                        only_if, s));
  return SFK_OK;
}

// ---- ROI validation ----

sfk_status validate_roi(sfk_ctx c, sfk_tree t, const sfk_roi* r, int idx) {
  if (!r) {
    set_err(c, "roi %d: NULL descriptor", idx);
    return SFK_E_INVAL;
  }
  if (!r->d_out) {
    set_err(c, "roi %d: d_out is NULL", idx);
    return SFK_E_INVAL;
  }
  int64_t m = 1;
  for (int k = 0; k < 3; ++k) {
    if (!(std::isfinite(r->lo[k]) && std::isfinite(r->hi[k]) && r->hi[k] > r->lo[k])) {
      set_err(c, "roi %d: box axis %d needs finite lo < hi", idx, k);
      return SFK_E_INVAL;
    }
    if (r->res[k] < 2) {
      set_err(c, "roi %d: res[%d] = %d (each must be >= 2)", idx, k, r->res[k]);
      return SFK_E_INVAL;
    }
    m *= r->res[k];
  }
  if (m > (int64_t)1 << 31) {
    set_err(c, "roi %d: grid of %lld nodes exceeds 2^31", idx, (long long)m);
    return SFK_E_INVAL;
  }
  if (r->kernel != SFK_KERNEL_EPANECHNIKOV && r->kernel != SFK_KERNEL_GAUSS_TRUNC3) {
    set_err(c, "roi %d: unknown kernel %d", idx, r->kernel);
    return SFK_E_INVAL;
  }
  if (r->norm != SFK_NORM_PAPER && r->norm != SFK_NORM_COUNT) {
    set_err(c, "roi %d: unknown norm %d", idx, r->norm);
    return SFK_E_INVAL;
  }
  if (r->set != SFK_SET_CLOUD && r->set != SFK_SET_IN_ROI) {
    set_err(c, "roi %d: unknown set %d", idx, r->set);
    return SFK_E_INVAL;
  }
  switch (r->bw) {
    case SFK_BW_FIXED:
      for (int k = 0; k < 3; ++k)
        if (!(r->h[k] > 0.0f) || !std::isfinite(r->h[k])) {
          set_err(c, "roi %d: fixed bandwidth h[%d] must be finite and > 0", idx, k);
          return SFK_E_INVAL;
        }
      break;
    case SFK_BW_ROI_SCALED:
      if (!(r->h[0] > 0.0f) || !std::isfinite(r->h[0])) {
        set_err(c, "roi %d: ROI-scaled bandwidth factor h[0] must be finite and > 0", idx);
        return SFK_E_INVAL;
      }
      break;
    case SFK_BW_PER_POINT:
      if (t && t->pp_mode != PP_ISO && t->n > 0) {
        set_err(c, "roi %d: per-point bandwidth requested but the tree has none "
                   "(build with knn_k > 0 or d_h)", idx);
        return SFK_E_INVAL;
      }
      break;
    case SFK_BW_MBE:
      if (r->kernel != SFK_KERNEL_EPANECHNIKOV) {
        set_err(c, "roi %d: MBE is defined for the Epanechnikov kernel", idx);
        return SFK_E_UNSUPPORTED;
      }
      if (r->set != SFK_SET_IN_ROI) {
        set_err(c, "roi %d: MBE uses the particles inside B (set = SFK_SET_IN_ROI)", idx);
        return SFK_E_INVAL;
      }
      break;
    default:
      set_err(c, "roi %d: unknown bandwidth mode %d", idx, r->bw);
      return SFK_E_INVAL;
  }
  return SFK_OK;
}

sfk_status validate_disjoint_outputs(sfk_ctx c, const sfk_roi* rois, int n) {
  std::vector<std::pair<uintptr_t, uintptr_t>> iv;
  iv.reserve(n);
  for (int i = 0; i < n; ++i) {
    const uintptr_t a = (uintptr_t)rois[i].d_out;
    const uintptr_t m = (uintptr_t)rois[i].res[0] * rois[i].res[1] * rois[i].res[2];
    iv.push_back({a, a + m * sizeof(float)});
  }
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].first < iv[i - 1].second) {
      set_err(c, "output grids of two ROIs overlap");
      return SFK_E_INVAL;
    }
  return SFK_OK;
}

// ---- one group of ROIs through count -> plan -> fill -> evaluate ----

struct GroupRoi {
  const sfk_roi* roi;
  int kk, pp;
  bool count_mode;
  float ih[3];
  float c2;
  double scale;
};

// Nodes per axis one particle's support can span in the particle sweep (the
// kernel's half-width in node steps, rounded outwards as the kernel rounds
// it, with a further 1e-6 margin; the kernel reports a wider span as an
// internal error). 0 for per-particle bandwidths.
int sweep_nm(const GroupRoi& g) {
  if (g.pp != PP_UNIFORM) return 0;
  int nm = 1;
  for (int k = 0; k < 3; ++k) {
    const sfk_roi* r = g.roi;
    const double inv_s = (double)(r->res[k] - 1) / (r->hi[k] - r->lo[k]);
    const double h = std::sqrt((double)g.c2) * inv_s / (double)g.ih[k];
    const double half = h * (1.0 + 1e-9) + 1e-9;
    nm = std::max(nm, (int)std::floor(2.0 * half + 1e-6) + 1);
  }
  return nm;
}

int chunk_leaves_of(sfk_ctx c) {
  return c->opts.chunk_leaves > 0 ? c->opts.chunk_leaves : kDefaultChunkLeaves;
}

// Fill RoiDev descriptors for rois[0..n) and the per-group tile total.
void make_roidev(const GroupRoi* g, size_t n, TileShape ts, RoiDev* out, int64_t* n_tiles,
                 int64_t* n_coords) {
  int64_t tb = 0, co = 0;
  for (size_t i = 0; i < n; ++i) {
    const sfk_roi* r = g[i].roi;
    RoiDev d{};
    for (int k = 0; k < 3; ++k) {
      d.lo[k] = r->lo[k];
      d.hi[k] = r->hi[k];
      d.res[k] = r->res[k];
    }
    d.ntile[0] = (r->res[0] + ts.tx - 1) / ts.tx;
    d.ntile[1] = (r->res[1] + ts.ty - 1) / ts.ty;
    d.ntile[2] = (r->res[2] + ts.tz - 1) / ts.tz;
    d.tile_base = tb;
    for (int k = 0; k < 3; ++k) d.ih[k] = g[i].ih[k];
    d.c2 = g[i].c2;
    d.scale = g[i].scale;
    d.kernel = g[i].kk;
    d.count_mode = g[i].count_mode ? 1 : 0;
    d.coord_off = (int32_t)co;
    d.out = r->d_out;
    d.pp_mode = g[i].pp;
    out[i] = d;
    tb += (int64_t)d.ntile[0] * d.ntile[1] * d.ntile[2];
    co += r->res[0] + r->res[1] + r->res[2];
  }
  *n_tiles = tb;
  *n_coords = co;
}

void make_roidev(const std::vector<GroupRoi>& g, TileShape ts, RoiDev* out, int64_t* n_tiles,
                 int64_t* n_coords) {
  make_roidev(g.data(), g.size(), ts, out, n_tiles, n_coords);
}

struct Caps {
  int64_t leaf_cap, partial_cap, item_cap, tiles_cap, rois_cap, coords_cap;
  int32_t slot_cap;
  int32_t splat;
};

// Leaves the count pass keeps per tile for a tile shape: 16 per node of the
// tile, at least 32 and at most kTileSlotCap (a tile of few nodes meets few
// leaves: 1x1x1 keeps 32, 2x2x2 128, larger tiles 256; 4x4x4 tiles of the
// 10M per-point workload average ~124 leaves, 4x2x2 tiles of dense 1e9-point
// ROIs several hundred).
int32_t slot_cap_of(TileShape ts) {
  if (sfk::is_sweep(ts)) return 32;  // the sweep keeps no per-tile lists
  const int t = ts.tx * ts.ty * ts.tz;
  return std::min(kTileSlotCap, std::max(32, 16 * t));
}

// Reserve every buffer of a group (n_rois descriptors, n_tiles tiles,
// n_coords coordinates; `headroom` > 1 over-allocates so later batches fit a
// captured graph) and report the capacities the buffers actually have.
// The default leaf-list capacity is 4 entries per leaf of the tree (and at
// least 64 per tile), so ROIs of any size over the cloud usually fit at the
// first call; overflowing batches still complete (walk fallback) and grow
// the capacities for the next one.
sfk_status reserve_group(sfk_ctx c, Workspace& ws, TileShape ts, int64_t n_rois, int64_t n_tiles,
                         int64_t n_coords, double headroom, int64_t tree_leaves, Caps* caps) {
  const int CH = chunk_leaves_of(c);
  const int T = ts.tx * ts.ty * ts.tz;
  const int64_t tiles = (int64_t)std::ceil((double)n_tiles * headroom);
  const int64_t nr = std::max<int64_t>(64, (int64_t)std::ceil((double)n_rois * headroom));
  const int64_t nc = std::max<int64_t>(1024, (int64_t)std::ceil((double)n_coords * headroom));
  int64_t leaf_cap = std::max<int64_t>({ws.want_leaf_cap, (int64_t)1 << 20, 64 * tiles,
                                        4 * tree_leaves});
  // partial slots are small (T doubles per chunk): room for twice the
  // chunks the leaf lists hold, so a batch whose lists overflow still splits
  // its heavy tiles over work items (walking per chunk)
  const bool brick = sfk::is_brick(ts);
  const bool sweep = sfk::is_sweep(ts);
  // a brick's partial slot holds its kBrick^3 node sums (32 KB): one per
  // split brick, up to 8192 of them; bricks beyond walk their whole tile in
  // one work item (which needs no slot)
  int64_t partial_cap =
      brick ? std::max<int64_t>(64, std::min<int64_t>(tiles, 8192))
            : std::max<int64_t>({ws.want_partial_cap, (int64_t)1 << 14, tiles / 4,
                                 2 * leaf_cap / CH});
  // the sweep: the node sums of every tile, and the (ROI, box) items of
  // every descriptor the header may hold (two int32 per item)
  const int64_t sweep_boxes = tree_leaves > SFK_FANOUT
                                  ? (tree_leaves + SFK_FANOUT - 1) / SFK_FANOUT
                                  : tree_leaves;
  if (sweep) {
    partial_cap = std::max<int64_t>(1, tiles);
    leaf_cap = std::max<int64_t>(leaf_cap, 2 * nr * std::max<int64_t>(1, sweep_boxes));
  }
  if (c->opts.list_capacity > 0 && !sweep) {
    leaf_cap = c->opts.list_capacity;
    partial_cap = std::max<int64_t>(1, c->opts.list_capacity / CH);
  }
  if (c->opts.partial_capacity > 0 && !sweep) partial_cap = c->opts.partial_capacity;
  SFK_TRY(ws_reserve(c, ws, ws.tile_cnt, sizeof(int32_t) * (size_t)tiles, "tile counts"));
  SFK_TRY(ws_reserve(c, ws, ws.tile_fit, sizeof(int32_t) * (size_t)tiles, "tile flags"));
  SFK_TRY(ws_reserve(c, ws, ws.tile_done, sizeof(int32_t) * (size_t)tiles, "tile counters"));
  const int32_t slot_cap = slot_cap_of(ts);
  SFK_TRY(ws_reserve(c, ws, ws.tile_slots, sizeof(int32_t) * slot_cap * (size_t)tiles,
                     "tile leaf slots"));
  SFK_TRY(ws_reserve(c, ws, ws.leaf_off, sizeof(int64_t) * (size_t)(tiles + 1), "leaf offsets"));
  SFK_TRY(ws_reserve(c, ws, ws.partial_off, sizeof(int64_t) * (size_t)(tiles + 1), "partial offsets"));
  SFK_TRY(ws_reserve(c, ws, ws.chunk_off, sizeof(int64_t) * (size_t)(tiles + 1), "item offsets"));
  SFK_TRY(ws_reserve(c, ws, ws.leaves, sizeof(int32_t) * (size_t)leaf_cap, "leaf lists"));
  SFK_TRY(ws_reserve(c, ws, ws.partials, sizeof(double) * (size_t)partial_cap * T, "partial sums"));
  SFK_TRY(ws_reserve(c, ws, ws.hdr_rois, sizeof(BatchHdr) + sizeof(RoiDev) * (size_t)nr,
                     "ROI descriptors"));
  SFK_TRY(ws_reserve(c, ws, ws.coords, sizeof(double) * (size_t)nc, "node coordinates"));
  SFK_TRY(ws_reserve(c, ws, ws.claims, kClaimBytes, "work-claim counters"));
  if (ws.claims_cleared != ws.claims.p) {
    // a new buffer: its error word starts at zero (no kernel clears it)
    SFK_HIP(c, hipMemsetAsync(ws.claims.p, 0, ws.claims.bytes, nullptr));
    SFK_HIP(c, hipStreamSynchronize(nullptr));
    ws.claims_cleared = ws.claims.p;
  }
  SFK_TRY(ws_reserve(c, ws, ws.roi_leaves, sizeof(int32_t) * kRoiListCap * (size_t)nr,
                     "ROI leaf lists"));
  SFK_TRY(ws_reserve(c, ws, ws.roi_nl, sizeof(int32_t) * (size_t)nr, "ROI list lengths"));
  SFK_TRY(ws_reserve(c, ws, ws.plan_tmp, 3 * sizeof(int64_t) * (size_t)sfk::plan_blocks(tiles),
                     "plan block sums"));
  Caps k;
  k.tiles_cap = std::min<int64_t>({(int64_t)(ws.plan_tmp.bytes / (3 * sizeof(int64_t))) * 1024,
                                   (int64_t)(ws.tile_cnt.bytes / sizeof(int32_t)),
                                   (int64_t)(ws.tile_fit.bytes / sizeof(int32_t)),
                                   (int64_t)(ws.tile_done.bytes / sizeof(int32_t)),
                                   (int64_t)(ws.tile_slots.bytes / (sizeof(int32_t) * slot_cap)),
                                   (int64_t)(ws.leaf_off.bytes / sizeof(int64_t)) - 1,
                                   (int64_t)(ws.partial_off.bytes / sizeof(int64_t)) - 1,
                                   (int64_t)(ws.chunk_off.bytes / sizeof(int64_t)) - 1});
  k.leaf_cap = c->opts.list_capacity > 0 && !sweep ? leaf_cap
                                                  : (int64_t)(ws.leaves.bytes / sizeof(int32_t));
  k.partial_cap = c->opts.list_capacity > 0 && !sweep
                      ? partial_cap
                      : (int64_t)(ws.partials.bytes / (sizeof(double) * (size_t)T));
  // the sweep's node sums live in the partial slots: one slot per tile
  if (sweep) k.tiles_cap = std::min(k.tiles_cap, k.partial_cap);
  k.rois_cap = std::min<int64_t>({(int64_t)((ws.hdr_rois.bytes - sizeof(BatchHdr)) / sizeof(RoiDev)),
                                  (int64_t)(ws.roi_leaves.bytes / (sizeof(int32_t) * kRoiListCap)),
                                  (int64_t)(ws.roi_nl.bytes / sizeof(int32_t))});
  k.coords_cap = (int64_t)(ws.coords.bytes / sizeof(double));
  k.slot_cap = slot_cap;
  // work items: one per tile plus one per partial slot (a split tile has one
  // item per chunk and one partial slot per chunk, whether it evaluates its
  // list or walks per chunk), so the plan can never exceed this. A split
  // brick has one slot for all its chunks and never walks per chunk, so its
  // extra items are bounded by the listed leaves / chunk_leaves.
  k.item_cap = k.tiles_cap + k.partial_cap + 1 + (brick ? k.leaf_cap / CH + 1 : 0);
  if (sweep) k.item_cap = k.leaf_cap / 2;  // the item list lives in the leaf-list buffer
  k.splat = brick ? 1 : 0;
  SFK_TRY(ws_reserve(c, ws, ws.item_tile, sizeof(int32_t) * (size_t)k.item_cap, "work items"));
  *caps = k;
  return SFK_OK;
}

// The batch header a group stages in front of its descriptors.
BatchHdr make_hdr(sfk_ctx c, const Caps& k, int64_t n_rois, int64_t n_tiles) {
  BatchHdr h{};
  h.debug_poison = c->debug_poison;
  h.n_tiles = n_tiles;
  h.leaf_cap = k.leaf_cap;
  h.partial_cap = k.partial_cap;
  h.item_cap = k.item_cap;
  h.n_rois = (int32_t)n_rois;
  h.slot_cap = k.slot_cap;
  h.splat = k.splat;
  return h;
}

// Enqueue the kernels of one group whose header + descriptors are already
// (being) copied into ws.hdr_rois. roi_grid: blocks of the coordinate
// kernel (one per ROI); max_tiles: a bound on the batch's tiles that sizes the
// tile and plan grids (exact for direct launches, the capacities for a
// captured graph).
sfk_status launch_kernels(sfk_ctx c, const TreeView& tv, TileShape ts, int kk, int pp, bool cnt,
                          Workspace& ws, int roi_grid, int64_t max_tiles, hipStream_t s,
                          int nm = 0) {
  if (sfk::is_sweep(ts)) {
    BatchHdr* hdr = (BatchHdr*)ws.hdr_rois.p;
    const RoiDev* rois = (const RoiDev*)((char*)ws.hdr_rois.p + sizeof(BatchHdr));
    double* coords = (double*)ws.coords.p;
    SFK_HIP(c, sfk::launch_roi_coords(tv, hdr, rois, roi_grid, coords, (int32_t*)ws.roi_leaves.p,
                                      (int32_t*)ws.roi_nl.p, s));
    {
      ProfScope p(c, PK_TILE_COUNT, s);
      SFK_HIP(c, sfk::launch_sweep_list(tv, hdr, rois, coords, (int64_t*)ws.leaves.p,
                                        (unsigned long long*)ws.partials.p, (int32_t*)ws.claims.p,
                                        roi_grid, max_tiles, s));
    }
    const int grid = c->opts.persistent_waves_per_cu > 0
                         ? c->n_cu * std::max(1, c->opts.persistent_waves_per_cu / 4)
                         : 0;
    ProfScope p(c, PK_EVAL, s, hdr);
    SFK_HIP(c, sfk::launch_sweep_eval(tv, hdr, rois, coords, kk, cnt, nm, (const int64_t*)ws.leaves.p,
                                      (unsigned long long*)ws.partials.p, (int32_t*)ws.claims.p,
                                      grid, c->n_cu, max_tiles, s));
    return SFK_OK;
  }
  const int tile_grid = sfk::tile_grid_blocks(max_tiles);
  const int CH = chunk_leaves_of(c);
  BatchHdr* hdr = (BatchHdr*)ws.hdr_rois.p;
  const RoiDev* rois = (const RoiDev*)((char*)ws.hdr_rois.p + sizeof(BatchHdr));
  double* coords = (double*)ws.coords.p;
  int32_t* tile_cnt = (int32_t*)ws.tile_cnt.p;
  int32_t* tile_fit = (int32_t*)ws.tile_fit.p;
  int32_t* tile_done = (int32_t*)ws.tile_done.p;
  int64_t* leaf_off = (int64_t*)ws.leaf_off.p;
  int64_t* partial_off = (int64_t*)ws.partial_off.p;
  int64_t* chunk_off = (int64_t*)ws.chunk_off.p;
  int32_t* roi_leaves = (int32_t*)ws.roi_leaves.p;
  int32_t* roi_nl = (int32_t*)ws.roi_nl.p;
  SFK_HIP(c, sfk::launch_roi_coords(tv, hdr, rois, roi_grid, coords, roi_leaves, roi_nl, s));
  {
    ProfScope p(c, PK_TILE_COUNT, s);
    SFK_HIP(c, sfk::launch_tile_count(tv, hdr, rois, coords, roi_leaves, roi_nl, ts, tile_grid,
                                      tile_cnt, tile_done, (int32_t*)ws.tile_slots.p, s));
  }
  {
    ProfScope p(c, PK_PLAN, s);
    SFK_HIP(c, sfk::launch_plan(tile_cnt, hdr, (int32_t*)ws.claims.p, CH, leaf_off, partial_off,
                                chunk_off, tile_fit, (int64_t*)ws.plan_tmp.p, max_tiles, s));
  }
  {
    ProfScope p(c, PK_TILE_FILL, s);
    SFK_HIP(c, sfk::launch_tile_fill(tv, hdr, rois, coords, roi_leaves, roi_nl,
                                      (const int32_t*)ws.tile_slots.p, ts, tile_grid,
                                      tile_cnt, tile_fit,
                                      leaf_off, chunk_off, (int32_t*)ws.leaves.p,
                                      (int32_t*)ws.item_tile.p, (int32_t*)ws.claims.p,
                                      (double*)ws.partials.p, partial_off, s));
  }
  // 0: resident blocks per CU from the occupancy query, capped at one wave
  // per tile (the tile kernels' grid) but at least one block per CU, so a
  // small batch does not launch (and drain) a full-device persistent grid
  // Serving with `interleave`: one wave per tile, so the workgroups of a
  // heavy request retire as they finish their items and the hardware can
  // interleave the kernels of requests on the other streams (measured on the
  // 1B-point trace: p50 0.54 -> 3.7 ms, saturated throughput -12%, p99 no
  // better, so persistent grids stay the default).
  const int grid = c->serve_interleave ? std::max(1, tile_grid)
                   : c->opts.persistent_waves_per_cu > 0
                       ? c->n_cu * std::max(1, c->opts.persistent_waves_per_cu / 4)
                       : 0;
  {
    ProfScope p(c, PK_EVAL, s, hdr);
    SFK_HIP(c, sfk::launch_eval(tv, hdr, rois, coords, ts, kk, pp, cnt, CH, leaf_off, chunk_off,
                                 partial_off, tile_cnt, tile_fit, (int32_t*)ws.leaves.p,
                                 (int32_t*)ws.item_tile.p, (double*)ws.partials.p, tile_done,
                                 hdr, (int32_t*)ws.claims.p, grid, c->n_cu,
                                 std::max(c->n_cu, tile_grid), s));
  }
  return SFK_OK;
}

// Resolve the per-ROI parameters of a CLOUD-set, non-MBE ROI.
GroupRoi resolve_cloud_roi(sfk_tree t, const sfk_roi* r, bool count_mode) {
  GroupRoi g{};
  g.roi = r;
  g.kk = r->kernel == SFK_KERNEL_GAUSS_TRUNC3 ? KK_GAUSS : KK_EPAN;
  g.count_mode = count_mode;
  g.c2 = g.kk == KK_GAUSS ? 9.0f : 1.0f;
  const double ck = g.kk == KK_GAUSS ? ck_gauss_trunc3() : ck_epanechnikov();
  const double nu = (r->norm == SFK_NORM_COUNT || t->n == 0) ? 1.0 : 1.0 / (double)t->n;
  if (r->bw == SFK_BW_PER_POINT) {
    g.pp = PP_ISO;
    g.ih[0] = g.ih[1] = g.ih[2] = 1.0f;
    g.scale = ck * nu;
  } else {
    float h[3];
    for (int k = 0; k < 3; ++k) {
      if (r->bw == SFK_BW_FIXED)
        h[k] = r->h[k];
      else
        h[k] = (float)((double)r->h[0] * (r->hi[k] - r->lo[k]));
    }
    g.pp = PP_UNIFORM;
    for (int k = 0; k < 3; ++k) g.ih[k] = (float)(1.0 / (double)h[k]);
    const double w = 1.0 / ((double)h[0] * (double)h[1] * (double)h[2]);
    g.scale = ck * nu * w;
  }
  if (count_mode) g.scale = 1.0;
  return g;
}

// Group CLOUD-set ROIs by (kernel, bandwidth source), in a fixed order.
// One evaluation pipeline per (kernel, bandwidth source, tile shape). The
// shape of a ROI depends on that ROI alone (the autotuned or default choice
// for its key), so a ROI is evaluated the same way alone and in any batch.
struct GroupKey {
  int kk, pp;
  TileShape ts;
  int nm;  // particle sweep: nodes per axis a support spans (0 otherwise)
  bool operator==(const GroupKey& o) const {
    return kk == o.kk && pp == o.pp && ts.tx == o.ts.tx && ts.ty == o.ts.ty &&
           ts.tz == o.ts.tz && nm == o.nm;
  }
};

TileShape choose_shape(sfk_ctx c, sfk_tree t, const sfk_roi* r);

void group_rois(sfk_ctx c, sfk_tree t, const std::vector<const sfk_roi*>& rois, bool count_mode,
                std::vector<std::vector<GroupRoi>>* groups, std::vector<GroupKey>* keys,
                const TileShape* force_ts = nullptr) {
  for (const sfk_roi* r : rois) {
    GroupRoi g = resolve_cloud_roi(t, r, count_mode);
    const TileShape ts = force_ts ? *force_ts : choose_shape(c, t, r);
    const GroupKey key{count_mode ? 0 : g.kk, g.pp, ts, sfk::is_sweep(ts) ? sweep_nm(g) : 0};
    size_t gi = 0;
    while (gi < keys->size() && !((*keys)[gi] == key)) ++gi;
    if (gi == keys->size()) {
      keys->push_back(key);
      groups->emplace_back();
    }
    (*groups)[gi].push_back(g);
  }
}

// Enqueue CLOUD-set ROIs, one pipeline per group, with direct launches sized
// to the batch. Every group's buffers are reserved before the first launch:
// the groups run one after another on the same workspace, and growing a
// buffer frees the old one.
sfk_status enqueue_groups(sfk_ctx c, sfk_tree t, std::vector<std::vector<GroupRoi>>& groups,
                          std::vector<GroupKey>& keys, bool count_mode, Workspace& ws,
                          Staging& st, hipStream_t s);

sfk_status enqueue_cloud_rois(sfk_ctx c, sfk_tree t, const std::vector<const sfk_roi*>& rois,
                              bool count_mode, Workspace& ws, Staging& st, hipStream_t s,
                              const TileShape* force_ts = nullptr) {
  if (rois.empty()) return SFK_OK;
  std::vector<std::vector<GroupRoi>> groups;
  std::vector<GroupKey> keys;
  group_rois(c, t, rois, count_mode, &groups, &keys, force_ts);
  return enqueue_groups(c, t, groups, keys, count_mode, ws, st, s);
}

// Enqueue groups formed by group_rois (one pipeline per group, direct
// launches, every group's buffers reserved before the first launch).
sfk_status enqueue_groups(sfk_ctx c, sfk_tree t, std::vector<std::vector<GroupRoi>>& groups,
                          std::vector<GroupKey>& keys, bool count_mode, Workspace& ws,
                          Staging& st, hipStream_t s) {
  size_t bytes = 0;
  for (auto& g : groups) bytes += sizeof(BatchHdr) + sizeof(RoiDev) * g.size();
  SFK_TRY(staging_reserve(c, st, bytes));
  if (st.ev_valid) SFK_HIP(c, hipEventSynchronize(st.ev));
  TreeView tv = view_of(t);
  std::vector<int64_t> tiles(groups.size());
  size_t off = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const int64_t n = (int64_t)groups[gi].size();
    RoiDev* rd = (RoiDev*)(st.host + off + sizeof(BatchHdr));
    int64_t n_coords = 0;
    make_roidev(groups[gi], keys[gi].ts, rd, &tiles[gi], &n_coords);
    Caps k;
    SFK_TRY(reserve_group(c, ws, keys[gi].ts, n, tiles[gi], n_coords, 1.0, t->n_leaves, &k));
    *(BatchHdr*)(st.host + off) = make_hdr(c, k, n, tiles[gi]);
    off += sizeof(BatchHdr) + sizeof(RoiDev) * (size_t)n;
  }
  off = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const int64_t n = (int64_t)groups[gi].size();
    const size_t gb = sizeof(BatchHdr) + sizeof(RoiDev) * (size_t)n;
    SFK_HIP(c, hipMemcpyAsync(ws.hdr_rois.p, st.host + off, gb, hipMemcpyHostToDevice, s));
    SFK_TRY(launch_kernels(c, tv, keys[gi].ts, keys[gi].kk, keys[gi].pp, count_mode, ws, (int)n,
                           tiles[gi], s, keys[gi].nm));
    off += gb;
  }
  SFK_HIP(c, hipMemcpyAsync(st.hdr_host, ws.hdr_rois.p, sizeof(BatchHdr), hipMemcpyDeviceToHost, s));
  SFK_HIP(c, hipMemcpyAsync(st.err_host(), (int32_t*)ws.claims.p + kErrWord, sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
  SFK_HIP(c, hipEventRecord(st.ev, s));
  st.ev_valid = true;
  st.stats_pending = true;
  return SFK_OK;
}

void drop_graph(GraphCache& gc) {
  if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
  if (gc.graph) (void)hipGraphDestroy(gc.graph);
  gc = GraphCache();
}

// Enqueue a single-group batch on an idle slot through its captured graph,
// capturing (again) when the key, the workspace or the capacities changed.
sfk_status enqueue_cloud_rois_graph(sfk_ctx c, sfk_tree t,
                                    const std::vector<const sfk_roi*>& rois, Slot& sl) {
  std::vector<std::vector<GroupRoi>> groups;
  std::vector<GroupKey> keys;
  group_rois(c, t, rois, false, &groups, &keys);
  if (groups.size() != 1) return enqueue_groups(c, t, groups, keys, false, sl.ws, sl.st, sl.stream);
  const int64_t n = (int64_t)groups[0].size();
  const TileShape ts = keys[0].ts;
  const int kk = keys[0].kk, pp = keys[0].pp, ch = chunk_leaves_of(c), nm = keys[0].nm;
  std::vector<RoiDev> rd((size_t)n);
  int64_t n_tiles = 0, n_coords = 0;
  make_roidev(groups[0], ts, rd.data(), &n_tiles, &n_coords);
  GraphCache& gc = sl.gc;
  const bool fits = gc.valid && gc.gen == sl.ws.gen && gc.st_gen == sl.st.gen && gc.tree == t &&
                    gc.kk == kk && gc.nm == nm &&
                    gc.pp == pp && gc.ch == ch && !gc.cnt && gc.interleave == c->serve_interleave &&
                    gc.ts.tx == ts.tx &&
                    gc.ts.ty == ts.ty && gc.ts.tz == ts.tz && n <= gc.rois_cap &&
                    n_tiles <= gc.tiles_cap && n_coords <= gc.coords_cap;
  Caps k;
  if (!fits) {
    drop_graph(gc);
    SFK_TRY(reserve_group(c, sl.ws, ts, n, n_tiles, n_coords, 2.0, t->n_leaves, &k));
  } else {
    SFK_TRY(reserve_group(c, sl.ws, ts, n, n_tiles, n_coords, 1.0, t->n_leaves, &k));
    if (sl.ws.gen != gc.gen) {  // a buffer moved after all
      drop_graph(gc);
      SFK_TRY(reserve_group(c, sl.ws, ts, n, n_tiles, n_coords, 2.0, t->n_leaves, &k));
    }
  }
  const size_t full = sizeof(BatchHdr) + sizeof(RoiDev) * (size_t)k.rois_cap;
  SFK_TRY(staging_reserve(c, sl.st, full));
  if (gc.valid && gc.st_gen != sl.st.gen) drop_graph(gc);
  BatchHdr* h = (BatchHdr*)sl.st.host;
  *h = make_hdr(c, k, n, n_tiles);
  std::memcpy(sl.st.host + sizeof(BatchHdr), rd.data(), sizeof(RoiDev) * (size_t)n);
  if (!gc.valid) {
    // profiling events cannot be recorded inside a capture
    const bool prof = c->prof_on;
    c->prof_on = false;
    const hipStream_t s = sl.stream;
    SFK_HIP(c, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    sfk_status st = SFK_OK;
    if (hipMemcpyAsync(sl.ws.hdr_rois.p, sl.st.host, full, hipMemcpyHostToDevice, s) != hipSuccess)
      st = SFK_E_DEVICE;
    if (st == SFK_OK)
      st = launch_kernels(c, view_of(t), ts, kk, pp, false, sl.ws, (int)k.rois_cap, k.tiles_cap,
                          s, nm);
    if (st == SFK_OK && hipMemcpyAsync(sl.st.hdr_host, sl.ws.hdr_rois.p, sizeof(BatchHdr),
                                       hipMemcpyDeviceToHost, s) != hipSuccess)
      st = SFK_E_DEVICE;
    if (st == SFK_OK &&
        hipMemcpyAsync(sl.st.err_host(), (int32_t*)sl.ws.claims.p + kErrWord, sizeof(int32_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess)
      st = SFK_E_DEVICE;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    c->prof_on = prof;
    if (st != SFK_OK || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      set_err(c, "capturing the batch graph failed");
      return st != SFK_OK ? st : SFK_E_DEVICE;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      set_err(c, "instantiating the batch graph failed");
      return SFK_E_DEVICE;
    }
    gc.valid = true;
    gc.ts = ts;
    gc.kk = kk;
    gc.nm = nm;
    gc.pp = pp;
    gc.ch = ch;
    gc.cnt = false;
    gc.interleave = c->serve_interleave;
    gc.tree = t;
    gc.gen = sl.ws.gen;
    gc.st_gen = sl.st.gen;
    gc.tiles_cap = k.tiles_cap;
    gc.rois_cap = k.rois_cap;
    gc.coords_cap = k.coords_cap;
    gc.graph = graph;
    gc.exec = exec;
  }
  SFK_HIP(c, hipGraphLaunch(gc.exec, sl.stream));
  return SFK_OK;
}

// Grow the list capacities from the direct-path batches whose header
// readback has completed, oldest first, stopping at the first one still in
// flight (never blocks; about one event query per call in steady state).
bool absorb_stats(Workspace& ws, const Staging& st);
// Returns true if one of the absorbed batches set the error word.
bool absorb_ready(Workspace& ws, Staging* ring, int n, int oldest) {
  bool err = false;
  for (int i = 0; i < n; ++i) {
    Staging& st = ring[(oldest + i) % n];
    if (!st.stats_pending || !st.ev_valid) continue;
    if (hipEventQuery(st.ev) != hipSuccess) break;
    err |= absorb_stats(ws, st);
    st.stats_pending = false;
  }
  return err;
}

// After a batch completed: grow the list capacities if they overflowed.
// Returns true (once) if the batch read back a set error word.
bool absorb_stats(Workspace& ws, const Staging& st) {
  if (!st.hdr_host) return false;
  const BatchHdr& h = *st.hdr_host;
  if (h.total_leaves > h.leaf_cap) ws.want_leaf_cap = h.total_leaves + h.total_leaves / 4;
  if (h.total_partials > h.partial_cap)
    ws.want_partial_cap = h.total_partials + h.total_partials / 4;
  int32_t* e = st.err_host();
  const bool err = *e != 0;
  *e = 0;
  return err;
}

// Clear the workspace's error word, stream-ordered (never inside a capture).
sfk_status clear_err_word(sfk_ctx c, Workspace& ws, hipStream_t s) {
  SFK_HIP(c, hipMemsetAsync((int32_t*)ws.claims.p + kErrWord, 0, sizeof(int32_t), s));
  return SFK_OK;
}

constexpr const char* kErrLeafIds =
    "internal error: a tile's leaf list held an id outside the tree (the batch's grids are "
    "not valid)";

// ---- IN_ROI set and MBE: a sub-cloud of the particles inside B ----

struct SubCloud {
  int64_t n_b = 0;
  int32_t n_leaves = 0, n_levels = 0, total_nodes = 0;
  int32_t off[SFK_MAX_LEVELS], cnt[SFK_MAX_LEVELS];
  TmpBuf pts, perm, nodes, node_ih, pparam, axes;
  explicit SubCloud(sfk_ctx c) : pts(c), perm(c), nodes(c), node_ih(c), pparam(c), axes(c) {}
  TreeView view(int pp) const {
    TreeView tv{};
    tv.pts = pts.as<const float4>();
    tv.pparam = pparam.as<const float4>();
    tv.nodes = nodes.as<const NodeBox>();
    tv.node_ih = node_ih.as<const float4>();
    for (int l = 0; l < SFK_MAX_LEVELS; ++l) {
      tv.level_off[l] = off[l];
      tv.level_cnt[l] = cnt[l];
    }
    tv.n_levels = n_levels;
    tv.n_leaves = n_leaves;
    tv.n = n_b;
    tv.pp_mode = pp;
    return tv;
  }
};

sfk_status make_subcloud(sfk_ctx c, sfk_tree t, const sfk_roi* r, bool want_axes, SubCloud& sc,
                         hipStream_t s) {
  // Only the leaves whose box meets B can hold particles in B: find them
  // first, then examine their slots alone (in leaf order, so the particles
  // come out in the tree's order as a scan of every slot would give them).
  // Work and scratch then grow with the box's leaves, not with the cloud.
  const int32_t nl = t->n_leaves;
  TmpBuf lflags(c), lpos(c), ltotal(c), cand(c), flags(c), pos(c), stmp(c), total(c);
  SFK_TRY(lflags.get(sizeof(int32_t) * (size_t)std::max(nl, 1), "leaf flags"));
  SFK_TRY(lpos.get(sizeof(int64_t) * (size_t)std::max(nl, 1), "leaf positions"));
  SFK_TRY(ltotal.get(sizeof(int64_t), "leaf total"));
  SFK_TRY(stmp.get(sfk::scan_tmp_bytes((int64_t)nl * SFK_LEAF), "scan scratch"));
  int64_t n_cand = 0;
  if (nl > 0) {
    SFK_HIP(c, sfk::launch_leaf_overlap((const NodeBox*)t->nodes.p + t->level_off[0], nl, r->lo,
                                         r->hi, lflags.as<int32_t>(), s));
    SFK_HIP(c, sfk::scan_exclusive_i32_i64(lflags.as<int32_t>(), lpos.as<int64_t>(), nl,
                                            ltotal.as<int64_t>(), stmp.b.p, stmp.b.bytes, s));
    SFK_HIP(c, hipMemcpyAsync(&n_cand, ltotal.b.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SFK_HIP(c, hipStreamSynchronize(s));
  }
  const int64_t n_slots = n_cand * SFK_LEAF;  // examined slots
  SFK_TRY(cand.get(sizeof(int32_t) * (size_t)std::max<int64_t>(n_cand, 1), "candidate leaves"));
  SFK_TRY(flags.get(sizeof(int32_t) * (size_t)std::max<int64_t>(n_slots, 1), "in-box flags"));
  SFK_TRY(pos.get(sizeof(int64_t) * (size_t)std::max<int64_t>(n_slots, 1), "in-box positions"));
  SFK_TRY(total.get(sizeof(int64_t), "in-box total"));
  if (n_cand > 0) {
    SFK_HIP(c, sfk::launch_compact_leaves(lflags.as<int32_t>(), lpos.as<int64_t>(), nl,
                                           cand.as<int32_t>(), s));
    SFK_HIP(c, sfk::launch_inbox_flags((const float4*)t->pts.p, cand.as<int32_t>(), n_slots,
                                        r->lo, r->hi, flags.as<int32_t>(), s));
    SFK_HIP(c, sfk::scan_exclusive_i32_i64(flags.as<int32_t>(), pos.as<int64_t>(), n_slots,
                                            total.as<int64_t>(), stmp.b.p, stmp.b.bytes, s));
  }
  int64_t n_b = 0;
  if (n_cand > 0) {
    SFK_HIP(c, hipMemcpyAsync(&n_b, total.b.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SFK_HIP(c, hipStreamSynchronize(s));
  }
  sc.n_b = n_b;
  sc.n_leaves = (int32_t)((n_b + SFK_LEAF - 1) / SFK_LEAF);
  level_layout(sc.n_leaves, sc.off, sc.cnt, &sc.n_levels, &sc.total_nodes);
  const int64_t out_slots = (int64_t)sc.n_leaves * SFK_LEAF;
  SFK_TRY(sc.pts.get(sizeof(float4) * (size_t)std::max<int64_t>(out_slots, 1), "in-box particles"));
  SFK_TRY(sc.perm.get(sizeof(int32_t) * (size_t)std::max<int64_t>(n_b, 1), "in-box indices"));
  SFK_TRY(sc.nodes.get(sizeof(NodeBox) * (size_t)std::max(sc.total_nodes, 1), "in-box boxes"));
  SFK_TRY(sc.node_ih.get(sizeof(float4) * (size_t)std::max(sc.total_nodes, 1), "in-box node bandwidths"));
  if (want_axes)
    SFK_TRY(sc.axes.get(sizeof(float) * 3 * (size_t)std::max<int64_t>(n_b, 1), "in-box axes"));
  if (n_b == 0) return SFK_OK;
  SFK_HIP(c, sfk::launch_compact((const float4*)t->pts.p, (const int32_t*)t->perm.p,
                                  cand.as<int32_t>(), flags.as<int32_t>(), pos.as<int64_t>(),
                                  n_slots, out_slots,
                                  sc.pts.as<float4>(), sc.perm.as<int32_t>(),
                                  want_axes ? sc.axes.as<float>() : nullptr, n_b, s));
  SFK_TRY(build_boxes(c, sc.pts.as<float4>(), n_b, sc.n_leaves, sc.nodes.as<NodeBox>(), sc.off,
                      sc.cnt, sc.n_levels, s));
  // keep the temporaries alive until the kernels that read them are done
  SFK_HIP(c, hipStreamSynchronize(s));
  return SFK_OK;
}

struct MbeDebug {
  float* ell0 = nullptr;
  int64_t* n_b = nullptr;
  int64_t* idx_b = nullptr;
  float* pilot = nullptr;
  float* pden = nullptr;
  double* aveden = nullptr;
  float* ell_j = nullptr;
  int64_t cap_b = 0;
};

// Evaluate one IN_ROI-set ROI (any bandwidth mode, MBE included). Blocking.
sfk_status eval_subcloud(sfk_ctx c, sfk_tree t, const sfk_roi* r, bool count_mode, TileShape ts,
                         Workspace& ws, Staging& st, hipStream_t s, MbeDebug* dbg) {
  const bool mbe = r->bw == SFK_BW_MBE;
  SubCloud sc(c);
  SFK_TRY(make_subcloud(c, t, r, mbe, sc, s));
  const int64_t n_b = sc.n_b;
  const int64_t m = (int64_t)r->res[0] * r->res[1] * r->res[2];
  if (dbg && dbg->n_b) *dbg->n_b = n_b;
  if (n_b == 0) {
    SFK_HIP(c, sfk::launch_fill_f32(r->d_out, m, 0.0f, s));
    if (dbg && dbg->aveden) *dbg->aveden = 0.0;
    if (dbg && dbg->ell0) dbg->ell0[0] = dbg->ell0[1] = dbg->ell0[2] = 0.0f;
    SFK_HIP(c, hipStreamSynchronize(s));
    return SFK_OK;
  }
  const double ck = r->kernel == SFK_KERNEL_GAUSS_TRUNC3 ? ck_gauss_trunc3() : ck_epanechnikov();
  const double nu = r->norm == SFK_NORM_COUNT ? 1.0 : 1.0 / (double)n_b;
  const bool kg = r->kernel == SFK_KERNEL_GAUSS_TRUNC3;

  auto run_one = [&](TreeView tv, const GroupRoi& g, float* out) -> sfk_status {
    sfk_roi rr = *g.roi;
    rr.d_out = out;
    GroupRoi gg = g;
    gg.roi = &rr;
    std::vector<GroupRoi> v{gg};
    const size_t gb = sizeof(BatchHdr) + sizeof(RoiDev);
    SFK_TRY(staging_reserve(c, st, gb));
    if (st.ev_valid) SFK_HIP(c, hipEventSynchronize(st.ev));
    int64_t n_tiles = 0, n_coords = 0;
    make_roidev(v, ts, (RoiDev*)(st.host + sizeof(BatchHdr)), &n_tiles, &n_coords);
    Caps k;
    SFK_TRY(reserve_group(c, ws, ts, 1, n_tiles, n_coords, 1.0, tv.n_leaves, &k));
    *(BatchHdr*)st.host = make_hdr(c, k, 1, n_tiles);
    SFK_HIP(c, hipMemcpyAsync(ws.hdr_rois.p, st.host, gb, hipMemcpyHostToDevice, s));
    SFK_HIP(c, hipEventRecord(st.ev, s));
    st.ev_valid = true;
    return launch_kernels(c, tv, ts, g.count_mode ? 0 : g.kk, g.pp, g.count_mode, ws, 1,
                          n_tiles, s);
  };

  if (!mbe) {
    GroupRoi g{};
    g.roi = r;
    g.kk = kg ? KK_GAUSS : KK_EPAN;
    g.count_mode = count_mode;
    g.c2 = kg ? 9.0f : 1.0f;
    if (r->bw == SFK_BW_PER_POINT) {
      g.pp = PP_ISO;
      g.ih[0] = g.ih[1] = g.ih[2] = 1.0f;
      g.scale = ck * nu;
      SFK_HIP(c, sfk::launch_node_ih(sc.pts.as<float4>(), nullptr, PP_ISO, n_b,
                                      sc.nodes.as<NodeBox>(), sc.off, sc.cnt, sc.n_levels,
                                      sc.node_ih.as<float4>(), 0, s));
    } else {
      float h[3];
      for (int k = 0; k < 3; ++k)
        h[k] = r->bw == SFK_BW_FIXED ? r->h[k] : (float)((double)r->h[0] * (r->hi[k] - r->lo[k]));
      g.pp = PP_UNIFORM;
      for (int k = 0; k < 3; ++k) g.ih[k] = (float)(1.0 / (double)h[k]);
      g.scale = ck * nu / ((double)h[0] * (double)h[1] * (double)h[2]);
    }
    if (count_mode) g.scale = 1.0;
    SFK_TRY(run_one(sc.view(g.pp), g, r->d_out));
    SFK_HIP(c, hipStreamSynchronize(s));
    return SFK_OK;
  }

  // ---- MBE (Section 3.1) ----
  // Eq. 1: exact order statistics from one radix sort of the three axes
  TmpBuf keys(c), keys2(c), vals(c), vals2(c), stmp(c), ell_d(c), flag_d(c), pilot(c), pden(c),
      bsum(c), ave_d(c), ellj_d(c);
  const int64_t m3 = 3 * n_b;
  SFK_TRY(keys.get(sizeof(uint64_t) * (size_t)m3, "axis keys"));
  SFK_TRY(keys2.get(sizeof(uint64_t) * (size_t)m3, "axis keys"));
  SFK_TRY(vals.get(sizeof(uint32_t) * (size_t)m3, "axis values"));
  SFK_TRY(vals2.get(sizeof(uint32_t) * (size_t)m3, "axis values"));
  SFK_TRY(stmp.get(sfk::radix_sort_tmp_bytes(m3), "sort scratch"));
  SFK_TRY(ell_d.get(4 * sizeof(float), "smoothing lengths"));
  SFK_TRY(flag_d.get(sizeof(int32_t), "flags"));
  SFK_HIP(c, sfk::launch_axis_keys(sc.axes.as<float>(), n_b, keys.as<uint64_t>(),
                                    vals.as<uint32_t>(), s));
  int alt = 0;
  SFK_HIP(c, sfk::radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), keys2.as<uint64_t>(),
                                    vals2.as<uint32_t>(), m3, 34, stmp.b.p, stmp.b.bytes, s, &alt));
  const uint64_t* sorted = alt ? keys2.as<uint64_t>() : keys.as<uint64_t>();
  SFK_HIP(c, sfk::launch_mbe_ell(sorted, n_b, r->lo, r->hi, r->res, ell_d.as<float>(),
                                  flag_d.as<int32_t>(), s));
  float ell0[3];
  SFK_HIP(c, hipMemcpyAsync(ell0, ell_d.b.p, 3 * sizeof(float), hipMemcpyDeviceToHost, s));
  SFK_HIP(c, hipStreamSynchronize(s));
  if (dbg && dbg->ell0) std::memcpy(dbg->ell0, ell0, sizeof ell0);

  // pilot grid (Eq. 2): uniform ellipsoid l_k over the particles in B
  SFK_TRY(pilot.get(sizeof(float) * (size_t)m, "pilot grid"));
  GroupRoi gp{};
  gp.roi = r;
  gp.kk = KK_EPAN;
  gp.pp = PP_UNIFORM;
  gp.c2 = 1.0f;
  for (int k = 0; k < 3; ++k) gp.ih[k] = (float)(1.0 / (double)ell0[k]);
  gp.scale = ck * nu / ((double)ell0[0] * (double)ell0[1] * (double)ell0[2]);
  SFK_TRY(run_one(sc.view(PP_UNIFORM), gp, pilot.as<float>()));

  // ASL (Eqs. 5-6): trilinear pilot at each particle, mean, lengths
  const int nblk = (int)((n_b + 255) / 256);
  SFK_TRY(pden.get(sizeof(double) * (size_t)n_b, "pilot at particles"));
  SFK_TRY(bsum.get(sizeof(double) * (size_t)nblk, "block sums"));
  SFK_TRY(ave_d.get(sizeof(double), "mean pilot"));
  SFK_TRY(sc.pparam.get(sizeof(float4) * (size_t)sc.n_leaves * SFK_LEAF, "adaptive parameters"));
  SFK_TRY(ellj_d.get(sizeof(float) * 3 * (size_t)n_b, "adaptive lengths"));
  SFK_HIP(c, sfk::launch_trilinear_mean(sc.pts.as<float4>(), n_b, pilot.as<float>(), r->lo, r->hi,
                                         r->res, pden.as<double>(), bsum.as<double>(),
                                         ave_d.as<double>(), s));
  SFK_HIP(c, sfk::launch_asl2(pden.as<double>(), n_b, ave_d.as<double>(), ell0, r->lo, r->hi,
                               r->res, sc.pparam.as<float4>(), ellj_d.as<float>(), s));
  SFK_HIP(c, sfk::launch_node_ih(sc.pts.as<float4>(), sc.pparam.as<float4>(), PP_ANISO, n_b,
                                  sc.nodes.as<NodeBox>(), sc.off, sc.cnt, sc.n_levels,
                                  sc.node_ih.as<float4>(), 0, s));

  // final grid (Eq. 7): per-particle ellipsoids
  GroupRoi gf{};
  gf.roi = r;
  gf.kk = KK_EPAN;
  gf.pp = PP_ANISO;
  gf.c2 = 1.0f;
  gf.ih[0] = gf.ih[1] = gf.ih[2] = 1.0f;
  gf.count_mode = count_mode;
  gf.scale = count_mode ? 1.0 : ck * nu;
  SFK_TRY(run_one(sc.view(PP_ANISO), gf, r->d_out));

  if (dbg) {
    std::vector<double> pd;
    std::vector<float> ej;
    std::vector<int32_t> ix;
    if (dbg->pilot)
      SFK_HIP(c, hipMemcpyAsync(dbg->pilot, pilot.b.p, sizeof(float) * (size_t)m,
                                hipMemcpyDeviceToHost, s));
    if (dbg->aveden)
      SFK_HIP(c, hipMemcpyAsync(dbg->aveden, ave_d.b.p, sizeof(double), hipMemcpyDeviceToHost, s));
    const bool per_particle = dbg->idx_b || dbg->pden || dbg->ell_j;
    if (per_particle && n_b <= dbg->cap_b) {
      pd.resize(n_b);
      ej.resize(3 * n_b);
      ix.resize(n_b);
      SFK_HIP(c, hipMemcpyAsync(pd.data(), pden.b.p, sizeof(double) * n_b, hipMemcpyDeviceToHost, s));
      SFK_HIP(c, hipMemcpyAsync(ej.data(), ellj_d.b.p, sizeof(float) * 3 * n_b,
                                hipMemcpyDeviceToHost, s));
      SFK_HIP(c, hipMemcpyAsync(ix.data(), sc.perm.b.p, sizeof(int32_t) * n_b,
                                hipMemcpyDeviceToHost, s));
    }
    SFK_HIP(c, hipStreamSynchronize(s));
    if (per_particle) {
      if (n_b > dbg->cap_b) {
        set_err(c, "debug capacity %lld below the %lld particles in B", (long long)dbg->cap_b,
                (long long)n_b);
        return SFK_E_INVAL;
      }
      std::vector<int64_t> order(n_b);
      for (int64_t i = 0; i < n_b; ++i) order[i] = i;
      std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return ix[a] < ix[b]; });
      for (int64_t q = 0; q < n_b; ++q) {
        const int64_t i = order[q];
        if (dbg->idx_b) dbg->idx_b[q] = ix[i];
        if (dbg->pden) dbg->pden[q] = (float)pd[i];
        if (dbg->ell_j)
          for (int k = 0; k < 3; ++k) dbg->ell_j[3 * q + k] = ej[3 * i + k];
      }
    }
  }
  SFK_HIP(c, hipStreamSynchronize(s));
  int32_t err = 0;
  SFK_HIP(c, hipMemcpy(&err, (int32_t*)ws.claims.p + kErrWord, sizeof(int32_t),
                       hipMemcpyDeviceToHost));
  if (err) {
    SFK_TRY(clear_err_word(c, ws, s));
    SFK_HIP(c, hipStreamSynchronize(s));
    set_err(c, "%s", kErrLeafIds);
    return SFK_E_INTERNAL;
  }
  return SFK_OK;
}

constexpr int kEstGrid = 32;  // cells per axis of the particle-count table

// The count table of a tree: the finest host level's box counts spread over
// a kEstGrid^3 lattice of cells on the bounding box, each box's count shared
// among the cells it overlaps in proportion to the overlap (a flat box axis
// goes whole to its cell), then summed into a summed-volume table. Boxes of
// one level partition the particles, so the spreading touches about
// kEstGrid^3 cells plus the boxes' boundary cells.
void build_est_table(sfk_tree_s* t) {
  constexpr int G = kEstGrid, G1 = kEstGrid + 1;
  t->est_sat.assign((size_t)G1 * G1 * G1, 0.0);
  if (t->n_levels <= 0 || t->host_nodes.empty()) return;
  std::vector<double> h((size_t)G * G * G, 0.0);
  const int lvl = t->host_level;
  std::vector<double> w[3];
  int c0[3];
  for (int i = 0; i < t->level_cnt[lvl]; ++i) {
    const NodeBox& b = t->host_nodes[(size_t)(t->level_off[lvl] - t->host_base + i)];
    if (b.count <= 0) continue;
    for (int k = 0; k < 3; ++k) {
      const double ext = t->bbox[3 + k] - t->bbox[k];
      const double u0 = ext > 0.0 ? ((double)b.lo[k] - t->bbox[k]) / ext * G : 0.0;
      const double u1 = ext > 0.0 ? ((double)b.hi[k] - t->bbox[k]) / ext * G : 0.0;
      const double a0 = std::min<double>(G, std::max(0.0, u0));
      const double a1 = std::min<double>(G, std::max(a0, u1));
      const int i0 = std::min(G - 1, (int)a0), i1 = std::min(G - 1, std::max(i0, (int)a1));
      c0[k] = i0;
      w[k].assign((size_t)(i1 - i0 + 1), 0.0);
      if (a1 - a0 <= 0.0) {
        w[k][0] = 1.0;
        continue;
      }
      for (int c = i0; c <= i1; ++c)
        w[k][(size_t)(c - i0)] =
            (std::min<double>(a1, c + 1) - std::max<double>(a0, c)) / (a1 - a0);
    }
    const double n = (double)b.count;
    for (size_t z = 0; z < w[2].size(); ++z)
      for (size_t y = 0; y < w[1].size(); ++y) {
        const double wyz = n * w[1][y] * w[2][z];
        double* row = &h[(size_t)c0[0] + G * ((size_t)(c0[1] + y) + G * (size_t)(c0[2] + z))];
        for (size_t x = 0; x < w[0].size(); ++x) row[x] += wyz * w[0][x];
      }
  }
  auto S = [&](int i, int j, int k) -> double& {
    return t->est_sat[(size_t)i + G1 * ((size_t)j + G1 * (size_t)k)];
  };
  for (int k = 1; k <= G; ++k)
    for (int j = 1; j <= G; ++j)
      for (int i = 1; i <= G; ++i)
        S(i, j, k) = h[(size_t)(i - 1) + G * ((size_t)(j - 1) + G * (size_t)(k - 1))] +
                     S(i - 1, j, k) + S(i, j - 1, k) + S(i, j, k - 1) - S(i - 1, j - 1, k) -
                     S(i - 1, j, k - 1) - S(i, j - 1, k - 1) + S(i - 1, j - 1, k - 1);
}

// Particles of the tree in the closed box [lo, hi], estimated in O(1) from
// the count table: counts spread evenly over their cells, so the count below
// a point is the table interpolated multilinearly, and a box's count is the
// eight-corner difference. A flat axis of the bounding box counts whole when
// [lo, hi] holds it. The estimate feeds log2 buckets (the tile shape's key)
// and the serving loop's work estimate.
double est_particles(const sfk_tree_s* t, const double* lo, const double* hi) {
  if (t->est_sat.empty()) return 0.0;
  constexpr int G = kEstGrid, G1 = kEstGrid + 1;
  double a[3], b[3];
  for (int k = 0; k < 3; ++k) {
    const double ext = t->bbox[3 + k] - t->bbox[k];
    if (ext > 0.0) {
      a[k] = std::min<double>(G, std::max(0.0, (lo[k] - t->bbox[k]) / ext * G));
      b[k] = std::min<double>(G, std::max(0.0, (hi[k] - t->bbox[k]) / ext * G));
    } else {
      const bool in = lo[k] <= t->bbox[k] && t->bbox[k] <= hi[k];
      a[k] = 0.0;
      b[k] = in ? G : 0.0;
    }
    if (!(b[k] > a[k])) return 0.0;
  }
  auto F = [&](double x, double y, double z) {
    const int i = std::min(G - 1, (int)x), j = std::min(G - 1, (int)y), k = std::min(G - 1, (int)z);
    const double fx = x - i, fy = y - j, fz = z - k;
    double v = 0.0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          v += (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz) *
               t->est_sat[(size_t)(i + dx) + G1 * ((size_t)(j + dy) + G1 * (size_t)(k + dz))];
    return v;
  };
  const double c = F(b[0], b[1], b[2]) - F(a[0], b[1], b[2]) - F(b[0], a[1], b[2]) -
                   F(b[0], b[1], a[2]) + F(a[0], a[1], b[2]) + F(a[0], b[1], a[2]) +
                   F(b[0], a[1], a[2]) - F(a[0], a[1], a[2]);
  return std::max(0.0, c);
}

// Estimated particles per grid node of a ROI: the particles in its box
// widened by the support, over its nodes (sparse ROIs below about one).
double particles_per_node(sfk_tree t, const sfk_roi* r) {
  if (!t || !uniform_bw(r)) return 0.0;
  double lo[3], hi[3], m = 1.0;
  for (int k = 0; k < 3; ++k) {
    const double h = r->bw == SFK_BW_FIXED ? (double)r->h[k]
                                           : (double)r->h[0] * (r->hi[k] - r->lo[k]);
    const double reach = h * (r->kernel == SFK_KERNEL_GAUSS_TRUNC3 ? 3.0 : 1.0);
    lo[k] = r->lo[k] - reach;
    hi[k] = r->hi[k] + reach;
    m *= (double)r->res[k];
  }
  return est_particles(t, lo, hi) / m;
}

// Autotuner key: kernel, bandwidth mode, the support radius measured in
// node spacings (log2 bucket; per-point bandwidths share one bucket) and,
// for uniform bandwidths, the estimated particles per grid node (log2
// bucket, 0 = below 1/8 ... 7 = 16 or more).
int tune_key(sfk_tree t, const sfk_roi* r) {
  double hs = 0.0;
  if (r->bw == SFK_BW_FIXED || r->bw == SFK_BW_ROI_SCALED) {
    double rs = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double h = r->bw == SFK_BW_FIXED ? (double)r->h[k] : (double)r->h[0] * (r->hi[k] - r->lo[k]);
      rs = std::max(rs, h / ((r->hi[k] - r->lo[k]) / (r->res[k] - 1)));
    }
    hs = r->kernel == SFK_KERNEL_GAUSS_TRUNC3 ? 3.0 * rs : rs;
  }
  const int bucket = hs <= 0.0 ? 0 : std::min(7, std::max(1, (int)std::floor(std::log2(hs)) + 4));
  const double ppn = particles_per_node(t, r);
  const int dens = ppn <= 0.0 ? 0 : std::min(7, std::max(0, (int)std::floor(std::log2(ppn)) + 4));
  return ((r->kernel * 4 + r->bw) * 8 + bucket) * 8 + dens;
}

// Untuned default tile shape. Smaller tiles pay off only where a node's
// support holds many particles (measured on clumpy clouds of 1e7-1e9 points:
// below about 2048 expected particles per node support the per-tile work
// dominates and 4x4x4 wins at every support/spacing ratio). Above that, per
// support/spacing bucket: a support below half the node spacing reaches at
// most one node per particle, so one node per wavefront reads only the
// particles near nodes; larger supports share each particle among more nodes.
int default_shape(int key, double particles_per_support, bool sweep_ok) {
  // sparse uniform-bandwidth ROIs (under about one particle per node) take
  // bricks: a tile's fixed costs (claim, range query, reduction) would
  // dominate its few pairs (measured: a 256^3 box of side 1/64 around a
  // clump of a 100M cloud, 0.27 ms in bricks vs 1.40 ms in 4x4x4 tiles)
  const int dens = key & 7, kb = (key >> 6) & 3, hs_bucket = (key >> 3) & 7;
  const bool uniform = kb == SFK_BW_FIXED || kb == SFK_BW_ROI_SCALED;
  // dense uniform-bandwidth ROIs (1 or more particles per node) whose
  // supports span at most kSweepMaxNM nodes per axis: the particle sweep
  // (autotuned on the served 1e9-point trace, 108 requests: the sweep is
  // fastest in 8 of the 10 keys from 1 particle per node up, by 1.6-7x at
  // 16 or more; below 1, bricks or 4x4x4 tiles). Supports of radius 2
  // spacings or more give each particle 30 or more nodes, which pays for
  // the sweep's per-box costs from half a particle per node (measured on a
  // 100M cloud at 256^3 and radius 2.55 spacings: a box of side 0.5 at 0.8
  // particles per node, 2.1 ms in the sweep vs 2.9 in tiles and 4.2 in
  // bricks; at radius 1.27 and 0.74 particles per node bricks still win)
  if (uniform && sweep_ok && (dens >= 4 || (dens == 3 && hs_bucket >= 5)))
    return kSweepShape;
  // Supports of radius 2 spacings or more from 1/8 to 1/2 particle per node
  // take 4x4x4 tiles (shape 1): a 100M cloud at 256^3, box of side 1/4, 1.97
  // ms vs 2.41 in bricks. Sparser ROIs keep bricks (side 1/16: 0.95 vs 1.63
  // ms). (Radius 1-2 spacings at 1/2 to 1 particle per node also favoured
  // tiles on zoom boxes, but the served trace and the 256-ROI batch, whose
  // requests fall there, were faster with bricks: 5.52e11 vs 5.42e11 evals/s
  // and 12.7 vs 13.6 ms.)
  if (uniform && dens < 4) return dens >= 1 && hs_bucket >= 5 ? 1 : kBrickShape;
  // Dense ROIs keep wavefront tiles, by support/spacing ratio: below 0.5 a
  // particle reaches at most one node, so one node per wavefront reads only
  // the particles near nodes (where a node's support holds many particles);
  // between 0.5 and 2, 4x2x2 tiles waste fewer pairs than 4x4x4 (measured on
  // 1e8 and 1e9-point clouds: 10-30% less time for boxes of side 0.6-1 at
  // 75^3-128^3); above 2, 4x4x4.
  const int bucket = (key >> 3) & 7;
  if (bucket == 0) return 1;
  if (bucket <= 2) return particles_per_support >= 2048.0 ? 5 : 1;
  if (bucket <= 4) return 3;
  return 1;
}

// Expected particles in the support box of one node at the cloud's mean
// density (0 for per-particle bandwidths).
double particles_per_support(sfk_tree t, const sfk_roi* r) {
  if (!t || (r->bw != SFK_BW_FIXED && r->bw != SFK_BW_ROI_SCALED)) return 0.0;
  double vol = 1.0, sup = 1.0;
  for (int k = 0; k < 3; ++k) {
    vol *= std::max(1e-30, (double)t->bbox[3 + k] - (double)t->bbox[k]);
    const double h = r->bw == SFK_BW_FIXED ? (double)r->h[k] : (double)r->h[0] * (r->hi[k] - r->lo[k]);
    sup *= 2.0 * h * (r->kernel == SFK_KERNEL_GAUSS_TRUNC3 ? 3.0 : 1.0);
  }
  return (double)t->n * sup / vol;
}

// The particle sweep takes uniform bandwidths whose supports span at most
// kSweepMaxNM nodes per axis.
bool sweep_ok(sfk_tree t, const sfk_roi* r) {
  if (!uniform_bw(r)) return false;
  const int nm = sweep_nm(resolve_cloud_roi(t, r, false));
  return nm >= 1 && nm <= kSweepMaxNM;
}

// The untuned default of a ROI when the sweep is not an option.
int default_shape_no_sweep(sfk_tree t, const sfk_roi* r) {
  return default_shape(tune_key(t, r), particles_per_support(t, r), false);
}

TileShape choose_shape(sfk_ctx c, sfk_tree t, const sfk_roi* r) {
  int id = 0;
  if (c->opts.tile_shape > 0) {
    id = c->opts.tile_shape;
  } else {
    const int key = tune_key(t, r);
    auto it = c->tune.find(key);
    id = it != c->tune.end() ? it->second
                             : default_shape(key, particles_per_support(t, r), sweep_ok(t, r));
  }
  if (id == kBrickShape && !uniform_bw(r)) id = 1;  // bricks need a uniform bandwidth
  if (id == kSweepShape && !sweep_ok(t, r)) id = default_shape_no_sweep(t, r);
  return shape_of(id);
}

// Launch everything a ticket needs on a slot. CLOUD ROIs go through one
// persistent pipeline per (kernel, bandwidth) group; IN_ROI ROIs through
// the sub-cloud path (blocking on the slot's stream).
sfk_status launch_ticket(sfk_ctx c, Ticket& tk, Slot& sl) {
  std::vector<const sfk_roi*> cloud;
  std::vector<const sfk_roi*> sub;
  for (const sfk_roi& r : tk.rois) (r.set == SFK_SET_IN_ROI ? sub : cloud).push_back(&r);
  (void)absorb_stats(sl.ws, sl.st);  // an error word was reported at completion
  if (!cloud.empty()) {
    // profiling events cannot be recorded inside a captured graph: while
    // profiling, batches use direct launches (the same kernels)
    if (c->opts.disable_graphs || c->prof_on)
      SFK_TRY(enqueue_cloud_rois(c, tk.tree, cloud, false, sl.ws, sl.st, sl.stream));
    else
      SFK_TRY(enqueue_cloud_rois_graph(c, tk.tree, cloud, sl));
  }
  for (const sfk_roi* r : sub)
    SFK_TRY(eval_subcloud(c, tk.tree, r, false, shape_of(1), sl.ws, sl.st, sl.stream, nullptr));
  SFK_HIP(c, hipEventRecord(sl.done, sl.stream));
  return SFK_OK;
}

int free_slot(sfk_ctx c) {
  for (int i = 0; i < kNumSlots; ++i)
    if (!c->slots[i].busy) return i;
  return -1;
}

// Retire finished slots and start pending tickets. Never blocks.
sfk_status pump(sfk_ctx c) {
  for (int i = 0; i < kNumSlots; ++i) {
    Slot& sl = c->slots[i];
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) {
      set_err(c, "batch failed on the device: %s", hipGetErrorString(q));
      auto it = c->tickets.find(sl.ticket);
      if (it != c->tickets.end()) {
        it->second.state = 4;
        it->second.status = SFK_E_DEVICE;
      }
      sl.busy = false;
      continue;
    }
    auto it = c->tickets.find(sl.ticket);
    const bool bad = absorb_stats(sl.ws, sl.st);
    if (it != c->tickets.end()) {
      it->second.state = bad ? 4 : 2;
      if (bad) it->second.status = SFK_E_INTERNAL;
    }
    if (bad) {
      set_err(c, "%s", kErrLeafIds);
      SFK_TRY(clear_err_word(c, sl.ws, sl.stream));
    }
    sl.busy = false;
    sl.ticket = -1;
  }
  while (!c->pending.empty()) {
    const int si = free_slot(c);
    if (si < 0) break;
    const int64_t id = c->pending.front();
    c->pending.pop_front();
    auto it = c->tickets.find(id);
    if (it == c->tickets.end() || it->second.state != 0) continue;
    Slot& sl = c->slots[si];
    sl.busy = true;
    sl.ticket = id;
    it->second.slot = si;
    it->second.state = 1;
    const sfk_status st = launch_ticket(c, it->second, sl);
    if (st != SFK_OK) {
      it->second.state = 4;
      it->second.status = st;
      (void)hipStreamSynchronize(sl.stream);
      sl.busy = false;
      sl.ticket = -1;
      return st;
    }
  }
  return SFK_OK;
}

sfk_status check_ctx(sfk_ctx c) {
  if (!c) {
    set_err(nullptr, "NULL context");
    return SFK_E_INVAL;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    set_err(c, "hipSetDevice(%d) failed", c->device);
    return SFK_E_DEVICE;
  }
  return SFK_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* sfk_version(void) { return "sfkde 0.1 (gfx950)"; }

const char* sfk_status_string(sfk_status s) {
  switch (s) {
    case SFK_OK: return "ok";
    case SFK_E_INVAL: return "invalid argument";
    case SFK_E_NOMEM: return "out of device memory";
    case SFK_E_BUDGET: return "device-memory budget exceeded";
    case SFK_E_DEVICE: return "device error";
    case SFK_E_NOT_READY: return "not ready";
    case SFK_E_CANCELLED: return "cancelled";
    case SFK_E_UNSUPPORTED: return "unsupported";
    case SFK_E_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* sfk_last_error(sfk_ctx ctx) {
  if (ctx) return ctx->err.c_str();
  return g_tls_err.c_str();
}

sfk_status sfk_ctx_create(int device, const sfk_allocator* alloc, size_t hbm_budget_bytes,
                          sfk_ctx* out) {
  SFK_GUARD_BEGIN
  if (!out) {
    set_err(nullptr, "out is NULL");
    return SFK_E_INVAL;
  }
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) {
    set_err(nullptr, "allocator needs both alloc and free");
    return SFK_E_INVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    set_err(nullptr, "no HIP device available");
    return SFK_E_DEVICE;
  }
  if (device < 0 || device >= ndev) {
    set_err(nullptr, "device %d out of range (%d devices)", device, ndev);
    return SFK_E_INVAL;
  }
  if (hipSetDevice(device) != hipSuccess) {
    set_err(nullptr, "hipSetDevice(%d) failed", device);
    return SFK_E_DEVICE;
  }
  sfk_ctx c = new sfk_ctx_s();
  c->device = device;
  if (alloc) {
    c->alloc = *alloc;
    c->use_alloc = true;
  }
  c->budget = hbm_budget_bytes;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    if (prop.multiProcessorCount > 0) c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);  // drop feature suffixes
  }
  for (int i = 0; i < kNumSlots; ++i) {
    if (hipStreamCreateWithFlags(&c->slots[i].stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->slots[i].done, hipEventDisableTiming) != hipSuccess) {
      set_err(nullptr, "stream creation failed");
      sfk_ctx_destroy(c);
      return SFK_E_DEVICE;
    }
  }
  if (hipEventCreateWithFlags(&c->direct_last, hipEventDisableTiming) != hipSuccess) {
    set_err(nullptr, "event creation failed");
    sfk_ctx_destroy(c);
    return SFK_E_DEVICE;
  }
  // Every staging slot's event and pinned buffers now, not at its first use
  // (an event and two pinned allocations cost ~0.15 ms of host time, which
  // the first calls of a fresh context would otherwise pay one by one).
  const size_t st_min = sizeof(BatchHdr) + 64 * sizeof(RoiDev);
  sfk_status st_ok = SFK_OK;
  for (int i = 0; i < kStagingRing && st_ok == SFK_OK; ++i)
    st_ok = staging_reserve(c, c->direct_st[i], st_min);
  for (int i = 0; i < kNumSlots && st_ok == SFK_OK; ++i)
    st_ok = staging_reserve(c, c->slots[i].st, st_min);
  if (st_ok != SFK_OK) {
    set_err(nullptr, "pinned staging allocation failed");
    sfk_ctx_destroy(c);
    return st_ok;
  }
  // sfk_eval_roi_noalloc: the scratch address of this device (the device is
  // current), a pinned descriptor ring and its events
  c->na_scratch = noalloc_scratch_of(device);
  if (hipEventCreateWithFlags(&c->na_last, hipEventDisableTiming) != hipSuccess) {
    set_err(nullptr, "event creation failed");
    sfk_ctx_destroy(c);
    return SFK_E_DEVICE;
  }
  for (int i = 0; i < kStagingRing; ++i) {
    if (hipHostMalloc((void**)&c->na_host[i], sizeof(BatchHdr) + sizeof(RoiDev)) != hipSuccess ||
        hipEventCreateWithFlags(&c->na_ev[i], hipEventDisableTiming) != hipSuccess) {
      set_err(nullptr, "pinned staging allocation failed");
      sfk_ctx_destroy(c);
      return SFK_E_NOMEM;
    }
  }
  *out = c;
  return SFK_OK;
  SFK_GUARD_END(nullptr)
}

static void release_ws(sfk_ctx c, Workspace& ws) {
  DevBuf* bufs[] = {&ws.hdr_rois, &ws.coords, &ws.tile_cnt, &ws.tile_fit, &ws.tile_done,
                    &ws.leaf_off, &ws.partial_off, &ws.chunk_off, &ws.leaves, &ws.item_tile,
                    &ws.partials, &ws.claims, &ws.plan_tmp, &ws.roi_leaves, &ws.roi_nl,
                    &ws.tile_slots};
  for (DevBuf* b : bufs) ws_release(c, *b);
}

static void release_staging(Staging& st) {
  if (st.ev_valid) (void)hipEventSynchronize(st.ev);
  if (st.host) (void)hipHostFree(st.host);
  if (st.hdr_host) (void)hipHostFree(st.hdr_host);
  if (st.ev) (void)hipEventDestroy(st.ev);
  st = Staging();
}

sfk_status sfk_ctx_destroy(sfk_ctx c) {
  SFK_GUARD_BEGIN
  if (!c) return SFK_OK;
  (void)hipSetDevice(c->device);
  for (int i = 0; i < kNumSlots; ++i) {
    Slot& sl = c->slots[i];
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    drop_graph(sl.gc);
    release_ws(c, sl.ws);
    release_staging(sl.st);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (c->direct_last_valid) (void)hipEventSynchronize(c->direct_last);
  release_ws(c, c->direct_ws);
  for (int i = 0; i < kStagingRing; ++i) release_staging(c->direct_st[i]);
  if (c->direct_last) (void)hipEventDestroy(c->direct_last);
  if (c->na_last_valid) (void)hipEventSynchronize(c->na_last);
  if (c->na_last) (void)hipEventDestroy(c->na_last);
  for (int i = 0; i < kStagingRing; ++i) {
    if (c->na_ev[i]) (void)hipEventDestroy(c->na_ev[i]);
    if (c->na_host[i]) (void)hipHostFree(c->na_host[i]);
  }
  for (const ProfRec& r : c->prof_pending) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  delete c;
  return SFK_OK;
  SFK_GUARD_END(nullptr)
}

sfk_status sfk_build_tree(sfk_ctx c, const float* d_xyz, int64_t n, const float* d_h,
                          const sfk_tree_opts* opts, void* hip_stream, sfk_tree* out) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!out) {
    set_err(c, "out is NULL");
    return SFK_E_INVAL;
  }
  *out = nullptr;
  if (n < 0 || n >= (int64_t)INT32_MAX - SFK_LEAF) {
    set_err(c, "n = %lld out of range [0, 2^31 - 64)", (long long)n);
    return SFK_E_INVAL;
  }
  if (n > 0 && !d_xyz) {
    set_err(c, "d_xyz is NULL");
    return SFK_E_INVAL;
  }
  sfk_tree_opts o{};
  if (opts) o = *opts;
  if (o.leaf_size != 0 && o.leaf_size != SFK_LEAF) {
    set_err(c, "leaf_size %d unsupported (0 or 64)", o.leaf_size);
    return SFK_E_UNSUPPORTED;
  }
  if (o.knn_k < 0 || o.knn_k > 64) {
    set_err(c, "knn_k = %d out of range [0, 64]", o.knn_k);
    return SFK_E_INVAL;
  }
  if (o.knn_k > 0 && n > 0 && o.knn_k >= n) {
    set_err(c, "knn_k = %d needs at least k + 1 = %d particles (n = %lld)", o.knn_k,
            o.knn_k + 1, (long long)n);
    return SFK_E_INVAL;
  }
  if (o.knn_k > 0 && d_h) {
    set_err(c, "give either knn_k or d_h, not both");
    return SFK_E_INVAL;
  }
  if (o.key_bits < 0 || o.key_bits > 21) {
    set_err(c, "key_bits = %d out of range [0, 21]", o.key_bits);
    return SFK_E_INVAL;
  }
  if (o.curve != SFK_CURVE_HILBERT && o.curve != SFK_CURVE_MORTON) {
    set_err(c, "unknown curve %d", o.curve);
    return SFK_E_INVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  sfk_tree t = new sfk_tree_s();
  t->ctx = c;
  t->n = n;
  t->knn_k = o.knn_k;
  auto fail = [&](sfk_status st) {
    (void)hipStreamSynchronize(s);
    tree_free(c, t, t->pts);
    tree_free(c, t, t->perm);
    tree_free(c, t, t->nodes);
    tree_free(c, t, t->node_ih);
    tree_free(c, t, t->h2);
    delete t;
    return st;
  };
  t->n_leaves = (int32_t)((n + SFK_LEAF - 1) / SFK_LEAF);
  int32_t total_nodes = 0;
  level_layout(t->n_leaves, t->level_off, t->level_cnt, &t->n_levels, &total_nodes);
  if (t->n_levels > 6) return fail((set_err(c, "hierarchy too deep"), SFK_E_INTERNAL));
  const int64_t n_slots = (int64_t)t->n_leaves * SFK_LEAF;
  sfk_status st;
  if ((st = tree_alloc(c, t, t->pts, sizeof(float4) * (size_t)n_slots, "particles")) != SFK_OK ||
      (st = tree_alloc(c, t, t->perm, sizeof(int32_t) * (size_t)n, "permutation")) != SFK_OK ||
      (st = tree_alloc(c, t, t->nodes, sizeof(NodeBox) * (size_t)total_nodes, "boxes")) != SFK_OK)
    return fail(st);
  if (n == 0) {
    *out = t;
    return SFK_OK;
  }
  if (d_h) {
    TmpBuf bad(c);
    if ((st = bad.get(sizeof(int32_t), "check")) != SFK_OK) return fail(st);
    int32_t nbad = 0;
    if (sfk::launch_count_nonpositive(d_h, n, bad.as<int32_t>(), s) != hipSuccess ||
        hipMemcpyAsync(&nbad, bad.b.p, sizeof nbad, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail((set_err(c, "bandwidth check failed"), SFK_E_DEVICE));
    if (nbad > 0)
      return fail((set_err(c, "%d per-particle bandwidths are not finite and > 0", nbad), SFK_E_INVAL));
  }
  // Build scratch lives until the build's last synchronisation, and each
  // stage's buffers are taken while the GPU runs the stage before, so no
  // allocation (a host callback under a caller's allocator) or release sits
  // between two launches.
  TmpBuf part(c), res(c), keys(c), keys2(c), vals(c), vals2(c), stmp(c), sub(c), moved(c);
  const bool per_point = o.knn_k > 0 || d_h;
  // bounding box (6 floats) and the count of non-finite coordinates, read at
  // the build's one synchronisation at the end: nothing before needs them on
  // the host (the key kernel reads the box on the device, and the k-NN returns
  // at once when the count is non-zero)
  float bb[7];
  {
    // bounding box + finiteness
    const int nblk = 1024;
    if ((st = part.get(sizeof(float) * 7 * nblk, "bbox partials")) != SFK_OK ||
        (st = res.get(sizeof(float) * 8, "bbox")) != SFK_OK)
      return fail(st);
    if (sfk::launch_bbox(d_xyz, n, part.as<float>(), nblk, res.as<float>(), s) != hipSuccess)
      return fail((set_err(c, "bounding box kernel failed"), SFK_E_DEVICE));
    // curve keys and the sort
    // automatic: about 4x finer per axis than n^(1/3), at least 10 bits
    // (10M points: 30-bit keys, four 8-bit sort passes)
    int bits = o.key_bits;
    if (bits == 0) {
      const int lg = (int)std::ceil(std::log2((double)std::max<int64_t>(n, 2)));
      bits = std::min(21, std::max(10, (lg + 2) / 3 + 2));
    }
    if ((st = keys.get(sizeof(uint64_t) * (size_t)n, "sort keys")) != SFK_OK ||
        (st = keys2.get(sizeof(uint64_t) * (size_t)n, "sort keys")) != SFK_OK ||
        (st = vals.get(sizeof(uint32_t) * (size_t)n, "sort values")) != SFK_OK ||
        (st = vals2.get(sizeof(uint32_t) * (size_t)n, "sort values")) != SFK_OK ||
        (st = stmp.get(sfk::radix_sort_tmp_bytes(n), "sort scratch")) != SFK_OK)
      return fail(st);
    int alt = 0;
    ProfScope prof(c, PK_BUILD, s);
    // keys of at most 32 bits are sorted as uint32 (a third less traffic per pass)
    const bool narrow = 3 * bits <= 32;
    if (sfk::launch_curve_keys(d_xyz, n, res.as<float>(), bits, o.curve == SFK_CURVE_HILBERT,
                               keys.b.p, vals.as<uint32_t>(), s) != hipSuccess ||
        (narrow ? sfk::radix_sort_pairs_u32(keys.as<uint32_t>(), vals.as<uint32_t>(),
                                            keys2.as<uint32_t>(), vals2.as<uint32_t>(), n,
                                            3 * bits, stmp.b.p, stmp.b.bytes, s, &alt)
                : sfk::radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(),
                                        keys2.as<uint64_t>(), vals2.as<uint32_t>(), n, 3 * bits,
                                        stmp.b.p, stmp.b.bytes, s, &alt)) != hipSuccess)
      return fail((set_err(c, "sort failed"), SFK_E_DEVICE));
    // the k-NN's sub-block boxes come out of the gather, from the same registers
    const bool knn = per_point && o.knn_k > 0;
    if (knn &&
        (st = sub.get(sfk::knn_sub_box_bytes(t->n_leaves), "k-NN sub-block boxes")) != SFK_OK)
      return fail(st);
    if (sfk::launch_gather(d_xyz, alt ? vals2.as<uint32_t>() : vals.as<uint32_t>(), n,
                           t->n_leaves, (float4*)t->pts.p, (int32_t*)t->perm.p,
                           (NodeBox*)t->nodes.p + t->level_off[0],
                           knn ? sub.as<float>() : nullptr, s) != hipSuccess)
      return fail((set_err(c, "gather failed"), SFK_E_DEVICE));
    if ((st = build_boxes(c, (const float4*)t->pts.p, n, t->n_leaves, (NodeBox*)t->nodes.p,
                          t->level_off, t->level_cnt, t->n_levels, s, nullptr, true)) != SFK_OK)
      return fail(st);
    if (per_point) {
      // the per-point stage's buffers, while the sort runs
      if ((st = tree_alloc(c, t, t->node_ih, sizeof(float4) * (size_t)total_nodes,
                           "node bandwidths")) != SFK_OK ||
          (st = moved.get(sizeof(int32_t), "moved-particle flag")) != SFK_OK)
        return fail(st);
      if (knn && (st = tree_alloc(c, t, t->h2, sizeof(float) * (size_t)n_slots,
                                  "k-NN distances")) != SFK_OK)
        return fail(st);
    }
  }
  if (per_point) {
    if (o.knn_k > 0) {
      ProfScope prof(c, PK_KNN, s);
      if (sfk::launch_knn(view_of(t), sub.as<float>(), o.knn_k, (float*)t->h2.p,
                          res.as<float>() + 6, s) != hipSuccess)
        return fail((set_err(c, "k-NN kernel failed"), SFK_E_DEVICE));
    }
    if (sfk::launch_iso_params((float4*)t->pts.p, (const float*)t->h2.p, d_h,
                               (const int32_t*)t->perm.p, n, t->n_leaves,
                               (float4*)t->node_ih.p + t->level_off[0], moved.as<int32_t>(),
                               s) != hipSuccess)
      return fail((set_err(c, "bandwidth kernel failed"), SFK_E_DEVICE));
    // zero-bandwidth particles moved to the sentinel: refresh the boxes (the
    // kernels return at once when no particle moved)
    if ((st = build_boxes(c, (const float4*)t->pts.p, n, t->n_leaves, (NodeBox*)t->nodes.p,
                          t->level_off, t->level_cnt, t->n_levels, s,
                          moved.as<int32_t>())) != SFK_OK)
      return fail(st);
    if (sfk::launch_node_ih((const float4*)t->pts.p, nullptr, PP_ISO, n,
                            (const NodeBox*)t->nodes.p, t->level_off, t->level_cnt, t->n_levels,
                            (float4*)t->node_ih.p, 1, s) != hipSuccess)
      return fail((set_err(c, "node bandwidth kernel failed"), SFK_E_DEVICE));
    t->pp_mode = PP_ISO;
  }
  // the coarse box levels for host-side particle-count estimates
  if (t->n_levels > 0) {
    int hl = 0;
    while (hl + 1 < t->n_levels && t->level_cnt[hl] > kHostLevelNodes) ++hl;
    t->host_level = hl;
    t->host_base = t->level_off[hl];
    t->host_nodes.resize((size_t)(total_nodes - t->host_base));
    if (hipMemcpyAsync(t->host_nodes.data(), (const NodeBox*)t->nodes.p + t->host_base,
                       sizeof(NodeBox) * t->host_nodes.size(), hipMemcpyDeviceToHost,
                       s) != hipSuccess)
      return fail((set_err(c, "tree build failed on the device"), SFK_E_DEVICE));
  }
  // pageable destination: the copy returns once the stream has run up to it
  if (hipMemcpyAsync(bb, res.b.p, sizeof bb, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail((set_err(c, "tree build failed on the device"), SFK_E_DEVICE));
  if (bb[6] > 0.0f)
    return fail((set_err(c, "%.0f non-finite coordinates", (double)bb[6]), SFK_E_INVAL));
  for (int k = 0; k < 6; ++k) t->bbox[k] = bb[k];
  build_est_table(t);
  if (c->prof_on) ++c->prof_builds;
  *out = t;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_profile_enable(sfk_ctx c, int32_t on) {
  SFK_TRY(check_ctx(c));
  c->prof_on = on != 0;
  return SFK_OK;
}

sfk_status sfk_profile_read(sfk_ctx c, sfk_profile* out, int32_t reset) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  for (const ProfRec& r : c->prof_pending) {
    SFK_HIP(c, hipEventSynchronize(r.b));
    float ms = 0.0f;
    SFK_HIP(c, hipEventElapsedTime(&ms, r.a, r.b));
    c->prof_ms[r.kind] += ms;
    if (r.kind == PK_EVAL) {
      ++c->prof_evals;
      if (r.hdr_dev) {
        BatchHdr h;
        if (hipMemcpy(&h, r.hdr_dev, sizeof h, hipMemcpyDeviceToHost) == hipSuccess) {
          c->prof_last_leaves = h.total_leaves;
          c->prof_last_items = h.n_items;
        }
      }
    }
    c->prof_pool.push_back(r.a);
    c->prof_pool.push_back(r.b);
  }
  c->prof_pending.clear();
  if (out) {
    out->tile_count_ms = c->prof_ms[PK_TILE_COUNT];
    out->plan_ms = c->prof_ms[PK_PLAN];
    out->tile_fill_ms = c->prof_ms[PK_TILE_FILL];
    out->eval_ms = c->prof_ms[PK_EVAL];
    out->build_ms = c->prof_ms[PK_BUILD];
    out->knn_ms = c->prof_ms[PK_KNN];
    out->eval_launches = c->prof_evals;
    out->builds = c->prof_builds;
    out->last_total_leaves = c->prof_last_leaves;
    out->last_items = c->prof_last_items;
  }
  if (reset) {
    for (int k = 0; k < PK_N; ++k) c->prof_ms[k] = 0.0;
    c->prof_evals = c->prof_builds = 0;
  }
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_tree_info(sfk_tree t, int64_t* n, double bbox[6], size_t* device_bytes) {
  if (!t) {
    set_err(nullptr, "NULL tree");
    return SFK_E_INVAL;
  }
  if (n) *n = t->n;
  if (bbox)
    for (int k = 0; k < 6; ++k) bbox[k] = t->bbox[k];
  if (device_bytes) *device_bytes = t->bytes;
  return SFK_OK;
}

sfk_status sfk_tree_destroy(sfk_tree t) {
  SFK_GUARD_BEGIN
  if (!t) return SFK_OK;
  sfk_ctx c = t->ctx;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  // graphs captured against this tree hold its device pointers
  for (int i = 0; i < kNumSlots; ++i)
    if (c->slots[i].gc.tree == t) drop_graph(c->slots[i].gc);
  tree_free(c, t, t->pts);
  tree_free(c, t, t->perm);
  tree_free(c, t, t->nodes);
  tree_free(c, t, t->node_ih);
  tree_free(c, t, t->h2);
  delete t;
  return SFK_OK;
  SFK_GUARD_END(nullptr)
}

sfk_status sfk_set_eval_opts(sfk_ctx c, const sfk_eval_opts* opts) {
  SFK_TRY(check_ctx(c));
  if (!opts) {
    set_err(c, "opts is NULL");
    return SFK_E_INVAL;
  }
  if (opts->tile_shape < 0 || opts->tile_shape > kNumShapes || opts->chunk_leaves < 0 ||
      opts->chunk_leaves > (1 << 20) || opts->persistent_waves_per_cu < 0 ||
      opts->persistent_waves_per_cu > 64 || opts->list_capacity < 0 ||
      opts->partial_capacity < 0 ||
      opts->disable_graphs < 0 || opts->disable_graphs > 1) {
    set_err(c, "evaluation options out of range");
    return SFK_E_INVAL;
  }
  c->opts = *opts;
  return SFK_OK;
}

// Stream-ordered single ROI on the caller's stream.
// CLOUD-set ROIs in one batch on the caller's stream (the direct path's
// workspace and staging ring), optionally all with one tile shape.
static sfk_status eval_direct_cloud(sfk_ctx c, sfk_tree t, const std::vector<const sfk_roi*>& v,
                                    hipStream_t s, bool count_mode, const TileShape* force_ts) {
  if (c->direct_last_valid && c->direct_last_stream != s)
    SFK_HIP(c, hipStreamWaitEvent(s, c->direct_last, 0));
  const int oldest = c->direct_next;
  Staging& st = c->direct_st[c->direct_next];
  c->direct_next = (c->direct_next + 1) % kStagingRing;
  if (absorb_ready(c->direct_ws, c->direct_st, kStagingRing, oldest)) {
    // an earlier stream-ordered evaluation of this context found a bad leaf id
    SFK_TRY(clear_err_word(c, c->direct_ws, s));
    set_err(c, "%s (reported by the next call on the context)", kErrLeafIds);
    return SFK_E_INTERNAL;
  }
  SFK_TRY(enqueue_cloud_rois(c, t, v, count_mode, c->direct_ws, st, s, force_ts));
  SFK_HIP(c, hipEventRecord(c->direct_last, s));
  c->direct_last_valid = true;
  c->direct_last_stream = s;
  c->direct_ws.last_use = c->direct_last;
  c->direct_ws.last_use_valid = true;
  return SFK_OK;
}

static sfk_status eval_direct(sfk_ctx c, sfk_tree t, const sfk_roi* roi, hipStream_t s,
                              bool count_mode) {
  if (roi->set != SFK_SET_IN_ROI) {
    std::vector<const sfk_roi*> v{roi};
    return eval_direct_cloud(c, t, v, s, count_mode, nullptr);
  }
  if (c->direct_last_valid && c->direct_last_stream != s)
    SFK_HIP(c, hipStreamWaitEvent(s, c->direct_last, 0));
  Staging& st = c->direct_st[c->direct_next];
  c->direct_next = (c->direct_next + 1) % kStagingRing;
  SFK_TRY(eval_subcloud(c, t, roi, count_mode, shape_of(1), c->direct_ws, st, s, nullptr));
  SFK_HIP(c, hipEventRecord(c->direct_last, s));
  c->direct_last_valid = true;
  c->direct_last_stream = s;
  c->direct_ws.last_use = c->direct_last;
  c->direct_ws.last_use_valid = true;
  return SFK_OK;
}

sfk_status sfk_eval_roi(sfk_ctx c, sfk_tree t, const sfk_roi* roi, void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t) {
    set_err(c, "NULL tree");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  return eval_direct(c, t, roi, (hipStream_t)hip_stream, false);
  SFK_GUARD_END(c)
}

// sfk_eval_roi with its workspace carved from this device's static scratch
// array: no device or host allocation. Layout, in order: descriptors, node
// coordinates, claim counters, the ROI leaf list, plan block sums, the
// per-tile arrays and leaf slots (fixed by the tile count), then the work
// items, partial sums and leaf lists share what is left. Smaller list and
// partial capacities than the allocating path's only move tiles to the
// walking modes, which visit the same leaves in the same order and chunks,
// so the grid is bitwise the same.
sfk_status sfk_eval_roi_noalloc(sfk_ctx c, sfk_tree t, const sfk_roi* roi, void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t) {
    set_err(c, "NULL tree");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  if (roi->set != SFK_SET_CLOUD || roi->bw == SFK_BW_MBE) {
    set_err(c, "the no-allocation path evaluates CLOUD-set, non-MBE ROIs (the in-box "
               "sub-cloud needs its own buffers)");
    return SFK_E_UNSUPPORTED;
  }
  if (!c->na_scratch) {
    set_err(c, "the scratch array of device %d has no device address", c->device);
    return SFK_E_DEVICE;
  }
  const hipStream_t s = (hipStream_t)hip_stream;
  const GroupRoi g = resolve_cloud_roi(t, roi, false);
  TileShape ts = choose_shape(c, t, roi);
  const size_t cap = SFK_NOALLOC_SCRATCH_BYTES;
  auto rb = [](size_t b) { return round_bytes(std::max<size_t>(b, 256)); };
  RoiDev rd;
  int64_t n_tiles = 0, n_coords = 0;
  make_roidev(&g, 1, ts, &rd, &n_tiles, &n_coords);
  if (sfk::is_sweep(ts)) {
    // the particle sweep needs the node sums of all its tiles and one item
    // per box of the hierarchy's first interior level
    const int64_t boxes = t->n_leaves > SFK_FANOUT
                              ? ((int64_t)t->n_leaves + SFK_FANOUT - 1) / SFK_FANOUT
                              : (int64_t)t->n_leaves;
    const size_t need = rb(sizeof(BatchHdr) + sizeof(RoiDev)) + rb(sizeof(double) * n_coords) +
                        rb(kClaimBytes) + rb(sizeof(int32_t) * kRoiListCap) + rb(sizeof(int32_t)) +
                        rb(sizeof(unsigned long long) * kSweep * kSweep * kSweep * (size_t)n_tiles) +
                        rb(sizeof(int64_t) * (size_t)std::max<int64_t>(1, boxes));
    if (need <= cap) {
      Workspace wv;
      size_t used = 0;
      auto take = [&](DevBuf& b, size_t bytes) {
        b.p = c->na_scratch + used;
        b.bytes = bytes;
        used += rb(bytes);
      };
      take(wv.hdr_rois, sizeof(BatchHdr) + sizeof(RoiDev));
      take(wv.coords, sizeof(double) * (size_t)n_coords);
      take(wv.claims, kClaimBytes);
      take(wv.roi_leaves, sizeof(int32_t) * kRoiListCap);
      take(wv.roi_nl, sizeof(int32_t));
      take(wv.partials, sizeof(unsigned long long) * kSweep * kSweep * kSweep * (size_t)n_tiles);
      take(wv.leaves, sizeof(int64_t) * (size_t)std::max<int64_t>(1, boxes));
      BatchHdr h{};
      h.n_tiles = n_tiles;
      h.item_cap = std::max<int64_t>(1, boxes);
      h.n_rois = 1;
      h.slot_cap = slot_cap_of(ts);
      h.debug_poison = c->debug_poison;
      const int si = c->na_next;
      c->na_next = (c->na_next + 1) % kStagingRing;
      if (c->na_ev_valid[si]) SFK_HIP(c, hipEventSynchronize(c->na_ev[si]));
      std::memcpy(c->na_host[si], &h, sizeof h);
      std::memcpy(c->na_host[si] + sizeof(BatchHdr), &rd, sizeof rd);
      if (c->na_last_valid && c->na_last_stream != s)
        SFK_HIP(c, hipStreamWaitEvent(s, c->na_last, 0));
      SFK_HIP(c, hipMemcpyAsync(wv.hdr_rois.p, c->na_host[si], sizeof(BatchHdr) + sizeof(RoiDev),
                                hipMemcpyHostToDevice, s));
      const bool prof = c->prof_on;
      c->prof_on = false;
      const sfk_status st =
          launch_kernels(c, view_of(t), ts, g.kk, g.pp, false, wv, 1, n_tiles, s, sweep_nm(g));
      c->prof_on = prof;
      SFK_TRY(st);
      SFK_HIP(c, hipEventRecord(c->na_ev[si], s));
      c->na_ev_valid[si] = true;
      SFK_HIP(c, hipEventRecord(c->na_last, s));
      c->na_last_valid = true;
      c->na_last_stream = s;
      return SFK_OK;
    }
    // too large for the array: the shape the ROI would take without the sweep
    ts = shape_of(default_shape_no_sweep(t, roi));
    make_roidev(&g, 1, ts, &rd, &n_tiles, &n_coords);
  }
  const int T = ts.tx * ts.ty * ts.tz;
  const size_t nt = (size_t)n_tiles;
  const size_t fixed0 = rb(sizeof(BatchHdr) + sizeof(RoiDev)) + rb(sizeof(double) * n_coords) +
                        rb(kClaimBytes) + rb(sizeof(int32_t) * kRoiListCap) +
                        rb(sizeof(int32_t)) +
                        rb(3 * sizeof(int64_t) * (size_t)sfk::plan_blocks(n_tiles)) +
                        3 * rb(sizeof(int32_t) * nt) + 3 * rb(sizeof(int64_t) * (nt + 1));
  // leaf slots: the tile shape's capacity, halved until the fixed part
  // leaves at least half of the array to the lists (0: the fill pass walks)
  int32_t slot_cap = slot_cap_of(ts);
  while (slot_cap > 0 && fixed0 + rb(sizeof(int32_t) * slot_cap * nt) > cap / 2)
    slot_cap = slot_cap > 16 ? slot_cap / 2 : 0;
  const size_t fixed = fixed0 + rb(sizeof(int32_t) * (size_t)slot_cap * nt);
  const size_t min_var = rb(sizeof(int32_t) * (nt + 2)) + rb(sizeof(double) * T) + 256;
  if (fixed + min_var > cap) {
    set_err(c, "ROI of %lld tiles needs more than the %zu-byte scratch array of the "
               "no-allocation path", (long long)n_tiles, cap);
    return SFK_E_BUDGET;
  }
  // what is left: a quarter to partial slots (with their work items), the
  // rest to leaf-list entries (for bricks, with one work item per
  // chunk_leaves entries); 4 x 256 bytes of rounding and item slack
  const bool brick = sfk::is_brick(ts);
  const int CH = chunk_leaves_of(c);
  const size_t rest = cap - fixed - rb(sizeof(int32_t) * (nt + 1)) - 4 * 256;
  const int64_t partial_cap =
      std::max<int64_t>(1, (int64_t)(rest / 4 / (sizeof(double) * T + sizeof(int32_t))));
  const double per_leaf = sizeof(int32_t) * (1.0 + (brick ? 1.0 / CH : 0.0));
  const int64_t leaf_cap = std::max<int64_t>(
      1, (int64_t)((double)(rest - (size_t)partial_cap * (sizeof(double) * T + sizeof(int32_t))) /
                   per_leaf));
  const int64_t item_cap = n_tiles + partial_cap + 1 + (brick ? leaf_cap / CH + 1 : 0);
  Workspace wv;  // a view of the scratch array; owns nothing
  size_t used = 0;
  auto take = [&](DevBuf& b, size_t bytes) {
    b.p = c->na_scratch + used;
    b.bytes = bytes;
    used += rb(bytes);
  };
  take(wv.hdr_rois, sizeof(BatchHdr) + sizeof(RoiDev));
  take(wv.coords, sizeof(double) * (size_t)n_coords);
  take(wv.claims, kClaimBytes);
  take(wv.roi_leaves, sizeof(int32_t) * kRoiListCap);
  take(wv.roi_nl, sizeof(int32_t));
  take(wv.plan_tmp, 3 * sizeof(int64_t) * (size_t)sfk::plan_blocks(n_tiles));
  take(wv.tile_cnt, sizeof(int32_t) * nt);
  take(wv.tile_fit, sizeof(int32_t) * nt);
  take(wv.tile_done, sizeof(int32_t) * nt);
  take(wv.leaf_off, sizeof(int64_t) * (nt + 1));
  take(wv.partial_off, sizeof(int64_t) * (nt + 1));
  take(wv.chunk_off, sizeof(int64_t) * (nt + 1));
  take(wv.tile_slots, sizeof(int32_t) * (size_t)slot_cap * nt);
  take(wv.item_tile, sizeof(int32_t) * (size_t)item_cap);
  take(wv.partials, sizeof(double) * (size_t)T * (size_t)partial_cap);
  take(wv.leaves, sizeof(int32_t) * (size_t)leaf_cap);
  if (used > cap) {
    set_err(c, "internal: no-allocation layout of %zu bytes exceeds the scratch array", used);
    return SFK_E_INTERNAL;
  }
  BatchHdr h{};
  h.n_tiles = n_tiles;
  h.leaf_cap = leaf_cap;
  h.partial_cap = partial_cap;
  h.item_cap = item_cap;
  h.n_rois = 1;
  h.slot_cap = slot_cap;
  h.debug_poison = c->debug_poison;
  h.splat = brick ? 1 : 0;
  // descriptors through a pinned ring set up at context creation
  const int si = c->na_next;
  c->na_next = (c->na_next + 1) % kStagingRing;
  if (c->na_ev_valid[si]) SFK_HIP(c, hipEventSynchronize(c->na_ev[si]));
  std::memcpy(c->na_host[si], &h, sizeof h);
  std::memcpy(c->na_host[si] + sizeof(BatchHdr), &rd, sizeof rd);
  // consecutive calls of this context share the array: order them
  if (c->na_last_valid && c->na_last_stream != s)
    SFK_HIP(c, hipStreamWaitEvent(s, c->na_last, 0));
  SFK_HIP(c, hipMemcpyAsync(wv.hdr_rois.p, c->na_host[si], sizeof(BatchHdr) + sizeof(RoiDev),
                            hipMemcpyHostToDevice, s));
  // profiling events may be created on demand: none here
  const bool prof = c->prof_on;
  c->prof_on = false;
  const sfk_status st = launch_kernels(c, view_of(t), ts, g.kk, g.pp, false, wv, 1, n_tiles, s);
  c->prof_on = prof;
  SFK_TRY(st);
  SFK_HIP(c, hipEventRecord(c->na_ev[si], s));
  c->na_ev_valid[si] = true;
  SFK_HIP(c, hipEventRecord(c->na_last, s));
  c->na_last_valid = true;
  c->na_last_stream = s;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_submit(sfk_ctx c, sfk_tree t, const sfk_roi* rois, int32_t n_rois,
                      sfk_ticket* out) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !out || (!rois && n_rois > 0) || n_rois < 0) {
    set_err(c, "invalid submit arguments");
    return SFK_E_INVAL;
  }
  for (int i = 0; i < n_rois; ++i) SFK_TRY(validate_roi(c, t, &rois[i], i));
  SFK_TRY(validate_disjoint_outputs(c, rois, n_rois));
  Ticket tk;
  tk.tree = t;
  tk.rois.assign(rois, rois + n_rois);
  const int64_t id = c->next_ticket++;
  c->tickets[id] = std::move(tk);
  c->pending.push_back(id);
  *out = id;
  return pump(c);
  SFK_GUARD_END(c)
}

sfk_status sfk_poll(sfk_ctx c, sfk_ticket tid, int32_t* done) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!done) {
    set_err(c, "done is NULL");
    return SFK_E_INVAL;
  }
  auto it = c->tickets.find(tid);
  if (it == c->tickets.end()) {
    set_err(c, "unknown ticket %lld", (long long)tid);
    return SFK_E_INVAL;
  }
  SFK_TRY(pump(c));
  it = c->tickets.find(tid);
  const int state = it->second.state;
  *done = (state >= 2) ? 1 : 0;
  if (state == 3) return SFK_E_CANCELLED;
  if (state == 4) return it->second.status;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_wait(sfk_ctx c, sfk_ticket tid, int64_t timeout_us) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  auto it = c->tickets.find(tid);
  if (it == c->tickets.end()) {
    set_err(c, "unknown ticket %lld", (long long)tid);
    return SFK_E_INVAL;
  }
  const double t0 = now_s();
  while (true) {
    SFK_TRY(pump(c));
    it = c->tickets.find(tid);
    const int state = it->second.state;
    if (state == 2) {
      c->tickets.erase(it);
      return SFK_OK;
    }
    if (state == 3) {
      c->tickets.erase(it);
      return SFK_E_CANCELLED;
    }
    if (state == 4) {
      const sfk_status st = it->second.status;
      c->tickets.erase(it);
      return st;
    }
    if (timeout_us >= 0 && (now_s() - t0) * 1e6 >= (double)timeout_us) {
      set_err(c, "ticket %lld not finished within %lld us", (long long)tid, (long long)timeout_us);
      return SFK_E_NOT_READY;
    }
    if (state == 1) {
      const Slot& sl = c->slots[it->second.slot];
      if (timeout_us < 0) {
        (void)hipEventSynchronize(sl.done);
      }
    }
  }
  SFK_GUARD_END(c)
}

sfk_status sfk_cancel(sfk_ctx c, sfk_ticket tid) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  auto it = c->tickets.find(tid);
  if (it == c->tickets.end()) {
    set_err(c, "unknown ticket %lld", (long long)tid);
    return SFK_E_INVAL;
  }
  if (it->second.state == 0) {
    it->second.state = 3;
    return SFK_OK;
  }
  if (it->second.state == 3) return SFK_OK;
  set_err(c, "ticket %lld already started", (long long)tid);
  return SFK_E_NOT_READY;
  SFK_GUARD_END(c)
}

// ---------------------------------------------------------------- debug

// ---- consumers of a grid: density at points, selection, Marching Cubes cells ----

namespace {
sfk_status validate_grid_args(sfk_ctx c, const sfk_roi* roi, const float* grid, int64_t n,
                              const void* a, const void* b) {
  if (!roi || !grid) {
    set_err(c, "NULL ROI or grid");
    return SFK_E_INVAL;
  }
  if (n < 0 || (n > 0 && (!a || !b))) {
    set_err(c, "invalid point arguments (n = %lld)", (long long)n);
    return SFK_E_INVAL;
  }
  int64_t m = 1;
  for (int k = 0; k < 3; ++k) {
    if (!(std::isfinite(roi->lo[k]) && std::isfinite(roi->hi[k]) && roi->hi[k] > roi->lo[k]) ||
        roi->res[k] < 2) {
      set_err(c, "grid axis %d needs finite lo < hi and res >= 2", k);
      return SFK_E_INVAL;
    }
    m *= roi->res[k];
  }
  if (m > (int64_t)1 << 31) {
    set_err(c, "grid of %lld nodes exceeds 2^31", (long long)m);
    return SFK_E_INVAL;
  }
  return SFK_OK;
}
}  // namespace

sfk_status sfk_sample_density(sfk_ctx c, const sfk_roi* roi, const float* d_grid,
                              const float* d_xyz, int64_t n, float* d_out, void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  SFK_TRY(validate_grid_args(c, roi, d_grid, n, d_xyz, d_out));
  SFK_HIP(c, sfk::launch_sample(d_grid, roi->lo, roi->hi, roi->res, d_xyz, n, d_out,
                                (hipStream_t)hip_stream));
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_select_points(sfk_ctx c, const sfk_roi* roi, const float* d_grid, double iso,
                             const float* d_xyz, int64_t n, int64_t* d_idx, int64_t cap,
                             int64_t* h_count, void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  SFK_TRY(validate_grid_args(c, roi, d_grid, n, d_xyz, d_idx));
  if (!h_count || cap < 0 || !std::isfinite(iso)) {
    set_err(c, "invalid selection arguments");
    return SFK_E_INVAL;
  }
  *h_count = 0;
  if (n == 0) return SFK_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  TmpBuf flags(c), pos(c), tmp(c), total(c);
  sfk_status st;
  if ((st = flags.get(sizeof(int32_t) * (size_t)n, "selection flags")) != SFK_OK ||
      (st = pos.get(sizeof(int64_t) * (size_t)n, "selection offsets")) != SFK_OK ||
      (st = tmp.get(sfk::scan_tmp_bytes(n), "scan scratch")) != SFK_OK ||
      (st = total.get(sizeof(int64_t), "selection count")) != SFK_OK)
    return st;
  int64_t cnt = 0;
  if (sfk::launch_select_flags(d_grid, roi->lo, roi->hi, roi->res, iso, d_xyz, n,
                               flags.as<int32_t>(), s) != hipSuccess ||
      sfk::scan_exclusive_i32_i64(flags.as<int32_t>(), pos.as<int64_t>(), n, total.as<int64_t>(),
                                  tmp.b.p, tmp.b.bytes, s) != hipSuccess ||
      sfk::launch_compact_index(flags.as<int32_t>(), pos.as<int64_t>(), n, d_idx, cap, s) !=
          hipSuccess ||
      hipMemcpyAsync(&cnt, total.b.p, sizeof cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    set_err(c, "selection kernels failed");
    return SFK_E_DEVICE;
  }
  *h_count = cnt;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_iso_cells(sfk_ctx c, const sfk_roi* roi, const float* d_grid, double iso,
                         int64_t* d_cells, uint8_t* d_cases, int64_t cap, int64_t* h_count,
                         void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  SFK_TRY(validate_grid_args(c, roi, d_grid, 0, nullptr, nullptr));
  if (!h_count || cap < 0 || (cap > 0 && (!d_cells || !d_cases)) || !std::isfinite(iso)) {
    set_err(c, "invalid iso-cell arguments");
    return SFK_E_INVAL;
  }
  const int64_t nc = (int64_t)(roi->res[0] - 1) * (roi->res[1] - 1) * (roi->res[2] - 1);
  hipStream_t s = (hipStream_t)hip_stream;
  TmpBuf flags(c), pos(c), cases(c), tmp(c), total(c);
  sfk_status st;
  if ((st = flags.get(sizeof(int32_t) * (size_t)nc, "cell flags")) != SFK_OK ||
      (st = pos.get(sizeof(int64_t) * (size_t)nc, "cell offsets")) != SFK_OK ||
      (st = cases.get((size_t)nc, "cell cases")) != SFK_OK ||
      (st = tmp.get(sfk::scan_tmp_bytes(nc), "scan scratch")) != SFK_OK ||
      (st = total.get(sizeof(int64_t), "cell count")) != SFK_OK)
    return st;
  int64_t cnt = 0;
  if (sfk::launch_iso_flags(d_grid, roi->res, iso, nc, flags.as<int32_t>(), cases.as<uint8_t>(),
                            s) != hipSuccess ||
      sfk::scan_exclusive_i32_i64(flags.as<int32_t>(), pos.as<int64_t>(), nc, total.as<int64_t>(),
                                  tmp.b.p, tmp.b.bytes, s) != hipSuccess ||
      sfk::launch_compact_cells(flags.as<int32_t>(), pos.as<int64_t>(), cases.as<uint8_t>(), nc,
                                d_cells, d_cases, cap, s) != hipSuccess ||
      hipMemcpyAsync(&cnt, total.b.p, sizeof cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    set_err(c, "iso-cell kernels failed");
    return SFK_E_DEVICE;
  }
  *h_count = cnt;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_iso_surface(sfk_ctx c, const sfk_roi* roi, const float* d_grid, double iso,
                           float* d_tris, int64_t cap, int64_t* h_count, void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  SFK_TRY(validate_grid_args(c, roi, d_grid, 0, nullptr, nullptr));
  if (!h_count || cap < 0 || (cap > 0 && !d_tris) || !std::isfinite(iso)) {
    set_err(c, "invalid iso-surface arguments");
    return SFK_E_INVAL;
  }
  const int64_t nc = (int64_t)(roi->res[0] - 1) * (roi->res[1] - 1) * (roi->res[2] - 1);
  hipStream_t s = (hipStream_t)hip_stream;
  TmpBuf flags(c), cnt(c), pos(c), cases(c), tmp(c), total(c);
  sfk_status st;
  if ((st = flags.get(sizeof(int32_t) * (size_t)nc, "cell flags")) != SFK_OK ||
      (st = cnt.get(sizeof(int32_t) * (size_t)nc, "cell triangle counts")) != SFK_OK ||
      (st = pos.get(sizeof(int64_t) * (size_t)nc, "cell offsets")) != SFK_OK ||
      (st = cases.get((size_t)nc, "cell cases")) != SFK_OK ||
      (st = tmp.get(sfk::scan_tmp_bytes(nc), "scan scratch")) != SFK_OK ||
      (st = total.get(sizeof(int64_t), "triangle count")) != SFK_OK)
    return st;
  int64_t n = 0;
  if (sfk::launch_iso_flags(d_grid, roi->res, iso, nc, flags.as<int32_t>(), cases.as<uint8_t>(),
                            s) != hipSuccess ||
      sfk::launch_iso_tri_count(cases.as<uint8_t>(), nc, cnt.as<int32_t>(), s) != hipSuccess ||
      sfk::scan_exclusive_i32_i64(cnt.as<int32_t>(), pos.as<int64_t>(), nc, total.as<int64_t>(),
                                  tmp.b.p, tmp.b.bytes, s) != hipSuccess ||
      sfk::launch_iso_emit(d_grid, roi->lo, roi->hi, roi->res, iso, cases.as<uint8_t>(),
                           pos.as<int64_t>(), nc, d_tris, cap, s) != hipSuccess ||
      hipMemcpyAsync(&n, total.b.p, sizeof n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    set_err(c, "iso-surface kernels failed");
    return SFK_E_DEVICE;
  }
  *h_count = n;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_mc_case(int32_t cs, int8_t* h_edges, int32_t* n_tri) {
  if (cs < 0 || cs > 255 || !h_edges || !n_tri) {
    set_err(nullptr, "case must be in 0..255, pointers non-NULL");
    return SFK_E_INVAL;
  }
  *n_tri = sfk::mc_case_host(cs, h_edges);
  return SFK_OK;
}

sfk_status sfk_debug_poison(sfk_ctx c, int32_t bits) {
  SFK_TRY(check_ctx(c));
  if (bits < 0 || bits > 3) {
    set_err(c, "poison bits must be in 0..3");
    return SFK_E_INVAL;
  }
  c->debug_poison = bits;
  return SFK_OK;
}

sfk_status sfk_debug_tree_order(sfk_ctx c, sfk_tree t, int32_t* h_perm) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || (!h_perm && t->n > 0)) {
    set_err(c, "invalid arguments");
    return SFK_E_INVAL;
  }
  if (t->n > 0)
    SFK_HIP(c, hipMemcpy(h_perm, t->perm.p, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost));
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_curve_keys(int32_t curve, int32_t bits, const uint32_t* h_cells, int64_t n,
                                uint64_t* h_keys) {
  SFK_GUARD_BEGIN
  if (n < 0 || (n > 0 && (!h_cells || !h_keys)) || bits < 1 || bits > 21 ||
      (curve != SFK_CURVE_HILBERT && curve != SFK_CURVE_MORTON)) {
    set_err(nullptr, "invalid arguments");
    return SFK_E_INVAL;
  }
  for (int64_t i = 0; i < 3 * n; ++i)
    if (h_cells[i] >> bits) {
      set_err(nullptr, "cell coordinate %u >= 2^%d", h_cells[i], bits);
      return SFK_E_INVAL;
    }
  sfk::curve_keys_host(h_cells, n, bits, curve == SFK_CURVE_HILBERT, h_keys);
  return SFK_OK;
  SFK_GUARD_END(nullptr)
}

sfk_status sfk_debug_point_h2(sfk_ctx c, sfk_tree t, float* h_h2) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !h_h2) {
    set_err(c, "invalid arguments");
    return SFK_E_INVAL;
  }
  if (!t->h2.p) {
    set_err(c, "tree was built without k-NN bandwidths");
    return SFK_E_INVAL;
  }
  std::vector<float> h2(t->n);
  std::vector<int32_t> perm(t->n);
  SFK_HIP(c, hipMemcpy(h2.data(), t->h2.p, sizeof(float) * t->n, hipMemcpyDeviceToHost));
  SFK_HIP(c, hipMemcpy(perm.data(), t->perm.p, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < t->n; ++i) h_h2[perm[i]] = h2[i];
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_candidates(sfk_ctx c, sfk_tree t, const sfk_roi* roi, int64_t node_begin,
                                int64_t node_end, int64_t* h_offsets, int64_t* h_idx, int64_t cap,
                                int64_t* needed) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !h_offsets || !needed) {
    set_err(c, "invalid arguments");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  if (roi->set != SFK_SET_CLOUD || roi->bw == SFK_BW_MBE) {
    set_err(c, "candidate export covers CLOUD-set, non-MBE ROIs");
    return SFK_E_UNSUPPORTED;
  }
  const int64_t m = (int64_t)roi->res[0] * roi->res[1] * roi->res[2];
  if (node_begin < 0 || node_end > m || node_begin > node_end) {
    set_err(c, "node range out of bounds");
    return SFK_E_INVAL;
  }
  const int64_t nn = node_end - node_begin;
  hipStream_t s = c->slots[0].stream;
  SFK_HIP(c, hipStreamSynchronize(s));
  TileShape ts = choose_shape(c, t, roi);
  // the sweep has no tiles: its support sets are found with the brick's
  // (support sets do not depend on the tile shape)
  if (sfk::is_sweep(ts)) ts = shape_of(kBrickShape);
  GroupRoi g = resolve_cloud_roi(t, roi, false);
  std::vector<GroupRoi> v{g};
  RoiDev rd;
  int64_t n_tiles, n_coords;
  make_roidev(v, ts, &rd, &n_tiles, &n_coords);
  TmpBuf hdev(c), coords(c), cnt(c), off(c), idx(c), rlist(c);
  SFK_TRY(hdev.get(sizeof(BatchHdr) + sizeof(RoiDev), "descriptor"));
  SFK_TRY(coords.get(sizeof(double) * (size_t)n_coords, "coordinates"));
  SFK_TRY(rlist.get(sizeof(int32_t) * (kRoiListCap + 1), "ROI leaf list"));
  SFK_TRY(cnt.get(sizeof(int64_t) * (size_t)std::max<int64_t>(nn, 1), "counts"));
  {
    BatchHdr h{};
    h.n_rois = 1;
    h.n_tiles = n_tiles;
    SFK_HIP(c, hipMemcpy(hdev.b.p, &h, sizeof h, hipMemcpyHostToDevice));
    SFK_HIP(c, hipMemcpy((char*)hdev.b.p + sizeof(BatchHdr), &rd, sizeof rd, hipMemcpyHostToDevice));
  }
  const RoiDev* rdev_p = (const RoiDev*)((char*)hdev.b.p + sizeof(BatchHdr));
  TreeView tv = view_of(t);
  SFK_HIP(c, sfk::launch_roi_coords(tv, hdev.as<BatchHdr>(), rdev_p, 1, coords.as<double>(),
                                    rlist.as<int32_t>() + 1, rlist.as<int32_t>(), s));
  SFK_HIP(c, sfk::launch_debug_candidates2(tv, (const int32_t*)t->perm.p, rdev_p,
                                            coords.as<double>(), ts, node_begin, node_end,
                                            cnt.as<int64_t>(), nullptr, nullptr, s));
  std::vector<int64_t> counts(nn);
  SFK_HIP(c, hipMemcpyAsync(counts.data(), cnt.b.p, sizeof(int64_t) * nn, hipMemcpyDeviceToHost, s));
  SFK_HIP(c, hipStreamSynchronize(s));
  h_offsets[0] = 0;
  for (int64_t i = 0; i < nn; ++i) h_offsets[i + 1] = h_offsets[i] + counts[i];
  *needed = h_offsets[nn];
  if (!h_idx || *needed > cap) return SFK_OK;
  SFK_TRY(off.get(sizeof(int64_t) * (size_t)std::max<int64_t>(nn, 1), "offsets"));
  SFK_TRY(idx.get(sizeof(int32_t) * (size_t)std::max<int64_t>(*needed, 1), "indices"));
  SFK_HIP(c, hipMemcpy(off.b.p, h_offsets, sizeof(int64_t) * nn, hipMemcpyHostToDevice));
  SFK_HIP(c, sfk::launch_debug_candidates2(tv, (const int32_t*)t->perm.p, rdev_p,
                                            coords.as<double>(), ts, node_begin, node_end, nullptr,
                                            off.as<int64_t>(), idx.as<int32_t>(), s));
  std::vector<int32_t> ix(*needed);
  SFK_HIP(c, hipMemcpyAsync(ix.data(), idx.b.p, sizeof(int32_t) * ix.size(), hipMemcpyDeviceToHost, s));
  SFK_HIP(c, hipStreamSynchronize(s));
  for (int64_t i = 0; i < nn; ++i) {
    std::sort(ix.begin() + h_offsets[i], ix.begin() + h_offsets[i + 1]);
    for (int64_t q = h_offsets[i]; q < h_offsets[i + 1]; ++q) h_idx[q] = ix[q];
  }
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_support_counts(sfk_ctx c, sfk_tree t, const sfk_roi* roi, float* d_counts,
                                    void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t) {
    set_err(c, "NULL tree");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  if (!d_counts) {
    set_err(c, "d_counts is NULL");
    return SFK_E_INVAL;
  }
  sfk_roi r = *roi;
  r.d_out = d_counts;
  return eval_direct(c, t, &r, (hipStream_t)hip_stream, true);
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_particle_estimate(sfk_ctx c, sfk_tree t, const double* lo, const double* hi,
                                       double* particles) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !lo || !hi || !particles) {
    set_err(c, "NULL argument");
    return SFK_E_INVAL;
  }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || lo[k] > hi[k]) {
      set_err(c, "box must be finite with lo <= hi");
      return SFK_E_INVAL;
    }
  *particles = est_particles(t, lo, hi);
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_eval_count(sfk_ctx c, sfk_tree t, const sfk_roi* roi, int64_t* useful_pairs,
                                int64_t* tested_pairs) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t) {
    set_err(c, "NULL tree");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  const int64_t m = (int64_t)roi->res[0] * roi->res[1] * roi->res[2];
  hipStream_t s = c->slots[0].stream;
  SFK_HIP(c, hipStreamSynchronize(s));
  TmpBuf cnt(c);
  SFK_TRY(cnt.get(sizeof(float) * (size_t)m, "support counts"));
  sfk_roi r = *roi;
  r.d_out = cnt.as<float>();
  SFK_TRY(eval_direct(c, t, &r, s, true));
  std::vector<float> h(m);
  SFK_HIP(c, hipMemcpyAsync(h.data(), cnt.b.p, sizeof(float) * m, hipMemcpyDeviceToHost, s));
  SFK_HIP(c, hipStreamSynchronize(s));
  int64_t useful = 0;
  for (int64_t i = 0; i < m; ++i) useful += (int64_t)h[i];
  if (useful_pairs) *useful_pairs = useful;
  if (tested_pairs) {
    // leaves listed per tile x 64 particles x nodes per tile (CLOUD path)
    int64_t tested = 0;
    if (roi->set == SFK_SET_CLOUD) {
      BatchHdr hh;
      SFK_HIP(c, hipMemcpy(&hh, c->direct_ws.hdr_rois.p, sizeof hh, hipMemcpyDeviceToHost));
      const TileShape ts = choose_shape(c, t, roi);
      if (sfk::is_sweep(ts)) {
        // listed boxes x their particles x the unrolled node span
        const int nm = sweep_nm(resolve_cloud_roi(t, roi, false));
        const int64_t per_box = t->n_leaves > SFK_FANOUT ? (int64_t)SFK_FANOUT * SFK_LEAF : SFK_LEAF;
        tested = hh.n_items * per_box * (int64_t)(nm * nm * nm);
      } else {
        tested = hh.total_leaves * SFK_LEAF * (int64_t)(ts.tx * ts.ty * ts.tz);
      }
    }
    *tested_pairs = tested;
  }
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_tile_leaves(sfk_ctx c, sfk_tree t, const sfk_roi* roi, int32_t* h_shape,
                                 int64_t* h_tile_cnt, int64_t tiles_cap, int32_t* h_leaves,
                                 int64_t cap, int64_t* n_tiles_out, int64_t* total_out) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !n_tiles_out || !total_out || tiles_cap < 0 || cap < 0) {
    set_err(c, "invalid arguments");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  if (roi->set != SFK_SET_CLOUD || roi->bw == SFK_BW_MBE) {
    set_err(c, "tile leaf lists are exported for CLOUD-set, non-MBE ROIs");
    return SFK_E_UNSUPPORTED;
  }
  hipStream_t s = c->slots[0].stream;
  SFK_HIP(c, hipStreamSynchronize(s));
  if (c->direct_last_valid) SFK_HIP(c, hipEventSynchronize(c->direct_last));
  const TileShape ts = choose_shape(c, t, roi);
  BatchHdr hh{};
  if (sfk::is_sweep(ts)) {
    // the sweep keeps no tile lists: its work items, the boxes of the
    // hierarchy's first interior level (the leaves for a tree of at most 64
    // leaves) that pass the box test, ascending
    SFK_TRY(eval_direct(c, t, roi, s, false));
    SFK_HIP(c, hipStreamSynchronize(s));
    SFK_HIP(c, hipMemcpy(&hh, c->direct_ws.hdr_rois.p, sizeof hh, hipMemcpyDeviceToHost));
    if (hh.n_items > hh.item_cap) {
      set_err(c, "sweep item list overflowed");
      return SFK_E_INTERNAL;
    }
    *n_tiles_out = hh.n_tiles;
    *total_out = hh.n_items;
    if (h_shape) {
      h_shape[0] = ts.tx;
      h_shape[1] = ts.ty;
      h_shape[2] = ts.tz;
    }
    if (h_tile_cnt && hh.n_tiles <= tiles_cap)
      for (int64_t i = 0; i < hh.n_tiles; ++i) h_tile_cnt[i] = 0;
    if (h_leaves && hh.n_items <= cap) {
      std::vector<int64_t> it((size_t)hh.n_items);
      if (hh.n_items > 0)
        SFK_HIP(c, hipMemcpy(it.data(), c->direct_ws.leaves.p, sizeof(int64_t) * hh.n_items,
                             hipMemcpyDeviceToHost));
      std::vector<int32_t> boxes((size_t)hh.n_items);
      for (size_t i = 0; i < it.size(); ++i) boxes[i] = (int32_t)(it[i] & 0xffffffff);
      std::sort(boxes.begin(), boxes.end());
      std::copy(boxes.begin(), boxes.end(), h_leaves);
    }
    return SFK_OK;
  }
  // the direct path's pipeline; a second run with room for every list if
  // the first overflowed (every tile then keeps its list)
  for (int attempt = 0; attempt < 2; ++attempt) {
    SFK_TRY(eval_direct(c, t, roi, s, false));
    SFK_HIP(c, hipStreamSynchronize(s));
    SFK_HIP(c, hipMemcpy(&hh, c->direct_ws.hdr_rois.p, sizeof hh, hipMemcpyDeviceToHost));
    if (!hh.overflow) break;
    c->direct_ws.want_leaf_cap = std::max(c->direct_ws.want_leaf_cap, hh.total_leaves);
    c->direct_ws.want_partial_cap = std::max(c->direct_ws.want_partial_cap, hh.total_partials);
  }
  if (hh.overflow) {
    set_err(c, "leaf lists overflowed twice");
    return SFK_E_INTERNAL;
  }
  *n_tiles_out = hh.n_tiles;
  *total_out = hh.total_leaves;
  if (h_shape) {
    h_shape[0] = ts.tx;
    h_shape[1] = ts.ty;
    h_shape[2] = ts.tz;
  }
  if (h_tile_cnt && hh.n_tiles <= tiles_cap) {
    std::vector<int32_t> cnt((size_t)hh.n_tiles);
    SFK_HIP(c, hipMemcpy(cnt.data(), c->direct_ws.tile_cnt.p, sizeof(int32_t) * hh.n_tiles,
                         hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < hh.n_tiles; ++i) h_tile_cnt[i] = cnt[(size_t)i];
  }
  if (h_leaves && hh.total_leaves <= cap)
    SFK_HIP(c, hipMemcpy(h_leaves, c->direct_ws.leaves.p, sizeof(int32_t) * hh.total_leaves,
                         hipMemcpyDeviceToHost));
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_leaf_boxes(sfk_ctx c, sfk_tree t, float* h_boxes) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || (!h_boxes && t->n_leaves > 0)) {
    set_err(c, "invalid arguments");
    return SFK_E_INVAL;
  }
  if (t->n_leaves == 0) return SFK_OK;
  std::vector<NodeBox> b((size_t)t->n_leaves);
  SFK_HIP(c, hipMemcpy(b.data(), (const NodeBox*)t->nodes.p + t->level_off[0],
                       sizeof(NodeBox) * t->n_leaves, hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < t->n_leaves; ++i)
    for (int k = 0; k < 3; ++k) {
      h_boxes[6 * (int64_t)i + k] = b[(size_t)i].lo[k];
      h_boxes[6 * (int64_t)i + 3 + k] = b[(size_t)i].hi[k];
    }
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_debug_mbe(sfk_ctx c, sfk_tree t, const sfk_roi* roi, float* h_ell0, int64_t* n_b,
                         int64_t* h_idx_b, float* h_pilot, float* h_pden, double* aveden,
                         float* h_ell_j, int64_t cap_b) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t) {
    set_err(c, "NULL tree");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  if (roi->bw != SFK_BW_MBE) {
    set_err(c, "sfk_debug_mbe needs an MBE ROI");
    return SFK_E_INVAL;
  }
  MbeDebug d;
  d.ell0 = h_ell0;
  d.n_b = n_b;
  d.idx_b = h_idx_b;
  d.pilot = h_pilot;
  d.pden = h_pden;
  d.aveden = aveden;
  d.ell_j = h_ell_j;
  d.cap_b = cap_b;
  hipStream_t s = c->slots[0].stream;
  SFK_HIP(c, hipStreamSynchronize(s));
  if (c->direct_last_valid) SFK_HIP(c, hipEventSynchronize(c->direct_last));
  Staging& st = c->direct_st[c->direct_next];
  c->direct_next = (c->direct_next + 1) % kStagingRing;
  SFK_TRY(eval_subcloud(c, t, roi, false, shape_of(1), c->direct_ws, st, s, &d));
  SFK_HIP(c, hipEventRecord(c->direct_last, s));
  c->direct_last_valid = true;
  c->direct_last_stream = s;
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_autotune(sfk_ctx c, sfk_tree t, const sfk_roi* sample, int32_t n) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || (!sample && n > 0) || n < 0) {
    set_err(c, "invalid autotune arguments");
    return SFK_E_INVAL;
  }
  for (int i = 0; i < n; ++i) {
    SFK_TRY(validate_roi(c, t, &sample[i], i));
    if (sample[i].set != SFK_SET_CLOUD || sample[i].bw == SFK_BW_MBE) {
      set_err(c, "autotune samples must be CLOUD-set, non-MBE ROIs");
      return SFK_E_UNSUPPORTED;
    }
  }
  hipStream_t s = c->slots[0].stream;
  SFK_HIP(c, hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  SFK_HIP(c, hipEventCreate(&e0));
  SFK_HIP(c, hipEventCreate(&e1));
  const sfk_eval_opts saved = c->opts;
  // per key: summed time of each shape over that key's samples
  std::map<int, std::vector<double>> cost;
  sfk_status st = SFK_OK;
  for (int i = 0; i < n && st == SFK_OK; ++i) {
    const int key = tune_key(t, &sample[i]);
    auto& v = cost[key];
    if (v.empty()) v.assign(kNumShapes + 1, 0.0);
    for (int shape = 1; shape <= kNumShapes && st == SFK_OK; ++shape) {
      if ((shape == kBrickShape && !uniform_bw(&sample[i])) ||
          (shape == kSweepShape && !sweep_ok(t, &sample[i]))) {
        v[shape] = 1e30;  // bricks and the sweep take uniform bandwidths only
        continue;
      }
      c->opts.tile_shape = shape;
      float best = 1e30f;
      for (int rep = 0; rep < 3 && st == SFK_OK; ++rep) {
        (void)hipEventRecord(e0, s);
        st = eval_direct(c, t, &sample[i], s, false);
        (void)hipEventRecord(e1, s);
        if (st == SFK_OK && hipEventSynchronize(e1) == hipSuccess) {
          float ms = 0.0f;
          if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && rep > 0) best = std::min(best, ms);
        }
      }
      v[shape] += best;
    }
  }
  c->opts = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SFK_OK) return st;
  for (auto& kv : cost) {
    int best = 1;
    for (int shape = 1; shape <= kNumShapes; ++shape)
      if (kv.second[shape] < kv.second[best]) best = shape;
    c->tune[kv.first] = best;
    c->tune_cost[kv.first] = kv.second;
  }
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_autotune_costs(sfk_ctx c, int32_t* keys, double* ms, int32_t cap, int32_t* n_out) {
  SFK_TRY(check_ctx(c));
  if (!n_out || cap < 0) {
    set_err(c, "invalid arguments");
    return SFK_E_INVAL;
  }
  int32_t i = 0;
  for (auto& kv : c->tune_cost) {
    if (keys && ms && i < cap) {
      keys[i] = kv.first;
      for (int sh = 1; sh <= kNumShapes; ++sh)
        ms[(size_t)i * kNumShapes + sh - 1] = sh < (int)kv.second.size() ? kv.second[sh] : 0.0;
    }
    ++i;
  }
  *n_out = i;
  return SFK_OK;
}

// Text file: a header line "sfkde-autotune 2 <arch> <shapes>", then one line
// per key: "<key> <shape>".
sfk_status sfk_autotune_save(sfk_ctx c, const char* path) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!path) {
    set_err(c, "path is NULL");
    return SFK_E_INVAL;
  }
  FILE* f = std::fopen(path, "w");
  if (!f) {
    set_err(c, "cannot write %s", path);
    return SFK_E_INVAL;
  }
  std::fprintf(f, "sfkde-autotune 2 %s %d\n", c->arch.empty() ? "unknown" : c->arch.c_str(),
               kNumShapes);
  for (auto& kv : c->tune) std::fprintf(f, "%d %d\n", kv.first, kv.second);
  const bool ok = std::fclose(f) == 0;
  if (!ok) {
    set_err(c, "cannot write %s", path);
    return SFK_E_INVAL;
  }
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_autotune_load(sfk_ctx c, const char* path) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!path) {
    set_err(c, "path is NULL");
    return SFK_E_INVAL;
  }
  FILE* f = std::fopen(path, "r");
  if (!f) {
    set_err(c, "cannot read %s", path);
    return SFK_E_INVAL;
  }
  char magic[32] = {0}, arch[64] = {0};
  int ver = 0, shapes = 0;
  if (std::fscanf(f, "%31s %d %63s %d", magic, &ver, arch, &shapes) != 4 ||
      std::strcmp(magic, "sfkde-autotune") != 0 || ver != 2 || shapes != kNumShapes) {
    std::fclose(f);
    set_err(c, "%s is not a tuning table of this library version", path);
    return SFK_E_INVAL;
  }
  if (c->arch != arch) {
    std::fclose(f);
    set_err(c, "%s was tuned on %s, this device is %s", path, arch, c->arch.c_str());
    return SFK_E_UNSUPPORTED;
  }
  std::map<int, int> t;
  int key = 0, shape = 0;
  while (std::fscanf(f, "%d %d", &key, &shape) == 2) {
    if (shape < 1 || shape > kNumShapes || key < 0) {
      std::fclose(f);
      set_err(c, "%s: entry %d %d out of range", path, key, shape);
      return SFK_E_INVAL;
    }
    t[key] = shape;
  }
  std::fclose(f);
  for (auto& kv : t) c->tune[kv.first] = kv.second;
  return SFK_OK;
  SFK_GUARD_END(c)
}

/* Autotuner table: (key, tile shape) pairs. */
sfk_status sfk_autotune_table(sfk_ctx c, int32_t* keys, int32_t* shapes, int32_t cap,
                              int32_t* n_out) {
  SFK_TRY(check_ctx(c));
  if (!n_out) {
    set_err(c, "n_out is NULL");
    return SFK_E_INVAL;
  }
  int32_t i = 0;
  for (auto& kv : c->tune) {
    if (keys && shapes && i < cap) {
      keys[i] = kv.first;
      shapes[i] = kv.second;
    }
    ++i;
  }
  *n_out = i;
  return SFK_OK;
}

// Estimated useful pairs of a request: the particles the host box levels put
// in its box widened by the support, times the nodes one support covers
// (an ellipsoid of semi-axes reach_k / s_k node steps, at least one node).
static double est_useful(sfk_tree t, const sfk_roi& r) {
  double lo[3], hi[3], vol = 4.0 / 3.0 * M_PI;
  const double c = r.kernel == SFK_KERNEL_GAUSS_TRUNC3 ? 3.0 : 1.0;
  for (int k = 0; k < 3; ++k) {
    double h = 0.0;
    if (r.bw == SFK_BW_FIXED) h = r.h[k];
    else if (r.bw == SFK_BW_ROI_SCALED) h = (double)r.h[0] * (r.hi[k] - r.lo[k]);
    else h = (r.hi[k] - r.lo[k]) / 64.0;  // per-point: a guess of one 64th of the box
    const double s = (r.hi[k] - r.lo[k]) / (double)(r.res[k] - 1);
    lo[k] = r.lo[k] - c * h;
    hi[k] = r.hi[k] + c * h;
    vol *= c * h / s;
  }
  return est_particles(t, lo, hi) * std::max(1.0, vol);
}

// Device bytes one request holds while in flight: its grid plus an estimate
// of its share of the batch workspace (per-tile arrays and leaf lists).
static double request_bytes(const sfk_roi& r, TileShape ts) {
  const double m = (double)r.res[0] * r.res[1] * r.res[2];
  const double tiles = std::ceil((double)r.res[0] / ts.tx) * std::ceil((double)r.res[1] / ts.ty) *
                       std::ceil((double)r.res[2] / ts.tz);
  const double sums = sfk::is_sweep(ts) ? 8.0 * kSweep * kSweep * kSweep : 0.0;
  return 4.0 * m + tiles * (3 * 4 + 3 * 8 + 64 * 4 + 4.0 * slot_cap_of(ts) + sums);
}

sfk_status sfk_serve(sfk_ctx c, sfk_tree t, const sfk_request* reqs, int64_t n,
                     const sfk_serve_opts* opts, sfk_request_result* res,
                     sfk_serve_summary* summ) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || (!reqs && n > 0) || n < 0 || !opts || (!res && n > 0)) {
    set_err(c, "invalid serve arguments");
    return SFK_E_INVAL;
  }
  if (opts->mode < 0 || opts->mode > 1 || opts->n_slots < 1 || opts->n_slots > kNumSlots ||
      opts->max_batch < 1 || !(opts->budget_bytes >= 0.0) || opts->interleave < 0 ||
      opts->interleave > 1 || !std::isfinite(opts->max_batch_work)) {
    set_err(c, "serve options out of range (mode 0|1, 1 <= n_slots <= %d, max_batch >= 1)",
            kNumSlots);
    return SFK_E_INVAL;
  }
  std::vector<sfk_roi> rois((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    SFK_TRY(validate_roi(c, t, &reqs[i].roi, (int)i));
    if (reqs[i].roi.set != SFK_SET_CLOUD || reqs[i].roi.bw == SFK_BW_MBE) {
      set_err(c, "request %lld: the serving loop takes CLOUD-set, non-MBE requests", (long long)i);
      return SFK_E_UNSUPPORTED;
    }
    if (i > 0 && reqs[i].arrival_s < reqs[i - 1].arrival_s) {
      set_err(c, "requests must be sorted by arrival time");
      return SFK_E_INVAL;
    }
    rois[i] = reqs[i].roi;
  }
  SFK_TRY(validate_disjoint_outputs(c, rois.data(), (int)n));
  // drain anything the context still runs
  for (int i = 0; i < kNumSlots; ++i)
    if (c->slots[i].busy) SFK_HIP(c, hipEventSynchronize(c->slots[i].done));
  SFK_TRY(pump(c));
  if (c->direct_last_valid) SFK_HIP(c, hipEventSynchronize(c->direct_last));

  const double budget = opts->budget_bytes > 0 ? opts->budget_bytes : (double)c->budget;
  struct Interleave {
    sfk_ctx c;
    bool saved;
    Interleave(sfk_ctx cc, bool on) : c(cc), saved(cc->serve_interleave) { c->serve_interleave = on; }
    ~Interleave() { c->serve_interleave = saved; }
  } interleave(c, opts->interleave != 0);
  for (int64_t i = 0; i < n; ++i) {
    res[i] = sfk_request_result{};
    res[i].arrival_s = reqs[i].arrival_s;
    res[i].batch = -1;
  }
  int64_t n_batches = 0, budget_waits = 0, batched_reqs = 0;
  double in_flight_area = 0.0;  // integral of batches in flight over time
  const double t0 = now_s();
  double last_t = 0.0;
  int64_t next = 0, done_cnt = 0;

  if (opts->mode == 1) {
    // one ROI per launch, in arrival order, on one stream
    hipStream_t s = c->slots[0].stream;
    std::vector<hipEvent_t> evs((size_t)n, nullptr);
    for (auto& e : evs) SFK_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int64_t retire = 0;
    sfk_status st = SFK_OK;
    while (done_cnt < n) {
      const double now = now_s() - t0;
      bool acted = false;
      if (next < n && reqs[next].arrival_s <= now) {
        res[next].admit_s = now;
        res[next].batch = (int32_t)n_batches++;
        st = eval_direct(c, t, &rois[next], s, false);
        if (st != SFK_OK) break;
        SFK_HIP(c, hipEventRecord(evs[next], s));
        ++next;
        acted = true;
      }
      while (retire < next) {
        const hipError_t q = hipEventQuery(evs[retire]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          set_err(c, "request %lld failed on the device", (long long)retire);
          st = SFK_E_DEVICE;
          break;
        }
        const double tnow = now_s() - t0;
        res[retire].done_s = tnow;
        res[retire].latency_ms = (tnow - reqs[retire].arrival_s) * 1e3;
        res[retire].status = SFK_OK;
        ++retire;
        ++done_cnt;
        acted = true;
      }
      if (st != SFK_OK) break;
      const double tnow = now_s() - t0;
      in_flight_area += (double)(next - retire) * (tnow - last_t);
      last_t = tnow;
      if (!acted) std::this_thread::yield();
    }
    (void)hipStreamSynchronize(s);
    for (auto& e : evs) (void)hipEventDestroy(e);
    if (st != SFK_OK) return st;
    batched_reqs = n;
  } else {
    const int ns = opts->n_slots;
    const double work_cap = opts->max_batch_work == 0.0 ? 2e8 : opts->max_batch_work;
    std::vector<double> work((size_t)n);
    for (int64_t i = 0; i < n; ++i) work[(size_t)i] = est_useful(t, rois[(size_t)i]);
    std::vector<std::vector<int64_t>> in_slot((size_t)ns);
    std::vector<double> slot_bytes((size_t)ns, 0.0);
    std::deque<int64_t> pending;
    double in_flight = 0.0;
    std::vector<const sfk_roi*> batch;
    while (done_cnt < n) {
      const double now = now_s() - t0;
      bool acted = false;
      while (next < n && reqs[next].arrival_s <= now) pending.push_back(next++);
      // retire finished batches
      int busy = 0;
      for (int si = 0; si < ns; ++si) {
        Slot& sl = c->slots[si];
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) {
          ++busy;
          continue;
        }
        if (q != hipSuccess) {
          set_err(c, "a batch failed on the device: %s", hipGetErrorString(q));
          return SFK_E_DEVICE;
        }
        const double tnow = now_s() - t0;
        const bool bad = absorb_stats(sl.ws, sl.st);
        if (bad) {
          set_err(c, "%s", kErrLeafIds);
          SFK_TRY(clear_err_word(c, sl.ws, sl.stream));
        }
        for (int64_t i : in_slot[si]) {
          res[i].done_s = tnow;
          res[i].latency_ms = (tnow - reqs[i].arrival_s) * 1e3;
          res[i].status = bad ? SFK_E_INTERNAL : SFK_OK;
          ++done_cnt;
        }
        in_flight -= slot_bytes[si];
        slot_bytes[si] = 0.0;
        in_slot[si].clear();
        sl.busy = false;
        acted = true;
      }
      // admit: every free slot takes the waiting requests that fit
      for (int si = 0; si < ns && !pending.empty(); ++si) {
        Slot& sl = c->slots[si];
        if (sl.busy) continue;
        batch.clear();
        double bytes = 0.0, bwork = 0.0;
        while (!pending.empty() && (int)batch.size() < opts->max_batch) {
          const int64_t i = pending.front();
          const double rb = request_bytes(rois[i], choose_shape(c, t, &rois[i]));
          const bool fits = budget <= 0.0 || in_flight + bytes + rb <= budget;
          if (!fits && !(batch.empty() && in_flight == 0.0)) break;
          // a heavy request closes the batch (it runs alone or starts the next)
          if (!batch.empty() && work_cap > 0.0 && bwork + work[(size_t)i] > work_cap) break;
          bwork += work[(size_t)i];
          batch.push_back(&rois[i]);
          in_slot[si].push_back(i);
          bytes += rb;
          pending.pop_front();
        }
        if (batch.empty()) {
          ++budget_waits;
          break;
        }
        const double tnow = now_s() - t0;
        for (int64_t i : in_slot[si]) {
          res[i].admit_s = tnow;
          res[i].batch = (int32_t)n_batches;
        }
        ++n_batches;
        batched_reqs += (int64_t)batch.size();
        sl.busy = true;
        sl.ticket = -1;
        if (c->opts.disable_graphs || c->prof_on)
          SFK_TRY(enqueue_cloud_rois(c, t, batch, false, sl.ws, sl.st, sl.stream));
        else
          SFK_TRY(enqueue_cloud_rois_graph(c, t, batch, sl));
        SFK_HIP(c, hipEventRecord(sl.done, sl.stream));
        slot_bytes[si] = bytes;
        in_flight += bytes;
        ++busy;
        acted = true;
      }
      const double tnow = now_s() - t0;
      in_flight_area += (double)busy * (tnow - last_t);
      last_t = tnow;
      if (!acted) std::this_thread::yield();
    }
  }
  const double wall = now_s() - t0;
  if (summ) {
    std::vector<double> lat((size_t)n);
    for (int64_t i = 0; i < n; ++i) lat[i] = res[i].latency_ms;
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double q) {
      if (lat.empty()) return 0.0;
      const double pos = q * (double)(lat.size() - 1);
      const size_t i = (size_t)pos;
      const double f = pos - (double)i;
      return i + 1 < lat.size() ? lat[i] + f * (lat[i + 1] - lat[i]) : lat[i];
    };
    summ->wall_s = wall;
    summ->p50_ms = pct(0.50);
    summ->p99_ms = pct(0.99);
    summ->max_ms = lat.empty() ? 0.0 : lat.back();
    summ->evals_per_s = 0.0;
    summ->n_batches = n_batches;
    summ->mean_batch = n_batches ? (double)batched_reqs / (double)n_batches : 0.0;
    summ->mean_in_flight = wall > 0 ? in_flight_area / wall : 0.0;
    summ->budget_waits = budget_waits;
  }
  return SFK_OK;
  SFK_GUARD_END(c)
}

}  // extern "C"

// ---------------------------------------------------------------------------
// View cache: lattices of nodes o + g*s cut into blocks of B^3 nodes, each
// block an ordinary ROI evaluated by the batch path with one tile shape per
// lattice, kept in a device-resident LRU cache across frames.
// ---------------------------------------------------------------------------

namespace {

struct ViewLattice {
  int64_t id;
  double s;        // spacing
  float h[3];      // FIXED / ROI_SCALED bandwidth of the lattice
  TileShape ts;    // tile shape every block of the lattice is evaluated with
};

struct BlockKey {
  int64_t lat, b[3];
  bool operator==(const BlockKey& o) const {
    return lat == o.lat && b[0] == o.b[0] && b[1] == o.b[1] && b[2] == o.b[2];
  }
};
struct BlockKeyHash {
  size_t operator()(const BlockKey& k) const {
    uint64_t h = (uint64_t)k.lat * 0x9E3779B97F4A7C15ull;
    for (int a = 0; a < 3; ++a) h = (h ^ (uint64_t)k.b[a]) * 0xBF58476D1CE4E5B9ull + 0x94D049BB133111EBull;
    return (size_t)(h ^ (h >> 31));
  }
};
struct BlockEntry {
  int32_t slot;
  int64_t stamp;  // frame that last needed the block
};

int64_t floor_div64(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// What a frame does, from the box and the view's state (pure host logic).
struct FramePlan {
  int lat = -1;            // index into the view's lattices, -1 = a new lattice
  double s = 0.0;
  int64_t g_lo[3], g_hi[3];  // lattice nodes of the returned grid
  int64_t m_lo[3], m_hi[3];  // blocks covering the box plus margin
  int64_t v_lo[3], v_hi[3];  // blocks covering the grid
  int64_t nodes = 0, blocks = 0;
};

}  // namespace

struct sfk_view_s {
  sfk_ctx ctx = nullptr;
  sfk_tree tree = nullptr;
  sfk_view_opts o{};
  int B = 32;
  double origin[3] = {0, 0, 0};
  int chunk_leaves = 0;  // chunking the cached blocks were evaluated with
  DevBuf cache;
  int64_t n_slots = 0;
  std::vector<ViewLattice> lattices;
  int64_t next_lattice = 0;
  std::unordered_map<BlockKey, BlockEntry, BlockKeyHash> map;
  std::vector<int32_t> free_slots;
  int64_t stamp = 0;
  DevBuf table;  // per-frame block -> slot table of the returned grid
  hipEvent_t last = nullptr;
  bool last_valid = false;
  hipStream_t last_stream = nullptr;
};

namespace {

sfk_status view_plan(sfk_view v, const double lo[3], const double hi[3], FramePlan* p) {
  sfk_ctx c = v->ctx;
  double side = 0.0;
  for (int k = 0; k < 3; ++k) {
    if (!(std::isfinite(lo[k]) && std::isfinite(hi[k]) && hi[k] > lo[k])) {
      set_err(c, "view box axis %d needs finite lo < hi", k);
      return SFK_E_INVAL;
    }
    side = std::max(side, hi[k] - lo[k]);
  }
  const double sw = side / (double)(v->o.res - 1);
  // the cached lattice closest in ratio, if within the threshold
  const double lim = std::log(v->o.scale_threshold);
  double best = 0.0;
  p->lat = -1;
  for (size_t i = 0; i < v->lattices.size(); ++i) {
    const double d = std::fabs(std::log(v->lattices[i].s / sw));
    if (d <= lim && (p->lat < 0 || d < best)) {
      p->lat = (int)i;
      best = d;
    }
  }
  const double s = p->lat >= 0 ? v->lattices[p->lat].s : sw;
  p->s = s;
  const int64_t B = v->B;
  const double lim_g = 1099511627776.0;  // 2^40: keeps o + g*s exact enough and products in range
  p->nodes = 1;
  p->blocks = 1;
  for (int k = 0; k < 3; ++k) {
    const double o = v->origin[k];
    const double ql = std::floor((lo[k] - o) / s), qh = std::ceil((hi[k] - o) / s);
    const double mg = v->o.margin * side;
    const double ml = std::floor((lo[k] - mg - o) / s), mh = std::ceil((hi[k] + mg - o) / s);
    if (!(std::fabs(ql) < lim_g && std::fabs(qh) < lim_g && std::fabs(ml) < lim_g &&
          std::fabs(mh) < lim_g)) {
      set_err(c, "view box axis %d lies too far from the tree at this spacing", k);
      return SFK_E_INVAL;
    }
    int64_t gl = (int64_t)ql, gh = (int64_t)qh;
    // the largest node at or below lo, the smallest at or above hi
    while (o + (double)(gl + 1) * s <= lo[k]) ++gl;
    while (o + (double)gl * s > lo[k]) --gl;
    while (o + (double)(gh - 1) * s >= hi[k]) --gh;
    while (o + (double)gh * s < hi[k]) ++gh;
    p->g_lo[k] = gl;
    p->g_hi[k] = gh;
    const int64_t mlo = std::min<int64_t>((int64_t)ml, gl), mhi = std::max<int64_t>((int64_t)mh, gh);
    p->m_lo[k] = floor_div64(mlo, B);
    p->m_hi[k] = floor_div64(mhi, B);
    p->v_lo[k] = floor_div64(gl, B);
    p->v_hi[k] = floor_div64(gh, B);
    const int64_t nn = gh - gl + 1, nb = p->m_hi[k] - p->m_lo[k] + 1;
    if (nn > ((int64_t)1 << 31) || nb > ((int64_t)1 << 21)) {
      set_err(c, "view grid axis %d: %lld nodes / %lld blocks is too many", k, (long long)nn,
              (long long)nb);
      return SFK_E_INVAL;
    }
    p->nodes = std::min<int64_t>(p->nodes * nn, (int64_t)1 << 62);
    p->blocks = std::min<int64_t>(p->blocks * nb, (int64_t)1 << 62);
  }
  if (p->nodes > ((int64_t)1 << 31)) {
    set_err(c, "view grid of %lld nodes exceeds 2^31", (long long)p->nodes);
    return SFK_E_INVAL;
  }
  return SFK_OK;
}

void view_fill_info(sfk_view v, const FramePlan& p, int64_t evaluated, sfk_view_frame_info* info) {
  if (!info) return;
  *info = sfk_view_frame_info{};
  for (int k = 0; k < 3; ++k) {
    info->g0[k] = p.g_lo[k];
    info->res[k] = (int32_t)(p.g_hi[k] - p.g_lo[k] + 1);
    info->lo[k] = v->origin[k] + (double)p.g_lo[k] * p.s;
    info->hi[k] = v->origin[k] + (double)p.g_hi[k] * p.s;
  }
  info->new_lattice = p.lat < 0 ? 1 : 0;
  info->spacing = p.s;
  info->lattice_id = p.lat >= 0 ? v->lattices[p.lat].id : v->next_lattice;
  info->blocks_needed = p.blocks;
  info->blocks_evaluated = evaluated;
}

// The ROI of block b of lattice L.
sfk_roi block_roi(sfk_view v, const ViewLattice& L, const int64_t b[3], float* out) {
  sfk_roi r{};
  for (int k = 0; k < 3; ++k) {
    r.lo[k] = v->origin[k] + (double)(b[k] * v->B) * L.s;
    r.hi[k] = v->origin[k] + (double)(b[k] * v->B + v->B - 1) * L.s;
    r.res[k] = v->B;
    r.h[k] = L.h[k];
  }
  r.kernel = v->o.kernel;
  r.bw = v->o.bw == SFK_BW_PER_POINT ? SFK_BW_PER_POINT : SFK_BW_FIXED;
  r.norm = v->o.norm;
  r.set = SFK_SET_CLOUD;
  r.d_out = out;
  return r;
}

void view_flush(sfk_view v) {
  v->map.clear();
  v->lattices.clear();
  v->free_slots.clear();
  for (int64_t i = v->n_slots - 1; i >= 0; --i) v->free_slots.push_back((int32_t)i);
}

}  // namespace

extern "C" {

sfk_status sfk_view_create(sfk_ctx c, sfk_tree t, const sfk_view_opts* o, sfk_view* out) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !o || !out) {
    set_err(c, "NULL view argument");
    return SFK_E_INVAL;
  }
  *out = nullptr;
  if (t->n <= 0) {
    set_err(c, "view of an empty tree");
    return SFK_E_INVAL;
  }
  if (o->kernel != SFK_KERNEL_EPANECHNIKOV && o->kernel != SFK_KERNEL_GAUSS_TRUNC3) {
    set_err(c, "view: unknown kernel %d", o->kernel);
    return SFK_E_INVAL;
  }
  if (o->norm != SFK_NORM_PAPER && o->norm != SFK_NORM_COUNT) {
    set_err(c, "view: unknown norm %d", o->norm);
    return SFK_E_INVAL;
  }
  if (o->bw == SFK_BW_FIXED) {
    for (int k = 0; k < 3; ++k)
      if (!(o->h[k] > 0.0f) || !std::isfinite(o->h[k])) {
        set_err(c, "view: fixed bandwidth h[%d] must be finite and > 0", k);
        return SFK_E_INVAL;
      }
  } else if (o->bw == SFK_BW_ROI_SCALED) {
    if (!(o->h[0] > 0.0f) || !std::isfinite(o->h[0])) {
      set_err(c, "view: bandwidth factor h[0] must be finite and > 0");
      return SFK_E_INVAL;
    }
  } else if (o->bw == SFK_BW_PER_POINT) {
    if (t->pp_mode != PP_ISO) {
      set_err(c, "view: per-point bandwidth requested but the tree has none");
      return SFK_E_INVAL;
    }
  } else {
    set_err(c, "view: bandwidth mode %d is not supported (FIXED, ROI_SCALED, PER_POINT)", o->bw);
    return SFK_E_INVAL;
  }
  const int B = o->block == 0 ? 32 : o->block;
  if (o->res < 2 || !(B == 8 || B == 16 || B == 32 || B == 64) ||
      !(o->scale_threshold >= 1.0) || !std::isfinite(o->scale_threshold) ||
      !(o->margin >= 0.0) || !std::isfinite(o->margin) || o->max_blocks < 1 ||
      o->max_blocks > ((int64_t)1 << 31) - 1) {
    set_err(c, "view: need res >= 2, block in {8, 16, 32, 64}, finite scale_threshold >= 1, "
               "finite margin >= 0, 1 <= max_blocks < 2^31");
    return SFK_E_INVAL;
  }
  const size_t bytes = round_bytes(sizeof(float) * (size_t)B * B * B * (size_t)o->max_blocks);
  if (c->budget && c->ws_bytes + bytes > c->budget) {
    set_err(c, "view cache of %zu bytes exceeds the device-memory budget", bytes);
    return SFK_E_BUDGET;
  }
  std::unique_ptr<sfk_view_s> v(new sfk_view_s());
  v->ctx = c;
  v->tree = t;
  v->o = *o;
  v->B = B;
  for (int k = 0; k < 3; ++k) v->origin[k] = t->bbox[k];
  v->cache.p = raw_alloc(c, bytes);
  if (!v->cache.p) {
    set_err(c, "device allocation of %zu bytes for the view cache failed", bytes);
    return SFK_E_NOMEM;
  }
  v->cache.bytes = bytes;
  c->ws_bytes += bytes;
  v->n_slots = o->max_blocks;
  if (hipEventCreateWithFlags(&v->last, hipEventDisableTiming) != hipSuccess) {
    raw_free(c, v->cache.p, v->cache.bytes);
    c->ws_bytes -= bytes;
    set_err(c, "event creation failed");
    return SFK_E_DEVICE;
  }
  view_flush(v.get());
  *out = v.release();
  return SFK_OK;
  SFK_GUARD_END(c)
}

sfk_status sfk_view_destroy(sfk_view v) {
  SFK_GUARD_BEGIN
  if (!v) return SFK_OK;
  sfk_ctx c = v->ctx;
  if (v->last_valid) (void)hipEventSynchronize(v->last);
  if (v->last) (void)hipEventDestroy(v->last);
  raw_free(c, v->cache.p, v->cache.bytes);
  c->ws_bytes -= v->cache.bytes;
  raw_free(c, v->table.p, v->table.bytes);
  delete v;
  return SFK_OK;
  SFK_GUARD_END(nullptr)
}

sfk_status sfk_view_frame(sfk_view v, const double lo[3], const double hi[3], float* d_out,
                          int64_t cap, sfk_view_frame_info* info, void* hip_stream) {
  if (!v) return SFK_E_INVAL;
  sfk_ctx c = v->ctx;
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!lo || !hi) {
    set_err(c, "view frame: NULL box");
    return SFK_E_INVAL;
  }
  // blocks evaluated with another chunking would not be bitwise reproducible
  if (chunk_leaves_of(c) != v->chunk_leaves) {
    view_flush(v);
    v->chunk_leaves = chunk_leaves_of(c);
  }
  FramePlan p;
  SFK_TRY(view_plan(v, lo, hi, &p));
  if (!d_out) {
    int64_t missing = 0;
    if (p.lat < 0) {
      missing = p.blocks;
    } else {
      const int64_t id = v->lattices[p.lat].id;
      for (int64_t bz = p.m_lo[2]; bz <= p.m_hi[2]; ++bz)
        for (int64_t by = p.m_lo[1]; by <= p.m_hi[1]; ++by)
          for (int64_t bx = p.m_lo[0]; bx <= p.m_hi[0]; ++bx)
            if (!v->map.count(BlockKey{id, {bx, by, bz}})) ++missing;
    }
    view_fill_info(v, p, missing, info);
    return SFK_OK;
  }
  if (cap < p.nodes) {
    view_fill_info(v, p, 0, info);
    set_err(c, "view frame: the grid needs %lld floats, cap is %lld", (long long)p.nodes,
            (long long)cap);
    return SFK_E_INVAL;
  }
  if (p.blocks > v->n_slots) {
    view_fill_info(v, p, 0, info);
    set_err(c, "view frame: box plus margin needs %lld blocks, the cache holds %lld",
            (long long)p.blocks, (long long)v->n_slots);
    return SFK_E_BUDGET;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (v->last_valid && v->last_stream != s) SFK_HIP(c, hipStreamWaitEvent(s, v->last, 0));
  const bool created = p.lat < 0;
  if (created) {
    ViewLattice L{};
    L.id = v->next_lattice++;
    L.s = p.s;
    for (int k = 0; k < 3; ++k)
      L.h[k] = v->o.bw == SFK_BW_FIXED ? v->o.h[k]
               : v->o.bw == SFK_BW_ROI_SCALED
                   ? (float)((double)v->o.h[0] * (double)(v->o.res - 1) * p.s)
                   : 1.0f;
    const int64_t b0[3] = {p.m_lo[0], p.m_lo[1], p.m_lo[2]};
    const sfk_roi r = block_roi(v, L, b0, (float*)v->cache.p);
    L.ts = choose_shape(c, v->tree, &r);
    v->lattices.push_back(L);
    p.lat = (int)v->lattices.size() - 1;
  }
  const ViewLattice& L = v->lattices[p.lat];
  const int64_t cur = ++v->stamp;
  std::vector<BlockKey> missing;
  for (int64_t bz = p.m_lo[2]; bz <= p.m_hi[2]; ++bz)
    for (int64_t by = p.m_lo[1]; by <= p.m_hi[1]; ++by)
      for (int64_t bx = p.m_lo[0]; bx <= p.m_hi[0]; ++bx) {
        const BlockKey key{L.id, {bx, by, bz}};
        auto it = v->map.find(key);
        if (it != v->map.end())
          it->second.stamp = cur;
        else
          missing.push_back(key);
      }
  // slots: free ones first, then the least recently used blocks this frame
  // does not need (earlier frames' reads of them are ordered before this
  // frame's writes on the stream)
  if ((int64_t)missing.size() > (int64_t)v->free_slots.size()) {
    std::vector<std::pair<int64_t, BlockKey>> old;
    for (const auto& kv : v->map)
      if (kv.second.stamp < cur) old.push_back({kv.second.stamp, kv.first});
    std::sort(old.begin(), old.end(), [](const std::pair<int64_t, BlockKey>& a,
                                         const std::pair<int64_t, BlockKey>& b) {
      if (a.first != b.first) return a.first < b.first;
      for (int k = 2; k >= 0; --k)
        if (a.second.b[k] != b.second.b[k]) return a.second.b[k] < b.second.b[k];
      return a.second.lat < b.second.lat;
    });
    size_t i = 0;
    while ((int64_t)missing.size() > (int64_t)v->free_slots.size() && i < old.size()) {
      auto it = v->map.find(old[i++].second);
      v->free_slots.push_back(it->second.slot);
      v->map.erase(it);
    }
    if ((int64_t)missing.size() > (int64_t)v->free_slots.size()) {
      set_err(c, "view cache: no slot left");
      return SFK_E_INTERNAL;
    }
  }
  std::vector<sfk_roi> rois;
  rois.reserve(missing.size());
  const size_t per_block = (size_t)v->B * v->B * v->B;
  for (const BlockKey& key : missing) {
    const int32_t slot = v->free_slots.back();
    v->free_slots.pop_back();
    v->map[key] = BlockEntry{slot, cur};
    rois.push_back(block_roi(v, L, key.b, (float*)v->cache.p + per_block * (size_t)slot));
  }
  if (!rois.empty()) {
    std::vector<const sfk_roi*> ptrs;
    for (const sfk_roi& r : rois) ptrs.push_back(&r);
    const sfk_status st = eval_direct_cloud(c, v->tree, ptrs, s, false, &L.ts);
    if (st != SFK_OK) {
      // the blocks may be partly written: forget them
      for (const BlockKey& key : missing) {
        auto it = v->map.find(key);
        if (it != v->map.end()) {
          v->free_slots.push_back(it->second.slot);
          v->map.erase(it);
        }
      }
      return st;
    }
  }
  // block -> slot table of the returned grid's blocks
  int32_t nb[3];
  int64_t nt = 1;
  for (int k = 0; k < 3; ++k) {
    nb[k] = (int32_t)(p.v_hi[k] - p.v_lo[k] + 1);
    nt *= nb[k];
  }
  std::vector<int32_t> tab((size_t)nt);
  for (int64_t bz = 0; bz < nb[2]; ++bz)
    for (int64_t by = 0; by < nb[1]; ++by)
      for (int64_t bx = 0; bx < nb[0]; ++bx) {
        auto it = v->map.find(BlockKey{L.id, {p.v_lo[0] + bx, p.v_lo[1] + by, p.v_lo[2] + bz}});
        tab[(size_t)(bx + nb[0] * (by + nb[1] * bz))] = it != v->map.end() ? it->second.slot : -1;
      }
  const size_t tb = sizeof(int32_t) * (size_t)nt;
  if (v->table.bytes < tb) {
    if (v->last_valid) SFK_HIP(c, hipEventSynchronize(v->last));
    raw_free(c, v->table.p, v->table.bytes);
    v->table = DevBuf();
    const size_t nbytes = round_bytes(std::max<size_t>(tb, 4096));
    v->table.p = raw_alloc(c, nbytes);
    if (!v->table.p) {
      set_err(c, "device allocation of %zu bytes for the view table failed", nbytes);
      return SFK_E_NOMEM;
    }
    v->table.bytes = nbytes;
  }
  // pageable source: the copy has read it when the call returns
  SFK_HIP(c, hipMemcpyAsync(v->table.p, tab.data(), tb, hipMemcpyHostToDevice, s));
  int32_t res[3];
  for (int k = 0; k < 3; ++k) res[k] = (int32_t)(p.g_hi[k] - p.g_lo[k] + 1);
  SFK_HIP(c, sfk::launch_view_gather((const float*)v->cache.p, v->n_slots, v->B,
                                     (const int32_t*)v->table.p, p.v_lo, nb, p.g_lo, res, d_out, s));
  SFK_HIP(c, hipEventRecord(v->last, s));
  v->last_valid = true;
  v->last_stream = s;
  view_fill_info(v, p, (int64_t)missing.size(), info);
  if (info) info->new_lattice = created ? 1 : 0;
  return SFK_OK;
  SFK_GUARD_END(c)
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adaptive resolution: bricks of a grid whose value range is large relative
// to the base grid's peak are re-evaluated at half the spacing, level by
// level.
// ---------------------------------------------------------------------------

namespace {

using sfk::BrickDesc;

// A grid whose cells may be refined: its device values and geometry.
struct AdaptiveGrid {
  const float* grid;
  double lo[3], hi[3];
  int32_t res[3];
  int32_t index;  // in the brick list, -1 = the base grid
};

// Node i of a grid axis, as the evaluation kernels place it.
double node_coord(double lo, double hi, int32_t res, int32_t i) {
  return lo + ((double)i * (hi - lo)) / (double)(res - 1);
}

}  // namespace

extern "C" {

sfk_status sfk_eval_adaptive(sfk_ctx c, sfk_tree t, const sfk_roi* roi,
                             const sfk_adaptive_opts* o, float* d_bricks, int64_t cap_floats,
                             sfk_brick* h_bricks, int32_t cap_bricks,
                             sfk_adaptive_result* res_out, void* hip_stream) {
  SFK_GUARD_BEGIN
  SFK_TRY(check_ctx(c));
  if (!t || !o || !res_out || (cap_floats > 0 && !d_bricks) || (cap_bricks > 0 && !h_bricks) ||
      cap_floats < 0 || cap_bricks < 0) {
    set_err(c, "invalid adaptive-evaluation arguments");
    return SFK_E_INVAL;
  }
  SFK_TRY(validate_roi(c, t, roi, 0));
  if (roi->bw == SFK_BW_MBE || roi->set != SFK_SET_CLOUD) {
    set_err(c, "adaptive evaluation takes CLOUD-set ROIs with fixed, ROI-scaled or per-point "
               "bandwidths");
    return SFK_E_UNSUPPORTED;
  }
  if (o->brick < 2 || o->brick > 64 || o->max_level < 1 || o->max_level > 4 ||
      !(o->threshold > 0.0f) || !std::isfinite(o->threshold)) {
    set_err(c, "adaptive options: brick in 2..64, max_level in 1..4, finite threshold > 0");
    return SFK_E_INVAL;
  }
  *res_out = sfk_adaptive_result{};
  res_out->complete = 1;
  hipStream_t s = (hipStream_t)hip_stream;
  SFK_TRY(eval_direct(c, t, roi, s, false));
  // the bricks' ROI template: same kernel and normalisation; a ROI-scaled
  // bandwidth becomes the base ROI's fixed h
  sfk_roi tmpl = *roi;
  if (roi->bw == SFK_BW_ROI_SCALED) {
    tmpl.bw = SFK_BW_FIXED;
    for (int k = 0; k < 3; ++k) tmpl.h[k] = (float)((double)roi->h[0] * (roi->hi[k] - roi->lo[k]));
  }
  std::vector<AdaptiveGrid> parents(1);
  for (int k = 0; k < 3; ++k) {
    parents[0].lo[k] = roi->lo[k];
    parents[0].hi[k] = roi->hi[k];
    parents[0].res[k] = roi->res[k];
  }
  parents[0].grid = roi->d_out;
  parents[0].index = -1;
  const int B = o->brick;
  float thr = 0.0f;
  int64_t used = 0;
  int32_t n_listed = 0;
  TmpBuf d_desc(c), d_mm(c);
  for (int level = 1; level <= o->max_level && !parents.empty(); ++level) {
    // bricks of every parent grid, in (parent, z, y, x) order
    std::vector<BrickDesc> descs;
    std::vector<int32_t> owner;
    for (size_t pi = 0; pi < parents.size(); ++pi) {
      const AdaptiveGrid& P = parents[pi];
      int32_t nb[3];
      for (int k = 0; k < 3; ++k) nb[k] = (P.res[k] - 1 + B - 1) / B;
      for (int32_t bz = 0; bz < nb[2]; ++bz)
        for (int32_t by = 0; by < nb[1]; ++by)
          for (int32_t bx = 0; bx < nb[0]; ++bx) {
            BrickDesc d{};
            d.grid = P.grid;
            const int32_t bb[3] = {bx, by, bz};
            for (int k = 0; k < 3; ++k) {
              d.res[k] = P.res[k];
              d.n0[k] = bb[k] * B;
              d.cells[k] = std::min(B, P.res[k] - 1 - bb[k] * B);
            }
            descs.push_back(d);
            owner.push_back((int32_t)pi);
          }
    }
    const int32_t nd = (int32_t)descs.size();
    if (nd == 0) break;
    if (d_desc.b.bytes < sizeof(BrickDesc) * (size_t)nd) {
      raw_free(c, d_desc.b.p, d_desc.b.bytes);
      d_desc.b = DevBuf();
      SFK_TRY(d_desc.get(sizeof(BrickDesc) * (size_t)nd, "brick descriptors"));
    }
    if (d_mm.b.bytes < 2 * sizeof(float) * (size_t)nd) {
      raw_free(c, d_mm.b.p, d_mm.b.bytes);
      d_mm.b = DevBuf();
      SFK_TRY(d_mm.get(2 * sizeof(float) * (size_t)nd, "brick ranges"));
    }
    std::vector<float> mm(2 * (size_t)nd);
    SFK_HIP(c, hipMemcpyAsync(d_desc.b.p, descs.data(), sizeof(BrickDesc) * (size_t)nd,
                              hipMemcpyHostToDevice, s));
    SFK_HIP(c, sfk::launch_brick_minmax(d_desc.as<BrickDesc>(), nd, d_mm.as<float>(),
                                        d_mm.as<float>() + nd, s));
    SFK_HIP(c, hipMemcpyAsync(mm.data(), d_mm.b.p, 2 * sizeof(float) * (size_t)nd,
                              hipMemcpyDeviceToHost, s));
    SFK_HIP(c, hipStreamSynchronize(s));
    if (level == 1) {
      float peak = -__builtin_huge_valf();
      for (int32_t i = 0; i < nd; ++i) peak = std::max(peak, mm[(size_t)nd + i]);
      res_out->peak = peak;
      thr = (float)((double)o->threshold * (double)peak);
      if (!(peak > 0.0f)) break;  // an empty field has nothing to refine
    }
    // the refined bricks of this level
    std::vector<sfk_brick> lvl;
    std::vector<AdaptiveGrid> next;
    int64_t lvl_floats = 0;
    for (int32_t i = 0; i < nd; ++i) {
      const float range = mm[(size_t)nd + i] - mm[i];
      if (!(range > thr)) continue;
      const BrickDesc& d = descs[i];
      const AdaptiveGrid& P = parents[owner[i]];
      sfk_brick b{};
      b.level = level;
      b.parent = P.index;
      int64_t nodes = 1;
      for (int k = 0; k < 3; ++k) {
        b.cell0[k] = d.n0[k];
        b.res[k] = 2 * d.cells[k] + 1;
        b.lo[k] = node_coord(P.lo[k], P.hi[k], P.res[k], d.n0[k]);
        b.hi[k] = node_coord(P.lo[k], P.hi[k], P.res[k], d.n0[k] + d.cells[k]);
        nodes *= b.res[k];
      }
      b.offset = used + lvl_floats;
      lvl_floats += nodes;
      lvl.push_back(b);
    }
    if (lvl.empty()) break;
    if (used + lvl_floats > cap_floats || (int64_t)n_listed + (int64_t)lvl.size() > cap_bricks) {
      res_out->complete = 0;
      break;
    }
    std::vector<sfk_roi> rois(lvl.size());
    std::vector<const sfk_roi*> ptrs(lvl.size());
    for (size_t i = 0; i < lvl.size(); ++i) {
      sfk_roi r = tmpl;
      for (int k = 0; k < 3; ++k) {
        r.lo[k] = lvl[i].lo[k];
        r.hi[k] = lvl[i].hi[k];
        r.res[k] = lvl[i].res[k];
      }
      r.d_out = d_bricks + lvl[i].offset;
      r.tag = 0;
      rois[i] = r;
      ptrs[i] = &rois[i];
    }
    for (size_t i = 0; i < lvl.size(); ++i) SFK_TRY(validate_roi(c, t, &rois[i], (int)i));
    SFK_TRY(eval_direct_cloud(c, t, ptrs, s, false, nullptr));
    for (size_t i = 0; i < lvl.size(); ++i) {
      h_bricks[n_listed + (int32_t)i] = lvl[i];
      AdaptiveGrid g{};
      g.grid = rois[i].d_out;
      for (int k = 0; k < 3; ++k) {
        g.lo[k] = lvl[i].lo[k];
        g.hi[k] = lvl[i].hi[k];
        g.res[k] = lvl[i].res[k];
      }
      g.index = n_listed + (int32_t)i;
      next.push_back(g);
    }
    n_listed += (int32_t)lvl.size();
    used += lvl_floats;
    res_out->levels = level;
    parents.swap(next);
  }
  // the descriptor and range buffers are freed on return: let the last
  // kernels that read them finish first
  SFK_HIP(c, hipStreamSynchronize(s));
  res_out->n_bricks = n_listed;
  res_out->floats_used = used;
  return SFK_OK;
  SFK_GUARD_END(c)
}

}  // extern "C"
