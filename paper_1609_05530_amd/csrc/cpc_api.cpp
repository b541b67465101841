// cpc_api.cpp — host side of the libcpc C ABI (include/cpc.h): argument
// validation, planning (subsets -> size classes -> launch lists, largest
// subsets first), workspace carving, and the launch sequence
//   rank -> fit -> variance -> combine
// for the partition-and-combine MPL estimator of arXiv:1609.05530
// (eq. 12-16). No device memory is allocated here: every buffer comes from
// the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cpc.h"
#include "kernels.h"

using namespace cpc;

// phases of a fit: ranks (eq. 12), maximisation of eq. (13), variance
// (Sec. 2.3), combine (eq. 15)
static constexpr int kPhases = 4;

struct cpc_context {
  int device;
  int magic;
  void* plan;               // host copy of the last call's launch tables, kept alive past the call
  hipEvent_t ev[kPhases + 1];  // phase boundaries of the last fit (CPC_FLAG_PHASE_TIMES)
  int have_times;
  int* pending_host;        // pinned: subsets of the streaming path still iterating
  hipStream_t cap_stream;   // the fit is captured here in graph mode (default priority)
  // second branch of a phase: the buckets after the first run here, forked
  // from and joined back to the call's stream (default priority)
  hipStream_t aux_stream;
  hipEvent_t fork_ev[kPhases], join_ev[kPhases];
  void* graph;              // GraphCache: the instantiated graph of the last graph-mode call
  void* tuner;              // Tuner: rank-kernel launch shapes chosen per workload signature
};

static constexpr int kMagic = 0x43504331;

// Scratch of the allocation-free entry point (cpc_fit_batched_noalloc): the
// workspace of such a call lives in this array. Each device the library runs
// on holds its own copy, at its own address, until the process ends. Host
// code never passes the array's name to a kernel (on the host it stands for
// a host-side shadow); it uses the device address that cpc_create looks up
// once per device with that device current.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;

namespace {
// Device address of `scratch` per device (nullptr until looked up) and the
// error of a failed lookup.
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Looks up the device's copy of `scratch` once (the device is current).
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  if (e == hipSuccess) g_scratch_ptr[device] = p;
}
}  // namespace

namespace {

thread_local char g_last_error[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_OK(expr)                                                                \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(CPC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

struct Options {
  int prec, ties, var, max_iter;
  double tol;
  int64_t n_min;
  int schedule;
  int flags;
};

int read_options(const cpc_options_t* o, Options& r) {
  cpc_options_t d;
  cpc_default_options(&d);
  if (!o) o = &d;
  if (o->prec != CPC_PREC_FP64 && o->prec != CPC_PREC_FP32C) return fail(CPC_E_ENUM, "unknown precision %d", o->prec);
  if (o->ties != CPC_TIES_AVERAGE && o->ties != CPC_TIES_FIRST) return fail(CPC_E_ENUM, "unknown tie rule %d", o->ties);
  if (o->var != CPC_VAR_GGR && o->var != CPC_VAR_INVINFO) return fail(CPC_E_ENUM, "unknown variance method %d", o->var);
  if (o->max_iter < 1) return fail(CPC_E_OPTIONS, "max_iter must be >= 1 (got %d)", o->max_iter);
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(CPC_E_OPTIONS, "tol must be finite and >= 0");
  if (o->n_min < 0) return fail(CPC_E_OPTIONS, "n_min must be >= 0");
  if (o->schedule < -1 || o->schedule > kNumRankShapes)
    return fail(CPC_E_OPTIONS, "schedule must be -1, 0 or 1 + a rank shape index below %d (got %d)", kNumRankShapes,
                o->schedule);
  r.prec = o->prec;
  r.ties = o->ties;
  r.var = o->var;
  r.max_iter = o->max_iter;
  r.tol = o->tol > 0.0 ? o->tol : (o->prec == CPC_PREC_FP64 ? 1e-12 : 1e-9);
  r.n_min = o->n_min < 2 ? 2 : o->n_min;
  r.schedule = o->schedule;
  r.flags = o->flags;
  return CPC_SUCCESS;
}

int check_offsets(const int64_t* offsets, int64_t K, int64_t n) {
  if (offsets[0] != 0) return fail(CPC_E_OFFSETS, "offsets[0] = %lld, expected 0", (long long)offsets[0]);
  for (int64_t m = 0; m < K; ++m) {
    if (offsets[m + 1] < offsets[m])
      return fail(CPC_E_OFFSETS, "offsets decrease at subset %lld", (long long)m);
    if (offsets[m + 1] - offsets[m] >= ((int64_t)1 << 31))
      return fail(CPC_E_UNSUPPORTED, "subset %lld has >= 2^31 rows", (long long)m);
  }
  if (offsets[K] != n) return fail(CPC_E_OFFSETS, "offsets[K] = %lld, expected n = %lld", (long long)offsets[K], (long long)n);
  return CPC_SUCCESS;
}

int size_class(int64_t rows) {
  for (int c = 0; c < kNumClasses; ++c)
    if (rows <= (int64_t)kClassThreads[c] * kClassItems[c]) return c;
  return -1;
}

// Workspace layout shared by all entry points.
struct Layout {
  size_t subs, order_rank, order_fit, state, gofs, r1, r2, e1, e2, l1, l2, s, g;
  // streaming path (subsets above kResidentMaxRows)
  size_t bsegs, btiles, bxorder, bflags, bgsum, bst, bpending, bhist, bpart, btsum, brow32[12], brow64[5];
  size_t total;
};

// Rows and subsets of the streaming path (subsets above kResidentMaxRows).
struct BigShare {
  int64_t rows = 0, subsets = 0;
};
BigShare big_share(const int64_t* offsets, int64_t K) {
  BigShare b;
  for (int64_t m = 0; m < K; ++m) {
    const int64_t rows = offsets[m + 1] - offsets[m];
    if (rows > kResidentMaxRows) {
      b.rows += rows;
      b.subsets += 1;
    }
  }
  return b;
}
// The most any partition of n rows into K subsets can put on the streaming path.
BigShare big_bound(int64_t n, int64_t K) {
  BigShare b;
  b.rows = n;
  b.subsets = std::min<int64_t>(K, n / (kResidentMaxRows + 1));
  return b;
}

int64_t max_tiles(int64_t rows, int64_t subsets) { return rows / kBigTile + subsets + 1; }

// The per-row arrays of the workgroup path are indexed by row and span all
// n rows; those of the streaming path are indexed by the compact position
// of a row among the streaming path's rows and span only those.
Layout layout(int64_t n, int64_t K, int64_t G, const BigShare& big) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.subs = take(sizeof(SubDesc) * (size_t)K);
  L.order_rank = take(sizeof(int32_t) * (size_t)K);
  L.order_fit = take(sizeof(int32_t) * (size_t)K);
  L.state = take(sizeof(SubState) * (size_t)K);
  L.gofs = take(sizeof(int64_t) * (size_t)(G + 1));
  L.r1 = take(2 * (size_t)n);
  L.r2 = take(2 * (size_t)n);
  L.e1 = take(2 * (size_t)n);
  L.e2 = take(2 * (size_t)n);
  L.l1 = take(2 * (size_t)n);
  L.l2 = take(2 * (size_t)n);
  L.s = take(8 * (size_t)n);
  L.g = take(8 * (size_t)n);
  const int64_t T = max_tiles(big.rows, big.subsets);
  const size_t nb = (size_t)big.rows;
  L.bsegs = take(sizeof(BigSeg) * (size_t)K);
  L.btiles = take(sizeof(BigTile) * (size_t)T);
  L.bxorder = take(sizeof(int64_t) * 8 * (size_t)T);
  L.bflags = take(sizeof(int32_t) * (size_t)K);
  L.bgsum = take(2 * sizeof(double) * (size_t)K);
  L.bst = take(sizeof(NewtonState) * (size_t)K);
  L.bpending = take(sizeof(int));
  L.bhist = take(256 * sizeof(uint32_t) * (size_t)T);
  L.bpart = take(5 * sizeof(double) * (size_t)T);
  L.btsum = take(2 * sizeof(double) * (size_t)T);
  for (int i = 0; i < 12; ++i) L.brow32[i] = take(4 * nb);
  for (int i = 0; i < 5; ++i) L.brow64[i] = take(8 * nb);
  L.total = off;
  return L;
}

// A launch list: subsets of one size class (and family) in decreasing size.
struct Bucket {
  int cls, fam;
  int32_t first, count;  // range in the order array
  int shape;             // rank buckets: launch shape (-1 = the class default)
};

struct Plan {
  std::vector<SubDesc> subs;
  std::vector<int32_t> order_rank, order_fit;
  std::vector<Bucket> rank_buckets, fit_buckets;
  std::vector<int64_t> gofs;
  std::vector<BigSeg> bsegs;
  std::vector<BigTile> btiles;
  std::vector<int64_t> bxorder;
  std::vector<int64_t> part_rep;  // replicate bounds of cpc_partition
};

// Deals per-subset work items to 8 queues (one per XCD: block b runs on XCD
// b mod 8) and interleaves them into launch slots, -1 for an idle slot. A
// subset goes whole to the least-loaded queue; one with more than 1/16 of all
// items is spread round-robin over the queues instead (else one XCD would
// carry it alone).
std::vector<int64_t> xcd_slots(const std::vector<std::vector<int64_t>>& items_of_seg) {
  int64_t total = 0;
  for (const auto& v : items_of_seg) total += (int64_t)v.size();
  std::vector<int64_t> q[8];
  int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int rr = 0;
  for (const auto& v : items_of_seg) {
    if ((int64_t)v.size() * 16 > total) {
      for (int64_t it : v) {
        q[rr].push_back(it);
        load[rr] += 1;
        rr = (rr + 1) & 7;
      }
      continue;
    }
    int best = 0;
    for (int x = 1; x < 8; ++x)
      if (load[x] < load[best]) best = x;
    for (int64_t it : v) q[best].push_back(it);
    load[best] += (int64_t)v.size();
  }
  size_t len = 0;
  for (int x = 0; x < 8; ++x) len = std::max(len, q[x].size());
  std::vector<int64_t> slots;
  slots.reserve(8 * len);
  for (size_t k = 0; k < len; ++k)
    for (int x = 0; x < 8; ++x) slots.push_back(k < q[x].size() ? q[x][k] : -1);
  return slots;
}

int make_plan(const int64_t* offsets, int64_t K, const int32_t* fam_of_subset, Plan& P) {
  P.subs.resize((size_t)K);
  P.bsegs.clear();
  P.btiles.clear();
  P.bxorder.clear();
  std::vector<int> cls((size_t)K);
  int64_t roff = 0;
  for (int64_t m = 0; m < K; ++m) {
    const int64_t rows = offsets[m + 1] - offsets[m];
    P.subs[m].begin = offsets[m];
    P.subs[m].n = (int32_t)rows;
    P.subs[m].family = (int16_t)fam_of_subset[m];
    P.subs[m].group = 0;
    cls[m] = size_class(rows);
    if (cls[m] < 0) {  // streaming path
      BigSeg b;
      b.begin = offsets[m];
      b.n = rows;
      b.roff = roff;
      b.tile0 = (int64_t)P.btiles.size();
      b.ntiles = (int32_t)((rows + kBigTile - 1) / kBigTile);
      b.sid = (int32_t)m;
      b.family = fam_of_subset[m];
      b.pad = 0;
      const int32_t g = (int32_t)P.bsegs.size();
      for (int64_t st = 0; st < rows; st += kBigTile) {
        BigTile t;
        t.seg = g;
        t.start = st;
        t.count = (int32_t)std::min<int64_t>(kBigTile, rows - st);
        P.btiles.push_back(t);
      }
      P.bsegs.push_back(b);
      roff += rows;
    }
  }
  // Tile slots in XCD order: the tiles of one subset then share an XCD's
  // L2, which holds the subset's arrays they scatter into or all read.
  if (!P.bsegs.empty()) {
    std::vector<std::vector<int64_t>> items(P.bsegs.size());
    for (size_t g = 0; g < P.bsegs.size(); ++g)
      for (int32_t k = 0; k < P.bsegs[g].ntiles; ++k) items[g].push_back(P.bsegs[g].tile0 + k);
    P.bxorder = xcd_slots(items);
  }
  std::vector<int32_t> ids;
  ids.reserve((size_t)K);
  for (int64_t m = 0; m < K; ++m)
    if (cls[m] >= 0) ids.push_back((int32_t)m);
  const int64_t KR = (int64_t)ids.size();
  // rank lists: by class, largest first
  std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
    if (cls[a] != cls[b]) return cls[a] > cls[b];
    return P.subs[a].n > P.subs[b].n;
  });
  P.order_rank = ids;
  P.rank_buckets.clear();
  for (int64_t i = 0; i < KR;) {
    int64_t j = i;
    while (j < KR && cls[ids[j]] == cls[ids[i]]) ++j;
    P.rank_buckets.push_back({cls[ids[i]], 0, (int32_t)i, (int32_t)(j - i), -1});
    i = j;
  }
  // fit / variance lists: by (class, family), largest first
  std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
    if (cls[a] != cls[b]) return cls[a] > cls[b];
    if (P.subs[a].family != P.subs[b].family) return P.subs[a].family < P.subs[b].family;
    return P.subs[a].n > P.subs[b].n;
  });
  P.order_fit = ids;
  P.fit_buckets.clear();
  for (int64_t i = 0; i < KR;) {
    int64_t j = i;
    while (j < KR && cls[ids[j]] == cls[ids[i]] && P.subs[ids[j]].family == P.subs[ids[i]].family) ++j;
    P.fit_buckets.push_back({cls[ids[i]], P.subs[ids[i]].family, (int32_t)i, (int32_t)(j - i), -1});
    i = j;
  }
  return CPC_SUCCESS;
}

struct Carved {
  SubDesc* subs;
  int32_t *order_rank, *order_fit;
  SubState* state;
  int64_t* gofs;
  RowArrays rows;
  BigParams big;
  BigBuffers bb;
};

Carved carve(void* ws, const Layout& L) {
  unsigned char* b = (unsigned char*)ws;
  Carved c;
  c.subs = (SubDesc*)(b + L.subs);
  c.order_rank = (int32_t*)(b + L.order_rank);
  c.order_fit = (int32_t*)(b + L.order_fit);
  c.state = (SubState*)(b + L.state);
  c.gofs = (int64_t*)(b + L.gofs);
  c.rows.R1 = (uint16_t*)(b + L.r1);
  c.rows.R2 = (uint16_t*)(b + L.r2);
  c.rows.E1 = (uint16_t*)(b + L.e1);
  c.rows.E2 = (uint16_t*)(b + L.e2);
  c.rows.L1 = (uint16_t*)(b + L.l1);
  c.rows.L2 = (uint16_t*)(b + L.l2);
  c.rows.S = (void*)(b + L.s);
  c.rows.G = (void*)(b + L.g);
  std::memset(&c.big, 0, sizeof(c.big));
  c.big.segs = (const BigSeg*)(b + L.bsegs);
  c.big.tiles = (const BigTile*)(b + L.btiles);
  c.big.xorder = (const int64_t*)(b + L.bxorder);
  c.big.flags = (int32_t*)(b + L.bflags);
  c.big.gsum = (double*)(b + L.bgsum);
  uint32_t** r32[12] = {&c.bb.ka, &c.bb.kb, &c.bb.kc, &c.bb.kd, &c.bb.va, &c.bb.vb,
                        &c.bb.R1, &c.bb.R2, &c.bb.E1, &c.bb.E2, &c.bb.L1, &c.bb.L2};
  for (int i = 0; i < 12; ++i) *r32[i] = (uint32_t*)(b + L.brow32[i]);
  void** r64[5] = {&c.bb.LX, &c.bb.LY, &c.bb.A1, &c.bb.A2, &c.bb.S};
  for (int i = 0; i < 5; ++i) *r64[i] = (void*)(b + L.brow64[i]);
  c.bb.hist = (uint32_t*)(b + L.bhist);
  c.bb.part = (double*)(b + L.bpart);
  c.bb.tsum = (double*)(b + L.btsum);
  c.bb.st = (NewtonState*)(b + L.bst);
  c.bb.pending = (int*)(b + L.bpending);
  return c;
}

int upload_tables(cpc_context* h, const Plan& P, const Carved& c, const int64_t* gofs, int64_t G,
                  hipStream_t s) {
  // the launch orders list only the subsets of the workgroup path (possibly none)
  if (!P.subs.empty())
    HIP_OK(hipMemcpyAsync(c.subs, P.subs.data(), sizeof(SubDesc) * P.subs.size(), hipMemcpyHostToDevice, s));
  if (!P.order_rank.empty())
    HIP_OK(hipMemcpyAsync(c.order_rank, P.order_rank.data(), sizeof(int32_t) * P.order_rank.size(),
                          hipMemcpyHostToDevice, s));
  if (!P.order_fit.empty())
    HIP_OK(hipMemcpyAsync(c.order_fit, P.order_fit.data(), sizeof(int32_t) * P.order_fit.size(),
                          hipMemcpyHostToDevice, s));
  if (gofs) HIP_OK(hipMemcpyAsync(c.gofs, gofs, sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
  if (!P.bsegs.empty()) {
    HIP_OK(hipMemcpyAsync((void*)c.big.segs, P.bsegs.data(), sizeof(BigSeg) * P.bsegs.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void*)c.big.tiles, P.btiles.data(), sizeof(BigTile) * P.btiles.size(),
                          hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync((void*)c.big.xorder, P.bxorder.data(), sizeof(int64_t) * P.bxorder.size(),
                          hipMemcpyHostToDevice, s));
  }
  (void)h;
  (void)G;
  return CPC_SUCCESS;
}

// Fills the counts of the streaming-path parameter block from the plan.
void set_big(Carved& c, const Plan& P, int64_t n_min) {
  c.big.nsegs = (int32_t)P.bsegs.size();
  c.big.ntiles = (int64_t)P.btiles.size();
  c.big.nslots = (int64_t)P.bxorder.size();
  c.big.n_min = n_min;
}

Plan& plan_of(cpc_handle_t h) { return *(Plan*)h->plan; }

int check_handle(cpc_handle_t h) {
  if (!h || h->magic != kMagic) return fail(CPC_E_HANDLE, "invalid handle");
  return CPC_SUCCESS;
}

// Graph mode (CPC_FLAG_GRAPH): the kernels of a fit are captured once into a
// hipGraph and replayed while the call's arguments stay the same. The launch
// tables are uploaded before capture, so the graph holds kernels only. The
// key is every pointer, size and option of the call plus the offsets, group
// offsets and families; a replay also requires that the workspace still
// holds the tables of the capture, so any other call through this handle
// with the same workspace drops the cached graph. With CPC_FLAG_PHASE_TIMES
// each phase is a graph of its own (events recorded inside a graph cannot be
// timed), launched back to back with the phase events recorded between them.
struct GraphCache {
  bool valid = false;
  const void *x = nullptr, *y = nullptr;
  int32_t dtype = 0;
  int64_t n = 0, K = 0, G = 0;
  std::vector<int64_t> offsets, gofs;
  std::vector<int32_t> fam;
  Options o{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void *out = nullptr, *comb = nullptr;
  hipGraphExec_t exec[kPhases] = {};
  int nexec = 0;

  void drop() {
    for (int i = 0; i < nexec; ++i) (void)hipGraphExecDestroy(exec[i]);
    nexec = 0;
    valid = false;
  }
  // replay: one graph, or the phase graphs between the handle's events
  hipError_t launch(hipEvent_t* ev, hipStream_t s) const {
    hipError_t e = hipSuccess;
    if (nexec == 1) return hipGraphLaunch(exec[0], s);
    for (int i = 0; i < nexec && e == hipSuccess; ++i) {
      e = hipEventRecord(ev[i], s);
      if (e == hipSuccess) e = hipGraphLaunch(exec[i], s);
    }
    return e == hipSuccess ? hipEventRecord(ev[nexec], s) : e;
  }
  bool same(const void* x_, const void* y_, int32_t dtype_, int64_t n_, const int64_t* off_, int64_t K_,
            const int64_t* gofs_, int64_t G_, const std::vector<int32_t>& fam_, const Options& o_, void* ws_,
            size_t ws_bytes_, void* out_, void* comb_) const {
    return valid && x == x_ && y == y_ && dtype == dtype_ && n == n_ && K == K_ && G == G_ && ws == ws_ &&
           ws_bytes == ws_bytes_ && out == out_ && comb == comb_ && o.prec == o_.prec && o.ties == o_.ties &&
           o.var == o_.var && o.max_iter == o_.max_iter && o.tol == o_.tol && o.n_min == o_.n_min && o.schedule == o_.schedule &&
           o.flags == o_.flags && std::equal(offsets.begin(), offsets.end(), off_) &&
           std::equal(gofs.begin(), gofs.end(), gofs_) && fam == fam_;
  }
};

GraphCache& graph_of(cpc_handle_t h) { return *(GraphCache*)h->graph; }

// Any call that writes into `ws` invalidates a graph captured over it.
void touch_workspace(cpc_handle_t h, const void* ws) {
  GraphCache& gc = graph_of(h);
  if (gc.valid && gc.ws == ws) gc.drop();
}

int enqueue_phase(int ph, cpc_handle_t h, const Plan& P, Carved& c, const void* x, const void* y, int32_t dtype,
                  int64_t G, const Options& o, cpc_subset_result_t* out, cpc_combined_t* comb, bool graph,
                  hipStream_t s);
int enqueue_fit(cpc_handle_t h, const Plan& P, Carved& c, const void* x, const void* y, int32_t dtype, int64_t G,
                const Options& o, cpc_subset_result_t* out, cpc_combined_t* comb, hipStream_t s, bool host_sync);

// Autotuner: the rank kernel's launch shape per size class, chosen by timing
// each candidate shape on the call's own subsets (the rank kernel is exact
// and idempotent, so trial launches leave nothing behind that the real run
// does not rewrite). A decision is keyed by (class, key width, log2 of the
// bucket's subset count, mean fill of the class capacity in eighths), kept
// in the handle and, when CPC_AUTOTUNE_CACHE names a file, appended there and
// read back by later handles. Tuning synchronises the stream once per new
// key; it runs before any graph capture.
struct Tuner {
  std::map<std::tuple<int, int, int, int>, int> choice;
  std::string path;
  std::string arch;
};
Tuner& tuner_of(cpc_handle_t h) { return *(Tuner*)h->tuner; }

void tuner_load(Tuner& t, int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) t.arch = prop.gcnArchName;
  const size_t colon = t.arch.find(':');
  if (colon != std::string::npos) t.arch.resize(colon);
  const char* p = std::getenv("CPC_AUTOTUNE_CACHE");
  if (!p || !*p) return;
  t.path = p;
  FILE* f = std::fopen(p, "r");
  if (!f) return;
  char arch[64];
  int cls, kw, cb, fb, shape;
  while (std::fscanf(f, "%63s %d %d %d %d %d", arch, &cls, &kw, &cb, &fb, &shape) == 6) {
    if (t.arch == arch && cls >= 0 && cls < kNumClasses && shape >= 0 && shape < kNumRankShapes &&
        kRankShapes[shape].cap >= (int)(kClassThreads[cls] * kClassItems[cls]))
      t.choice[{cls, kw, cb, fb}] = shape;
  }
  std::fclose(f);
}

RankParams rank_params(const Carved& c, const void* x, const void* y, const Options& o) {
  RankParams rp;
  std::memset(&rp, 0, sizeof(rp));
  rp.x = x;
  rp.y = y;
  rp.subs = c.subs;
  rp.mode = MODE_FIT;
  rp.ties = o.ties;
  rp.int_keys = 0;
  rp.n_min = o.n_min;
  rp.rows = c.rows;
  rp.state = c.state;
  return rp;
}

// With trials = false (a call that must not synchronise) a signature without
// a recorded decision takes the built-in shape and records nothing.
int choose_rank_shapes(cpc_handle_t h, Plan& P, const Carved& c, const void* x, const void* y, int kw,
                       const Options& o, hipStream_t s, bool trials) {
  Tuner& t = tuner_of(h);
  for (Bucket& b : P.rank_buckets) {
    b.shape = kRankDefaultShape[b.cls];
    if (o.schedule > 0) {  // a forced shape, for the classes whose capacity it has
      if (kw == 1 && kRankShapes[o.schedule - 1].cap == kClassThreads[b.cls] * kClassItems[b.cls])
        b.shape = o.schedule - 1;
      continue;
    }
    if (o.schedule == 0 || kw != 1 || b.count <= 0) continue;
    double mean = 0.0;
    for (int32_t i = 0; i < b.count; ++i) mean += P.subs[P.order_rank[b.first + i]].n;
    mean /= b.count;
    const int cap = kClassThreads[b.cls] * kClassItems[b.cls];
    const int cb = (int)std::floor(std::log2((double)b.count));
    const int fb = std::min(7, (int)(8.0 * mean / cap));
    const auto key = std::make_tuple(b.cls, kw, cb, fb);
    auto it = t.choice.find(key);
    if (it != t.choice.end()) {
      b.shape = it->second;
      continue;
    }
    if (!trials) continue;
    RankParams rp = rank_params(c, x, y, o);
    rp.order = c.order_rank + b.first;
    float best = 0.0f;
    for (int k = 0; k < 6 && kRankCandidates[b.cls][k] >= 0; ++k) {
      const int shape = kRankCandidates[b.cls][k];
      HIP_OK(launch_rank_shape(shape, kw, rp, b.count, s));  // warm-up
      HIP_OK(hipEventRecord(h->ev[0], s));
      HIP_OK(launch_rank_shape(shape, kw, rp, b.count, s));
      HIP_OK(launch_rank_shape(shape, kw, rp, b.count, s));
      HIP_OK(hipEventRecord(h->ev[1], s));
      HIP_OK(hipEventSynchronize(h->ev[1]));
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
      if (k == 0 || ms < best) {
        best = ms;
        b.shape = shape;
      }
    }
    t.choice[key] = b.shape;
    if (!t.path.empty()) {
      if (FILE* f = std::fopen(t.path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d %d %d %d\n", t.arch.c_str(), b.cls, kw, cb, fb, b.shape);
        std::fclose(f);
      }
    }
  }
  return CPC_SUCCESS;
}

// The full fit path for validated arguments.
// noalloc: the workspace is the static scratch and the call must neither
// synchronise nor build a graph (no autotuning trials, no host wait in the
// streaming path's Newton loop).
int run_fit(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n, const int64_t* offsets,
            int64_t K, const int64_t* gofs, int64_t G, const std::vector<int32_t>& fam_of_subset,
            const Options& o, void* ws, size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb,
            hipStream_t s, bool noalloc = false) {
  const Layout L = layout(n, K, G, big_share(offsets, K));
  if (!ws) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < L.total)
    return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, L.total);
  const bool graph = (o.flags & CPC_FLAG_GRAPH) != 0;
  const bool timed = (o.flags & CPC_FLAG_PHASE_TIMES) != 0;
  GraphCache& gc = graph_of(h);
  HIP_OK(hipSetDevice(h->device));
  if (graph && gc.same(x, y, dtype, n, offsets, K, gofs, G, fam_of_subset, o, ws, ws_bytes, out, comb)) {
    h->have_times = timed ? 1 : 0;
    HIP_OK(gc.launch(h->ev, s));
    return CPC_SUCCESS;
  }
  touch_workspace(h, ws);
  Plan& P = plan_of(h);
  int rc = make_plan(offsets, K, fam_of_subset.data(), P);
  if (rc) return rc;
  Carved c = carve(ws, L);
  h->have_times = 0;
  P.gofs.assign(gofs, gofs + G + 1);
  rc = upload_tables(h, P, c, P.gofs.data(), G, s);
  if (rc) return rc;
  set_big(c, P, o.n_min);
  rc = choose_rank_shapes(h, P, c, x, y, dtype == CPC_F64 ? 2 : 1, o, s, !noalloc);
  if (rc) return rc;
  if (!graph) return enqueue_fit(h, P, c, x, y, dtype, G, o, out, comb, s, !noalloc);

  // capture on the handle's stream once the uploads on `s` are done: one
  // graph, or one per phase when the phases are timed
  HIP_OK(hipStreamSynchronize(s));
  const int nexec = timed ? kPhases : 1;
  hipGraphExec_t ex[kPhases] = {};
  for (int e = 0; e < nexec; ++e) {
    hipError_t he = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    const char* what = "hipStreamBeginCapture";
    if (he == hipSuccess) {
      for (int ph = timed ? e : 0; ph < (timed ? e + 1 : kPhases) && rc == CPC_SUCCESS; ++ph)
        rc = enqueue_phase(ph, h, P, c, x, y, dtype, G, o, out, comb, true, h->cap_stream);
      hipGraph_t g = nullptr;
      he = hipStreamEndCapture(h->cap_stream, &g);
      what = "hipStreamEndCapture";
      if (rc == CPC_SUCCESS && he == hipSuccess) {
        he = hipGraphInstantiate(&ex[e], g, nullptr, nullptr, 0);
        what = "hipGraphInstantiate";
      }
      if (g) (void)hipGraphDestroy(g);
    }
    if (rc != CPC_SUCCESS || he != hipSuccess) {
      for (int i = 0; i < e; ++i) (void)hipGraphExecDestroy(ex[i]);
      return rc != CPC_SUCCESS ? rc : fail(CPC_E_HIP, "%s: %s", what, hipGetErrorString(he));
    }
  }
  gc.drop();
  gc.x = x; gc.y = y; gc.dtype = dtype; gc.n = n; gc.K = K; gc.G = G;
  gc.offsets.assign(offsets, offsets + K + 1);
  gc.gofs.assign(gofs, gofs + G + 1);
  gc.fam = fam_of_subset;
  gc.o = o; gc.ws = ws; gc.ws_bytes = ws_bytes; gc.out = out; gc.comb = comb;
  for (int e = 0; e < nexec; ++e) gc.exec[e] = ex[e];
  gc.nexec = nexec;
  gc.valid = true;
  h->have_times = timed ? 1 : 0;
  HIP_OK(gc.launch(h->ev, s));
  return CPC_SUCCESS;
}

// The launch sequence of a fit (tables already in the workspace), one phase
// at a time: rank -> fit -> variance -> combine. In graph mode nothing here
// waits on the host: the streaming path's Newton loop runs its full pass
// budget, its kernels returning at once when every subset is done.
// The buckets of a launch list touch disjoint subsets: they run on two
// streams at once, the call's stream s and the handle's auxiliary one (a
// captured graph gets two branches), so that a bucket does not wait for the
// previous one's last workgroups; the join puts the end back on s. Buckets
// are dealt longest first to the branch with less work, the work of a
// bucket taken as its rows times the family's cost per row relative to the
// Gaussian's (fit and variance passes measured on the benchmark workload:
// Frank about 1.3, Gumbel 1.6; ranks cost the same for every family).
struct Branches {
  bool two = false;
  std::vector<char> on_aux;
  hipStream_t stream(cpc_handle_t h, const std::vector<Bucket>& bl, const Bucket& b, hipStream_t s) const {
    return two && on_aux[(size_t)(&b - bl.data())] ? h->aux_stream : s;
  }
};

int fork_buckets(cpc_handle_t h, const Plan& P, const std::vector<Bucket>& bl, const int32_t* ord, bool by_family,
                 int ev, hipStream_t s, Branches& br) {
  br.two = bl.size() > 1;
  br.on_aux.assign(bl.size(), 0);
  if (!br.two) return CPC_SUCCESS;
  std::vector<std::pair<double, size_t>> w(bl.size());
  for (size_t i = 0; i < bl.size(); ++i) {
    double rows = 0.0;
    for (int32_t k = 0; k < bl[i].count; ++k) rows += (double)P.subs[ord[bl[i].first + k]].n;
    const double f = (!by_family || bl[i].fam == FAM_GAUSSIAN) ? 1.0 : (bl[i].fam == FAM_FRANK ? 1.3 : 1.6);
    w[i] = {rows * f, i};
  }
  std::stable_sort(w.begin(), w.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  double load[2] = {0.0, 0.0};
  for (const auto& e : w) {
    const int side = load[1] < load[0] ? 1 : 0;
    br.on_aux[e.second] = (char)side;
    load[side] += e.first;
  }
  HIP_OK(hipEventRecord(h->fork_ev[ev], s));
  HIP_OK(hipStreamWaitEvent(h->aux_stream, h->fork_ev[ev], 0));
  return CPC_SUCCESS;
}

int join_buckets(cpc_handle_t h, const Branches& br, int ev, hipStream_t s) {
  if (!br.two) return CPC_SUCCESS;
  HIP_OK(hipEventRecord(h->join_ev[ev], h->aux_stream));
  HIP_OK(hipStreamWaitEvent(s, h->join_ev[ev], 0));
  return CPC_SUCCESS;
}

int enqueue_phase(int ph, cpc_handle_t h, const Plan& P, Carved& c, const void* x, const void* y, int32_t dtype,
                  int64_t G, const Options& o, cpc_subset_result_t* out, cpc_combined_t* comb, bool graph,
                  hipStream_t s) {
  const int kw = (dtype == CPC_F64) ? 2 : 1;
  const int fp64 = (o.prec == CPC_PREC_FP64) ? 1 : 0;
  const std::vector<Bucket>& bl = (ph == 0) ? P.rank_buckets : P.fit_buckets;
  Branches br;
  if (ph < 3) {
    if (int rc = fork_buckets(h, P, bl, (ph == 0) ? P.order_rank.data() : P.order_fit.data(), ph != 0, ph, s, br))
      return rc;
  }
  auto stream_of = [&](const Bucket& b) { return br.stream(h, bl, b, s); };
  auto join = [&]() -> int { return join_buckets(h, br, ph, s); };
  switch (ph) {
    case 0: {
      RankParams rp = rank_params(c, x, y, o);
      for (const Bucket& b : P.rank_buckets) {
        rp.order = c.order_rank + b.first;
        HIP_OK(launch_rank_shape(b.shape >= 0 ? b.shape : kRankDefaultShape[b.cls], kw, rp, b.count, stream_of(b)));
      }
      HIP_OK(big_rank(c.big, c.bb, x, y, kw, 0, o.ties, nullptr, nullptr, s));
      return join();
    }
    case 1: {
      FitParams fp;
      std::memset(&fp, 0, sizeof(fp));
      fp.subs = c.subs;
      fp.rows = c.rows;
      fp.state = c.state;
      fp.max_iter = o.max_iter;
      fp.tol = o.tol;
      for (const Bucket& b : P.fit_buckets) {
        fp.order = c.order_fit + b.first;
        HIP_OK(launch_fit_wg(b.cls, b.fam, fp64, fp, b.count, stream_of(b)));
      }
      HIP_OK(big_solve(c.big, c.bb, o.tol, o.max_iter, fp64, graph ? nullptr : h->pending_host, s));
      return join();
    }
    case 2: {
      VarParams vp;
      std::memset(&vp, 0, sizeof(vp));
      vp.subs = c.subs;
      vp.rows = c.rows;
      vp.state = c.state;
      vp.mode = MODE_FIT;
      vp.var_method = o.var;
      vp.out = (ResultOut*)out;
      for (const Bucket& b : P.fit_buckets) {
        vp.order = c.order_fit + b.first;
        HIP_OK(launch_var_wg(b.cls, b.fam, fp64, vp, b.count, stream_of(b)));
      }
      HIP_OK(big_variance(c.big, c.bb, fp64, nullptr, o.var, MODE_FIT, nullptr, (ResultOut*)out, s));
      return join();
    }
    default:
      HIP_OK(launch_combine((const ResultOut*)out, c.gofs, G, (CombinedOut*)comb, s));
      return CPC_SUCCESS;
  }
}

// Eager launch of every phase, with the phase events when asked for. Without
// host_sync the streaming path enqueues its whole Newton pass budget (as in
// graph capture) instead of waiting on its convergence counter.
int enqueue_fit(cpc_handle_t h, const Plan& P, Carved& c, const void* x, const void* y, int32_t dtype, int64_t G,
                const Options& o, cpc_subset_result_t* out, cpc_combined_t* comb, hipStream_t s, bool host_sync) {
  const bool timed = (o.flags & CPC_FLAG_PHASE_TIMES) != 0;
  for (int ph = 0; ph < kPhases; ++ph) {
    if (timed) HIP_OK(hipEventRecord(h->ev[ph], s));
    const int rc = enqueue_phase(ph, h, P, c, x, y, dtype, G, o, out, comb, !host_sync, s);
    if (rc) return rc;
  }
  if (timed) {
    HIP_OK(hipEventRecord(h->ev[kPhases], s));
    h->have_times = 1;
  }
  return CPC_SUCCESS;
}

}  // namespace

extern "C" {

void cpc_default_options(cpc_options_t* o) {
  if (!o) return;
  o->prec = CPC_PREC_FP64;
  o->ties = CPC_TIES_AVERAGE;
  o->var = CPC_VAR_GGR;
  o->max_iter = 60;
  o->tol = 0.0;
  o->n_min = 2;
  o->schedule = -1;
  o->flags = 0;
}

int cpc_create(int device, cpc_handle_t* out) {
  if (!out) return fail(CPC_E_NULL, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_OK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(CPC_E_SIZE, "device %d out of range (%d devices)", device, count);
  HIP_OK(hipSetDevice(device));
  scratch_setup(device);
  cpc_context* h = new cpc_context();
  h->device = device;
  h->magic = kMagic;
  h->plan = new Plan();
  h->have_times = 0;
  h->pending_host = nullptr;
  h->graph = new GraphCache();
  h->tuner = new Tuner();
  tuner_load(tuner_of(h), device);
  if (hipHostMalloc((void**)&h->pending_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
    delete (Tuner*)h->tuner;
    delete (GraphCache*)h->graph;
    delete (Plan*)h->plan;
    delete h;
    return fail(CPC_E_HIP, "hipHostMalloc failed");
  }
  if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipHostFree(h->pending_host);
    delete (Tuner*)h->tuner;
    delete (GraphCache*)h->graph;
    delete (Plan*)h->plan;
    delete h;
    return fail(CPC_E_HIP, "hipStreamCreateWithFlags failed");
  }
  for (int i = 0; i <= kPhases; ++i) {
    if (hipEventCreate(&h->ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(h->ev[j]);
      (void)hipStreamDestroy(h->cap_stream);
      (void)hipHostFree(h->pending_host);
      delete (Tuner*)h->tuner;
      delete (GraphCache*)h->graph;
      delete (Plan*)h->plan;
      delete h;
      return fail(CPC_E_HIP, "hipEventCreate failed");
    }
  }
  bool ok = hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking) == hipSuccess;
  int made = 0;
  for (; ok && made < kPhases; ++made)
    ok = hipEventCreateWithFlags(&h->fork_ev[made], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&h->join_ev[made], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    *out = h;
    (void)cpc_destroy(h);  // (destroys what was made; the rest is null)
    *out = nullptr;
    return fail(CPC_E_HIP, "creating the auxiliary stream or its events failed");
  }
  *out = h;
  return CPC_SUCCESS;
}

int cpc_destroy(cpc_handle_t h) {
  if (int rc = check_handle(h)) return rc;
  h->magic = 0;
  (void)hipSetDevice(h->device);
  graph_of(h).drop();
  delete (GraphCache*)h->graph;
  delete (Tuner*)h->tuner;
  (void)hipStreamDestroy(h->cap_stream);
  if (h->aux_stream) (void)hipStreamDestroy(h->aux_stream);
  for (int i = 0; i < kPhases; ++i) {
    if (h->fork_ev[i]) (void)hipEventDestroy(h->fork_ev[i]);
    if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
  }
  for (int i = 0; i <= kPhases; ++i) (void)hipEventDestroy(h->ev[i]);
  (void)hipHostFree(h->pending_host);
  delete (Plan*)h->plan;
  delete h;
  return CPC_SUCCESS;
}

size_t cpc_workspace_bytes(int64_t n, int64_t K, int64_t G, int32_t dtype, const cpc_options_t* opt) {
  (void)dtype;
  (void)opt;
  if (n < 0 || K < 0 || G < 0) return 0;
  return layout(n, K, G < 1 ? 1 : G, big_bound(n, K)).total;
}

size_t cpc_workspace_bytes_for(const int64_t* offsets, int64_t K, int64_t G, int32_t dtype,
                               const cpc_options_t* opt) {
  (void)dtype;
  (void)opt;
  if (!offsets || K < 1 || G < 0) return 0;
  if (check_offsets(offsets, K, offsets[K]) != CPC_SUCCESS) return 0;
  return layout(offsets[K], K, G < 1 ? 1 : G, big_share(offsets, K)).total;
}

int cpc_fit(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n, const int64_t* offsets,
            int64_t K, int32_t family, const cpc_options_t* opt, void* workspace, size_t ws_bytes,
            cpc_subset_result_t* out, cpc_combined_t* comb, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !y || !offsets || !out || !comb) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1) return fail(CPC_E_SIZE, "K < 1");
  if (dtype != CPC_F64 && dtype != CPC_F32) return fail(CPC_E_ENUM, "unknown dtype %d", dtype);
  if (family < 0 || family > 2) return fail(CPC_E_ENUM, "unknown family %d", family);
  Options o;
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  std::vector<int32_t> fam((size_t)K, family);
  const int64_t gofs[2] = {0, K};
  return run_fit(h, x, y, dtype, n, offsets, K, gofs, 1, fam, o, workspace, ws_bytes, out, comb,
                 (hipStream_t)stream);
}

}  // extern "C"

namespace {
// Host checks of a batched fit's arguments; fills the options and the family
// of every subset.
int check_batched(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n, const int64_t* offsets,
                  int64_t K, const int64_t* group_offsets, int64_t G, const int32_t* family_per_group,
                  const cpc_options_t* opt, const cpc_subset_result_t* out, const cpc_combined_t* comb, Options& o,
                  std::vector<int32_t>& fam) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !y || !offsets || !group_offsets || !family_per_group || !out || !comb)
    return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1) return fail(CPC_E_SIZE, "K < 1");
  if (G < 1) return fail(CPC_E_SIZE, "G < 1");
  if (dtype != CPC_F64 && dtype != CPC_F32) return fail(CPC_E_ENUM, "unknown dtype %d", dtype);
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  if (group_offsets[0] != 0 || group_offsets[G] != K)
    return fail(CPC_E_OFFSETS, "group_offsets must run from 0 to K");
  fam.assign((size_t)K, 0);
  for (int64_t g = 0; g < G; ++g) {
    if (group_offsets[g + 1] < group_offsets[g]) return fail(CPC_E_OFFSETS, "group_offsets decrease at %lld", (long long)g);
    if (family_per_group[g] < 0 || family_per_group[g] > 2)
      return fail(CPC_E_ENUM, "unknown family %d for group %lld", family_per_group[g], (long long)g);
    for (int64_t m = group_offsets[g]; m < group_offsets[g + 1]; ++m) fam[m] = family_per_group[g];
  }
  return CPC_SUCCESS;
}
}  // namespace

extern "C" {

int cpc_fit_batched(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
                    const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
                    const int32_t* family_per_group, const cpc_options_t* opt, void* workspace,
                    size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb, void* stream) {
  Options o;
  std::vector<int32_t> fam;
  if (int rc = check_batched(h, x, y, dtype, n, offsets, K, group_offsets, G, family_per_group, opt, out, comb, o, fam))
    return rc;
  return run_fit(h, x, y, dtype, n, offsets, K, group_offsets, G, fam, o, workspace, ws_bytes, out, comb,
                 (hipStream_t)stream);
}

int cpc_fit_batched_noalloc(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
                            const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
                            const int32_t* family_per_group, const cpc_options_t* opt, cpc_subset_result_t* out,
                            cpc_combined_t* comb, void* stream) {
  Options o;
  std::vector<int32_t> fam;
  if (int rc = check_batched(h, x, y, dtype, n, offsets, K, group_offsets, G, family_per_group, opt, out, comb, o, fam))
    return rc;
  if (o.flags & CPC_FLAG_GRAPH)
    return fail(CPC_E_OPTIONS, "CPC_FLAG_GRAPH builds a graph (an allocation); capture the call instead");
  if (h->device >= kMaxDevices) return fail(CPC_E_UNSUPPORTED, "device %d: no scratch slot", h->device);
  void* ws = nullptr;
  hipError_t err = hipSuccess;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ws = g_scratch_ptr[h->device];
    err = g_scratch_err[h->device];
  }
  if (!ws) return fail(CPC_E_HIP, "scratch of device %d unavailable: %s", h->device, hipGetErrorString(err));
  const size_t need = layout(n, K, G, big_share(offsets, K)).total;
  if (need > kScratchBytes)
    return fail(CPC_E_WORKSPACE, "the call needs %zu bytes of scratch, the static scratch holds %zu", need,
                kScratchBytes);
  return run_fit(h, x, y, dtype, n, offsets, K, group_offsets, G, fam, o, ws, kScratchBytes, out, comb,
                 (hipStream_t)stream, true);
}

// The body of cpc_rank; margins = 1 leaves the y ranks of subsets above
// kResidentMaxRows unwritten (the workgroup kernels rank both margins). With
// big_sorted, x of those subsets is only sorted: their R1 is not written,
// and *big_sorted / *big receive the sorted order and the streaming path's
// tables (big->nsegs = 0 when there is no such subset).
static int rank_impl(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n, const int64_t* offsets,
                     int64_t K, const cpc_options_t* opt, void* workspace, size_t ws_bytes, uint32_t* R1,
                     uint32_t* R2, void* stream, int margins, BigSorted* big_sorted = nullptr,
                     BigParams* big = nullptr) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !y || !offsets || !R1 || !R2) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1) return fail(CPC_E_SIZE, "K < 1");
  if (dtype != CPC_F64 && dtype != CPC_F32) return fail(CPC_E_ENUM, "unknown dtype %d", dtype);
  Options o;
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  const Layout L = layout(n, K, 1, big_share(offsets, K));
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < L.total) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, L.total);
  std::vector<int32_t> fam((size_t)K, 0);
  Plan& P = plan_of(h);
  if (int rc = make_plan(offsets, K, fam.data(), P)) return rc;
  HIP_OK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  touch_workspace(h, workspace);
  Carved c = carve(workspace, L);
  if (int rc = upload_tables(h, P, c, nullptr, 0, s)) return rc;
  RankParams rp;
  std::memset(&rp, 0, sizeof(rp));
  rp.x = x;
  rp.y = y;
  rp.subs = c.subs;
  rp.mode = MODE_RANK;
  rp.ties = o.ties;
  rp.n_min = o.n_min;
  rp.rows = c.rows;
  rp.R1out = R1;
  rp.R2out = R2;
  rp.state = c.state;
  const int kw = (dtype == CPC_F64) ? 2 : 1;
  Branches br;
  if (int rc = fork_buckets(h, P, P.rank_buckets, P.order_rank.data(), false, 0, s, br)) return rc;
  for (const Bucket& b : P.rank_buckets) {
    rp.order = c.order_rank + b.first;
    // a shape forced through opt->schedule for the classes it serves; else the class default
    if (o.schedule > 0 && kw == 1 && kRankShapes[o.schedule - 1].cap == kClassThreads[b.cls] * kClassItems[b.cls])
      HIP_OK(launch_rank_shape(o.schedule - 1, kw, rp, b.count, br.stream(h, P.rank_buckets, b, s)));
    else
      HIP_OK(launch_rank_wg(b.cls, kw, rp, b.count, br.stream(h, P.rank_buckets, b, s)));
  }
  set_big(c, P, o.n_min);
  if (big) *big = c.big;
  HIP_OK(big_rank(c.big, c.bb, x, y, kw, 0, o.ties, R1, R2, s, margins, big_sorted));
  return join_buckets(h, br, 0, s);
}

int cpc_rank(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n, const int64_t* offsets,
             int64_t K, const cpc_options_t* opt, void* workspace, size_t ws_bytes, uint32_t* R1, uint32_t* R2,
             void* stream) {
  return rank_impl(h, x, y, dtype, n, offsets, K, opt, workspace, ws_bytes, R1, R2, stream, 2);
}

int cpc_variance(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n, const int64_t* offsets,
                 int64_t K, int32_t family, const double* theta, const cpc_options_t* opt, void* workspace,
                 size_t ws_bytes, double* var, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!R1 || !R2 || !offsets || !theta || !var) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1) return fail(CPC_E_SIZE, "K < 1");
  if (family < 0 || family > 2) return fail(CPC_E_ENUM, "unknown family %d", family);
  Options o;
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  const Layout L = layout(n, K, 1, big_share(offsets, K));
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < L.total) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, L.total);
  std::vector<int32_t> fam((size_t)K, family);
  Plan& P = plan_of(h);
  if (int rc = make_plan(offsets, K, fam.data(), P)) return rc;
  HIP_OK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  touch_workspace(h, workspace);
  Carved c = carve(workspace, L);
  if (int rc = upload_tables(h, P, c, nullptr, 0, s)) return rc;
  // re-rank from the given ranks (integer keys): sorted positions and tie groups
  RankParams rp;
  std::memset(&rp, 0, sizeof(rp));
  rp.x = R1;
  rp.y = R2;
  rp.subs = c.subs;
  rp.mode = MODE_VARIANCE;
  rp.ties = o.ties;
  rp.int_keys = 1;
  rp.n_min = o.n_min;
  rp.rows = c.rows;
  rp.state = c.state;
  Branches br;
  if (int rc = fork_buckets(h, P, P.rank_buckets, P.order_rank.data(), false, 0, s, br)) return rc;
  for (const Bucket& b : P.rank_buckets) {
    rp.order = c.order_rank + b.first;
    HIP_OK(launch_rank_wg(b.cls, 1, rp, b.count, br.stream(h, P.rank_buckets, b, s)));
  }
  set_big(c, P, o.n_min);
  HIP_OK(big_rank(c.big, c.bb, R1, R2, 1, 1, o.ties, nullptr, nullptr, s));
  if (int rc = join_buckets(h, br, 0, s)) return rc;
  VarParams vp;
  std::memset(&vp, 0, sizeof(vp));
  vp.subs = c.subs;
  vp.rows = c.rows;
  vp.state = c.state;
  vp.mode = MODE_VARIANCE;
  vp.var_method = o.var;
  vp.theta_in = theta;
  vp.var_out = var;
  const int fp64 = (o.prec == CPC_PREC_FP64) ? 1 : 0;
  Branches bv;
  if (int rc = fork_buckets(h, P, P.fit_buckets, P.order_fit.data(), true, 2, s, bv)) return rc;
  for (const Bucket& b : P.fit_buckets) {
    vp.order = c.order_fit + b.first;
    HIP_OK(launch_var_wg(b.cls, b.fam, fp64, vp, b.count, bv.stream(h, P.fit_buckets, b, s)));
  }
  HIP_OK(big_variance(c.big, c.bb, fp64, theta, o.var, MODE_VARIANCE, var, nullptr, s));
  return join_buckets(h, bv, 2, s);
}

int cpc_eval(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n, const int64_t* offsets, int64_t K,
             int32_t family, const double* theta, const cpc_options_t* opt, void* workspace, size_t ws_bytes,
             double* out, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!R1 || !R2 || !offsets || !theta || !out) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1) return fail(CPC_E_SIZE, "K < 1");
  if (family < 0 || family > 2) return fail(CPC_E_ENUM, "unknown family %d", family);
  Options o;
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  const Layout L = layout(n, K, 1, big_share(offsets, K));
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < L.total) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, L.total);
  std::vector<SubDesc> subs((size_t)K);
  for (int64_t m = 0; m < K; ++m) {
    subs[m].begin = offsets[m];
    subs[m].n = (int32_t)(offsets[m + 1] - offsets[m]);
    subs[m].family = (int16_t)family;
    subs[m].group = 0;
  }
  HIP_OK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  touch_workspace(h, workspace);
  Carved c = carve(workspace, L);
  HIP_OK(hipMemcpyAsync(c.subs, subs.data(), sizeof(SubDesc) * (size_t)K, hipMemcpyHostToDevice, s));
  int64_t n_max = 0;
  for (int64_t m = 0; m < K; ++m) n_max = std::max<int64_t>(n_max, offsets[m + 1] - offsets[m]);
  HIP_OK(launch_eval_wg(R1, R2, c.subs, K, family, o.prec == CPC_PREC_FP64 ? 1 : 0, n_max, theta, out, s));
  return CPC_SUCCESS;
}

int cpc_sample(cpc_handle_t h, int32_t family, double theta, uint64_t seed, int64_t row0, int64_t n, int32_t dtype,
               void* x, void* y, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (n < 0 || row0 < 0) return fail(CPC_E_SIZE, "n and row0 must be >= 0");
  if (n > 0 && (!x || !y)) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (dtype != CPC_F64 && dtype != CPC_F32) return fail(CPC_E_ENUM, "unknown dtype %d", dtype);
  if (family < 0 || family > 2) return fail(CPC_E_ENUM, "unknown family %d", family);
  const bool ok = family == CPC_GAUSSIAN ? (theta > -1.0 && theta < 1.0)
                                         : (family == CPC_FRANK ? std::isfinite(theta) : (theta >= 1.0 && std::isfinite(theta)));
  if (!ok) return fail(CPC_E_OPTIONS, "theta = %g is outside the family's parameter range", theta);
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(launch_sample(family, theta, seed, row0, n, dtype == CPC_F32 ? 1 : 0, x, y, (hipStream_t)stream));
  return CPC_SUCCESS;
}

int cpc_density_distance(cpc_handle_t h, int32_t family, int64_t P, const double* theta_a, const double* theta_b,
                         double box, int32_t panels, void* workspace, size_t ws_bytes, double* out, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!theta_a || !theta_b || !out) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (family < 0 || family > 2) return fail(CPC_E_ENUM, "unknown family %d", family);
  if (P < 1 || P > 65535) return fail(CPC_E_SIZE, "P must be in [1, 65535] (got %lld)", (long long)P);
  if (panels < 1 || panels > 65535) return fail(CPC_E_SIZE, "panels must be in [1, 65535] (got %d)", panels);
  if (!(box > 0.0) || !(box <= 40.0)) return fail(CPC_E_OPTIONS, "box must be in (0, 40] (got %g)", box);
  const size_t need = sizeof(double) * 4 * (size_t)P * (size_t)panels;
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(launch_density_distance(family, P, theta_a, theta_b, box, panels, (double*)workspace, out,
                                 (hipStream_t)stream));
  return CPC_SUCCESS;
}

int cpc_replicate_summary(cpc_handle_t h, int64_t S, const cpc_combined_t* combined, const cpc_combined_t* full,
                          double* out, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!combined || !full || !out) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (S < 1) return fail(CPC_E_SIZE, "S < 1");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(launch_replicate_summary(S, (const CombinedOut*)combined, (const CombinedOut*)full, out,
                                  (hipStream_t)stream));
  return CPC_SUCCESS;
}

// Rank options of cpc_partition: ties broken by row order, so that the
// doubled ranks are 2 (position + 1) in the x-order.
static cpc_options_t partition_rank_options() {
  cpc_options_t o;
  cpc_default_options(&o);
  o.ties = CPC_TIES_FIRST;
  return o;
}

size_t cpc_partition_workspace_bytes(const int64_t* rep_offsets, int64_t R, int32_t dtype, int32_t scheme) {
  if (!rep_offsets || R < 1) return 0;
  if (dtype != CPC_F64 && dtype != CPC_F32) return 0;
  if (scheme < CPC_PART_CONTIGUOUS || scheme > CPC_PART_STRIDED) return 0;
  if (check_offsets(rep_offsets, R, rep_offsets[R]) != CPC_SUCCESS) return 0;
  size_t need = align_up(sizeof(int64_t) * (size_t)(R + 1));
  // strided: the rows in blocks order before their transpose
  if (scheme == CPC_PART_STRIDED)
    need += 2 * align_up((dtype == CPC_F64 ? 8 : 4) * (size_t)rep_offsets[R]);
  if (scheme != CPC_PART_CONTIGUOUS) {
    const cpc_options_t o = partition_rank_options();
    need += 2 * align_up(sizeof(uint32_t) * (size_t)rep_offsets[R]) +
            cpc_workspace_bytes_for(rep_offsets, R, 1, dtype, &o);
  }
  return need;
}

int cpc_partition(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n, const int64_t* rep_offsets,
                  int64_t R, int64_t M, int32_t scheme, void* workspace, size_t ws_bytes, void* x_out, void* y_out,
                  int64_t* offsets_out, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!x || !y || !rep_offsets || !x_out || !y_out || !offsets_out) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (R < 1) return fail(CPC_E_SIZE, "R < 1");
  if (M < 1 || M >= ((int64_t)1 << 31)) return fail(CPC_E_SIZE, "M = %lld: expected 1 <= M < 2^31", (long long)M);
  if (M > (INT64_MAX - 1) / R) return fail(CPC_E_SIZE, "R M + 1 offsets do not fit in int64");
  if (dtype != CPC_F64 && dtype != CPC_F32) return fail(CPC_E_ENUM, "unknown dtype %d", dtype);
  if (scheme < CPC_PART_CONTIGUOUS || scheme > CPC_PART_STRIDED) return fail(CPC_E_ENUM, "unknown scheme %d", scheme);
  if (x_out == x || x_out == y || y_out == x || y_out == y || x_out == y_out)
    return fail(CPC_E_SIZE, "x_out and y_out must be buffers of their own");
  if (int rc = check_offsets(rep_offsets, R, n)) return rc;
  const size_t need = cpc_partition_workspace_bytes(rep_offsets, R, dtype, scheme);
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
  // subset bounds: contiguous and blocks split N evenly, floor(m N / M); the
  // strided scheme's subset m has ceil((N - m) / M) rows
  for (int64_t r = 0; r < R; ++r) {
    const int64_t b = rep_offsets[r], N = rep_offsets[r + 1] - b;
    const int64_t a = N / M, c = N % M;
    for (int64_t m = 0; m < M; ++m)
      offsets_out[r * M + m] =
          b + (scheme == CPC_PART_STRIDED ? m * a + (m < c ? m : c) : (int64_t)(((__int128)m * N) / M));
  }
  offsets_out[R * M] = n;
  if (n == 0) return CPC_SUCCESS;
  HIP_OK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  unsigned char* b = (unsigned char*)workspace;
  int64_t* drep = (int64_t*)b;
  b += align_up(sizeof(int64_t) * (size_t)(R + 1));
  void *tx = nullptr, *ty = nullptr;
  if (scheme == CPC_PART_STRIDED) {
    const size_t eb = align_up((dtype == CPC_F64 ? 8 : 4) * (size_t)n);
    tx = b;
    ty = b + eb;
    b += 2 * eb;
  }
  uint32_t* R1 = nullptr;
  // replicates above kResidentMaxRows: x sorted on the streaming path and
  // the rows gathered from the sorted payloads (no ranks formed)
  BigSorted big_sorted = {nullptr, nullptr, nullptr};
  BigParams big;
  std::memset(&big, 0, sizeof(big));
  if (scheme != CPC_PART_CONTIGUOUS) {
    R1 = (uint32_t*)b;
    b += align_up(sizeof(uint32_t) * (size_t)n);
    uint32_t* R2 = (uint32_t*)b;
    b += align_up(sizeof(uint32_t) * (size_t)n);
    const cpc_options_t o = partition_rank_options();
    const size_t used = (size_t)(b - (unsigned char*)workspace);
    if (int rc = rank_impl(h, x, y, dtype, n, rep_offsets, R, &o, b, ws_bytes - used, R1, R2, stream, 1,
                           &big_sorted, &big))
      return rc;
  }
  // the host table stays alive in the handle until the next call (the copy is asynchronous)
  Plan& P = plan_of(h);
  P.part_rep.assign(rep_offsets, rep_offsets + R + 1);
  HIP_OK(hipMemcpyAsync(drep, P.part_rep.data(), sizeof(int64_t) * (size_t)(R + 1), hipMemcpyHostToDevice, s));
  const int f32 = dtype == CPC_F32 ? 1 : 0;
  const bool gather = big.nsegs > 0 && big_sorted.rows != nullptr;
  bool small = !gather;  // a replicate left to the scatter kernel
  for (int64_t r = 0; r < R && !small; ++r) {
    const int64_t N = rep_offsets[r + 1] - rep_offsets[r];
    small = N > 0 && N <= kResidentMaxRows;
  }
  if (small) HIP_OK(launch_partition(f32, x, y, R1, drep, R, n, M, scheme, gather ? 1 : 0, x_out, y_out, s));
  if (gather && scheme == CPC_PART_STRIDED) {
    // the blocks order (whose x comes from the keys in order), then its
    // transpose into the strided order: both read and write along rows
    HIP_OK(launch_partition_gather(f32, big, big_sorted, x, y, M, CPC_PART_BLOCKS, tx, ty, s));
    int64_t max_tiles = 0;
    for (int64_t r = 0; r < R; ++r) {
      const int64_t N = rep_offsets[r + 1] - rep_offsets[r];
      if (N <= kResidentMaxRows) continue;
      const int64_t Q = (N + M - 1) / M, Mc = std::min<int64_t>(M, N);
      max_tiles = std::max<int64_t>(max_tiles, ((Q + 31) / 32) * ((Mc + 31) / 32));
    }
    if ((int64_t)big.nsegs * max_tiles >= ((int64_t)1 << 31))
      return fail(CPC_E_UNSUPPORTED, "too many transpose tiles");
    HIP_OK(launch_partition_transpose(f32, big, tx, ty, M, max_tiles, x_out, y_out, s));
  } else if (gather) {
    HIP_OK(launch_partition_gather(f32, big, big_sorted, x, y, M, scheme, x_out, y_out, s));
  }
  return CPC_SUCCESS;
}

size_t cpc_spearman_workspace_bytes(int64_t n, int64_t K, int64_t G) {
  if (n < 0 || K < 1 || G < 1) return 0;
  return align_up(sizeof(SubDesc) * (size_t)K) + align_up(sizeof(int64_t) * (size_t)(G + 1)) +
         2 * align_up(sizeof(long long) * 2 * (size_t)(n + K));
}

size_t cpc_kendall_workspace_bytes(int64_t n, int64_t K, int64_t G) {
  if (n < 0 || K < 1 || G < 1) return 0;
  return align_up(sizeof(SubDesc) * (size_t)K) + align_up(sizeof(int64_t) * (size_t)(G + 1)) +
         2 * align_up(sizeof(unsigned long long) * (size_t)n) + align_up(sizeof(int) * (size_t)n) +
         align_up(sizeof(int) * (size_t)K);
}

namespace {

constexpr int64_t kKendallMaxRows = int64_t(1) << 20;

// cpc_spearman_fit (kendall = false) and cpc_kendall_fit (kendall = true)
int moment_fit(bool kendall, cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n,
               const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
               const int32_t* family_per_group, const cpc_options_t* opt, void* workspace, size_t ws_bytes,
               cpc_subset_result_t* out, cpc_combined_t* comb, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!R1 || !R2 || !offsets || !group_offsets || !family_per_group || !out || !comb)
    return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1 || G < 1) return fail(CPC_E_SIZE, "K and G must be >= 1");
  Options o;
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  if (group_offsets[0] != 0 || group_offsets[G] != K) return fail(CPC_E_OFFSETS, "group_offsets must run from 0 to K");
  std::vector<SubDesc> subs((size_t)K);
  for (int64_t g = 0; g < G; ++g) {
    if (group_offsets[g + 1] < group_offsets[g]) return fail(CPC_E_OFFSETS, "group_offsets decrease at %lld", (long long)g);
    if (family_per_group[g] < 0 || family_per_group[g] > 2)
      return fail(CPC_E_ENUM, "unknown family %d for group %lld", family_per_group[g], (long long)g);
    for (int64_t m = group_offsets[g]; m < group_offsets[g + 1]; ++m) {
      const int64_t nm = offsets[m + 1] - offsets[m];
      if (kendall && nm > kKendallMaxRows)
        return fail(CPC_E_UNSUPPORTED, "subset %lld has %lld rows; the Kendall estimator takes at most %lld",
                    (long long)m, (long long)nm, (long long)kKendallMaxRows);
      subs[m].begin = offsets[m];
      subs[m].n = (int32_t)nm;
      subs[m].family = (int16_t)family_per_group[g];
      subs[m].group = 0;
    }
  }
  const size_t need = kendall ? cpc_kendall_workspace_bytes(n, K, G) : cpc_spearman_workspace_bytes(n, K, G);
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
  unsigned char* b = (unsigned char*)workspace;
  SubDesc* dsubs = (SubDesc*)b;
  b += align_up(sizeof(SubDesc) * (size_t)K);
  int64_t* dgofs = (int64_t*)b;
  b += align_up(sizeof(int64_t) * (size_t)(G + 1));
  long long* H1 = nullptr;
  long long* H2 = nullptr;
  unsigned long long* W0 = nullptr;
  unsigned long long* W1 = nullptr;
  int* C = nullptr;
  int* flag = nullptr;
  if (kendall) {
    W0 = (unsigned long long*)b;
    b += align_up(sizeof(unsigned long long) * (size_t)n);
    W1 = (unsigned long long*)b;
    b += align_up(sizeof(unsigned long long) * (size_t)n);
    C = (int*)b;
    b += align_up(sizeof(int) * (size_t)n);
    flag = (int*)b;
  } else {
    H1 = (long long*)b;
    b += align_up(sizeof(long long) * 2 * (size_t)(n + K));
    H2 = (long long*)b;
  }
  HIP_OK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  touch_workspace(h, workspace);
  // the host tables stay alive in the handle until the next call (the copies are asynchronous)
  Plan& P = plan_of(h);
  P.subs = subs;
  P.gofs.assign(group_offsets, group_offsets + G + 1);
  HIP_OK(hipMemcpyAsync(dsubs, P.subs.data(), sizeof(SubDesc) * (size_t)K, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dgofs, P.gofs.data(), sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
  // one launch per run of groups of one family (subsets in order); the runs
  // touch disjoint subsets and rows, so with more than one they are dealt,
  // most rows first, to the call's stream and the auxiliary one (each
  // launch otherwise ends with a partly idle last wave of workgroups)
  std::vector<std::pair<int64_t, int64_t>> runs;  // (first group, end group)
  for (int64_t g = 0; g < G;) {
    int64_t h2 = g;
    while (h2 < G && family_per_group[h2] == family_per_group[g]) ++h2;
    if (group_offsets[h2] > group_offsets[g]) runs.push_back({g, h2});
    g = h2;
  }
  const bool two = runs.size() > 1;
  std::vector<char> on_aux(runs.size(), 0);
  if (two) {
    std::vector<std::pair<int64_t, size_t>> w(runs.size());
    for (size_t i = 0; i < runs.size(); ++i)
      w[i] = {offsets[group_offsets[runs[i].second]] - offsets[group_offsets[runs[i].first]], i};
    std::stable_sort(w.begin(), w.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    int64_t load[2] = {0, 0};
    for (const auto& e : w) {
      const int side = load[1] < load[0] ? 1 : 0;
      on_aux[e.second] = (char)side;
      load[side] += e.first;
    }
    HIP_OK(hipEventRecord(h->fork_ev[1], s));
    HIP_OK(hipStreamWaitEvent(h->aux_stream, h->fork_ev[1], 0));
  }
  for (size_t i = 0; i < runs.size(); ++i) {
    const int64_t g = runs[i].first;
    const int64_t m0 = group_offsets[g], m1 = group_offsets[runs[i].second];
    hipStream_t rs = on_aux[i] ? h->aux_stream : s;
    if (kendall) {
      HIP_OK(launch_kendall(family_per_group[g], R1, R2, dsubs, m0, m1 - m0, o.n_min, W0, W1, C, flag,
                            (ResultOut*)out, rs));
    } else {
      int64_t n_max = 0;
      for (int64_t m = m0; m < m1; ++m) n_max = std::max<int64_t>(n_max, offsets[m + 1] - offsets[m]);
      HIP_OK(launch_spearman(family_per_group[g], R1, R2, dsubs, m0, m1 - m0, o.n_min, n_max, H1, H2,
                             (ResultOut*)out, rs));
    }
  }
  if (two) {
    HIP_OK(hipEventRecord(h->join_ev[1], h->aux_stream));
    HIP_OK(hipStreamWaitEvent(s, h->join_ev[1], 0));
  }
  HIP_OK(launch_combine((const ResultOut*)out, dgofs, G, (CombinedOut*)comb, s));
  return CPC_SUCCESS;
}

}  // namespace

int cpc_spearman_fit(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n, const int64_t* offsets,
                     int64_t K, const int64_t* group_offsets, int64_t G, const int32_t* family_per_group,
                     const cpc_options_t* opt, void* workspace, size_t ws_bytes, cpc_subset_result_t* out,
                     cpc_combined_t* comb, void* stream) {
  return moment_fit(false, h, R1, R2, n, offsets, K, group_offsets, G, family_per_group, opt, workspace, ws_bytes,
                    out, comb, stream);
}

int cpc_kendall_fit(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n, const int64_t* offsets,
                    int64_t K, const int64_t* group_offsets, int64_t G, const int32_t* family_per_group,
                    const cpc_options_t* opt, void* workspace, size_t ws_bytes, cpc_subset_result_t* out,
                    cpc_combined_t* comb, void* stream) {
  return moment_fit(true, h, R1, R2, n, offsets, K, group_offsets, G, family_per_group, opt, workspace, ws_bytes,
                    out, comb, stream);
}

size_t cpc_gaussk_workspace_bytes(int64_t n, int32_t k, int64_t K, int64_t G) {
  if (n < 0 || k < 2 || k > 8 || K < 1 || G < 1) return 0;
  const int64_t p = (int64_t)k * (k - 1) / 2;
  return align_up(sizeof(SubDesc) * (size_t)K) + align_up(sizeof(int64_t) * (size_t)(p * G + 1)) +
         align_up(sizeof(double) * (size_t)n * (size_t)k) + align_up(sizeof(double) * (size_t)n * (size_t)gaussk_ldx(k)) +
         align_up(sizeof(double) * (size_t)(n + K) * (size_t)k * (size_t)k);
}

int cpc_gaussk_fit(cpc_handle_t h, const uint32_t* R, int64_t n, int32_t k, const int64_t* offsets, int64_t K,
                   const int64_t* group_offsets, int64_t G, const cpc_options_t* opt, void* workspace, size_t ws_bytes,
                   cpc_subset_result_t* out, cpc_combined_t* comb, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!R || !offsets || !group_offsets || !out || !comb) return fail(CPC_E_NULL, "a required pointer is NULL");
  if (n < 0) return fail(CPC_E_SIZE, "n < 0");
  if (K < 1 || G < 1) return fail(CPC_E_SIZE, "K and G must be >= 1");
  if (k < 2) return fail(CPC_E_SIZE, "k = %d: at least two margins", (int)k);
  if (k > 8) return fail(CPC_E_UNSUPPORTED, "k = %d: at most 8 margins", (int)k);
  Options o;
  if (int rc = read_options(opt, o)) return rc;
  if (int rc = check_offsets(offsets, K, n)) return rc;
  if (group_offsets[0] != 0 || group_offsets[G] != K) return fail(CPC_E_OFFSETS, "group_offsets must run from 0 to K");
  for (int64_t g = 0; g < G; ++g)
    if (group_offsets[g + 1] < group_offsets[g]) return fail(CPC_E_OFFSETS, "group_offsets decrease at %lld", (long long)g);
  const size_t need = cpc_gaussk_workspace_bytes(n, k, K, G);
  if (!workspace) return fail(CPC_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(CPC_E_WORKSPACE, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
  const int64_t p = (int64_t)k * (k - 1) / 2;
  std::vector<SubDesc> subs((size_t)K);
  for (int64_t m = 0; m < K; ++m) {
    subs[m].begin = offsets[m];
    subs[m].n = (int32_t)(offsets[m + 1] - offsets[m]);
    subs[m].family = (int16_t)FAM_GAUSSIAN;
    subs[m].group = 0;
  }
  // eq. (15) per parameter and group: group (q, g) spans the entries
  // q K + group_offsets[g] .. q K + group_offsets[g + 1] of the parameter-major results
  std::vector<int64_t> gofs((size_t)(p * G + 1));
  for (int64_t q = 0; q < p; ++q)
    for (int64_t g = 0; g < G; ++g) gofs[(size_t)(q * G + g)] = q * K + group_offsets[g];
  gofs[(size_t)(p * G)] = p * K;
  unsigned char* b = (unsigned char*)workspace;
  SubDesc* dsubs = (SubDesc*)b;
  b += align_up(sizeof(SubDesc) * (size_t)K);
  int64_t* dgofs = (int64_t*)b;
  b += align_up(sizeof(int64_t) * (size_t)(p * G + 1));
  double* Z = (double*)b;
  b += align_up(sizeof(double) * (size_t)n * (size_t)k);
  double* X = (double*)b;
  b += align_up(sizeof(double) * (size_t)n * (size_t)gaussk_ldx(k));
  double* B = (double*)b;
  HIP_OK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  touch_workspace(h, workspace);
  // the host tables stay alive in the handle until the next call (the copies are asynchronous)
  Plan& P = plan_of(h);
  P.subs = subs;
  P.gofs = gofs;
  HIP_OK(hipMemcpyAsync(dsubs, P.subs.data(), sizeof(SubDesc) * (size_t)K, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dgofs, P.gofs.data(), sizeof(int64_t) * P.gofs.size(), hipMemcpyHostToDevice, s));
  HIP_OK(launch_gaussk(R, n, k, dsubs, K, o.n_min, Z, X, B, (ResultOut*)out, s));
  HIP_OK(launch_combine((const ResultOut*)out, dgofs, p * G, (CombinedOut*)comb, s));
  return CPC_SUCCESS;
}

int cpc_phase_times(cpc_handle_t h, float* ms) {
  if (int rc = check_handle(h)) return rc;
  if (!ms) return fail(CPC_E_NULL, "ms is NULL");
  if (!h->have_times) return fail(CPC_E_OPTIONS, "no fit with CPC_FLAG_PHASE_TIMES on this handle");
  HIP_OK(hipEventSynchronize(h->ev[kPhases]));
  for (int i = 0; i < kPhases; ++i) HIP_OK(hipEventElapsedTime(&ms[i], h->ev[i], h->ev[i + 1]));
  return CPC_SUCCESS;
}

const char* cpc_strerror(int code) {
  switch (code) {
    case CPC_SUCCESS: return "success";
    case CPC_E_NULL: return "a required pointer is NULL";
    case CPC_E_SIZE: return "size out of range";
    case CPC_E_OFFSETS: return "offsets are not a partition of the rows";
    case CPC_E_ENUM: return "unknown enumeration value";
    case CPC_E_WORKSPACE: return "workspace missing or too small";
    case CPC_E_HIP: return "HIP runtime error";
    case CPC_E_HANDLE: return "invalid handle";
    case CPC_E_OPTIONS: return "option out of range";
    case CPC_E_UNSUPPORTED: return "unsupported size or feature";
    default: return "unknown error code";
  }
}

const char* cpc_last_error(void) { return g_last_error; }

}  // extern "C"
