// C-ABI of libcum (declared in include/cum.h).
//
// Alg. 1 of the paper as library calls: cum_init computes the first window's
// moments (chunked contraction) and cumulants; every cum_update slides the
// window (Alg. 2), recomputes the cumulants (Alg. 3/4) and the norms (Alg. 5,
// Eq. (mef)) on the context's stream.  All argument checks happen before any
// HIP call, so invalid calls leave the context untouched.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/cum.h"
#include "adjoint.h"
#include "kernels.h"
#include "noalloc.h"
#include "tables.h"

using namespace cum;

namespace {

constexpr int64_t kRowChunk = 2048;  // rows per contraction before each compensated fold

}  // namespace

struct cum_ctx {
  int n = 0, d = 0, b = 0, prec = 0;
  int64_t t = 0;
  int device = 0;        // device current at cum_init
  hipStream_t stream = nullptr;
  bool ready = false;
  Tables T;
  int nitems = 0;
  int tm = 2, tn = 2;    // update tile in 16x16 fragments
  int chunk = 0, stride = 0;
  size_t st_size = 0;    // bytes per state element (4 or 8)
  size_t x_size = 0;     // bytes per input element (4 or 8)
  void* s_hi[CUM_MAXD + 1] = {};
  void* s_lo[CUM_MAXD + 1] = {};
  double* C[CUM_MAXD + 1] = {};
  double* partial[CUM_MAXD + 1] = {};
  int32_t* subrank[CUM_MAXD + 1] = {};
  double* mult[CUM_MAXD + 1] = {};
  LeftCol* left[CUM_MAXD + 1] = {};
  RightCol* right[CUM_MAXD + 1] = {};
  UpdItem* items = nullptr;
  double* norms = nullptr;
  void* stage = nullptr;
  size_t stage_bytes = 0;
  std::vector<void*> owned;
  // set while this context belongs to a batch: the batch's last step, and
  // whether the context was updated directly since (the batch then waits)
  hipEvent_t batch_done = nullptr;
  bool direct_since_batch = false;
  // optional per-kernel timing: (class, start, stop) per launch of the
  // classes in profile_mask; events are recycled through a pool
  void* zero = nullptr;  // UPD_ZERO_BYTES zeros: padding source of the update's direct loads
  // four tiles per workgroup: the items padded to groups of four with empty
  // tiles (M = N = 0)
  bool quad = false;
  UpdItem* qitems = nullptr;
  std::vector<UpdItem> h_qitems;
  // split contraction (init and recalculation of contexts with few tiles):
  // room for split_cap chunks' copies of the running sums, their argument
  // blocks, and the quad items repeated per chunk (ctx = chunk)
  int split_cap = 0;
  void* split_state = nullptr;
  UpdArgs* d_split_args = nullptr;
  UpdItem* d_split_items = nullptr;
  int split_args_cap = 0;
  std::vector<UpdArgs> h_split_args;
  std::vector<UpdArgs> h_split_prev;  // the blocks on the device
  // FIFO mode (fifo_p > 0): fifo_q = t / fifo_p slots of batch increments
  // per order, slot fifo_head holding the oldest batch of the window
  int64_t fifo_p = 0;
  int fifo_q = 0, fifo_head = 0;
  void* snap[CUM_MAXD + 1] = {};
  // fused combine over each order-d block's sub-block lattice (lat_lds > 0
  // when it fits in LDS): designation bits per order-d block, LDS offsets
  uint8_t* desig = nullptr;
  size_t lat_lds = 0;
  int lat_off[(1 << CUM_MAXD) + 1] = {};
  int combine = CUM_COMBINE_PARTITIONS;
  // norms of the last combine not yet formed: the next update launch forms
  // them in one extra workgroup, or flush_norms launches them alone
  bool norms_pending = false;
  NormArgs pending_na{};
  // pipelined sliding updates: the update launch stores its increment in
  // delta[slot] (slots alternate); on pstream the increment is folded into
  // the running sums, then the combine and the norms run, beside the next
  // update.  pipe_active: pstream holds work not yet ordered before stream.
  hipStream_t pstream = nullptr;
  void* delta[2] = {};
  hipEvent_t ev_upd[2] = {}, ev_fold[2] = {}, ev_join = nullptr;
  bool fold_pending[2] = {};
  int pipe_slot = 0;
  bool pipe_active = false;
  bool pipe_off = true;               // unless CUM_PIPELINE=1 in the environment
  // the device allocation the last update's rows were found in: rows inside
  // it need no pointer query
  uintptr_t dev_lo = 0, dev_hi = 0;
  int profile_mask = 0;
  bool no_events = false;             // set during cum_update_noalloc: no profiling events
  int profile_every = 1;              // bracket one launch in this many per class
  int64_t profile_seen[3] = {0, 0, 0};
  struct Ev { int cls; hipEvent_t a, b; };
  std::vector<Ev> events;
  std::vector<hipEvent_t> event_pool;
};

namespace {

thread_local char g_last_error[512] = "";

void note_error(hipError_t e, const char* what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "api.cpp:%d %s -> %s (%s)", line, what,
           hipGetErrorName(e), hipGetErrorString(e));
}

int map_err(hipError_t e) {
  if (e == hipSuccess) return CUM_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return CUM_ENOMEM;
  return CUM_EDEVICE;
}

#define CUM_TRY(expr)                    \
  do {                                   \
    hipError_t e_ = (expr);              \
    if (e_ != hipSuccess) {              \
      note_error(e_, #expr, __LINE__);   \
      (void)hipGetLastError();           \
      return map_err(e_);                \
    }                                    \
  } while (0)

#define CUM_NOTE(e, what) note_error((e), (what), __LINE__)

// Optional cap on the bytes one context may allocate (forces CUM_ENOMEM in
// tests without exhausting the device): CUM_DEVICE_MEM_CAP=<bytes>.
size_t mem_cap() {
  const char* s = getenv("CUM_DEVICE_MEM_CAP");
  if (!s || !*s) return 0;
  return (size_t)strtoull(s, nullptr, 10);
}

hipError_t dalloc(cum_ctx* c, void** p, size_t bytes, size_t* used) {
  *p = nullptr;
  const size_t cap = mem_cap();
  if (cap && *used + bytes > cap) return hipErrorOutOfMemory;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) { *p = nullptr; return e; }
  *used += bytes;
  c->owned.push_back(*p);
  return hipSuccess;
}

template <typename V>
hipError_t upload(cum_ctx* c, V** dst, const std::vector<V>& src, size_t* used) {
  void* p = nullptr;
  hipError_t e = dalloc(c, &p, src.size() * sizeof(V), used);
  if (e != hipSuccess) return e;
  *dst = (V*)p;
  if (!src.empty()) e = hipMemcpy(p, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice);
  return e;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) { (void)hipGetLastError(); return false; }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

void drop_events(cum_ctx* c) {
  for (auto& e : c->events) {
    c->event_pool.push_back(e.a);
    c->event_pool.push_back(e.b);
  }
  c->events.clear();
}

void release(cum_ctx* c) {
  if (c->pstream) (void)hipStreamSynchronize(c->pstream);
  for (int q = 0; q < 2; ++q) {
    if (c->ev_upd[q]) (void)hipEventDestroy(c->ev_upd[q]);
    if (c->ev_fold[q]) (void)hipEventDestroy(c->ev_fold[q]);
    c->ev_upd[q] = c->ev_fold[q] = nullptr;
  }
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  c->ev_join = nullptr;
  if (c->pstream) (void)hipStreamDestroy(c->pstream);
  c->pstream = nullptr;
  drop_events(c);
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  c->event_pool.clear();
  for (void* p : c->owned) (void)hipFree(p);
  c->owned.clear();
  if (c->stage) (void)hipFree(c->stage);
  c->stage = nullptr;
  if (c->split_state) (void)hipFree(c->split_state);
  if (c->d_split_args) (void)hipFree(c->d_split_args);
  if (c->d_split_items) (void)hipFree(c->d_split_items);
  c->split_state = nullptr;
  c->d_split_args = nullptr;
  c->d_split_items = nullptr;
  c->split_cap = 0;
  c->split_args_cap = 0;
}

int check_shape(int n, int d, int b) {
  if (n < 1 || n > CUM_MAX_COLS || d < 1 || d > CUM_MAX_ORDER || b < 1 || b > n) return CUM_EINVAL;
  return CUM_OK;
}

hipEvent_t pooled_event(cum_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Brackets one launch with HIP events when its class (0 = update,
// 1 = combine, 2 = norms) is being profiled.  With `own` the launch takes
// the events itself (start() / stop()) and they carry the kernel's own
// dispatch timestamps; otherwise they are recorded on the stream around it.
struct Timed {
  cum_ctx* c;
  int cls;
  bool own;
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st;
  Timed(cum_ctx* ctx, int k, bool own_events = false, hipStream_t on = nullptr)
      : c(ctx), cls(k), own(own_events), st(on ? on : ctx->stream) {
    if (!(c->profile_mask & (1 << cls)) || c->no_events) return;
    if (c->profile_seen[cls]++ % c->profile_every != c->profile_every - 1) return;
    a = pooled_event(c);
    b = pooled_event(c);
    if (!a || !b) {
      if (a) c->event_pool.push_back(a);
      if (b) c->event_pool.push_back(b);
      a = b = nullptr;
      return;
    }
    if (!own) (void)hipEventRecord(a, st);
  }
  hipEvent_t start() const { return a; }
  hipEvent_t stop() const { return b; }
  // With `own`: the launch went in and took the events.
  void launched() { taken = true; }
  ~Timed() {
    if (!a) return;
    if (own && !taken) {  // the launch failed: the events were never recorded
      c->event_pool.push_back(a);
      c->event_pool.push_back(b);
      return;
    }
    if (!own) (void)hipEventRecord(b, st);
    c->events.push_back({cls, a, b});
  }
  bool taken = false;
};

// Update tile shape: CUM_TILE=<TM>x<TN> overrides the default 2x2.
void pick_tile(cum_ctx* c) {
  c->tm = 2;
  c->tn = 2;
  const char* s = getenv("CUM_TILE");
  int tm = 0, tn = 0;
  if (s && sscanf(s, "%dx%d", &tm, &tn) == 2 && update_tile_supported(tm, tn)) {
    c->tm = tm;
    c->tn = tn;
  }
}

UpdArgs base_args(cum_ctx* c) {
  UpdArgs a{};
  a.n = c->n;
  a.shl = (16 % c->b == 0) ? 1 : 0;
  a.items = c->items;
  a.zero = c->zero;
  for (int k = 1; k <= c->d; ++k) {
    a.left[k] = c->left[k];
    a.right[k] = c->right[k];
    a.s_hi[k] = c->s_hi[k];
    a.s_lo[k] = c->s_lo[k];
  }
  return a;
}

// FIFO arguments of one update: mode (0 off, 1 store, 2 replace) and slot.
void set_fifo(const cum_ctx* c, UpdArgs& a, int mode, int slot) {
  a.fifo = mode;
  for (int k = 1; k <= c->d; ++k)
    a.snap[k] = mode ? (char*)c->snap[k] + (size_t)slot * (size_t)c->T.ord[k].nelems * c->st_size : nullptr;
}

int flush_norms(cum_ctx* c);

int64_t state_elems(const cum_ctx* c) {
  int64_t tot = 0;
  for (int k = 1; k <= c->d; ++k) tot += c->T.ord[k].nelems;
  return tot;
}

// Room for `nsplit` chunks' state copies and `nargs` argument blocks of a
// split contraction (grown on demand).
int ensure_split(cum_ctx* c, int nsplit, int nargs) {
  if (nsplit > c->split_cap) {
    if (c->split_state) (void)hipFree(c->split_state);
    if (c->d_split_items) (void)hipFree(c->d_split_items);
    c->split_state = nullptr;
    c->d_split_items = nullptr;
    c->split_cap = 0;
    const size_t sbytes = (size_t)nsplit * 2 * (size_t)state_elems(c) * c->st_size;
    const size_t nq = c->h_qitems.size();
    std::vector<UpdItem> rep((size_t)nsplit * nq);
    for (int s = 0; s < nsplit; ++s)
      for (size_t i = 0; i < nq; ++i) {
        rep[(size_t)s * nq + i] = c->h_qitems[i];
        rep[(size_t)s * nq + i].ctx = s;
      }
    if (hipMalloc(&c->split_state, sbytes) != hipSuccess ||
        hipMalloc((void**)&c->d_split_items, rep.size() * sizeof(UpdItem)) != hipSuccess) {
      (void)hipGetLastError();
      return CUM_ENOMEM;
    }
    CUM_TRY(hipMemcpy(c->d_split_items, rep.data(), rep.size() * sizeof(UpdItem), hipMemcpyHostToDevice));
    // zero once: every fold leaves the copies it read zeroed again
    CUM_TRY(hipMemset(c->split_state, 0, sbytes));
    c->split_cap = nsplit;
  }
  if (nargs > c->split_args_cap) {
    if (c->d_split_args) (void)hipFree(c->d_split_args);
    c->d_split_args = nullptr;
    c->split_args_cap = 0;
    if (hipMalloc((void**)&c->d_split_args, (size_t)nargs * sizeof(UpdArgs)) != hipSuccess) {
      (void)hipGetLastError();
      return CUM_ENOMEM;
    }
    c->split_args_cap = nargs;
    c->h_split_prev.clear();
  }
  return CUM_OK;
}

// Chunks of a plus-rows-only contraction in one launch when the context has
// too few tiles to fill the device chunk by chunk (see FoldArgs).  Chunks
// are at most kRowChunk rows, fewer (multiples of 256) when the tiles are
// so few that kRowChunk-row chunks would still leave the device idle.
constexpr int64_t kSplitWorkgroups = 512;                 // target workgroups per launch
constexpr int64_t kSplitMaxBytes = (int64_t)256 << 20;    // cap of the chunks' state copies

bool split_eligible(const cum_ctx* c, const char* xp, int64_t np, const char* xm, int64_t nm, int fifo) {
  (void)xm;
  return fifo == 0 && nm == 0 && np > 256 && c->quad && !c->no_events && (c->n * c->x_size) % 16 == 0 &&
         (uintptr_t)xp % 16 == 0 && (int64_t)c->h_qitems.size() / 4 * 2 < kSplitWorkgroups;
}

int64_t split_chunk_rows(const cum_ctx* c, int64_t np) {
  const int64_t nq = (int64_t)c->h_qitems.size() / 4;
  const int64_t want = (np * nq + kSplitWorkgroups - 1) / kSplitWorkgroups;
  return std::max<int64_t>(256, std::min<int64_t>(kRowChunk, (want + 255) / 256 * 256));
}

// fresh: the running sums are zero before this contraction (they are
// written, not read)
int run_contraction_split(cum_ctx* c, const char* xp, int64_t np, bool fresh) {
  const int64_t nq = (int64_t)c->h_qitems.size() / 4;
  const int64_t rows = split_chunk_rows(c, np);
  const int64_t nchunks = (np + rows - 1) / rows;
  const int64_t per = std::max<int64_t>(1, std::min<int64_t>(nchunks, (kSplitWorkgroups + nq - 1) / nq));
  const int64_t tot = state_elems(c);
  const int group = (int)std::min<int64_t>(per, std::max<int64_t>(1, kSplitMaxBytes / (2 * tot * (int64_t)c->st_size)));
  if (int rc = ensure_split(c, group, (int)nchunks)) return rc;
  if (c->norms_pending)
    if (int rc = flush_norms(c)) return rc;
  const size_t rb = (size_t)c->n * c->x_size;
  const int str = update_lds_stride(c->n);
  FoldArgs fa{};
  fa.d = c->d;
  fa.tot = tot;
  int64_t o = 0;
  for (int k = 1; k <= c->d; ++k) {
    fa.off[k] = o;
    o += c->T.ord[k].nelems;
    fa.s_hi[k] = c->s_hi[k];
    fa.s_lo[k] = c->s_lo[k];
  }
  fa.off[c->d + 1] = tot;
  fa.split = c->split_state;
  // every chunk's argument block (chunk i of a group uses state copy i mod group)
  c->h_split_args.resize((size_t)nchunks);
  for (int64_t ci = 0; ci < nchunks; ++ci) {
    const int64_t q0 = ci * rows;
    UpdArgs a = base_args(c);
    set_fifo(c, a, 0, 0);
    a.xp = xp + (size_t)q0 * rb;
    a.np = (int)std::min<int64_t>(rows, np - q0);
    a.xm = nullptr;
    a.nm = 0;
    a.vec = 1;
    a.quad = 1;
    a.items = nullptr;
    a.with_norms = 0;
    char* base = (char*)c->split_state + (size_t)(ci % group) * 2 * (size_t)tot * c->st_size;
    for (int k = 1; k <= c->d; ++k) {
      a.s_hi[k] = base + (size_t)fa.off[k] * c->st_size;
      a.s_lo[k] = base + (size_t)(tot + fa.off[k]) * c->st_size;
    }
    c->h_split_args[(size_t)ci] = a;
  }
  // uploaded only when they changed: a repeated recalculation of the same
  // buffer (as inside a captured graph) reuses the blocks on the device
  if (c->h_split_prev.size() != c->h_split_args.size() ||
      memcmp(c->h_split_prev.data(), c->h_split_args.data(), c->h_split_args.size() * sizeof(UpdArgs)) != 0) {
    CUM_TRY(hipMemcpyAsync(c->d_split_args, c->h_split_args.data(), c->h_split_args.size() * sizeof(UpdArgs),
                           hipMemcpyHostToDevice, c->stream));
    CUM_TRY(hipStreamSynchronize(c->stream));  // the host blocks may change on the next call
    c->h_split_prev = c->h_split_args;
  }
  for (int64_t g0 = 0; g0 < nchunks; g0 += group) {
    const int ns = (int)std::min<int64_t>(group, nchunks - g0);
    {
      Timed tm(c, 0);
      CUM_TRY(launch_update_quad_batch(c->prec, str, c->d, c->d_split_args + g0, c->d_split_items,
                                       (int)((int64_t)ns * nq * 4), (int)((int64_t)ns * nq), c->stream));
    }
    fa.nsplit = ns;
    fa.fresh = (fresh && g0 == 0) ? 1 : 0;
    CUM_TRY(launch_fold_splits(c->prec, fa, c->stream));
  }
  return CUM_OK;
}

// allow_split: a context with few tiles may contract a long plus-only run
// of rows chunk-parallel; fresh: the running sums are zero beforehand
int run_contraction(cum_ctx* c, const char* xp, int64_t np, const char* xm, int64_t nm, int fifo = 0,
                    int slot = 0, bool allow_split = false, bool fresh = false) {
  if (allow_split && split_eligible(c, xp, np, xm, nm, fifo)) return run_contraction_split(c, xp, np, fresh);
  UpdArgs a = base_args(c);
  set_fifo(c, a, fifo, slot);
  const int64_t rows = np > nm ? np : nm;
  const size_t rb = (size_t)c->n * c->x_size;
  for (int64_t q0 = 0; q0 < rows; q0 += kRowChunk) {
    const int64_t cp = np > q0 ? (np - q0 < kRowChunk ? np - q0 : kRowChunk) : 0;
    const int64_t cm = nm > q0 ? (nm - q0 < kRowChunk ? nm - q0 : kRowChunk) : 0;
    a.xp = cp ? xp + (size_t)q0 * rb : nullptr;
    a.xm = cm ? xm + (size_t)q0 * rb : nullptr;
    a.np = (int)cp;
    a.nm = (int)cm;
    a.vec = ((c->n * c->x_size) % 16 == 0) && ((uintptr_t)a.xp % 16 == 0) && ((uintptr_t)a.xm % 16 == 0);
    a.quad = c->quad && a.vec;
    a.items = a.quad ? c->qitems : c->items;
    a.with_norms = 0;
    if (c->norms_pending && c->nitems > 0) {
      a.with_norms = 1;
      a.na = c->pending_na;
      c->norms_pending = false;
    }
    Timed tm(c, 0, true);
    CUM_TRY(launch_update(c->prec, c->tm, c->tn, c->d, a, c->nitems, c->stream, tm.start(), tm.stop()));
    tm.launched();
  }
  return CUM_OK;
}

LatArgs lat_args(const cum_ctx* c) {
  LatArgs la{};
  la.b = c->b;
  la.log2b = ((c->b & (c->b - 1)) == 0) ? __builtin_ctz((unsigned)c->b) : -1;
  la.subrank = c->subrank[c->d];
  la.desig = c->desig;
  la.inv_t = 1.0 / (double)c->t;
  for (int k = 1; k <= c->d; ++k) {
    la.s_hi[k] = c->s_hi[k];
    la.s_lo[k] = c->s_lo[k];
    la.C[k] = c->C[k];
    la.mult[k] = c->mult[k];
    la.partial[k] = c->partial[k];
  }
  for (int m = 0; m <= (1 << c->d); ++m) la.off[m] = c->lat_off[m];
  la.rec = c->combine == CUM_COMBINE_RECURSION;
  return la;
}

int run_combine_and_norms(cum_ctx* c, hipStream_t st = nullptr) {
  if (!st) st = c->stream;
  if (c->lat_lds > 0) {
    const LatArgs la = lat_args(c);
    Timed tm(c, 1, false, st);
    CUM_TRY(launch_combine_lattice(c->prec, c->d, c->combine == CUM_COMBINE_RECURSION, la,
                                   c->T.ord[c->d].nblocks, c->lat_lds, st));
  }
  for (int s = 1; s <= c->d && c->lat_lds == 0; ++s) {
    CombArgs a{};
    a.b = c->b;
    a.nbar = c->T.nbar;
    a.log2b = ((c->b & (c->b - 1)) == 0) ? __builtin_ctz((unsigned)c->b) : -1;
    a.bs = c->T.ord[s].bk;
    a.subrank = c->subrank[s];
    a.s_hi = c->s_hi[s];
    a.s_lo = c->s_lo[s];
    a.inv_t = 1.0 / (double)c->t;
    for (int q = 1; q < s; ++q) {
      a.C[q] = c->C[q];
      a.Shi[q] = c->s_hi[q];
      a.Slo[q] = c->s_lo[q];
    }
    a.Cout = c->C[s];
    a.mult = c->mult[s];
    a.partial = c->partial[s];
    a.rec = c->combine == CUM_COMBINE_RECURSION;
    Timed tm(c, 1, false, st);
    if (combine_split_supported(s, c->b))
      CUM_TRY(launch_combine_split(c->prec, s, a, c->T.ord[s].nblocks, st));
    else
      CUM_TRY(launch_combine(c->prec, s, a, c->T.ord[s].nblocks, st));
  }
  NormArgs na{};
  na.d = c->d;
  na.kfirst = 1;
  for (int k = 1; k <= c->d; ++k) {
    na.nblocks[k] = c->T.ord[k].nblocks;
    na.partial[k] = c->partial[k];
  }
  na.out = c->norms;
  // formed by the next update launch (on an idle CU) or by flush_norms
  c->pending_na = na;
  c->norms_pending = true;
  return CUM_OK;
}

// Launches the pending norms on their own (before anything reads them).
int flush_norms(cum_ctx* c) {
  if (!c->norms_pending) return CUM_OK;
  c->norms_pending = false;
  Timed tm(c, 2);
  CUM_TRY(launch_norms(c->pending_na, c->stream));
  return CUM_OK;
}

// Work of a batch that contains this context must finish before its state
// is read on the host.
hipError_t wait_batch(cum_ctx* c) {
  if (!c->batch_done) return hipSuccess;
  return hipEventSynchronize(c->batch_done);
}

int ensure_stage(cum_ctx* c, size_t bytes) {
  if (bytes <= c->stage_bytes) return CUM_OK;
  CUM_TRY(hipStreamSynchronize(c->stream));
  if (c->stage) (void)hipFree(c->stage);
  c->stage = nullptr;
  c->stage_bytes = 0;
  const size_t cap = mem_cap();
  if (cap && bytes > cap) return CUM_ENOMEM;
  CUM_TRY(hipMalloc(&c->stage, bytes));
  c->stage_bytes = bytes;
  return CUM_OK;
}

}  // namespace

extern "C" {

const char* cum_last_error(void) { return g_last_error; }

const char* cum_strerror(int status) {
  switch (status) {
    case CUM_OK: return "ok";
    case CUM_EINVAL: return "invalid argument";
    case CUM_ENOMEM: return "out of memory";
    case CUM_EDEVICE: return "HIP device error";
    case CUM_ESTATE: return "context not initialised";
    case CUM_ENONFINITE: return "non-finite input";
    case CUM_ESIZE: return "size beyond capacity or limits";
    default: return "unknown status";
  }
}

int64_t cum_num_blocks(int n, int b, int k) {
  if (n < 1 || b < 1 || k < 0 || k > CUM_MAX_ORDER) return -1;
  const int64_t nbar = (n + b - 1) / b;
  return binom(nbar + k - 1, k);
}

int64_t cum_num_elems(int n, int b, int k) {
  const int64_t nb = cum_num_blocks(n, b, k);
  if (nb < 0) return -1;
  return nb * ipow64(b, k);
}

int64_t cum_plan_coverage(int n, int b, int k, int32_t* hits) {
  if (n < 1 || b < 1 || k < 1 || k > CUM_MAX_ORDER) return CUM_EINVAL;
  Tables T;
  if (build_tables(n, b, k, T) != 0) return CUM_EINVAL;
  std::vector<int32_t> h;
  const int64_t bad = coverage(T, k, h);
  if (hits) memcpy(hits, h.data(), h.size() * sizeof(int32_t));
  return bad;
}

int64_t cum_plan_items(int n, int d, int b) {
  if (check_shape(n, d, b) != CUM_OK) return CUM_EINVAL;
  Tables T;
  if (build_tables(n, b, d, T) != 0) return CUM_EINVAL;
  return (int64_t)build_items(T, 1, d, 32, 32).size();
}

int64_t cum_plan_groups(int n, int d, int b, int32_t* frags, int32_t* tiles) {
  if (check_shape(n, d, b) != CUM_OK) return CUM_EINVAL;
  Tables T;
  if (build_tables(n, b, d, T) != 0) return CUM_EINVAL;
  const std::vector<UpdItem> q = pack_quads(build_items(T, 1, d, 32, 32));
  const size_t ng = q.size() / 4;
  for (size_t g = 0; g < ng; ++g) {
    int32_t f = 0, t = 0;
    for (size_t j = 0; j < 4; ++j) {
      const UpdItem& it = q[g * 4 + j];
      if (it.M == 0) continue;
      f += (it.M - it.r0 > 16 ? 2 : 1) * (it.N - it.c0 > 16 ? 2 : 1);
      ++t;
    }
    if (frags) frags[g] = f;
    if (tiles) tiles[g] = t;
  }
  return (int64_t)ng;
}

namespace {

// Shared by cum_init and cum_init_fifo (fifo_p = 0: plain sliding mode).
int init_ctx(cum_ctx** out, int n, int d, int b, const void* X, int64_t t, int64_t fifo_p, int prec,
             void* hip_stream) {
  if (!out) return CUM_EINVAL;
  *out = nullptr;
  int rc = check_shape(n, d, b);
  if (rc != CUM_OK) return rc;
  if (prec != CUM_FP64 && prec != CUM_FP32 && prec != CUM_BF16X3) return CUM_EINVAL;
  if (!X || t < 1 || t > ((int64_t)1 << 40)) return CUM_EINVAL;
  if (fifo_p < 0 || (fifo_p > 0 && (t % fifo_p != 0))) return CUM_EINVAL;
  if (fifo_p > kRowChunk || t / (fifo_p ? fifo_p : 1) > (1 << 30)) return CUM_ESIZE;

  cum_ctx* c = new (std::nothrow) cum_ctx();
  if (!c) return CUM_ENOMEM;
  c->n = n; c->d = d; c->b = b; c->prec = prec; c->t = t;
  c->fifo_p = fifo_p;
  c->fifo_q = fifo_p ? (int)(t / fifo_p) : 0;
  c->stream = (hipStream_t)hip_stream;
  c->x_size = (prec == CUM_FP64) ? 8 : 4;
  {
    // CUM_PIPELINE=1: pipelined sliding updates.  Off by default: where the
    // update fills every CU (n = 60: one 1024-thread workgroup with 139 KB
    // of LDS per CU) the side stream's combine and norms only compete with
    // it, and a step took 67 us instead of 55 us.
    const char* pe = getenv("CUM_PIPELINE");
    c->pipe_off = !(pe && pe[0] == '1');
  }
  c->st_size = (prec == CUM_FP64) ? 8 : 4;
  if (hipGetDevice(&c->device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return CUM_EDEVICE;
  }
  if (build_tables(n, b, d, c->T) != 0) { delete c; return CUM_EINVAL; }
  c->stride = update_lds_stride(n);
  c->chunk = c->stride ? update_chunk_rows(prec, c->stride) : 0;
  if (c->chunk <= 0) { delete c; return CUM_ESIZE; }
  pick_tile(c);

  const std::vector<UpdItem> items = build_items(c->T, 1, d, 16 * c->tm, 16 * c->tn);
  c->nitems = (int)items.size();

  size_t used = 0;
  auto fail = [&](hipError_t e) {
    note_error(e, "cum_init allocation/upload", __LINE__);
    const int r = map_err(e);
    (void)hipGetLastError();
    release(c);
    delete c;
    return r;
  };
  hipError_t e;
  for (int k = 1; k <= d; ++k) {
    const OrderInfo& o = c->T.ord[k];
    if ((e = dalloc(c, &c->s_hi[k], (size_t)o.nelems * c->st_size, &used)) != hipSuccess) return fail(e);
    if ((e = dalloc(c, &c->s_lo[k], (size_t)o.nelems * c->st_size, &used)) != hipSuccess) return fail(e);
    if ((e = dalloc(c, (void**)&c->C[k], (size_t)o.nelems * 8, &used)) != hipSuccess) return fail(e);
    if ((e = dalloc(c, (void**)&c->partial[k], (size_t)o.nblocks * 8, &used)) != hipSuccess) return fail(e);
    if ((e = upload(c, &c->subrank[k], c->T.subrank[k], &used)) != hipSuccess) return fail(e);
    if ((e = upload(c, &c->mult[k], c->T.mult[k], &used)) != hipSuccess) return fail(e);
    if ((e = upload(c, &c->left[k], c->T.left[k], &used)) != hipSuccess) return fail(e);
    if ((e = upload(c, &c->right[k], c->T.right[k], &used)) != hipSuccess) return fail(e);
    if ((e = hipMemsetAsync(c->s_hi[k], 0, (size_t)o.nelems * c->st_size, c->stream)) != hipSuccess) return fail(e);
    if ((e = hipMemsetAsync(c->s_lo[k], 0, (size_t)o.nelems * c->st_size, c->stream)) != hipSuccess) return fail(e);
    if (c->fifo_q &&
        (e = dalloc(c, &c->snap[k], (size_t)c->fifo_q * (size_t)o.nelems * c->st_size, &used)) != hipSuccess)
      return fail(e);
  }
  if ((e = upload(c, &c->items, items, &used)) != hipSuccess) return fail(e);
  c->quad = update_quad_supported(prec, n) && !items.empty();
  if (c->quad) {
    c->h_qitems = pack_quads(items);
    if ((e = upload(c, &c->qitems, c->h_qitems, &used)) != hipSuccess) return fail(e);
  }
  if ((e = dalloc(c, (void**)&c->norms, (size_t)2 * (d + 1) * 8, &used)) != hipSuccess) return fail(e);
  if ((e = dalloc(c, &c->zero, UPD_ZERO_BYTES, &used)) != hipSuccess) return fail(e);
  if (lattice_lds_bytes(d, b) <= LAT_LDS_BYTES) {
    // order-d block j writes its prefix-s block when j_s = ... = j_d
    const OrderInfo& od = c->T.ord[d];
    std::vector<uint8_t> des((size_t)od.nblocks, 0);
    for (int64_t r = 0; r < od.nblocks; ++r) {
      const uint8_t* tu = &c->T.tuples[d][(size_t)r * d];
      for (int q = 1; q < d; ++q) {
        bool tail = true;
        for (int u = q; u < d; ++u) tail = tail && tu[u] == tu[q - 1];
        if (tail) des[(size_t)r] |= (uint8_t)(1 << q);
      }
    }
    if ((e = upload(c, &c->desig, des, &used)) != hipSuccess) return fail(e);
    int off = 0;
    for (int m = 1; m < (1 << d) - 1; ++m) {
      c->lat_off[m] = off;
      int bl = 1;
      for (int q = 0; q < __builtin_popcount(m); ++q) bl *= b;
      off += bl;
    }
    c->lat_off[(1 << d) - 1] = off;
    c->lat_off[1 << d] = off;
    c->lat_lds = lattice_lds_bytes(d, b);
    if (c->lat_lds == 0) c->lat_lds = 16;  // d = 1: no sub-blocks
  }
  if ((e = hipMemsetAsync(c->zero, 0, UPD_ZERO_BYTES, c->stream)) != hipSuccess) return fail(e);

  // the window, on the device
  const char* xw = (const char*)X;
  void* tmp = nullptr;
  const size_t wbytes = (size_t)t * n * c->x_size;
  if (!is_device_ptr(X)) {
    if ((e = dalloc(c, &tmp, wbytes, &used)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(tmp, X, wbytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return fail(e);
    xw = (const char*)tmp;
  }
  if (c->fifo_q) {
    // the window as t / p batches, oldest first: slot q holds batch q
    const size_t bb = (size_t)fifo_p * n * c->x_size;
    for (int q = 0; q < c->fifo_q && rc == CUM_OK; ++q)
      rc = run_contraction(c, xw + (size_t)q * bb, fifo_p, nullptr, 0, 1, q);
  } else {
    rc = run_contraction(c, xw, t, nullptr, 0, 0, 0, true, true);  // the sums were just zeroed
  }
  if (rc == CUM_OK) rc = run_combine_and_norms(c);
  if (rc == CUM_OK && (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
    CUM_NOTE(e, "hipStreamSynchronize after init");
    rc = map_err(e);
  }
  if (tmp) {
    (void)hipFree(tmp);
    for (size_t i = 0; i < c->owned.size(); ++i)
      if (c->owned[i] == tmp) { c->owned.erase(c->owned.begin() + (long)i); break; }
  }
  if (rc != CUM_OK) {
    (void)hipGetLastError();
    release(c);
    delete c;
    return rc;
  }
  c->ready = true;
  *out = c;
  return CUM_OK;
}

}  // namespace

int cum_init(cum_ctx** out, int n, int d, int b, const void* X, int64_t t, int prec, void* hip_stream) {
  return init_ctx(out, n, d, b, X, t, 0, prec, hip_stream);
}

int cum_init_fifo(cum_ctx** out, int n, int d, int b, const void* X, int64_t t, int64_t p, int prec,
                  void* hip_stream) {
  if (p < 1) return CUM_EINVAL;
  return init_ctx(out, n, d, b, X, t, p, prec, hip_stream);
}

}  // extern "C"

namespace {

// Shared by cum_update and cum_update_noalloc.  `stage`: where host inputs
// are copied (nullptr: the context's own buffer, grown on demand).
// Orders the pipelined work queued on pstream before whatever comes next on
// the context's stream (every entry point that reads or rewrites the state,
// the cumulants or the norms calls it first).
int join_pipe(cum_ctx* c) {
  if (!c->pipe_active) return CUM_OK;
  CUM_TRY(hipEventRecord(c->ev_join, c->pstream));
  CUM_TRY(hipStreamWaitEvent(c->stream, c->ev_join, 0));
  c->pipe_active = false;
  return CUM_OK;
}

// The increments and the side stream of pipelined updates (allocated on the
// first pipelined update).
int ensure_pipe(cum_ctx* c) {
  if (c->pstream) return CUM_OK;
  const size_t bytes = (size_t)state_elems(c) * c->st_size;
  size_t used = 0;
  // zeroed once: the update never writes the elements with a padded index
  // (b not dividing n), so they must fold in as zero
  for (int q = 0; q < 2; ++q)
    if (dalloc(c, &c->delta[q], bytes, &used) != hipSuccess || hipMemset(c->delta[q], 0, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return CUM_ENOMEM;
    }
  for (int q = 0; q < 2; ++q)
    if (hipEventCreateWithFlags(&c->ev_upd[q], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fold[q], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return CUM_EDEVICE;
    }
  if (hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&c->pstream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    c->pstream = nullptr;
    return CUM_EDEVICE;
  }
  return CUM_OK;
}

// A sliding update whose increment, fold, combine and norms overlap the next
// update: one four-tile launch on the context's stream stores the increment
// of every stored element in delta[slot]; on pstream the increment is folded
// into the running sums (the same compensated fold, in the same order, as
// the update's own), then the combine and the norms.  The next update writes
// the other slot; the one after waits for this slot's fold.
bool pipe_eligible(const cum_ctx* c, const char* xn, const char* xo, int64_t p) {
  if (c->pipe_off || c->fifo_q > 0 || c->no_events || c->batch_done || !c->quad || p < 1 || p > kRowChunk)
    return false;
  if ((c->n * c->x_size) % 16 != 0 || (uintptr_t)xn % 16 != 0 || (uintptr_t)xo % 16 != 0) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

int update_pipelined(cum_ctx* c, const char* xn, const char* xo, int64_t p) {
  if (int rc = ensure_pipe(c)) return rc;
  const int slot = c->pipe_slot;
  c->pipe_slot ^= 1;
  if (c->fold_pending[slot]) CUM_TRY(hipStreamWaitEvent(c->stream, c->ev_fold[slot], 0));
  if (c->norms_pending)  // a combine queued on the context's stream before this update
    if (int rc = flush_norms(c)) return rc;
  const int64_t tot = state_elems(c);
  FoldArgs fa{};
  fa.d = c->d;
  fa.nsplit = 1;
  fa.single = 1;
  fa.tot = tot;
  UpdArgs a = base_args(c);
  set_fifo(c, a, 3, 0);
  int64_t o = 0;
  for (int k = 1; k <= c->d; ++k) {
    fa.off[k] = o;
    fa.s_hi[k] = c->s_hi[k];
    fa.s_lo[k] = c->s_lo[k];
    a.s_hi[k] = (char*)c->delta[slot] + (size_t)o * c->st_size;
    a.s_lo[k] = nullptr;
    o += c->T.ord[k].nelems;
  }
  fa.off[c->d + 1] = tot;
  fa.split = c->delta[slot];
  a.xp = xn;
  a.xm = xo;
  a.np = (int)p;
  a.nm = (int)p;
  a.vec = 1;
  a.quad = 1;
  a.items = c->qitems;
  a.with_norms = 0;
  {
    Timed tm(c, 0, true);
    CUM_TRY(launch_update(c->prec, c->tm, c->tn, c->d, a, c->nitems, c->stream, tm.start(), tm.stop()));
    tm.launched();
  }
  CUM_TRY(hipEventRecord(c->ev_upd[slot], c->stream));
  CUM_TRY(hipStreamWaitEvent(c->pstream, c->ev_upd[slot], 0));
  CUM_TRY(launch_fold_splits(c->prec, fa, c->pstream));
  CUM_TRY(hipEventRecord(c->ev_fold[slot], c->pstream));
  c->fold_pending[slot] = true;
  c->pipe_active = true;
  if (int rc = run_combine_and_norms(c, c->pstream)) return rc;
  c->norms_pending = false;
  Timed tn(c, 2, false, c->pstream);
  CUM_TRY(launch_norms(c->pending_na, c->pstream));
  return CUM_OK;
}

int update_impl(cum_ctx* c, const void* X_new, const void* X_old, int64_t p, char* stage) {
  const bool fifo = c->fifo_q > 0;
  const char* xn = (const char*)X_new;
  const char* xo = fifo ? nullptr : (const char*)X_old;
  const size_t bytes = (size_t)p * c->n * c->x_size;
  const uintptr_t a0 = (uintptr_t)X_new, a1 = (uintptr_t)X_old;
  const bool cached = c->dev_lo && a0 >= c->dev_lo && a0 + bytes <= c->dev_hi &&
                      (fifo || (a1 >= c->dev_lo && a1 + bytes <= c->dev_hi));
  const bool dn = cached || is_device_ptr(X_new);
  const bool dob = fifo || cached || is_device_ptr(X_old);
  if (!cached) {
    c->dev_lo = c->dev_hi = 0;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (dn && dob) {
      if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)X_new) == hipSuccess && base &&
          (fifo || (a1 >= (uintptr_t)base && a1 + bytes <= (uintptr_t)base + size))) {
        c->dev_lo = (uintptr_t)base;
        c->dev_hi = (uintptr_t)base + size;
      } else {
        (void)hipGetLastError();
      }
    }
  }
  if (!dn || !dob) {
    if (!stage) {
      int rc = ensure_stage(c, 2 * bytes);
      if (rc != CUM_OK) return rc;
      stage = (char*)c->stage;
    }
    if (!dn) {
      CUM_TRY(hipMemcpyAsync(stage, X_new, bytes, hipMemcpyHostToDevice, c->stream));
      xn = stage;
    }
    if (!dob) {
      CUM_TRY(hipMemcpyAsync(stage + bytes, X_old, bytes, hipMemcpyHostToDevice, c->stream));
      xo = stage + bytes;
    }
    // host buffers are free for reuse once this returns
    CUM_TRY(hipStreamSynchronize(c->stream));
  }
  if (c->batch_done) {
    CUM_TRY(hipStreamWaitEvent(c->stream, c->batch_done, 0));
    c->direct_since_batch = true;
  }
  if (pipe_eligible(c, xn, xo, p)) return update_pipelined(c, xn, xo, p);
  if (int rj = join_pipe(c)) return rj;
  int rc;
  if (fifo) {
    rc = run_contraction(c, xn, p, nullptr, 0, 2, c->fifo_head);
    if (rc != CUM_OK) return rc;
    c->fifo_head = (c->fifo_head + 1) % c->fifo_q;
  } else {
    rc = run_contraction(c, xn, p, xo, p);
    if (rc != CUM_OK) return rc;
  }
  return run_combine_and_norms(c);
}

int check_update_args(cum_ctx* c, const void* X_new, const void* X_old, int64_t p) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (p < 0 || p > c->t) return CUM_EINVAL;
  const bool fifo = c->fifo_q > 0;
  if (p > 0 && fifo && p != c->fifo_p) return CUM_EINVAL;
  if (p > 0 && (!X_new || (!fifo && !X_old))) return CUM_EINVAL;
  return CUM_OK;
}

}  // namespace

extern "C" {

int cum_update(cum_ctx* c, const void* X_new, const void* X_old, int64_t p) {
  if (int rc = check_update_args(c, X_new, X_old, p)) return rc;
  if (p == 0) return CUM_OK;
  return update_impl(c, X_new, X_old, p, nullptr);
}

int cum_update_noalloc(cum_ctx* c, const void* X_new, const void* X_old, int64_t p) {
  if (int rc = check_update_args(c, X_new, X_old, p)) return rc;
  if (p == 0) return CUM_OK;
  const int nin = c->fifo_q > 0 ? 1 : 2;
  if ((size_t)nin * (size_t)p * c->n * c->x_size > NOALLOC_STAGE_BYTES) return CUM_ESIZE;
  int dev = -1;
  CUM_TRY(hipGetDevice(&dev));
  if (dev != c->device) return CUM_EINVAL;
  void* stage = nullptr;
  CUM_TRY(noalloc_stage(&stage));
  c->no_events = true;
  int rc = update_impl(c, X_new, X_old, p, (char*)stage);
  c->no_events = false;
  // the staging array is shared by every call on this device: the update
  // has finished reading it when this returns
  if (rc == CUM_OK) CUM_TRY(hipStreamSynchronize(c->stream));
  return rc;
}

int cum_recompute(cum_ctx* c, const void* X) {
  if (!c || !X) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  const size_t wbytes = (size_t)c->t * c->n * c->x_size;
  const char* xw = (const char*)X;
  if (!is_device_ptr(X)) {
    int rc = ensure_stage(c, wbytes);
    if (rc != CUM_OK) return rc;
    CUM_TRY(hipMemcpyAsync(c->stage, X, wbytes, hipMemcpyHostToDevice, c->stream));
    xw = (const char*)c->stage;
  }
  if (c->batch_done) {
    CUM_TRY(hipStreamWaitEvent(c->stream, c->batch_done, 0));
    c->direct_since_batch = true;
  }
  // the chunk-parallel contraction writes the running sums outright
  const bool split = !c->fifo_q && split_eligible(c, xw, c->t, nullptr, 0, 0);
  if (!split) {
    ZeroArgs za{};
    for (int k = 1; k <= c->d; ++k) {
      const int64_t words = c->T.ord[k].nelems * (int64_t)c->st_size / 4;
      za.ptr[za.count] = c->s_hi[k];
      za.words[za.count++] = words;
      za.ptr[za.count] = c->s_lo[k];
      za.words[za.count++] = words;
    }
    CUM_TRY(launch_zero(za, c->stream));
  }
  int rc = CUM_OK;
  if (c->fifo_q) {
    const size_t bb = (size_t)c->fifo_p * c->n * c->x_size;
    for (int q = 0; q < c->fifo_q && rc == CUM_OK; ++q)
      rc = run_contraction(c, xw + (size_t)q * bb, c->fifo_p, nullptr, 0, 1, q);
    c->fifo_head = 0;
  } else {
    rc = run_contraction(c, xw, c->t, nullptr, 0, 0, 0, true, split);
  }
  if (rc != CUM_OK) return rc;
  rc = run_combine_and_norms(c);
  if (rc == CUM_OK && xw != (const char*)X) CUM_TRY(hipStreamSynchronize(c->stream));
  return rc;
}

int cum_get(cum_ctx* c, int k, double* blocks, size_t capacity_elems) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  if (k < 1 || k > c->d || !blocks) return CUM_EINVAL;
  const size_t ne = (size_t)c->T.ord[k].nelems;
  if (capacity_elems < ne) return CUM_ESIZE;
  CUM_TRY(wait_batch(c));
  CUM_TRY(hipStreamSynchronize(c->stream));
  CUM_TRY(hipMemcpy(blocks, c->C[k], ne * 8, hipMemcpyDefault));
  return CUM_OK;
}

int cum_get_moments(cum_ctx* c, int k, double* blocks, size_t capacity_elems) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  if (k < 1 || k > c->d || !blocks) return CUM_EINVAL;
  const size_t ne = (size_t)c->T.ord[k].nelems;
  if (capacity_elems < ne) return CUM_ESIZE;
  CUM_TRY(wait_batch(c));
  CUM_TRY(hipStreamSynchronize(c->stream));
  std::vector<char> hi(ne * c->st_size), lo(ne * c->st_size);
  std::vector<double> m(ne);
  CUM_TRY(hipMemcpy(hi.data(), c->s_hi[k], ne * c->st_size, hipMemcpyDeviceToHost));
  CUM_TRY(hipMemcpy(lo.data(), c->s_lo[k], ne * c->st_size, hipMemcpyDeviceToHost));
  const double inv_t = 1.0 / (double)c->t;
  for (size_t i = 0; i < ne; ++i) {
    double h, l;
    if (c->st_size == 8) { h = ((double*)hi.data())[i]; l = ((double*)lo.data())[i]; }
    else { h = ((float*)hi.data())[i]; l = ((float*)lo.data())[i]; }
    m[i] = (h + l) * inv_t;
  }
  CUM_TRY(hipMemcpy(blocks, m.data(), ne * 8, hipMemcpyDefault));
  return CUM_OK;
}

int cum_norms(cum_ctx* c, double* fro, double* nu) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  if (!fro || !nu) return CUM_EINVAL;
  CUM_TRY(wait_batch(c));
  if (int rc = flush_norms(c)) return rc;
  CUM_TRY(hipStreamSynchronize(c->stream));
  std::vector<double> h((size_t)2 * (c->d + 1));
  CUM_TRY(hipMemcpy(h.data(), c->norms, h.size() * 8, hipMemcpyDeviceToHost));
  for (int k = 0; k <= c->d; ++k) {
    fro[k] = h[(size_t)k];
    nu[k] = h[(size_t)(c->d + 1 + k)];
  }
  return CUM_OK;
}

int cum_norms_device(cum_ctx* c, const double** dev_ptr) {
  if (!c || !dev_ptr) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  if (int rc = flush_norms(c)) return rc;
  *dev_ptr = c->norms;
  return CUM_OK;
}

int cum_sync(cum_ctx* c) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  CUM_TRY(wait_batch(c));
  if (int rc = flush_norms(c)) return rc;
  CUM_TRY(hipStreamSynchronize(c->stream));
  return CUM_OK;
}

int cum_profile_enable(cum_ctx* c, int on) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  CUM_TRY(hipStreamSynchronize(c->stream));
  drop_events(c);
  c->profile_mask = on & 7;
  c->profile_every = 1;
  for (int q = 0; q < 3; ++q) c->profile_seen[q] = 0;
  return CUM_OK;
}

int cum_profile_sample(cum_ctx* c, int every) {
  if (!c || every < 1) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  c->profile_every = every;
  for (int q = 0; q < 3; ++q) c->profile_seen[q] = 0;
  return CUM_OK;
}

int cum_profile_read(cum_ctx* c, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (int rj = join_pipe(c)) return rj;
  CUM_TRY(hipStreamSynchronize(c->stream));
  for (int q = 0; q < 3; ++q) { launches[q] = 0; total_ms[q] = 0.0; }
  for (auto& e : c->events) {
    float ms = 0.f;
    CUM_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    launches[e.cls] += 1;
    total_ms[e.cls] += ms;
  }
  drop_events(c);
  return CUM_OK;
}

int cum_set_combine(cum_ctx* c, int method) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (method != CUM_COMBINE_PARTITIONS && method != CUM_COMBINE_RECURSION) return CUM_EINVAL;
  c->combine = method;
  return CUM_OK;
}

int cum_free(cum_ctx* c) {
  if (!c) return CUM_OK;
  if (c->ready) (void)wait_batch(c);
  if (c->ready) (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
  return CUM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched streams: one graph per batch replays the update of every member
// context (persistent launches grouped by LDS stride, batched combine per
// order, batched norms).  Only the input pointers and row counts change
// between updates; they are copied into the device argument table first.

struct cum_batch {
  std::vector<cum_ctx*> ctx;
  int prec = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<UpdArgs> h_upd;
  UpdArgs* d_upd = nullptr;
  // pinned copies of the argument table, used in turn, each with the event
  // that marks its copy done (the host waits only when it is kRing steps ahead)
  static constexpr int kRing = 4;
  UpdArgs* ring[kRing] = {};
  hipEvent_t ring_done[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_next = 0;
  // per member, the device allocation its last inputs were found in (the
  // pointer check is skipped while later inputs stay inside it)
  std::vector<uintptr_t> alloc_lo, alloc_hi;
  // quad: four-tile workgroups (items in groups of four tiles of one member)
  struct Group { int str; bool vl; int kmax; UpdItem* items; int nitems; int grid; bool quad; };
  std::vector<Group> groups;
  CombArgs* d_comb[CUM_MAXD + 1] = {};
  int64_t* comb_items[CUM_MAXD + 1] = {};
  int ncomb[CUM_MAXD + 1] = {};
  int comb_grid[CUM_MAXD + 1] = {};
  size_t stage_bytes[CUM_MAXD + 1] = {};
  NormArgs* d_norm = nullptr;
  // fused combine of the members whose lattices fit, one launch per order d
  LatArgs* d_lat = nullptr;
  // fused-combine launches, one per (order d, lattice size): a launch's
  // workgroups all reserve its largest lattice, so members of small b do not
  // share the LDS reservation (and occupancy) of a b = 8 member
  struct LatGroup { int d; int64_t* items; int n; int grid; size_t lds; int b; };
  std::vector<LatGroup> lat_groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  std::vector<void*> owned;
};

namespace {

void batch_release(cum_batch* bt) {
  for (int r = 0; r < cum_batch::kRing; ++r) {
    if (bt->ring_done[r]) (void)hipEventDestroy(bt->ring_done[r]);
    if (bt->ring[r]) (void)hipHostFree(bt->ring[r]);
    bt->ring_done[r] = nullptr;
    bt->ring[r] = nullptr;
  }
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  for (cum_ctx* c : bt->ctx)
    if (c && c->batch_done == bt->done) c->batch_done = nullptr;
  if (bt->done) (void)hipEventDestroy(bt->done);
  for (void* p : bt->owned) (void)hipFree(p);
  bt->owned.clear();
  if (bt->own_stream && bt->stream) (void)hipStreamDestroy(bt->stream);
}

template <typename V>
hipError_t bupload(cum_batch* bt, V** dst, const V* src, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count ? count * sizeof(V) : 16);
  if (e != hipSuccess) return e;
  bt->owned.push_back(p);
  *dst = (V*)p;
  if (count) e = hipMemcpy(p, src, count * sizeof(V), hipMemcpyHostToDevice);
  return e;
}

int batch_launch_all(cum_batch* bt) {
  for (const auto& g : bt->groups)
    if (g.quad)
      CUM_TRY(launch_update_quad_batch(bt->prec, g.str, g.kmax, bt->d_upd, g.items, g.nitems, g.grid, bt->stream));
    else
      CUM_TRY(launch_update_batch(bt->prec, g.str, g.vl, g.kmax, bt->d_upd, g.items, g.nitems, g.grid, bt->stream));
  for (const auto& g : bt->lat_groups)
    CUM_TRY(launch_combine_lattice_batch(bt->prec, g.d, g.b, bt->d_lat, g.items, g.n, g.grid, g.lds, bt->stream));
  for (int s = 1; s <= CUM_MAXD; ++s)
    CUM_TRY(launch_combine_batch(bt->prec, s, bt->d_comb[s], bt->comb_items[s], bt->ncomb[s], bt->comb_grid[s],
                                 bt->stage_bytes[s], false, bt->stream));
  CUM_TRY(launch_norms_batch(bt->d_norm, (int)bt->ctx.size(), bt->stream));
  return CUM_OK;
}

}  // namespace

extern "C" {

int cum_batch_create(cum_batch** out, cum_ctx* const* ctxs, int m) {
  if (!out || !ctxs || m < 1 || m > (1 << 20)) return CUM_EINVAL;
  *out = nullptr;
  for (int i = 0; i < m; ++i) {
    if (!ctxs[i]) return CUM_EINVAL;
    if (!ctxs[i]->ready) return CUM_ESTATE;
    if (ctxs[i]->prec != ctxs[0]->prec) return CUM_EINVAL;
    if (ctxs[i]->batch_done) return CUM_EINVAL;  // already in a batch
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return CUM_EINVAL;
  }
  cum_batch* bt = new (std::nothrow) cum_batch();
  if (!bt) return CUM_ENOMEM;
  bt->ctx.assign(ctxs, ctxs + m);
  bt->prec = ctxs[0]->prec;
  auto fail = [&](int rc) {
    (void)hipGetLastError();
    batch_release(bt);
    delete bt;
    return rc;
  };
  for (int i = 0; i < m; ++i)
    if (join_pipe(ctxs[i]) != CUM_OK || hipStreamSynchronize(ctxs[i]->stream) != hipSuccess) return fail(CUM_EDEVICE);
  if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess) return fail(CUM_EDEVICE);
  bt->own_stream = true;
  if (hipEventCreateWithFlags(&bt->done, hipEventDisableTiming) != hipSuccess) return fail(CUM_EDEVICE);

  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  const int pgrid = ncu * 4;

  // per-context update arguments (inputs filled per update)
  bt->h_upd.resize((size_t)m);
  for (int i = 0; i < m; ++i) bt->h_upd[(size_t)i] = base_args(ctxs[i]);
  if (bupload(bt, &bt->d_upd, bt->h_upd.data(), bt->h_upd.size()) != hipSuccess) return fail(CUM_ENOMEM);
  for (int r = 0; r < cum_batch::kRing; ++r)
    if (hipHostMalloc((void**)&bt->ring[r], (size_t)m * sizeof(UpdArgs), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ring_done[r], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CUM_ENOMEM);
    }
  bt->alloc_lo.assign((size_t)m, 0);
  bt->alloc_hi.assign((size_t)m, 0);

  // update items grouped by (LDS stride, vector loader), longest windows first
  std::vector<int> order((size_t)m);
  for (int i = 0; i < m; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return ctxs[a]->t > ctxs[b2]->t; });
  struct Key { int str; bool vl; };
  std::vector<Key> keys;
  for (int i : order) {
    cum_ctx* c = ctxs[i];
    const Key k{c->stride, (c->n * (int)c->x_size) % 16 == 0};
    bool seen = false;
    for (const auto& q : keys) seen = seen || (q.str == k.str && q.vl == k.vl);
    if (!seen) keys.push_back(k);
  }
  for (const auto& k : keys) {
    std::vector<UpdItem> items;
    int kmax = 1;
    const bool quad = k.vl && update_quad_batch_supported(bt->prec, k.str);
    for (int i : order) {
      cum_ctx* c = ctxs[i];
      if (c->stride != k.str || ((c->n * (int)c->x_size) % 16 == 0) != k.vl) continue;
      if (c->tm != 2 || c->tn != 2) return fail(CUM_EINVAL);
      kmax = std::max(kmax, c->d);
      std::vector<UpdItem> ci = build_items(c->T, 1, c->d, 32, 32);
      if (quad) ci = pack_quads(ci);  // padding tiles keep the member's index
      for (auto& it : ci) {
        it.ctx = i;
        items.push_back(it);
      }
    }
    cum_batch::Group g{k.str, k.vl, kmax, nullptr, (int)items.size(), 0, quad};
    g.grid = quad ? std::min(g.nitems / 4, ncu) : std::min(g.nitems, pgrid);
    if (bupload(bt, &g.items, items.data(), items.size()) != hipSuccess) return fail(CUM_ENOMEM);
    bt->groups.push_back(g);
  }

  // fused combine: members whose lattices fit, items grouped by order d
  {
    std::vector<LatArgs> la((size_t)m);
    for (int i = 0; i < m; ++i)
      if (ctxs[i]->lat_lds > 0) la[(size_t)i] = lat_args(ctxs[i]);
    if (bupload(bt, &bt->d_lat, la.data(), la.size()) != hipSuccess) return fail(CUM_ENOMEM);
    for (int dd = 1; dd <= CUM_MAXD; ++dd) {
      std::vector<size_t> sizes;
      for (int i : order)
        if (ctxs[i]->lat_lds > 0 && ctxs[i]->d == dd &&
            std::find(sizes.begin(), sizes.end(), ctxs[i]->lat_lds) == sizes.end())
          sizes.push_back(ctxs[i]->lat_lds);
      for (size_t lds : sizes) {
        std::vector<int64_t> items;
        for (int i : order) {
          cum_ctx* c = ctxs[i];
          if (c->lat_lds != lds || c->d != dd) continue;
          for (int64_t blk = 0; blk < c->T.ord[dd].nblocks; ++blk) items.push_back(((int64_t)i << 40) | blk);
        }
        int gb = 0;  // every member of the group has this b (the lattice size fixes it)
        for (int i : order)
          if (ctxs[i]->lat_lds == lds && ctxs[i]->d == dd) gb = ctxs[i]->b;
        cum_batch::LatGroup g{dd, nullptr, (int)items.size(), 0, lds, gb};
        g.grid = g.n;  // one block per workgroup: the hardware keeps every CU full
        if (bupload(bt, &g.items, items.data(), items.size()) != hipSuccess) return fail(CUM_ENOMEM);
        bt->lat_groups.push_back(g);
      }
    }
  }
  // per-order combine of the other members (Alg. 4's partition sum): one
  // entry per context (unused when d < s or the member uses the fused
  // combine)
  for (int s = 1; s <= CUM_MAXD; ++s) {
    std::vector<CombArgs> args((size_t)m);
    std::vector<int64_t> items;
    size_t stage = 0;
    for (int i : order) {
      cum_ctx* c = ctxs[i];
      if (c->d < s || c->lat_lds > 0) continue;
      CombArgs& a = args[(size_t)i];
      a.b = c->b;
      a.nbar = c->T.nbar;
      a.log2b = ((c->b & (c->b - 1)) == 0) ? __builtin_ctz((unsigned)c->b) : -1;
      a.bs = c->T.ord[s].bk;
      a.subrank = c->subrank[s];
      a.s_hi = c->s_hi[s];
      a.s_lo = c->s_lo[s];
      a.inv_t = 1.0 / (double)c->t;
      for (int q = 1; q < s; ++q) a.C[q] = c->C[q];
      a.Cout = c->C[s];
      a.mult = c->mult[s];
      a.partial = c->partial[s];
      for (int64_t blk = 0; blk < c->T.ord[s].nblocks; ++blk) items.push_back(((int64_t)i << 40) | blk);
      int64_t tot = 1, bs = 1;
      for (int q = 0; q < s; ++q) { tot *= (c->b + 1); bs *= c->b; }
      stage = std::max(stage, (size_t)(tot - 1 - bs) * sizeof(double));
    }
    if (items.empty()) continue;
    bt->ncomb[s] = (int)items.size();
    bt->comb_grid[s] = std::min(bt->ncomb[s], pgrid * 2);
    bt->stage_bytes[s] = stage ? stage : 16;
    if (bupload(bt, &bt->d_comb[s], args.data(), args.size()) != hipSuccess) return fail(CUM_ENOMEM);
    if (bupload(bt, &bt->comb_items[s], items.data(), items.size()) != hipSuccess) return fail(CUM_ENOMEM);
  }
  std::vector<NormArgs> na((size_t)m);
  for (int i = 0; i < m; ++i) {
    cum_ctx* c = ctxs[i];
    na[(size_t)i].d = c->d;
    na[(size_t)i].kfirst = 1;
    for (int k = 1; k <= c->d; ++k) {
      na[(size_t)i].nblocks[k] = c->T.ord[k].nblocks;
      na[(size_t)i].partial[k] = c->partial[k];
    }
    na[(size_t)i].out = c->norms;
  }
  if (bupload(bt, &bt->d_norm, na.data(), na.size()) != hipSuccess) return fail(CUM_ENOMEM);

  // capture the whole step once
  if (hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(CUM_EDEVICE);
  const int lrc = batch_launch_all(bt);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(bt->stream, &g);
  if (lrc != CUM_OK || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(lrc != CUM_OK ? lrc : CUM_EDEVICE);
  }
  bt->graph = g;
  if (hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0) != hipSuccess) return fail(CUM_EDEVICE);
  for (cum_ctx* c : bt->ctx) c->batch_done = bt->done;
  *out = bt;
  return CUM_OK;
}

int cum_batch_update(cum_batch* bt, const void* const* X_new, const void* const* X_old, const int64_t* p) {
  if (!bt || !X_new || !X_old || !p) return CUM_EINVAL;
  const int m = (int)bt->ctx.size();
  for (int i = 0; i < m; ++i) {
    cum_ctx* c = bt->ctx[(size_t)i];
    const int64_t pi = p[i];
    if (pi < 0 || pi > c->t || pi > kRowChunk) return CUM_EINVAL;
    const bool fifo = c->fifo_q > 0;
    if (fifo && pi != 0 && pi != c->fifo_p) return CUM_EINVAL;
    if (pi > 0) {
      const void* xo = fifo ? X_new[i] : X_old[i];
      if (!X_new[i] || !xo) return CUM_EINVAL;
      const bool vl = (c->n * (int)c->x_size) % 16 == 0;
      if (vl && (((uintptr_t)X_new[i] | (uintptr_t)xo) % 16)) return CUM_EINVAL;
      // device memory: both row blocks inside the allocation the member's
      // last inputs were found in, or found by a query now
      const uintptr_t bytes = (uintptr_t)pi * c->n * c->x_size;
      const uintptr_t a0 = (uintptr_t)X_new[i], a1 = (uintptr_t)xo;
      uintptr_t& lo = bt->alloc_lo[(size_t)i];
      uintptr_t& hi = bt->alloc_hi[(size_t)i];
      const bool inside = lo && a0 >= lo && a0 + bytes <= hi && a1 >= lo && a1 + bytes <= hi;
      if (!inside) {
        if (!is_device_ptr(X_new[i]) || !is_device_ptr(xo)) return CUM_EINVAL;
        hipDeviceptr_t base = nullptr;
        size_t size = 0;
        if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)X_new[i]) == hipSuccess && base &&
            a1 >= (uintptr_t)base && a1 + bytes <= (uintptr_t)base + size) {
          lo = (uintptr_t)base;
          hi = (uintptr_t)base + size;
        } else {
          (void)hipGetLastError();
          lo = hi = 0;
        }
      }
    }
  }
  for (cum_ctx* c : bt->ctx)
    if (c->norms_pending) {  // the batch step rewrites the partials they need
      if (int rc = flush_norms(c)) return rc;
      c->direct_since_batch = true;
    }
  for (cum_ctx* c : bt->ctx)
    if (c->direct_since_batch || c->pipe_active) {
      if (int rj = join_pipe(c)) return rj;
      CUM_TRY(hipStreamSynchronize(c->stream));
      c->direct_since_batch = false;
    }
  for (int i = 0; i < m; ++i) {
    cum_ctx* c = bt->ctx[(size_t)i];
    UpdArgs& a = bt->h_upd[(size_t)i];
    const bool fifo = c->fifo_q > 0 && p[i] > 0;
    a.xp = p[i] ? X_new[i] : nullptr;
    a.xm = (p[i] && !fifo) ? X_old[i] : nullptr;
    a.np = (int)p[i];
    a.nm = fifo ? 0 : (int)p[i];
    a.vec = (c->n * (int)c->x_size) % 16 == 0;
    set_fifo(c, a, fifo ? 2 : 0, c->fifo_head);
  }
  // the table goes up from the next pinned slot (its previous copy done)
  const int r = bt->ring_next;
  bt->ring_next = (r + 1) % cum_batch::kRing;
  if (bt->ring_used[r]) CUM_TRY(hipEventSynchronize(bt->ring_done[r]));
  memcpy(bt->ring[r], bt->h_upd.data(), bt->h_upd.size() * sizeof(UpdArgs));
  CUM_TRY(hipMemcpyAsync(bt->d_upd, bt->ring[r], bt->h_upd.size() * sizeof(UpdArgs), hipMemcpyHostToDevice,
                         bt->stream));
  CUM_TRY(hipEventRecord(bt->ring_done[r], bt->stream));
  bt->ring_used[r] = true;
  CUM_TRY(hipGraphLaunch(bt->exec, bt->stream));
  CUM_TRY(hipEventRecord(bt->done, bt->stream));
  for (int i = 0; i < m; ++i) {
    cum_ctx* c = bt->ctx[(size_t)i];
    if (c->fifo_q > 0 && p[i] > 0) c->fifo_head = (c->fifo_head + 1) % c->fifo_q;
  }
  return CUM_OK;
}

int cum_batch_sync(cum_batch* bt) {
  if (!bt) return CUM_EINVAL;
  CUM_TRY(hipStreamSynchronize(bt->stream));
  return CUM_OK;
}

int cum_batch_free(cum_batch* bt) {
  if (!bt) return CUM_OK;
  (void)hipStreamSynchronize(bt->stream);
  batch_release(bt);
  delete bt;
  return CUM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint: L = sum_k w_k ||C_k(X W^T)||_F^2 and its gradients.

namespace {

// Y_bar work items: every stored block as (order << 28 | block), orders
// ascending, cut into `groups` contiguous ranges of equal element count.
void build_ybar_items(const Tables& T, int groups, std::vector<int32_t>& items, std::vector<int32_t>& gptr) {
  items.clear();
  std::vector<int64_t> wt;
  int64_t total = 0;
  for (int s = 1; s <= T.d; ++s)
    for (int64_t r = 0; r < T.ord[s].nblocks; ++r) {
      items.push_back((int32_t)(((int64_t)s << 28) | r));
      wt.push_back(T.ord[s].bk);
      total += T.ord[s].bk;
    }
  gptr.assign((size_t)groups + 1, (int32_t)items.size());
  gptr[0] = 0;
  int64_t acc = 0;
  int g = 1;
  for (size_t i = 0; i < items.size() && g < groups; ++i) {
    acc += wt[i];
    while (g < groups && acc * groups >= total * g) gptr[(size_t)g++] = (int32_t)(i + 1);
  }
}

// Reverse-combine gather lists of order s: for every block of the lower
// orders 1 .. s-1 (concatenated by order, bstart[q] = first block of order
// q), the (order-s block << 6 | mask) pairs whose sub-tuple is that block,
// in increasing (block, mask) order.
int build_rev_lists(const Tables& T, int s, std::vector<int64_t>& bstart, std::vector<int32_t>& ptr,
                    std::vector<int32_t>& ent) {
  const int nm = 1 << s;
  bstart.assign((size_t)s + 1, 0);
  int64_t nlow = 0;
  for (int q = 1; q < s; ++q) {
    bstart[(size_t)q] = nlow;
    nlow += T.ord[q].nblocks;
  }
  bstart[(size_t)s] = nlow;
  const int64_t nb = T.ord[s].nblocks;
  if (nb >= ((int64_t)1 << 25) || nb * (nm - 2) >= ((int64_t)1 << 31)) return CUM_ESIZE;
  std::vector<int64_t> cnt((size_t)nlow + 1, 0);
  for (int64_t r = 0; r < nb; ++r)
    for (int m = 1; m < nm - 1; ++m) {
      const int q = __builtin_popcount((unsigned)m);
      cnt[(size_t)(bstart[(size_t)q] + T.subrank[s][(size_t)r * nm + m] + 1)] += 1;
    }
  ptr.assign((size_t)nlow + 1, 0);
  for (int64_t i = 0; i < nlow; ++i) ptr[(size_t)i + 1] = (int32_t)(ptr[(size_t)i] + cnt[(size_t)i + 1]);
  ent.assign((size_t)ptr[(size_t)nlow], 0);
  std::vector<int32_t> pos(ptr.begin(), ptr.end() - 1);
  for (int64_t r = 0; r < nb; ++r)
    for (int m = 1; m < nm - 1; ++m) {
      const int q = __builtin_popcount((unsigned)m);
      const size_t at = (size_t)(bstart[(size_t)q] + T.subrank[s][(size_t)r * nm + m]);
      ent[(size_t)pos[at]++] = (int32_t)((r << 6) | m);
    }
  return CUM_OK;
}

// Tables of Y_bar = P G.  Rows of G: the sorted tuples J of orders 0 .. d-1
// over the n columns, in increasing order and lexicographic within an order
// (kpad rows, padded with empty rows); facs[row] holds J's columns, one per
// byte, then the index n (which reads 1).  Entry lists of G[row, j]: every
// stored element e (of the concatenated pyramids, offsets `base`) whose
// multi-index is J plus j, with the number of positions of e holding j.
int build_g_tables(const Tables& T, int n, int d, int64_t splits_max, const int64_t* base, int ncol,
                   int& splits, int64_t& kpad, std::vector<uint64_t>& facs, std::vector<int64_t>& gptr,
                   std::vector<int64_t>& gent, int64_t t) {
  std::unordered_map<uint64_t, int64_t> rowof;
  std::vector<std::vector<int>> rows;
  auto key = [](const int* J, int len) {
    uint64_t k = (uint64_t)len;
    for (int q = 0; q < len; ++q) k |= (uint64_t)(J[q] + 1) << (3 + 7 * q);
    return k;
  };
  for (int len = 0; len < d; ++len) {
    std::vector<int> J((size_t)len, 0);
    while (true) {
      rowof[key(J.data(), len)] = (int64_t)rows.size();
      rows.push_back(J);
      int q = len - 1;
      while (q >= 0 && J[(size_t)q] == n - 1) --q;
      if (q < 0) break;
      ++J[(size_t)q];
      for (int r = q + 1; r < len; ++r) J[(size_t)r] = J[(size_t)q];
    }
  }
  const int64_t K = (int64_t)rows.size();
  const int64_t tiles = (t + 127) / 128;  // row tiles of the Y_bar kernel
  splits = (int)std::max<int64_t>(1, std::min<int64_t>(splits_max, (1024 + tiles - 1) / tiles));
  kpad = (K + 32 * splits - 1) / (32 * splits) * (32 * splits);
  if (kpad * ncol > ((int64_t)1 << 24) || kpad / splits > YB_MAX_KPER) return CUM_ESIZE;
  facs.assign((size_t)kpad, 0);
  for (int64_t r = 0; r < kpad; ++r) {
    uint64_t f = 0;
    for (int q = 0; q < 8; ++q) {
      const int v = (r < K && q < (int)rows[(size_t)r].size()) ? rows[(size_t)r][(size_t)q] : n;
      f |= (uint64_t)v << (8 * q);
    }
    facs[(size_t)r] = f;
  }
  std::vector<std::pair<int64_t, int64_t>> pairs;  // (G index, element offset)
  int64_t total = 0;
  for (int k = 1; k <= d; ++k) total += T.ord[k].nelems * k;
  if (total > ((int64_t)1 << 26)) return CUM_ESIZE;
  pairs.reserve((size_t)total);
  int idx[CUM_MAXD], J[CUM_MAXD];
  for (int k = 1; k <= d; ++k) {
    const OrderInfo& o = T.ord[k];
    for (int64_t blk = 0; blk < o.nblocks; ++blk)
      for (int64_t l = 0; l < o.bk; ++l) {
        int64_t rem = l;
        bool pad = false;
        for (int q = k - 1; q >= 0; --q) {
          idx[q] = T.tuples[k][(size_t)blk * k + q] * T.b + (int)(rem % T.b);
          rem /= T.b;
          pad = pad || idx[q] >= n;
        }
        if (pad) continue;
        const int64_t off = base[k] + blk * o.bk + l;
        for (int q = 0; q < k; ++q) {
          int len = 0;
          for (int u = 0; u < k; ++u)
            if (u != q) J[len++] = idx[u];
          std::sort(J, J + len);
          const int64_t row = rowof.at(key(J, len));
          pairs.emplace_back(row * ncol + idx[q], off);
        }
      }
  }
  std::sort(pairs.begin(), pairs.end());
  gptr.assign((size_t)(kpad * ncol) + 1, 0);
  gent.clear();
  size_t i = 0;
  for (int64_t r = 0; r < kpad * ncol; ++r) {
    while (i < pairs.size() && pairs[i].first == r) {
      size_t j = i;
      while (j < pairs.size() && pairs[j] == pairs[i]) ++j;
      gent.push_back(pairs[i].second | ((int64_t)(j - i) << 48));
      i = j;
    }
    gptr[(size_t)r + 1] = (int64_t)gent.size();
  }
  return CUM_OK;
}

}  // namespace

extern "C" {

struct cum_loss_plan {
  int n = 0, d = 0, b = 0;
  int64_t t = 0;
  hipStream_t caller = nullptr;  // the stream the caller's X and W are ordered on
  hipStream_t st = nullptr;      // the plan's own stream (the pass is captured on it)
  hipEvent_t ev = nullptr;
  hipGraphExec_t graph = nullptr;
  bool eager_only = false;       // capture failed: every call runs the pass eagerly
  cum_ctx* c = nullptr;  // FP32 context over Y = X W^T
  float* Y = nullptr;
  // plan-owned copies of the inputs and outputs (the captured pass reads and
  // writes only these), the weights on the device and in pinned host memory,
  // and the norms read back
  float* Xp = nullptr;
  float* Wp = nullptr;
  float* dXp = nullptr;
  float* dWp = nullptr;
  double* d_w = nullptr;
  double* h_w = nullptr;
  double* h_norms = nullptr;
  double* Cbar[CUM_MAXD + 1] = {};  // views into one allocation, orders concatenated
  int64_t cbar_base[CUM_MAXD + 1] = {};
  // reverse combine
  double* rev_part = nullptr;
  RevCollectArgs rc[CUM_MAXD + 1] = {};
  int64_t rc_nblocks[CUM_MAXD + 1] = {};
  // Y_bar on matrix cores (mma) or block by block
  bool mma = false;
  int splits = 1, ncol = 16, F = 1;
  int64_t kpad = 0;
  uint64_t* facs = nullptr;
  double* G = nullptr;
  int64_t* gptr = nullptr;
  int64_t* gent = nullptr;
  uint8_t* tuples[CUM_MAXD + 1] = {};
  int32_t* items = nullptr;
  int32_t* bgptr = nullptr;
  int groups = 1;
  double* part = nullptr;    // splits (or groups) x t x n
  double* dwpart = nullptr;  // row tiles x n x n
  std::vector<void*> owned;
};

int cum_loss_plan_free(cum_loss_plan* pl) {
  if (!pl) return CUM_OK;
  if (pl->st) (void)hipStreamSynchronize(pl->st);
  if (pl->graph) (void)hipGraphExecDestroy(pl->graph);
  if (pl->c) cum_free(pl->c);
  for (void* p : pl->owned) (void)hipFree(p);
  if (pl->h_w) (void)hipHostFree(pl->h_w);
  if (pl->h_norms) (void)hipHostFree(pl->h_norms);
  if (pl->ev) (void)hipEventDestroy(pl->ev);
  if (pl->st) (void)hipStreamDestroy(pl->st);
  delete pl;
  return CUM_OK;
}

int cum_loss_plan_create(cum_loss_plan** out, int n, int d, int b, int64_t t, void* hip_stream) {
  if (!out) return CUM_EINVAL;
  *out = nullptr;
  int rc = check_shape(n, d, b);
  if (rc != CUM_OK) return rc;
  if (t < 1 || t > ((int64_t)1 << 31)) return CUM_EINVAL;
  // Y_bar stages 256 rows of Y (256 n floats) in LDS; the host table of
  // (element, column) pairs holds up to d entries per stored element
  if (n > 64) return CUM_ESIZE;
  // the reverse combine stages a block's moment lattice and gradients in LDS
  for (int s = 2; s <= d; ++s) {
    int64_t tot = 1;
    for (int q = 0; q < s; ++q) tot *= (b + 1);
    if (tot - 1 > REV_LDS_DOUBLES) return CUM_ESIZE;
  }
  {
    Tables probe;
    if (build_tables(n, b, d, probe) != 0) return CUM_EINVAL;
    int64_t tot = 0;
    for (int k = 1; k <= d; ++k) tot += probe.ord[k].nelems;
    if (tot > ((int64_t)1 << 24)) return CUM_ESIZE;
  }
  cum_loss_plan* pl = new (std::nothrow) cum_loss_plan();
  if (!pl) return CUM_ENOMEM;
  pl->n = n; pl->d = d; pl->b = b; pl->t = t;
  pl->caller = (hipStream_t)hip_stream;
  auto fail = [&](int r) {
    cum_loss_plan_free(pl);
    return r;
  };
  auto alloc = [&](void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e == hipSuccess) pl->owned.push_back(*p);
    else *p = nullptr;
    return e;
  };
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&pl->st, hipStreamNonBlocking)) != hipSuccess) {
    pl->st = nullptr;
    return fail(map_err(e));
  }
  if ((e = hipEventCreateWithFlags(&pl->ev, hipEventDisableTiming)) != hipSuccess) {
    pl->ev = nullptr;
    return fail(map_err(e));
  }
  if ((e = hipHostMalloc((void**)&pl->h_w, (size_t)(d + 1) * sizeof(double), hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&pl->h_norms, (size_t)2 * (d + 1) * sizeof(double), hipHostMallocDefault)) !=
          hipSuccess)
    return fail(map_err(e));
  if ((e = alloc((void**)&pl->Xp, (size_t)t * n * sizeof(float))) != hipSuccess ||
      (e = alloc((void**)&pl->dXp, (size_t)t * n * sizeof(float))) != hipSuccess ||
      (e = alloc((void**)&pl->Wp, (size_t)n * n * sizeof(float))) != hipSuccess ||
      (e = alloc((void**)&pl->dWp, (size_t)n * n * sizeof(float))) != hipSuccess ||
      (e = alloc((void**)&pl->d_w, (size_t)(d + 1) * sizeof(double))) != hipSuccess)
    return fail(map_err(e));
  if ((e = alloc((void**)&pl->Y, (size_t)t * n * sizeof(float))) != hipSuccess) return fail(map_err(e));
  if ((e = hipMemsetAsync(pl->Y, 0, (size_t)t * n * sizeof(float), pl->st)) != hipSuccess) return fail(map_err(e));
  if ((e = hipStreamSynchronize(pl->st)) != hipSuccess) return fail(map_err(e));
  rc = cum_init(&pl->c, n, d, b, pl->Y, t, CUM_FP32, pl->st);
  if (rc != CUM_OK) return fail(rc);
  const Tables& T = pl->c->T;
  int64_t ctot = 0;
  for (int k = 1; k <= d; ++k) {
    pl->cbar_base[k] = ctot;
    ctot += T.ord[k].nelems;
  }
  double* cbar_all = nullptr;
  if ((e = alloc((void**)&cbar_all, (size_t)ctot * sizeof(double))) != hipSuccess) return fail(map_err(e));
  for (int k = 1; k <= d; ++k) pl->Cbar[k] = cbar_all + pl->cbar_base[k];
  auto up = [&](void** dst, const void* src, size_t bytes) {
    hipError_t r = alloc(dst, bytes);
    if (r == hipSuccess && bytes) r = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return r;
  };
  // reverse combine: partials of the largest order, gather lists per order
  int64_t rev_max = 0;
  for (int s = 2; s <= d; ++s) {
    int64_t tot = 1, bs = 1;
    for (int q = 0; q < s; ++q) { tot *= (b + 1); bs *= b; }
    tot = tot - 1 - bs;
    rev_max = std::max(rev_max, T.ord[s].nblocks * tot);
    RevCollectArgs& ra = pl->rc[s];
    ra.b = b;
    ra.tot = (int)tot;
    int off = 0;
    for (int m = 1; m < (1 << s) - 1; ++m) {
      ra.moff[m] = off;
      int bl = 1;
      for (int q = 0; q < __builtin_popcount((unsigned)m); ++q) bl *= b;
      off += bl;
    }
    std::vector<int64_t> bstart;
    std::vector<int32_t> ptr, ent;
    if ((rc = build_rev_lists(T, s, bstart, ptr, ent)) != CUM_OK) return fail(rc);
    int64_t es = 0;
    for (int q = 1; q < s; ++q) {
      ra.estart[q] = es;
      ra.bstart[q] = bstart[(size_t)q];
      ra.bk[q] = T.ord[q].bk;
      es += T.ord[q].nelems;
    }
    ra.estart[s] = es;
    ra.bstart[s] = bstart[(size_t)s];
    pl->rc_nblocks[s] = bstart[(size_t)s];  // blocks of the lower orders
    if ((e = up((void**)&ra.ptr, ptr.data(), ptr.size() * sizeof(int32_t))) != hipSuccess) return fail(map_err(e));
    if ((e = up((void**)&ra.ent, ent.data(), ent.size() * sizeof(int32_t))) != hipSuccess) return fail(map_err(e));
    for (int k = 1; k <= d; ++k) ra.Cbar[k] = pl->Cbar[k];
  }
  if ((e = alloc((void**)&pl->rev_part, (size_t)std::max<int64_t>(rev_max, 1) * sizeof(double))) != hipSuccess)
    return fail(map_err(e));
  for (int s = 2; s <= d; ++s) pl->rc[s].part = pl->rev_part;
  // Y_bar: on matrix cores when its gathered matrix stays small, else block
  // by block (row tiles of 64 times block groups, partials capped at 256 MB)
  const int64_t tiles = (t + 63) / 64;
  int nsplit = 1;
  {
    pl->ncol = (n + 15) / 16 * 16;
    pl->F = d > 1 ? d - 1 : 1;
    std::vector<uint64_t> facs;
    std::vector<int64_t> gptr, gent;
    int64_t cap = 1;
    while (cap < 16 && (cap + 1) * t * n * 8 <= ((int64_t)256 << 20)) ++cap;
    if (build_g_tables(T, n, d, cap, pl->cbar_base, pl->ncol, pl->splits, pl->kpad, facs, gptr, gent, t) ==
        CUM_OK) {
      pl->mma = true;
      nsplit = pl->splits;
      if ((e = up((void**)&pl->facs, facs.data(), facs.size() * sizeof(uint64_t))) != hipSuccess)
        return fail(map_err(e));
      if ((e = up((void**)&pl->gptr, gptr.data(), gptr.size() * sizeof(int64_t))) != hipSuccess)
        return fail(map_err(e));
      if ((e = up((void**)&pl->gent, gent.data(), std::max<size_t>(gent.size(), 1) * sizeof(int64_t))) !=
          hipSuccess)
        return fail(map_err(e));
      if ((e = alloc((void**)&pl->G, (size_t)(pl->kpad * pl->ncol) * sizeof(double))) != hipSuccess)
        return fail(map_err(e));
    }
  }
  if (!pl->mma) {
    int groups = (int)std::max<int64_t>(1, std::min<int64_t>(64, (2048 + tiles - 1) / tiles));
    while (groups > 1 && (int64_t)groups * t * n * 8 > ((int64_t)256 << 20)) --groups;
    pl->groups = groups;
    nsplit = groups;
    std::vector<int32_t> items, gptr;
    build_ybar_items(T, groups, items, gptr);
    for (int k = 1; k <= d; ++k)
      if ((e = up((void**)&pl->tuples[k], T.tuples[k].data(), T.tuples[k].size())) != hipSuccess)
        return fail(map_err(e));
    if ((e = up((void**)&pl->items, items.data(), items.size() * sizeof(int32_t))) != hipSuccess)
      return fail(map_err(e));
    if ((e = up((void**)&pl->bgptr, gptr.data(), gptr.size() * sizeof(int32_t))) != hipSuccess)
      return fail(map_err(e));
  }
  if ((e = alloc((void**)&pl->part, (size_t)nsplit * t * n * sizeof(double))) != hipSuccess) return fail(map_err(e));
  if ((e = alloc((void**)&pl->dwpart, (size_t)tiles * n * n * sizeof(double))) != hipSuccess)
    return fail(map_err(e));
  *out = pl;
  return CUM_OK;
}

}  // extern "C"

namespace {

// One forward and reverse pass on the plan's buffers (Xp, Wp -> dXp, dWp,
// the norms in the context), every step a kernel on the plan's stream.
int loss_pass(cum_loss_plan* pl) {
  cum_ctx* c = pl->c;
  const int n = pl->n, d = pl->d, b = pl->b;
  const int64_t t = pl->t;
  hipStream_t st = pl->st;
  CUM_TRY(launch_linear(pl->Xp, pl->Wp, pl->Y, t, n, st));
  int rc = cum_recompute(c, pl->Y);
  if (rc != CUM_OK) return rc;
  // the norms (for the loss) are formed on the stream and read at the end
  if ((rc = flush_norms(c)) != CUM_OK) return rc;
  {
    CbarArgs ca{};
    ca.d = d;
    for (int k = 1; k <= d; ++k) {
      ca.off[k] = pl->cbar_base[k];
      ca.bk[k] = c->T.ord[k].bk;
      ca.C[k] = c->C[k];
      ca.mult[k] = c->mult[k];
    }
    ca.off[d + 1] = pl->cbar_base[d] + c->T.ord[d].nelems;
    ca.w = pl->d_w;
    ca.Cbar = pl->Cbar[1];
    CUM_TRY(launch_cbar_init(ca, st));
  }
  for (int s = d; s >= 2; --s) {
    RevBlockArgs ra{};
    ra.b = b;
    ra.bs = c->T.ord[s].bk;
    ra.tot = pl->rc[s].tot;
    ra.subrank = c->subrank[s];
    ra.Cbar_s = pl->Cbar[s];
    for (int k = 1; k < s; ++k) {
      ra.Shi[k] = (const float*)c->s_hi[k];
      ra.Slo[k] = (const float*)c->s_lo[k];
    }
    ra.inv_t = 1.0 / (double)t;
    ra.part = pl->rev_part;
    CUM_TRY(launch_rev_block(s, ra, c->T.ord[s].nblocks, st));
    CUM_TRY(launch_rev_collect(pl->rc[s], s, pl->rc_nblocks[s], st));
  }
  if (pl->mma) {
    GbuildArgs ga{};
    ga.rows = pl->kpad * pl->ncol;
    ga.ptr = pl->gptr;
    ga.ent = pl->gent;
    ga.Mbar = pl->Cbar[1];
    ga.inv_t = 1.0 / (double)t;
    ga.G = pl->G;
    CUM_TRY(launch_gbuild(ga, st));
    YbarMmaArgs ya{};
    ya.n = n;
    ya.ncol = pl->ncol;
    ya.t = t;
    ya.kper = (int)(pl->kpad / pl->splits);
    ya.Y = pl->Y;
    ya.facs = pl->facs;
    ya.G = pl->G;
    ya.part = pl->part;
    CUM_TRY(launch_ybar_mma(ya, pl->F, pl->splits, st));
    CUM_TRY(launch_ybar_finish(pl->part, pl->splits, 1.0, pl->Xp, pl->Wp, pl->dXp, pl->dwpart, pl->dWp, t, n, st));
  } else {
    YbarBlockArgs ya{};
    ya.n = n;
    ya.b = b;
    ya.ncols = c->T.nbar * b;
    ya.t = t;
    ya.Y = pl->Y;
    for (int k = 1; k <= d; ++k) {
      ya.Mbar[k] = pl->Cbar[k];
      ya.tuples[k] = pl->tuples[k];
    }
    ya.items = pl->items;
    ya.gptr = pl->bgptr;
    ya.part = pl->part;
    CUM_TRY(launch_ybar_blocks(ya, pl->groups, st));
    CUM_TRY(launch_ybar_finish(pl->part, pl->groups, 1.0 / (double)t, pl->Xp, pl->Wp, pl->dXp, pl->dwpart,
                               pl->dWp, t, n, st));
  }
  return CUM_OK;
}

}  // namespace

extern "C" {

// The first call runs the pass eagerly, then captures it into a HIP graph on
// the plan's stream; later calls copy the inputs in, launch the graph and
// copy the results out.
int cum_loss_plan_grad(cum_loss_plan* pl, const float* X, const float* W, const double* w, double* L, float* dX,
                       float* dW) {
  if (!pl || !X || !W || !w || !L || !dX || !dW) return CUM_EINVAL;
  if (!is_device_ptr(X) || !is_device_ptr(W) || !is_device_ptr(dX) || !is_device_ptr(dW)) return CUM_EINVAL;
  const int n = pl->n, d = pl->d;
  const int64_t t = pl->t;
  hipStream_t st = pl->st;
  for (int k = 0; k <= d; ++k) pl->h_w[k] = w[k];
  CUM_TRY(hipEventRecord(pl->ev, pl->caller));
  CUM_TRY(hipStreamWaitEvent(st, pl->ev, 0));
  CUM_TRY(hipMemcpyAsync(pl->d_w, pl->h_w, (size_t)(d + 1) * sizeof(double), hipMemcpyHostToDevice, st));
  CUM_TRY(hipMemcpyAsync(pl->Xp, X, (size_t)t * n * sizeof(float), hipMemcpyDeviceToDevice, st));
  CUM_TRY(hipMemcpyAsync(pl->Wp, W, (size_t)n * n * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (pl->graph) {
    CUM_TRY(hipGraphLaunch(pl->graph, st));
  } else {
    int rc = loss_pass(pl);
    if (rc != CUM_OK) return rc;
    if (!pl->eager_only) {
      // capture the same pass for the next calls (nothing runs during capture)
      CUM_TRY(hipStreamSynchronize(st));
      hipGraph_t g = nullptr;
      bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) == hipSuccess;
      const int prc = ok ? loss_pass(pl) : CUM_EDEVICE;
      ok = (hipStreamEndCapture(st, &g) == hipSuccess) && ok && prc == CUM_OK && g;
      if (ok) ok = hipGraphInstantiate(&pl->graph, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
      if (!ok) {
        (void)hipGetLastError();
        pl->graph = nullptr;
        pl->eager_only = true;
      }
    }
  }
  CUM_TRY(hipMemcpyAsync(dX, pl->dXp, (size_t)t * n * sizeof(float), hipMemcpyDeviceToDevice, st));
  CUM_TRY(hipMemcpyAsync(dW, pl->dWp, (size_t)n * n * sizeof(float), hipMemcpyDeviceToDevice, st));
  CUM_TRY(hipMemcpyAsync(pl->h_norms, pl->c->norms, (size_t)2 * (d + 1) * sizeof(double), hipMemcpyDeviceToHost,
                         st));
  CUM_TRY(hipStreamSynchronize(st));
  double loss = 0.0;
  for (int k = 1; k <= d; ++k)
    if (w[k] != 0.0) loss += w[k] * pl->h_norms[k] * pl->h_norms[k];
  *L = loss;
  return CUM_OK;
}

int cum_loss_grad(int n, int d, int b, const float* X, int64_t t, const float* W, const double* w, double* L,
                  float* dX, float* dW, void* hip_stream) {
  if (!X || !W || !w || !L || !dX || !dW) return CUM_EINVAL;
  if (!is_device_ptr(X) || !is_device_ptr(W) || !is_device_ptr(dX) || !is_device_ptr(dW)) return CUM_EINVAL;
  cum_loss_plan* pl = nullptr;
  int rc = cum_loss_plan_create(&pl, n, d, b, t, hip_stream);
  if (rc != CUM_OK) return rc;
  pl->eager_only = true;  // one call: nothing to capture for
  rc = cum_loss_plan_grad(pl, X, W, w, L, dX, dW);
  cum_loss_plan_free(pl);
  return rc;
}

}  // extern "C"
