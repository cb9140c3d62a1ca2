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

#include <new>
#include <vector>

#include "../../include/cum.h"
#include "kernels.h"
#include "tables.h"

using namespace cum;

namespace {

constexpr int64_t kRowChunk = 2048;  // rows per contraction before each compensated fold

}  // namespace

struct cum_ctx {
  int n = 0, d = 0, b = 0, prec = 0;
  int64_t t = 0;
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
  // optional per-kernel timing: (class, start, stop) per launch
  bool profiling = false;
  struct Ev { int cls; hipEvent_t a, b; };
  std::vector<Ev> events;
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
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->events.clear();
}

void release(cum_ctx* c) {
  drop_events(c);
  for (void* p : c->owned) (void)hipFree(p);
  c->owned.clear();
  if (c->stage) (void)hipFree(c->stage);
  c->stage = nullptr;
}

int check_shape(int n, int d, int b) {
  if (n < 1 || n > CUM_MAX_COLS || d < 1 || d > CUM_MAX_ORDER || b < 1 || b > n) return CUM_EINVAL;
  return CUM_OK;
}

// Brackets one launch with HIP events when profiling is on (class 0 =
// update, 1 = combine, 2 = norms).
struct Timed {
  cum_ctx* c;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(cum_ctx* ctx, int k) : c(ctx), cls(k) {
    if (!c->profiling) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
    (void)hipEventRecord(a, c->stream);
  }
  ~Timed() {
    if (!a) return;
    (void)hipEventRecord(b, c->stream);
    c->events.push_back({cls, a, b});
  }
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
  a.items = c->items;
  for (int k = 1; k <= c->d; ++k) {
    a.left[k] = c->left[k];
    a.right[k] = c->right[k];
    a.s_hi[k] = c->s_hi[k];
    a.s_lo[k] = c->s_lo[k];
  }
  return a;
}

int run_contraction(cum_ctx* c, const char* xp, int64_t np, const char* xm, int64_t nm) {
  UpdArgs a = base_args(c);
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
    Timed tm(c, 0);
    CUM_TRY(launch_update(c->prec, c->tm, c->tn, a, c->nitems, c->stream));
  }
  return CUM_OK;
}

int run_combine_and_norms(cum_ctx* c) {
  for (int s = 1; s <= c->d; ++s) {
    CombArgs a{};
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
    Timed tm(c, 1);
    CUM_TRY(launch_combine(c->prec, s, a, c->T.ord[s].nblocks, c->stream));
  }
  NormArgs na{};
  na.d = c->d;
  na.kfirst = 1;
  for (int k = 1; k <= c->d; ++k) {
    na.nblocks[k] = c->T.ord[k].nblocks;
    na.partial[k] = c->partial[k];
  }
  na.out = c->norms;
  Timed tm(c, 2);
  CUM_TRY(launch_norms(na, c->stream));
  return CUM_OK;
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

int cum_init(cum_ctx** out, int n, int d, int b, const void* X, int64_t t, int prec,
             void* hip_stream) {
  if (!out) return CUM_EINVAL;
  *out = nullptr;
  int rc = check_shape(n, d, b);
  if (rc != CUM_OK) return rc;
  if (prec != CUM_FP64 && prec != CUM_FP32 && prec != CUM_BF16X3) return CUM_EINVAL;
  if (!X || t < 1 || t > ((int64_t)1 << 40)) return CUM_EINVAL;

  cum_ctx* c = new (std::nothrow) cum_ctx();
  if (!c) return CUM_ENOMEM;
  c->n = n; c->d = d; c->b = b; c->prec = prec; c->t = t;
  c->stream = (hipStream_t)hip_stream;
  c->x_size = (prec == CUM_FP64) ? 8 : 4;
  c->st_size = (prec == CUM_FP64) ? 8 : 4;
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
  }
  if ((e = upload(c, &c->items, items, &used)) != hipSuccess) return fail(e);
  if ((e = dalloc(c, (void**)&c->norms, (size_t)2 * (d + 1) * 8, &used)) != hipSuccess) return fail(e);

  // the window, on the device
  const char* xw = (const char*)X;
  void* tmp = nullptr;
  const size_t wbytes = (size_t)t * n * c->x_size;
  if (!is_device_ptr(X)) {
    if ((e = dalloc(c, &tmp, wbytes, &used)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(tmp, X, wbytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return fail(e);
    xw = (const char*)tmp;
  }
  rc = run_contraction(c, xw, t, nullptr, 0);
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

int cum_update(cum_ctx* c, const void* X_new, const void* X_old, int64_t p) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (p < 0 || p > c->t) return CUM_EINVAL;
  if (p == 0) return CUM_OK;
  if (!X_new || !X_old) return CUM_EINVAL;
  const char* xn = (const char*)X_new;
  const char* xo = (const char*)X_old;
  const size_t bytes = (size_t)p * c->n * c->x_size;
  const bool dn = is_device_ptr(X_new), dob = is_device_ptr(X_old);
  if (!dn || !dob) {
    int rc = ensure_stage(c, 2 * bytes);
    if (rc != CUM_OK) return rc;
    char* st = (char*)c->stage;
    if (!dn) {
      CUM_TRY(hipMemcpyAsync(st, X_new, bytes, hipMemcpyHostToDevice, c->stream));
      xn = st;
    }
    if (!dob) {
      CUM_TRY(hipMemcpyAsync(st + bytes, X_old, bytes, hipMemcpyHostToDevice, c->stream));
      xo = st + bytes;
    }
    // host buffers are free for reuse once this returns
    CUM_TRY(hipStreamSynchronize(c->stream));
  }
  int rc = run_contraction(c, xn, p, xo, p);
  if (rc != CUM_OK) return rc;
  return run_combine_and_norms(c);
}

int cum_get(cum_ctx* c, int k, double* blocks, size_t capacity_elems) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (k < 1 || k > c->d || !blocks) return CUM_EINVAL;
  const size_t ne = (size_t)c->T.ord[k].nelems;
  if (capacity_elems < ne) return CUM_ESIZE;
  CUM_TRY(hipStreamSynchronize(c->stream));
  CUM_TRY(hipMemcpy(blocks, c->C[k], ne * 8, hipMemcpyDefault));
  return CUM_OK;
}

int cum_get_moments(cum_ctx* c, int k, double* blocks, size_t capacity_elems) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  if (k < 1 || k > c->d || !blocks) return CUM_EINVAL;
  const size_t ne = (size_t)c->T.ord[k].nelems;
  if (capacity_elems < ne) return CUM_ESIZE;
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
  if (!fro || !nu) return CUM_EINVAL;
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
  *dev_ptr = c->norms;
  return CUM_OK;
}

int cum_sync(cum_ctx* c) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  CUM_TRY(hipStreamSynchronize(c->stream));
  return CUM_OK;
}

int cum_profile_enable(cum_ctx* c, int on) {
  if (!c) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
  CUM_TRY(hipStreamSynchronize(c->stream));
  drop_events(c);
  c->profiling = on != 0;
  return CUM_OK;
}

int cum_profile_read(cum_ctx* c, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return CUM_EINVAL;
  if (!c->ready) return CUM_ESTATE;
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

int cum_free(cum_ctx* c) {
  if (!c) return CUM_OK;
  if (c->ready) (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
  return CUM_OK;
}

}  // extern "C"
