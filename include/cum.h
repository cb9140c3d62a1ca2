/*
 * cum.h -- C-ABI of libcum: sliding-window cumulant tensors on MI355X (gfx950).
 *
 * Method: Domino & Gawron, "Algorithm for an arbitrary-order cumulant tensor
 * calculation in a sliding window of data streams" (arXiv:1701.06446).
 *
 * Data convention (Sec. 2.1): a window X holds t rows (samples) of n columns
 * (marginals), row-major.  Each update appends p new rows X_new and drops the
 * window's p oldest rows X_old (the batches X_(+) and X_(-) of Sec. 2.1).
 *
 * Storage convention (Sec. 2.3 block structure, Alg. 5): an order-k tensor is
 * kept as the blocks whose block multi-index j_1 <= ... <= j_k is
 * non-decreasing, with nbar = ceil(n/b) blocks per mode; blocks are listed in
 * lexicographic order of j; every block is a full b^k array of doubles,
 * row-major in (a_1, ..., a_k) with a_1 slowest, holding the element at global
 * indices i_m = j_m*b + a_m.  Columns past n are zero padding and their
 * entries are exactly 0.  cum_num_blocks() gives the block count
 * C(nbar + k - 1, k); an order-k pyramid holds cum_num_blocks(n,b,k) * b^k
 * doubles.
 *
 * Estimators: raw plug-in moments m_i = (1/t) sum_rows prod x (Eq. (mom));
 * cumulants by the moment-cumulant recursion over all set partitions
 * (Alg. 3/4); no bias correction.
 *
 * Pointers: every input pointer may be host or device memory (detected with
 * hipPointerGetAttributes).  Inputs are FP64 when prec == CUM_FP64 and FP32
 * otherwise.  The caller owns every buffer it passes.  Host inputs are copied
 * before the call returns.  Device inputs are read by work queued on the
 * context's stream: keep them unchanged until that work has completed
 * (stream order, or cum_sync()).  The library owns its device state until
 * cum_free().
 *
 * Errors: every call returns CUM_OK (0) or a negative cum_status; nothing
 * aborts or throws across this boundary.  Arguments are validated before any
 * work is queued.  On a validation error the context's state is unchanged
 * and the context stays usable.  After CUM_EDEVICE the state is undefined.
 *
 * Threads: one context must not be used from two threads at once; distinct
 * contexts are independent.
 */
#ifndef CUM_H
#define CUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cum_ctx cum_ctx;

/* Precision of the moment contraction (the combine and norms are always FP64).
 *   CUM_FP64   - FP64 inputs, FP64 MFMA, FP64 compensated window sums.
 *   CUM_FP32   - FP32 inputs, FP32 MFMA, FP32 compensated (hi+lo) sums.
 *   CUM_BF16X3 - FP32 inputs; every Khatri-Rao operand is split into
 *                RNE-rounded bf16 hi + lo parts and each product is taken as
 *                hi*hi + hi*lo + lo*hi on bf16 MFMA with FP32 accumulation;
 *                FP32 compensated sums. */
typedef enum { CUM_FP64 = 0, CUM_FP32 = 1, CUM_BF16X3 = 2 } cum_prec;

typedef enum {
  CUM_OK = 0,
  CUM_EINVAL = -1,     /* bad argument (range, NULL pointer, p > t, ...) */
  CUM_ENOMEM = -2,     /* device or host allocation failed */
  CUM_EDEVICE = -3,    /* a HIP runtime call failed */
  CUM_ESTATE = -4,     /* context not initialised */
  CUM_ENONFINITE = -5, /* reserved: non-finite input detected */
  CUM_ESIZE = -6       /* output capacity too small, or shape beyond limits */
} cum_status;

/* Library limits: 1 <= d <= CUM_MAX_ORDER, 1 <= b <= n <= CUM_MAX_COLS. */
#define CUM_MAX_ORDER 6
#define CUM_MAX_COLS 255

/*
 * cum_init -- create a context and compute the moments M_1..M_d of the first
 * window X (t x n, row-major), then its cumulants C_1..C_d and norms (the
 * start of Alg. 1).  The window is contracted in chunks of at most 2048
 * rows, each folded into the compensated running sums.
 *   ctx        out: the new context (set to NULL on error)
 *   n, d, b    columns (1..255), maximal order (1..6), block size
 *              (1..n; b need not divide n: columns are zero-padded to
 *              ceil(n/b)*b)
 *   X          t x n window, FP64 if prec == CUM_FP64 else FP32
 *   t          window length (>= 1)
 *   prec       cum_prec
 *   hip_stream hipStream_t for all work of this context (NULL = null stream)
 */
int cum_init(cum_ctx **ctx, int n, int d, int b, const void *X, int64_t t, int prec,
             void *hip_stream);

/*
 * cum_update -- slide the window by p rows: M_k += (sum over X_new of x^(k) -
 * sum over X_old of x^(k)) / t for k = 1..d (Eq. (momupdate), Alg. 2), then
 * recompute C_1..C_d (Alg. 3/4) and the norms (Alg. 5, Eq. (mef)).
 * Asynchronous on the context's stream.  The norms' final reduction is
 * deferred: the next update launch forms it in one extra workgroup on a CU
 * its tiles leave idle, and cum_norms, cum_norms_device and cum_sync launch
 * it on its own if it is still pending.
 * With CUM_PIPELINE=1 in the environment at cum_init, a sliding update of
 * at most 2048 rows from 16-byte aligned rows (four-tile kernel) is
 * pipelined instead: the update launch stores the increment, and its fold
 * into the running sums (the same arithmetic, bitwise equal results), the
 * combine and the norms run on a stream of the context's own beside the
 * next update; every other entry point orders that work before its own.
 * Not while the stream is being captured, for FIFO contexts or batch
 * members.
 *   X_new  p x n rows entering the window
 *   X_old  p x n rows leaving it; precondition (not checked): these are the
 *          window's p oldest rows
 *   p      0 <= p <= t; p == 0 is a no-op
 */
int cum_update(cum_ctx *ctx, const void *X_new, const void *X_old, int64_t p);

/*
 * cum_update_noalloc -- cum_update for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, semantics and errors as cum_update,
 * but host inputs are staged through a fixed device array of the library
 * (16 MiB per GPU, held from the first call on that GPU until the process
 * ends) instead of a buffer allocated on demand: the call allocates nothing
 * (no hipMalloc / hipFree; profiling events are not recorded during it).
 *   - CUM_ESIZE, before any work, when the staged rows exceed the array:
 *     p * n * sizeof(element) * (2, or 1 on a FIFO context) > 16 MiB.
 *   - CUM_EINVAL when the current device is not the one cum_init ran on.
 *   - Synchronises the context's stream before returning, so the array is
 *     free again.  Every call on one GPU shares that GPU's array: calls that
 *     overlap on one GPU (from several threads) race.
 */
int cum_update_noalloc(cum_ctx *ctx, const void *X_new, const void *X_old, int64_t p);

/*
 * cum_recompute -- recalculate the context's moments from scratch over the
 * window X (t x n rows, the t of cum_init, host or device, same element type
 * as cum_init's), then its cumulants and norms: the recalculation that
 * Eq. (upcmplx) (Sec. 2.4) and Eq. (complxn) (Sec. 2.6) compare the update
 * with.  The running sums are zeroed first, so any rounding accumulated by
 * earlier updates is dropped;
 * a FIFO context (cum_init_fifo) refills its t/p batch slots from X's
 * batches, oldest first.  Asynchronous on the context's stream for device X;
 * host X is staged and the call synchronises.
 */
int cum_recompute(cum_ctx *ctx, const void *X);

/*
 * cum_init_fifo -- like cum_init, but the context keeps the FIFO of batch
 * moments that Sec. 2.4 describes (after Alg. 2) as the alternative to contracting the rows
 * that leave the window: the window is cut into t/p batches of p rows
 * (oldest first), and the increment sum_{batch} x^(k) of every batch is kept
 * per stored element (t/p slots per order: FP64 on the CUM_FP64 path, else
 * FP32, i.e. t/p * cum_num_elems * 4 or 8 bytes per order).  On such a
 * context cum_update contracts only X_new (half the multiply-adds), folds
 * its increment into the running sums, folds out the stored increment of
 * the batch leaving the window (bit-for-bit the value once added, so the
 * sums do not drift), and stores the new one in its slot.  X_old is not
 * read (may be NULL) and p must equal the context's batch size; otherwise
 * CUM_EINVAL.
 *   p      batch size: 1 <= p <= 2048 (CUM_ESIZE beyond) and t % p == 0
 *          (CUM_EINVAL otherwise); other arguments as for cum_init
 */
int cum_init_fifo(cum_ctx **ctx, int n, int d, int b, const void *X, int64_t t, int64_t p, int prec,
                  void *hip_stream);

/*
 * cum_get -- copy the order-k cumulant pyramid C_k (k = 1..d, FP64, layout
 * above) into `blocks` (host or device), which holds `capacity_elems`
 * doubles.  Synchronises the context's stream.  CUM_ESIZE if too small.
 */
int cum_get(cum_ctx *ctx, int k, double *blocks, size_t capacity_elems);

/*
 * cum_get_moments -- copy M_k = S_k / t (the running sums divided by the
 * window length, FP64) in the same layout.  Synchronises.
 */
int cum_get_moments(cum_ctx *ctx, int k, double *blocks, size_t capacity_elems);

/*
 * cum_norms -- fro[k] = ||C_k||_F over the full n^k tensor (Alg. 5 with
 * exponent 2) for k = 1..d, fro[0] = NaN; nu[k] = fro[k] / fro[2]^(k/2) for
 * 3 <= k <= d (Eq. (mef)), NaN for k < 3 (and NaN when ||C_2|| = 0).  Both
 * arrays hold d+1 doubles (host pointers).  Synchronises.
 */
int cum_norms(cum_ctx *ctx, double *fro, double *nu);

/*
 * cum_norms_device -- device address of the norms written by the last
 * init/update: 2(d+1) doubles, fro[0..d] then nu[0..d].  Enqueues their
 * final reduction on the context's stream if it is still pending, so work
 * enqueued on that stream afterwards reads them; call it after every update
 * whose norms are read on the device.  Does not synchronise; the buffer is
 * owned by the context and overwritten by the next update.
 */
int cum_norms_device(cum_ctx *ctx, const double **dev_ptr);

/*
 * cum_profile_enable -- `on` is a mask of kernel classes (bit 0 = moment
 * update, bit 1 = cumulant combine, bit 2 = norms; 0 switches profiling
 * off): every launch of a selected class is bracketed by HIP events on the
 * context's stream (each pair adds a short gap between launches).  The
 * norms' reduction usually rides on the next update launch and is timed
 * with it; class 2 sees only its launches on its own (cum_sync & co.).
 * Synchronises and clears earlier records.
 */
int cum_profile_enable(cum_ctx *ctx, int on);

/*
 * cum_profile_sample -- bracket only the last of every `every` launches of
 * each selected class (every >= 1; cum_profile_enable resets it to 1), so
 * that a long timed run pays for few event pairs and the first launch after
 * a synchronisation (which starts on an idle GPU) is not among them unless
 * every = 1.  Returns CUM_EINVAL for every < 1.  Does not synchronise.
 */
int cum_profile_sample(cum_ctx *ctx, int every);

/*
 * cum_profile_read -- per kernel class (0 = moment update, 1 = cumulant
 * combine, 2 = norms): launches[3] and total_ms[3] of the launches recorded
 * since profiling was enabled or last read; clears the records.
 * Synchronises.
 */
int cum_profile_read(cum_ctx *ctx, int64_t *launches, double *total_ms);

/*
 * cum_set_combine -- how the moment -> cumulant combine forms each element
 * (takes effect at the next cum_update):
 *   CUM_COMBINE_PARTITIONS  Alg. 4: c_I = m_I minus, over every partition of
 *                           I's positions into 2..|I| parts, the product of
 *                           the parts' cumulants (B(|I|) - 1 terms; default)
 *   CUM_COMBINE_RECURSION   c_I = m_I minus, over the proper subsets B that
 *                           hold I's first position, c_B * m_{I\B}
 *                           (2^(|I|-1) - 1 terms: the moment-cumulant
 *                           relation grouped by the part that holds the first
 *                           position; the same value up to FP64 rounding)
 * Both run in the fused combine when each order-d block's lower-order
 * sub-blocks fit its 64 KB of LDS, else order by order (e.g. d = 6 with
 * b = 4), where the recursion reads the moments m_{I\B} from the
 * lower-order running sums.  A batch (below) uses each member's method as
 * set when the batch was created for members whose sub-blocks fit, and
 * Alg. 4 for the others.
 */
enum { CUM_COMBINE_PARTITIONS = 0, CUM_COMBINE_RECURSION = 1 };
int cum_set_combine(cum_ctx *ctx, int method);

/* cum_sync -- finish the context's work: launch the last update's norms if
 * still pending, then wait for everything queued on the context's stream. */
int cum_sync(cum_ctx *ctx);

/* cum_free -- release the context and its device state; NULL is allowed. */
int cum_free(cum_ctx *ctx);

/* Block count of an order-k pyramid, C(ceil(n/b) + k - 1, k); -1 on bad args. */
int64_t cum_num_blocks(int n, int b, int k);

/* Stored doubles of an order-k pyramid, cum_num_blocks(n,b,k) * b^k. */
int64_t cum_num_elems(int n, int b, int k);

/* Static text for a status code. */
const char *cum_strerror(int status);

/* Text naming the last failing HIP call of the calling thread (empty if none);
 * valid until that thread's next failing call. */
const char *cum_last_error(void);

/*
 * Batched streams.  cum_batch_create groups m initialised contexts (same
 * precision, any n, d, b, t; each at most one batch) and captures one HIP
 * graph that updates all of them: persistent update launches over the
 * tiles of every member (longest windows first), the combine of every order
 * for every member, and every member's norms.  The batch runs on a stream of
 * its own; member contexts wait for it before cum_get / cum_norms /
 * cum_update.  Free the batch before its members.
 *
 * cum_batch_update(bt, X_new[m], X_old[m], p[m]) slides member i by p[i]
 * rows (0 <= p[i] <= min(t_i, 2048)); every pointer must be device memory
 * (16-byte aligned when n*sizeof(element) is a multiple of 16) and stay
 * unchanged until the work completes (cum_batch_sync).  A member made by
 * cum_init_fifo takes p[i] equal to its batch size (or 0) and its X_old[i]
 * is not read (may be NULL).  CUM_EINVAL on any violation, before any work
 * is queued.
 */
typedef struct cum_batch cum_batch;
int cum_batch_create(cum_batch **batch, cum_ctx *const *ctxs, int m);
int cum_batch_update(cum_batch *batch, const void *const *X_new, const void *const *X_old, const int64_t *p);
int cum_batch_sync(cum_batch *batch);
int cum_batch_free(cum_batch *batch);

/*
 * cum_loss_grad -- the contrast L = sum_{k=1..d} w[k] ||C_k(Y)||_F^2 of the
 * single window Y = X W^T (X: t x n, W: n x n, row-major FP32 device
 * memory) and its gradients dL/dX (t x n) and dL/dW (n x n), FP32 device
 * memory owned by the caller.  w holds d+1 host doubles (w[0] unused).
 * Forward: FP32 moment contraction, FP64 combine (Alg. 3/4) and norms
 * (Alg. 5); reverse: FP64 (Alg. 4 backwards, then the derivative of
 * Eq. (mom), the latter on FP64 matrix cores).  Every sum is taken in a
 * fixed order (no atomics): repeated calls on the same inputs return
 * bitwise equal results.  L (host) receives the loss.
 * Synchronises `hip_stream`; allocates and frees its own temporaries.
 * CUM_ESIZE when n > 64, when orders 1..d hold more than 2^24 stored
 * elements, or when a block's moment lattice does not fit the reverse
 * combine's LDS ((b+1)^s - 1 > 19200 for some s <= d).
 */
int cum_loss_grad(int n, int d, int b, const float *X, int64_t t, const float *W, const double *w,
                  double *L, float *dX, float *dW, void *hip_stream);

/*
 * The same contrast and gradients for repeated calls at one shape (an
 * optimisation loop over W): cum_loss_plan_create allocates, once, the
 * context over Y = X W^T, the reverse-pass buffers and the per-column table
 * of the derivative of Eq. (mom); cum_loss_plan_grad then runs one forward
 * and reverse pass (arguments and results as for cum_loss_grad; synchronises
 * the plan's stream); cum_loss_plan_free releases everything.  Limits and
 * errors as for cum_loss_grad; a plan is not thread-safe.
 */
typedef struct cum_loss_plan cum_loss_plan;
int cum_loss_plan_create(cum_loss_plan **plan, int n, int d, int b, int64_t t, void *hip_stream);
int cum_loss_plan_grad(cum_loss_plan *plan, const float *X, const float *W, const double *w, double *L,
                       float *dX, float *dW);
int cum_loss_plan_free(cum_loss_plan *plan);

/*
 * cum_plan_coverage -- host-only check of the update's pivot decomposition
 * (no GPU needed): for order k, counts how many (pivot, row, column)
 * products of the update land on each stored element (written to `hits`,
 * cum_num_elems(n,b,k) ints, may be NULL) and returns the number of products
 * that miss the pyramid or land on an element with other global indices
 * (0 when the decomposition is exact), or a negative status.
 */
int64_t cum_plan_coverage(int n, int b, int k, int32_t *hits);

/*
 * cum_plan_items -- number of update workgroups (tiles) one update of
 * orders 1..d launches; a negative status on bad arguments.  Host only.
 */
int64_t cum_plan_items(int n, int d, int b);

/*
 * cum_plan_groups -- host-only view of how one update launch of the
 * four-tile kernel packs those tiles into workgroups: returns the number of
 * workgroups (four tiles each, padded with empty tiles) and, when the arrays
 * are not NULL, fills per workgroup the 16x16 fragments its tiles multiply
 * (`frags`) and its real tiles (`tiles`), one int each.  A negative status
 * on bad arguments.
 */
int64_t cum_plan_groups(int n, int d, int b, int32_t *frags, int32_t *tiles);

#ifdef __cplusplus
}
#endif

#endif /* CUM_H */
