// Adjoint of L = sum_k w_k ||C_k(Y)||_F^2 with Y = X W^T (single window).
//
// Forward: Y = X W^T, then the library's moment contraction, combine and
// norms on Y.  Reverse, in FP64:
//   k_cbar_init     C_bar_k = 2 w_k mult(block) c  for every stored element
//                   (the loss of Alg. 5 differentiated element by element);
//   k_rev_block /   Alg. 4 run backwards, orders d..2: the gradient of an
//   k_rev_collect   order-s element w.r.t. a lower-order cumulant c_B of one
//                   of its sub-blocks is minus the product of the other parts
//                   summed over the partitions holding B, which is the
//                   moment of the complementary positions; per block and
//                   sub-block into partials, then gathered by every
//                   lower-order element in a fixed order (M_bar_s = the final
//                   C_bar_s);
//   k_gbuild /      Y_bar[l, j] = (1/t) sum over stored elements e containing
//   k_ybar_mma      column j of count_j(e) M_bar[e] prod of y[l, i] over e's
//                   other indices (the derivative of Eq. (mom)), as the
//                   product of the row products over sorted tuples with a
//                   gathered matrix, on FP64 matrix cores;
//   k_ybar_finish   dX = Y_bar W, dW = Y_bar^T X.
// (k_ybar_blocks is the block-by-block form of Y_bar for shapes whose
// gathered matrix would be too large.)  No atomics: every sum is taken in a
// fixed order.
#include <hip/hip_runtime.h>

#include "adjoint.h"
#include "partitions.h"

namespace cum {

// Y = X W^T for a tile of 64 rows, X's rows and W in LDS; each output sums
// over j in increasing order (one FP32 fused multiply-add per term).
__global__ __launch_bounds__(256) void k_linear(const float* __restrict__ X, const float* __restrict__ W,
                                                float* __restrict__ Y, int64_t t, int n) {
  __shared__ float xs[64 * 65];
  __shared__ float ws[64 * 65];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int rows = (int)(t - r0 < 64 ? t - r0 : 64);
  const int np = n + 1;  // padded rows: a wave's reads of one column spread over the banks
  for (int i = tid; i < rows * n; i += 256) {
    const int r = i / n, c = i - r * n;
    xs[r * np + c] = X[(r0 + r) * n + c];
  }
  for (int i = tid; i < n * n; i += 256) {
    const int r = i / n, c = i - r * n;
    ws[r * np + c] = W[i];
  }
  __syncthreads();
  for (int o = tid; o < rows * n; o += 256) {
    const int r = o / n, i = o - r * n;
    float acc = 0.0f;
    for (int j = 0; j < n; ++j) acc = fmaf(xs[r * np + j], ws[i * np + j], acc);
    Y[(r0 + r) * n + i] = acc;
  }
}

__global__ __launch_bounds__(256) void k_cbar_init(CbarArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.off[a.d + 1]) return;
  int k = 1;
  for (int q = 2; q <= a.d; ++q)
    if (i >= a.off[q]) k = q;
  const double* C = a.C[1];
  const double* mult = a.mult[1];
  int64_t bk = a.bk[1];
#pragma unroll
  for (int q = 2; q <= CUM_MAXD; ++q)
    if (k == q) {
      C = a.C[q];
      mult = a.mult[q];
      bk = a.bk[q];
    }
  const int64_t e = i - a.off[k];
  a.Cbar[i] = 2.0 * a.w[k] * mult[e / bk] * C[e];
}

// Y_bar by stored blocks.  For a block with columns c_q + a (q < S, a < b)
// and values Mb[a_0 .. a_{S-1}] (the row's derivative of Eq. (mom) is
// Mb * prod of the other positions' y), digit recursion from the outermost
// position: V_q(a_0..a_q) = sum over the inner digits of Mb * prod_{q' > q}
// y_{q'}; position q's column gains prefix_q * V_q, prefix_q = prod_{q' < q}
// y_{q'}; V_{S-1} = Mb and V_q = sum_{a_{q+1}} y_{q+1} V_{q+1}.  Each lane owns
// one row: ys / acc hold its y values and sums column-major (col * 64 + lane).
template <int S, int Q>
__device__ __forceinline__ double yb_rec(const double* __restrict__ Mb, int e, double pre, const int (&cb)[S],
                                         int b, const float* ys, double* acc, int lane) {
  double W = 0.0;
  for (int a = 0; a < b; ++a) {
    const int col = cb[Q] + a;
    const double y = (double)ys[col * 64 + lane];
    const int ee = e * b + a;
    double V;
    if constexpr (Q == S - 1) V = Mb[ee];
    else V = yb_rec<S, Q + 1>(Mb, ee, pre * y, cb, b, ys, acc, lane);
    acc[col * 64 + lane] += pre * V;
    W += y * V;
  }
  return W;
}

constexpr int YB_MSTAGE = 1024;  // block values staged in LDS (larger blocks read global memory)

// The same recursion with a compile-time block size B: fully unrolled, the
// block's y values and each position's column sums held in registers (added
// to the row's LDS sums once per block), the values read from LDS with
// immediate offsets.  For blocks of at most YB_MSTAGE values.
template <int S, int B, int Q>
__device__ __forceinline__ double yb_rec_fixed(const double* __restrict__ ms, int e, double pre,
                                               const float (&yv)[S][B], double (&av)[S][B]) {
  double W = 0.0;
#pragma unroll
  for (int a = 0; a < B; ++a) {
    const double y = (double)yv[Q][a];
    const int ee = e * B + a;
    double V;
    if constexpr (Q == S - 1) V = ms[ee];
    else V = yb_rec_fixed<S, B, Q + 1>(ms, ee, pre * y, yv, av);
    av[Q][a] += pre * V;
    W += y * V;
  }
  return W;
}

template <int S, int B>
__device__ __forceinline__ void yb_block_fixed(const double* ms, const int (&cb)[S], const float* ys, double* acc,
                                               int lane) {
  float yv[S][B];
  double av[S][B];
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int a = 0; a < B; ++a) {
      yv[q][a] = ys[(cb[q] + a) * 64 + lane];
      av[q][a] = 0.0;
    }
  (void)yb_rec_fixed<S, B, 0>(ms, 0, 1.0, yv, av);
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int a = 0; a < B; ++a) acc[(cb[q] + a) * 64 + lane] += av[q][a];
}

template <int S, int B>
constexpr bool yb_fixed_ok() {
  int bs = 1;
  for (int q = 0; q < S; ++q) bs *= B;
  return bs <= 256;
}

template <int S>
__device__ __forceinline__ void yb_block(const YbarBlockArgs& a, int64_t blk, const float* ys, double* acc,
                                         double* ms, int lane) {
  int cb[S];
  const uint8_t* tu = a.tuples[S] + blk * S;
#pragma unroll
  for (int q = 0; q < S; ++q) cb[q] = (int)tu[q] * a.b;
  int bs = 1;
#pragma unroll
  for (int q = 0; q < S; ++q) bs *= a.b;
  const double* src = a.Mbar[S] + blk * bs;
  if (bs <= YB_MSTAGE) {
    // the block's values once, coalesced, then broadcast reads from LDS
    __syncthreads();
    for (int i = lane; i < bs; i += 64) ms[i] = src[i];
    __syncthreads();
    if constexpr (yb_fixed_ok<S, 4>()) {
      if (a.b == 4) { yb_block_fixed<S, 4>(ms, cb, ys, acc, lane); return; }
    }
    if constexpr (yb_fixed_ok<S, 2>()) {
      if (a.b == 2) { yb_block_fixed<S, 2>(ms, cb, ys, acc, lane); return; }
    }
    if constexpr (yb_fixed_ok<S, 8>()) {
      if (a.b == 8) { yb_block_fixed<S, 8>(ms, cb, ys, acc, lane); return; }
    }
    (void)yb_rec<S, 0>(ms, 0, 1.0, cb, a.b, ys, acc, lane);
  } else {
    (void)yb_rec<S, 0>(src, 0, 1.0, cb, a.b, ys, acc, lane);
  }
}

__global__ __launch_bounds__(64) void k_ybar_blocks(YbarBlockArgs a) {
  // dynamic LDS: the block values, then the row sums, then the row values
  extern __shared__ __attribute__((aligned(16))) double yb_lds[];
  double* ms = yb_lds;
  double* acc = yb_lds + YB_MSTAGE;
  float* ys = (float*)(acc + a.ncols * 64);
  const int lane = threadIdx.x;
  const int64_t l = (int64_t)blockIdx.x * 64 + lane;
  const int g = blockIdx.y;
  for (int c = 0; c < a.ncols; ++c) {
    ys[c * 64 + lane] = (l < a.t && c < a.n) ? a.Y[l * a.n + c] : 0.0f;
    acc[c * 64 + lane] = 0.0;
  }
  for (int i = a.gptr[g]; i < a.gptr[g + 1]; ++i) {
    const int32_t it = a.items[i];
    const int s = it >> 28;
    const int64_t blk = it & ((1 << 28) - 1);
    switch (s) {
      case 1: yb_block<1>(a, blk, ys, acc, ms, lane); break;
      case 2: yb_block<2>(a, blk, ys, acc, ms, lane); break;
      case 3: yb_block<3>(a, blk, ys, acc, ms, lane); break;
      case 4: yb_block<4>(a, blk, ys, acc, ms, lane); break;
      case 5: yb_block<5>(a, blk, ys, acc, ms, lane); break;
      case 6: yb_block<6>(a, blk, ys, acc, ms, lane); break;
      default: break;
    }
  }
  if (l < a.t)
    for (int c = 0; c < a.n; ++c) a.part[((int64_t)g * a.t + l) * a.n + c] = acc[c * 64 + lane];
}

// ---------------------------------------------------------------------------
// Reverse combine.

// Offset, in an order-S block (positions ascending, the first slowest), of
// the base-b digits of v placed on the positions of mask (the mask's first
// position slowest); pw[q] = b^(S-1-q).
template <int S>
__device__ __forceinline__ int spread(int v, int mask, int b, int lb, const int (&pw)[S]) {
  int e = 0;
#pragma unroll
  for (int q = S - 1; q >= 0; --q) {
    if (mask & (1 << q)) {
      int d;
      if (lb >= 0) {
        d = v & (b - 1);
        v >>= lb;
      } else {
        d = v % b;
        v /= b;
      }
      e += d * pw[q];
    }
  }
  return e;
}

template <int S>
__global__ __launch_bounds__(256) void k_rev_block(RevBlockArgs a) {
  constexpr int NM = 1 << S;
  constexpr int FULL = NM - 1;
  // the moments m_R of every proper sub-block at moff[R], the block's C_bar at tot
  extern __shared__ __attribute__((aligned(16))) double lds[];
  __shared__ int moff[NM];
  __shared__ int64_t subbase[NM];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int b = a.b;
  const int lb = (b & (b - 1)) == 0 ? __builtin_ctz((unsigned)b) : -1;
  const int tot = a.tot;
  int pw[S];
  {
    int p = 1;
#pragma unroll
    for (int q = S - 1; q >= 0; --q) {
      pw[q] = p;
      p *= b;
    }
  }
  if (tid == 0) {
    int off = 0;
    for (int m = 1; m < FULL; ++m) {
      moff[m] = off;
      int bl = 1;
      for (int q = 0; q < __builtin_popcount(m); ++q) bl *= b;
      off += bl;
    }
    moff[FULL] = off;
  }
  if (tid > 0 && tid < FULL) {
    int64_t bl = 1;
    for (int q = 0; q < __builtin_popcount(tid); ++q) bl *= b;
    subbase[tid] = (int64_t)a.subrank[blk * NM + tid] * bl;
  }
  __syncthreads();
  // stage, four items per thread and pass with their loads issued together
  for (int i0 = tid; i0 < tot; i0 += 4 * 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 256;
      v[u] = 0.0;
      if (i < tot) {
        int lo = 1, hi = FULL - 1;  // the mask m with moff[m] <= i < moff[m + 1]
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (moff[mid] <= i) lo = mid;
          else hi = mid - 1;
        }
        const int q = __builtin_popcount(lo);
        const float* h = a.Shi[1];
        const float* l = a.Slo[1];
#pragma unroll
        for (int k = 2; k < S; ++k)
          if (q == k) {
            h = a.Shi[k];
            l = a.Slo[k];
          }
        const int64_t src = subbase[lo] + (i - moff[lo]);
        v[u] = ((double)h[src] + (double)l[src]) * a.inv_t;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * 256 < tot) lds[i0 + u * 256] = v[u];
  }
  for (int64_t i = tid; i < a.bs; i += 256) lds[tot + i] = a.Cbar_s[blk * a.bs + i];
  __syncthreads();
  const double* gbar = lds + tot;
  for (int m = 1; m < FULL; ++m) {
    const int rc = FULL & ~m;
    int size = 1, cnt = 1;
    for (int q = 0; q < S; ++q) {
      if (m & (1 << q)) size *= b;
      else cnt *= b;
    }
    // G lanes (a power of two dividing the wave) share one output
    int G = 1;
    while (G < 64 && G * 2 * size <= 256) G *= 2;
    const int lg = __builtin_ctz((unsigned)G);
    for (int base = 0; base < size * G; base += 256) {
      const int i = base + tid;
      const int x = i >> lg, g = i & (G - 1);
      double acc = 0.0;
      if (x < size) {
        const int ex = spread<S>(x, m, b, lb, pw);
        const double* mr = lds + moff[rc];
        for (int y = g; y < cnt; y += G) acc += gbar[ex + spread<S>(y, rc, b, lb, pw)] * mr[y];
      }
      for (int w = 1; w < G; w <<= 1) acc += __shfl_xor(acc, w, 64);
      if (x < size && g == 0) a.part[blk * tot + moff[m] + x] = -acc;
    }
  }
}

// One workgroup per lower-order block; T lanes (a power of two dividing the
// wave) share each of its elements, lane g summing entries g, g + T, ...,
// then a butterfly over the T lanes.
__global__ __launch_bounds__(256) void k_rev_collect(RevCollectArgs a, int s) {
  __shared__ int moff[64];
  const int tid = threadIdx.x;
  if (tid < 64) moff[tid] = a.moff[tid];
  __syncthreads();
  const int64_t q = blockIdx.x;  // block among the lower orders, concatenated
  int sp = 1;
  for (int k = 2; k < s; ++k)
    if (q >= a.bstart[k]) sp = k;
  const int64_t beta = q - a.bstart[sp];
  const int bk = (int)a.bk[sp];
  int T = 1;
  while (T < 64 && T * 2 * bk <= 256) T *= 2;
  const int lt = __builtin_ctz((unsigned)T);
  const int32_t e0 = a.ptr[q], e1 = a.ptr[q + 1];
  double* cb = a.Cbar[1];
#pragma unroll
  for (int k = 2; k < CUM_MAXD; ++k)
    if (sp == k) cb = a.Cbar[k];
  const int per = 256 >> lt;  // elements per pass
  for (int x0 = 0; x0 < bk; x0 += per) {
    const int x = x0 + (tid >> lt), g = tid & (T - 1);
    double sum = 0.0;
    if (x < bk)
      for (int32_t e = e0 + g; e < e1; e += T) {
        const int32_t v = a.ent[e];
        sum += a.part[(int64_t)(v >> 6) * a.tot + moff[v & 63] + x];
      }
    for (int w = 1; w < T; w <<= 1) sum += __shfl_xor(sum, w, 64);
    if (x < bk && g == 0) cb[beta * bk + x] += sum;
  }
}

// ---------------------------------------------------------------------------
// Y_bar on FP64 matrix cores.

__global__ __launch_bounds__(256) void k_gbuild(GbuildArgs a) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= a.rows) return;
  double acc = 0.0;
  for (int64_t e = a.ptr[r]; e < a.ptr[r + 1]; ++e) {
    const int64_t v = a.ent[e];
    acc += (double)(v >> 48) * a.Mbar[v & ((int64_t(1) << 48) - 1)];
  }
  a.G[r] = acc * a.inv_t;
}

typedef double f64x4v __attribute__((ext_vector_type(4)));

// One workgroup: YB_ROWS rows of Y (32 per wave: two 16-row fragments that
// share every B operand) times the split's rows of G.  A lane supplies
// A[row = lane % 16][k = lane / 16] = the product of its row's factors for
// G row k, and B[k = lane / 16][col = lane % 16].
constexpr int YB_ROWS = 128;

template <int NC, int F>
__global__ __launch_bounds__(256) void k_ybar_mma(YbarMmaArgs a) {
  extern __shared__ __attribute__((aligned(16))) double ys[];  // YB_ROWS x (n + 1)
  const int n = a.n, np = n + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * YB_ROWS;
  // the split's factor words follow the row tile in LDS
  uint64_t* fl = (uint64_t*)(ys + YB_ROWS * np);
  for (int i = tid; i < YB_ROWS * np; i += 256) {
    const int r = i / np, c = i - r * np;
    const int64_t l = r0 + r;
    ys[i] = c == n ? 1.0 : (l < a.t ? (double)a.Y[l * n + c] : 0.0);
  }
  for (int i = tid; i < a.kper; i += 256) fl[i] = a.facs[(int64_t)blockIdx.y * a.kper + i];
  __syncthreads();
  const double* yr0 = ys + (wave * 32 + (lane & 15)) * np;
  const double* yr1 = yr0 + 16 * np;
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t k0 = (int64_t)blockIdx.y * a.kper;
  const double* gp = a.G + (k0 + kq) * a.ncol + cl;
  f64x4v acc[2][NC];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[f][c] = f64x4v{0.0, 0.0, 0.0, 0.0};
  // four k-steps per batch, two batches per iteration (kper is a multiple of
  // 32); the next batch's global loads are issued before this batch's
  // products, unconditionally (clamped to the split's last batch, so the
  // loop has no branch and the load counters stay exact)
  uint64_t fc[2][4];
  double gv[2][4][NC];
  auto load = [&](int kk, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      fc[buf][u] = fl[kk + 4 * u + kq];
      const double* g = gp + (int64_t)(kk + 4 * u) * a.ncol;
#pragma unroll
      for (int c = 0; c < NC; ++c) gv[buf][u][c] = g[c * 16];
    }
    // keep the loads here: left alone, the scheduler sinks each to its use
    __builtin_amdgcn_sched_barrier(0);
  };
  auto step = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t f = fc[buf][u];
      double a0 = yr0[f & 0xff], a1 = yr1[f & 0xff];
#pragma unroll
      for (int q = 1; q < F; ++q) {
        const int j = (int)((f >> (8 * q)) & 0xff);
        a0 *= yr0[j];
        a1 *= yr1[j];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[0][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, gv[buf][u][c], acc[0][c], 0, 0, 0);
        acc[1][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, gv[buf][u][c], acc[1][c], 0, 0, 0);
      }
    }
  };
  const int last = a.kper - 16;
  load(0, 0);
  for (int kk = 0; kk < a.kper; kk += 32) {
    load(kk + 16, 1);
    step(0);
    load(min(kk + 32, last), 0);
    step(1);
  }
  // lane holds rows lane / 16 + 4 r of each fragment, column lane % 16
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t l = r0 + wave * 32 + f * 16 + kq + 4 * r;
        const int col = c * 16 + cl;
        if (l < a.t && col < n) a.part[((int64_t)blockIdx.y * a.t + l) * n + col] = acc[f][c][r];
      }
}

// Y_bar for a tile of 64 rows (its split partials summed in split order),
// then dX for the tile and the tile's dW partial.
__global__ __launch_bounds__(256) void k_ybar_finish(const double* __restrict__ part, int splits, double scale,
                                                     const float* __restrict__ X, const float* __restrict__ W,
                                                     float* __restrict__ dX, double* __restrict__ dwpart, int64_t t,
                                                     int n) {
  __shared__ double yb[64 * 64];
  __shared__ float xs[64 * 64];
  __shared__ float ws[64 * 64];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int rows = (int)(t - r0 < 64 ? t - r0 : 64);
  for (int i = tid; i < 64 * n; i += 256) {
    const int r = i / n, c = i - r * n;
    const int64_t l = r0 + r;
    double s = 0.0;
    if (r < rows) {
      // up to 16 splits' loads in flight, added in split order
      for (int k0 = 0; k0 < splits; k0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = k0 + u < splits ? part[((int64_t)(k0 + u) * t + l) * n + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (k0 + u < splits) s += v[u];
      }
    }
    yb[i] = s * scale;
    xs[i] = r < rows ? X[l * n + c] : 0.0f;
  }
  for (int i = tid; i < n * n; i += 256) ws[i] = W[i];
  __syncthreads();
  for (int i = tid; i < rows * n; i += 256) {
    const int r = i / n, j = i - r * n;
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc += yb[r * n + q] * (double)ws[q * n + j];
    dX[(r0 + r) * n + j] = (float)acc;
  }
  for (int i = tid; i < n * n; i += 256) {
    const int p = i / n, j = i - p * n;
    double acc = 0.0;
    for (int r = 0; r < rows; ++r) acc += yb[r * n + p] * (double)xs[r * n + j];
    dwpart[(int64_t)blockIdx.x * n * n + i] = acc;
  }
}

// dW: 64 outputs per workgroup (one per lane), wave w summing tiles w, w + 16,
// ...; the 16 wave sums then added in wave order.
__global__ __launch_bounds__(1024) void k_dw_sum(const double* __restrict__ dwpart, int tiles, int n,
                                                 float* __restrict__ dW) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int nn = n * n;
  double s = 0.0;
  if (i < nn)
    for (int k = wave; k < tiles; k += 16) s += dwpart[(int64_t)k * nn + i];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && i < nn) {
    double t = red[0][lane];
    for (int w = 1; w < 16; ++w) t += red[w][lane];
    dW[i] = (float)t;
  }
}

hipError_t launch_linear(const float* X, const float* W, float* Y, int64_t t, int n, hipStream_t st) {
  if (n < 1 || n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_linear, dim3((unsigned)((t + 63) / 64)), dim3(256), 0, st, X, W, Y, t, n);
  return hipGetLastError();
}

hipError_t launch_cbar_init(const CbarArgs& a, hipStream_t st) {
  const int64_t tot = a.off[a.d + 1];
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cbar_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_rev_block(int s, const RevBlockArgs& a, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), blk(256);
  const size_t lds = (size_t)(a.tot + a.bs) * sizeof(double);
  if (a.tot + a.bs > REV_LDS_DOUBLES) return hipErrorInvalidValue;
  switch (s) {
    case 2: hipLaunchKernelGGL(k_rev_block<2>, grid, blk, lds, st, a); break;
    case 3: hipLaunchKernelGGL(k_rev_block<3>, grid, blk, lds, st, a); break;
    case 4: hipLaunchKernelGGL(k_rev_block<4>, grid, blk, lds, st, a); break;
    case 5: hipLaunchKernelGGL(k_rev_block<5>, grid, blk, lds, st, a); break;
    case 6: hipLaunchKernelGGL(k_rev_block<6>, grid, blk, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rev_collect(const RevCollectArgs& a, int s, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rev_collect, dim3((unsigned)nblocks), dim3(256), 0, st, a, s);
  return hipGetLastError();
}

hipError_t launch_gbuild(const GbuildArgs& a, hipStream_t st) {
  if (a.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gbuild, dim3((unsigned)((a.rows + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int NC>
static hipError_t launch_mma_nc(const YbarMmaArgs& a, int F, dim3 grid, hipStream_t st) {
  const size_t lds = (size_t)YB_ROWS * (a.n + 1) * sizeof(double) + (size_t)a.kper * sizeof(uint64_t);
  switch (F) {
    case 1: hipLaunchKernelGGL((k_ybar_mma<NC, 1>), grid, dim3(256), lds, st, a); break;
    case 2: hipLaunchKernelGGL((k_ybar_mma<NC, 2>), grid, dim3(256), lds, st, a); break;
    case 3: hipLaunchKernelGGL((k_ybar_mma<NC, 3>), grid, dim3(256), lds, st, a); break;
    case 4: hipLaunchKernelGGL((k_ybar_mma<NC, 4>), grid, dim3(256), lds, st, a); break;
    case 5: hipLaunchKernelGGL((k_ybar_mma<NC, 5>), grid, dim3(256), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ybar_mma(const YbarMmaArgs& a, int F, int splits, hipStream_t st) {
  if (a.n < 1 || a.n > 64 || a.kper % 32 || a.kper < 32 || a.kper > YB_MAX_KPER || splits < 1)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.t + YB_ROWS - 1) / YB_ROWS), (unsigned)splits);
  switch (a.ncol / 16) {
    case 1: return launch_mma_nc<1>(a, F, grid, st);
    case 2: return launch_mma_nc<2>(a, F, grid, st);
    case 3: return launch_mma_nc<3>(a, F, grid, st);
    case 4: return launch_mma_nc<4>(a, F, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ybar_finish(const double* part, int splits, double scale, const float* X, const float* W,
                              float* dX, double* dwpart, float* dW, int64_t t, int n, hipStream_t st) {
  if (n < 1 || n > 64) return hipErrorInvalidValue;
  const int64_t tiles = (t + 63) / 64;
  hipLaunchKernelGGL(k_ybar_finish, dim3((unsigned)tiles), dim3(256), 0, st, part, splits, scale, X, W, dX, dwpart,
                     t, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dw_sum, dim3((unsigned)((n * n + 63) / 64)), dim3(1024), 0, st, dwpart, (int)tiles, n, dW);
  return hipGetLastError();
}

hipError_t launch_ybar_blocks(const YbarBlockArgs& a, int groups, hipStream_t st) {
  if (a.ncols > YB_MAXCOLS || groups < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.t + 63) / 64), (unsigned)groups);
  const size_t lds = (size_t)YB_MSTAGE * 8 + (size_t)a.ncols * 64 * 12;
  hipLaunchKernelGGL(k_ybar_blocks, grid, dim3(64), lds, st, a);
  return hipGetLastError();
}

}  // namespace cum
