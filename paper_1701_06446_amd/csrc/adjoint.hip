// Adjoint of L = sum_k w_k ||C_k(Y)||_F^2 with Y = X W^T (single window).
//
// Forward: Y = X W^T, then the library's moment contraction, combine and
// norms on Y.  Reverse, in FP64:
//   k_cbar_init     C_bar_k = 2 w_k mult(block) c  for every stored element
//                   (the loss of Alg. 5 differentiated element by element);
//   k_combine_rev   Alg. 4 run backwards, orders d..2: every stored element e
//                   of order s passes C_bar_s[e] to its moment (M_bar_s = the
//                   final C_bar_s) and -C_bar_s[e] * (product of the other
//                   parts) to the lower-order cumulant at every part of every
//                   partition;
//   k_ybar_blocks   Y_bar[l, j] = sum over stored elements e that contain
//                   column j: count_j(e) * M_bar[e] / t * prod of y[l, i] over
//                   e's other indices (the derivative of Eq. (mom)), block by
//                   block with a digit recursion, then k_ybar_sum;
//   k_dx / k_dw     dX = Y_bar W, dW = Y_bar^T X (fixed-order sums).
// The reverse combine adds contributions from many blocks into the same
// lower-order entries with FP64 atomics, so it is deterministic up to the
// order of those additions.
#include <hip/hip_runtime.h>

#include "adjoint.h"
#include "partitions.h"

namespace cum {

__global__ __launch_bounds__(256) void k_linear(const float* __restrict__ X, const float* __restrict__ W,
                                                float* __restrict__ Y, int64_t t, int n) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= t * n) return;
  const int64_t l = o / n;
  const int i = (int)(o - l * n);
  float acc = 0.0f;
  for (int j = 0; j < n; ++j) acc = fmaf(X[l * n + j], W[(int64_t)i * n + j], acc);
  Y[o] = acc;
}

__global__ __launch_bounds__(256) void k_cbar_init(const double* __restrict__ C, const double* __restrict__ mult,
                                                   double* __restrict__ Cbar, int64_t nelems, int64_t bk,
                                                   double two_w) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nelems) return;
  Cbar[e] = two_w * mult[e / bk] * C[e];
}

template <int S>
__global__ __launch_bounds__(256) void k_combine_rev(RevArgs a) {
  constexpr int NM = 1 << S;
  constexpr int FULL = NM - 1;
  extern __shared__ __attribute__((aligned(16))) double lds[];  // staged c, then gradients
  __shared__ int64_t subbase[NM];
  __shared__ int lds_off[NM + 1];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int b = a.b;
  if (tid == 0) {
    int off = 0;
    for (int mask = 1; mask < FULL; ++mask) {
      int bl = 1;
      for (int q = 0; q < __builtin_popcount(mask); ++q) bl *= b;
      lds_off[mask] = off;
      off += bl;
    }
    lds_off[FULL] = off;
  }
  if (tid > 0 && tid < FULL) {
    int64_t bl = 1;
    for (int q = 0; q < __builtin_popcount(tid); ++q) bl *= b;
    subbase[tid] = (int64_t)a.subrank[blk * NM + tid] * bl;
  }
  __syncthreads();
  const int total = lds_off[FULL];
  double* stage = lds;
  double* grad = lds + total;
  for (int i = tid; i < total; i += 256) {
    int mask = 1;
    while (mask + 1 < FULL && lds_off[mask + 1] <= i) ++mask;
    stage[i] = a.C[__builtin_popcount(mask)][subbase[mask] + (i - lds_off[mask])];
    grad[i] = 0.0;
  }
  __syncthreads();
  for (int64_t e = tid; e < a.bs; e += 256) {
    const double g = a.Cbar[S][blk * a.bs + e];
    int dig[S];
    int64_t rem = e;
#pragma unroll
    for (int q = S - 1; q >= 0; --q) {
      dig[q] = (int)(rem % b);
      rem /= b;
    }
    int off[NM];
    double cB[NM];
#pragma unroll
    for (int mask = 1; mask < FULL; ++mask) {
      int o = 0;
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (mask & (1 << q)) o = o * b + dig[q];
      off[mask] = lds_off[mask] + o;
      cB[mask] = stage[off[mask]];
    }
#pragma unroll
    for (int p = 0; p < kParts<S>.count; ++p) {
#pragma unroll
      for (int q = 0; q < S; ++q) {
        if (q < kParts<S>.nparts[p]) {
          double others = -g;
#pragma unroll
          for (int r = 0; r < S; ++r)
            if (r < kParts<S>.nparts[p] && r != q) others *= cB[kParts<S>.mask[p][r]];
          atomicAdd(&grad[off[kParts<S>.mask[p][q]]], others);
        }
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < total; i += 256) {
    int mask = 1;
    while (mask + 1 < FULL && lds_off[mask + 1] <= i) ++mask;
    const double v = grad[i];
    if (v != 0.0) atomicAdd(&a.Cbar[__builtin_popcount(mask)][subbase[mask] + (i - lds_off[mask])], v);
  }
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

__global__ __launch_bounds__(256) void k_ybar_sum(const double* __restrict__ part, int groups, int64_t t, int n,
                                                  double inv_t, double* __restrict__ Ybar) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= t * n) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += part[(int64_t)g * t * n + o];
  Ybar[o] = s * inv_t;
}

__global__ __launch_bounds__(256) void k_dx(const double* __restrict__ Ybar, const float* __restrict__ W,
                                            float* __restrict__ dX, int64_t t, int n) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= t * n) return;
  const int64_t l = o / n;
  const int j = (int)(o - l * n);
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += Ybar[l * n + i] * (double)W[(int64_t)i * n + j];
  dX[o] = (float)acc;
}

__global__ __launch_bounds__(256) void k_dw(const double* __restrict__ Ybar, const float* __restrict__ X,
                                            float* __restrict__ dW, int64_t t, int n) {
  __shared__ double red[256];
  const int i = blockIdx.x / n, j = blockIdx.x % n;
  double acc = 0.0;
  for (int64_t l = threadIdx.x; l < t; l += 256) acc += Ybar[l * n + i] * (double)X[l * n + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dW[blockIdx.x] = (float)red[0];
}

hipError_t launch_linear(const float* X, const float* W, float* Y, int64_t t, int n, hipStream_t st) {
  const int64_t tot = t * n;
  hipLaunchKernelGGL(k_linear, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, W, Y, t, n);
  return hipGetLastError();
}

hipError_t launch_cbar_init(const double* C, const double* mult, double* Cbar, int64_t nelems, int64_t bk,
                            double two_w, hipStream_t st) {
  if (nelems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cbar_init, dim3((unsigned)((nelems + 255) / 256)), dim3(256), 0, st, C, mult, Cbar,
                     nelems, bk, two_w);
  return hipGetLastError();
}

hipError_t launch_combine_rev(int s, const RevArgs& a, int64_t nblocks, size_t lds_bytes, hipStream_t st) {
  const dim3 grid((unsigned)nblocks), blk(256);
  switch (s) {
    case 2: hipLaunchKernelGGL(k_combine_rev<2>, grid, blk, lds_bytes, st, a); break;
    case 3: hipLaunchKernelGGL(k_combine_rev<3>, grid, blk, lds_bytes, st, a); break;
    case 4: hipLaunchKernelGGL(k_combine_rev<4>, grid, blk, lds_bytes, st, a); break;
    case 5: hipLaunchKernelGGL(k_combine_rev<5>, grid, blk, lds_bytes, st, a); break;
    case 6: hipLaunchKernelGGL(k_combine_rev<6>, grid, blk, lds_bytes, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ybar_blocks(const YbarBlockArgs& a, int groups, hipStream_t st) {
  if (a.ncols > YB_MAXCOLS || groups < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.t + 63) / 64), (unsigned)groups);
  const size_t lds = (size_t)YB_MSTAGE * 8 + (size_t)a.ncols * 64 * 12;
  hipLaunchKernelGGL(k_ybar_blocks, grid, dim3(64), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_ybar_sum(const double* part, int groups, int64_t t, int n, double inv_t, double* Ybar,
                           hipStream_t st) {
  const int64_t tot = t * n;
  hipLaunchKernelGGL(k_ybar_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part, groups, t, n, inv_t,
                     Ybar);
  return hipGetLastError();
}

hipError_t launch_dx_dw(const double* Ybar, const float* X, const float* W, float* dX, float* dW, int64_t t,
                        int n, hipStream_t st) {
  const int64_t tot = t * n;
  hipLaunchKernelGGL(k_dx, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Ybar, W, dX, t, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dw, dim3((unsigned)(n * n)), dim3(256), 0, st, Ybar, X, dW, t, n);
  return hipGetLastError();
}

}  // namespace cum
