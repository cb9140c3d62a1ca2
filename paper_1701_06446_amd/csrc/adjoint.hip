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
//   k_ybar          Y_bar[l, j] = sum over stored elements e that contain
//                   column j: count_j(e) * M_bar[e] / t * prod of y[l, i] over
//                   e's other indices (the derivative of Eq. (mom));
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

// Y_bar for a tile of 256 rows and one column j; the tile's rows of Y are
// staged in LDS.  Entries of column j: (order, element, count, other indices).
__global__ __launch_bounds__(256) void k_ybar(YbarArgs a) {
  extern __shared__ __attribute__((aligned(16))) float ytile[];
  const int tid = threadIdx.x;
  const int64_t l0 = (int64_t)blockIdx.x * 256;
  const int j = blockIdx.y;
  const int n = a.n;
  const int rows = (int)min((int64_t)256, a.t - l0);
  for (int i = tid; i < rows * n; i += 256) ytile[i] = a.Y[l0 * n + i];
  __syncthreads();
  if (tid >= rows) return;
  const float* yr = ytile + tid * n;
  double acc = 0.0;
  for (int64_t q = a.colptr[j]; q < a.colptr[j + 1]; ++q) {
    const YbarEntry en = a.entries[q];
    double v = (double)en.cnt * a.Mbar[en.s][en.off];
    for (int r = 0; r < en.s - 1; ++r) v *= (double)yr[en.oth[r]];
    acc += v;
  }
  a.Ybar[(l0 + tid) * n + j] = acc * a.inv_t;
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

hipError_t launch_ybar(const YbarArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.t + 255) / 256), (unsigned)a.n);
  hipLaunchKernelGGL(k_ybar, grid, dim3(256), (size_t)256 * a.n * sizeof(float), st, a);
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
