// Adjoint kernels for L = sum_k w_k ||C_k(X W^T)||_F^2 (argument blocks and
// launch wrappers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cum_internal.h"

namespace cum {

struct RevArgs {
  int b;
  int64_t bs;                       // b^s of the order being reversed
  const int32_t* subrank;           // order-s sub-tuple ranks
  const double* C[CUM_MAXD + 1];    // forward cumulants
  double* Cbar[CUM_MAXD + 1];       // gradients w.r.t. the stored cumulants
};

// Y_bar by stored blocks: grid (row tiles of 64, block groups); group g
// covers items[gptr[g] .. gptr[g+1]) of (order << 28 | block); partial sums
// part[g][row][col], then summed over g in index order.
constexpr int YB_MAXCOLS = 72;  // ceil(n/b)*b for n <= 64, b <= 8

struct YbarBlockArgs {
  int n, b, ncols;                  // ncols = ceil(n/b)*b
  int64_t t;
  const float* Y;
  const double* Mbar[CUM_MAXD + 1];
  const uint8_t* tuples[CUM_MAXD + 1];
  const int32_t* items;
  const int32_t* gptr;
  double* part;                     // groups x t x n
};

hipError_t launch_ybar_blocks(const YbarBlockArgs& a, int groups, hipStream_t st);
hipError_t launch_ybar_sum(const double* part, int groups, int64_t t, int n, double inv_t, double* Ybar,
                           hipStream_t st);

hipError_t launch_linear(const float* X, const float* W, float* Y, int64_t t, int n, hipStream_t st);
hipError_t launch_cbar_init(const double* C, const double* mult, double* Cbar, int64_t nelems, int64_t bk,
                            double two_w, hipStream_t st);
hipError_t launch_combine_rev(int s, const RevArgs& a, int64_t nblocks, size_t lds_bytes, hipStream_t st);
hipError_t launch_dx_dw(const double* Ybar, const float* X, const float* W, float* dX, float* dW, int64_t t,
                        int n, hipStream_t st);

}  // namespace cum
