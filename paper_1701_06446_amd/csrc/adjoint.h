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

// One (stored element, column) pair of Y_bar: the element's order and
// offset, how often the column occurs in it, and its other s-1 indices.
struct YbarEntry {
  int32_t off;
  uint8_t s, cnt;
  uint8_t oth[CUM_MAXD - 1];
};

struct YbarArgs {
  int n;
  int64_t t;
  double inv_t;
  const float* Y;
  const double* Mbar[CUM_MAXD + 1];
  const int64_t* colptr;            // n+1 offsets into entries
  const YbarEntry* entries;
  double* Ybar;                     // t x n
};

hipError_t launch_linear(const float* X, const float* W, float* Y, int64_t t, int n, hipStream_t st);
hipError_t launch_cbar_init(const double* C, const double* mult, double* Cbar, int64_t nelems, int64_t bk,
                            double two_w, hipStream_t st);
hipError_t launch_combine_rev(int s, const RevArgs& a, int64_t nblocks, size_t lds_bytes, hipStream_t st);
hipError_t launch_ybar(const YbarArgs& a, hipStream_t st);
hipError_t launch_dx_dw(const double* Ybar, const float* X, const float* W, float* dX, float* dW, int64_t t,
                        int n, hipStream_t st);

}  // namespace cum
