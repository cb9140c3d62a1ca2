// Adjoint kernels for L = sum_k w_k ||C_k(X W^T)||_F^2 (argument blocks and
// launch wrappers).  Every sum is taken in a fixed order: repeated calls on
// the same inputs give bitwise equal results.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cum_internal.h"

namespace cum {

// Reverse combine of one order s (Alg. 4 backwards), in two deterministic
// passes.  k_rev_block: one workgroup per order-s block computes, for every
// proper non-empty sub-block mask B and sub-block element x,
//   part[blk][moff(B) + x] = - sum_y C_bar_s[x (+) y] m_{B^c}[y],
// the gradient of the block's cumulants w.r.t. c_B at x (the parts of the
// partitions holding B other than B itself multiply to the moment m_{B^c}).
// k_rev_collect: every element of the lower orders adds, in increasing
// (block, mask) order, the partials of the (block, mask) pairs whose
// sub-tuple is its block.
struct RevBlockArgs {
  int b;
  int64_t bs;                       // b^s
  int tot;                          // (b+1)^s - 1 - b^s partials per block
  const int32_t* subrank;           // order-s sub-tuple ranks
  const double* Cbar_s;             // final C_bar of order s
  const float* Shi[CUM_MAXD + 1];   // running sums of the lower orders
  const float* Slo[CUM_MAXD + 1];
  double inv_t;
  double* part;                     // nblocks(s) x tot
};

struct RevCollectArgs {
  int b;
  int tot;
  int moff[64];                     // partial offset of each mask (masks 1 .. 2^s - 2)
  int64_t estart[CUM_MAXD + 1];     // first element of order s' among the lower orders; estart[s] = end
  int64_t bstart[CUM_MAXD + 1];     // first block of order s' in ptr
  int64_t bk[CUM_MAXD + 1];         // b^s'
  const int32_t* ptr;               // entries of lower-order block q: ent[ptr[q] .. ptr[q+1])
  const int32_t* ent;               // (order-s block << 6) | mask
  const double* part;
  double* Cbar[CUM_MAXD + 1];
};

// Y_bar = P G on FP64 matrix cores: P[l, J] = prod of y[l, i] over the
// sorted tuple J (orders 0 .. d-1; factor index n reads 1), formed per lane
// from the row tile in LDS; G[J, j] = (1/t) sum over the stored moments
// containing J and j of (multiplicity of j) M_bar (gathered by k_gbuild).
// Row tiles of 128 over grid.x, K split over grid.y; part[split][l][j] is
// summed in split order.
constexpr int YB_MAX_KPER = 4096;  // rows of G per split (their factor words sit in LDS)

struct YbarMmaArgs {
  int n, ncol;                      // ncol = G's padded width (16 per fragment)
  int64_t t;
  int kper;                         // rows of G per split (a multiple of 32)
  const float* Y;
  const uint64_t* facs;             // per G row: factor column indices, one byte each
  const double* G;                  // kpad x ncol
  double* part;                     // splits x t x n
};

struct GbuildArgs {
  int64_t rows;                     // kpad * ncol
  const int64_t* ptr;               // entries of G row r: ent[ptr[r] .. ptr[r+1])
  const int64_t* ent;               // offset into the concatenated M_bar | (count << 48)
  const double* Mbar;
  double inv_t;
  double* G;
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

hipError_t launch_linear(const float* X, const float* W, float* Y, int64_t t, int n, hipStream_t st);
// C_bar = 2 w_k mult(block) c for every stored element of every order, the
// orders concatenated in Cbar (at off[k]); w (device, d+1 values) is read
// by the kernel, so a captured launch follows the caller's weights.
struct CbarArgs {
  int d;
  int64_t off[CUM_MAXD + 2];
  int64_t bk[CUM_MAXD + 1];
  const double* C[CUM_MAXD + 1];
  const double* mult[CUM_MAXD + 1];
  const double* w;
  double* Cbar;
};
hipError_t launch_cbar_init(const CbarArgs& a, hipStream_t st);
hipError_t launch_rev_block(int s, const RevBlockArgs& a, int64_t nblocks, hipStream_t st);
// one workgroup per block of the lower orders (nblocks of them, concatenated)
hipError_t launch_rev_collect(const RevCollectArgs& a, int s, int64_t nblocks, hipStream_t st);
hipError_t launch_gbuild(const GbuildArgs& a, hipStream_t st);
// F = d - 1 factors per G row (1..5), ncol / 16 = 1..4 column fragments
hipError_t launch_ybar_mma(const YbarMmaArgs& a, int F, int splits, hipStream_t st);
// Y_bar = sum of the split partials (scaled by `scale`), then dX = Y_bar W
// and per 64-row tile dW partials Y_bar^T X, summed over tiles in order
hipError_t launch_ybar_finish(const double* part, int splits, double scale, const float* X, const float* W,
                              float* dX, double* dwpart, float* dW, int64_t t, int n, hipStream_t st);
// largest (b+1)^s - 1 the reverse block kernel stages (doubles in LDS)
constexpr int REV_LDS_DOUBLES = 19200;

}  // namespace cum
