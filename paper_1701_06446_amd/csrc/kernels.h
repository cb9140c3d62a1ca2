// Kernel argument blocks and launch wrappers (host <-> device interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cum_internal.h"

namespace cum {

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };

// Update tile: UPD_TM x UPD_TN fragments of 16x16 per workgroup; the four
// waves of a workgroup split the rows of every LDS chunk between them.
constexpr int UPD_TM = 2;
constexpr int UPD_TN = 2;
constexpr int UPD_LDS_BYTES = 32768;

struct UpdArgs {
  const void* xp;           // rows entering the window (+1), row-major np x n
  const void* xm;           // rows leaving the window (-1), row-major nm x n
  int np, nm;
  int n, npad;              // data columns, zero-padded columns (nbar*b)
  int stride;               // LDS row stride in elements (npad + 1)
  int chunk;                // rows per LDS chunk (multiple of the MFMA K step)
  const UpdItem* items;
  const LeftCol* left[CUM_MAXD + 1];
  const RightCol* right[CUM_MAXD + 1];
  void* s_hi[CUM_MAXD + 1]; // running window sums, compensated pair
  void* s_lo[CUM_MAXD + 1];
};

struct CombArgs {
  int b, nbar;
  int64_t bs;               // b^s
  const uint8_t* tuples;    // order-s block tuples
  const int64_t* ntab;      // N(q, y) table, (CUM_MAXD+1) x (nbar+1)
  const void* s_hi;         // order-s running sums (pair)
  const void* s_lo;
  double inv_t;             // 1/t
  const double* C[CUM_MAXD + 1];  // cumulants of orders 1..s-1
  double* Cout;             // order-s cumulants
  const double* mult;       // per-block multiplicity
  double* partial;          // per-block mult * sum(c^2)
};

struct NormArgs {
  int d;
  int64_t nblocks[CUM_MAXD + 1];
  const double* partial[CUM_MAXD + 1];
  double* out;              // [0..d] ||C_k||_F, [d+1 .. 2d+1] nu_k
};

hipError_t launch_update(int prec, const UpdArgs& a, int nitems, hipStream_t st);
hipError_t launch_combine(int prec, int s, const CombArgs& a, int64_t nblocks, hipStream_t st);
hipError_t launch_norms(const NormArgs& a, hipStream_t st);

}  // namespace cum
