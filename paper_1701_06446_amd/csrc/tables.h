// Host-side block enumerator: tables for the update, combine and norm kernels.
#pragma once
#include <stdint.h>

#include <vector>

#include "cum_internal.h"

namespace cum {

struct Pivot {
  int lrow0;   // first row of this pivot in the order's left table
  int nrows;   // M_v = (#left tuples ending at v) * b^h
  int rcol0;   // first column of this pivot in the order's right table
  int ncols;   // N_v = (#right tuples starting at >= v) * b^m
};

struct Tables {
  int n = 0, b = 0, d = 0, nbar = 0, npad = 0;
  OrderInfo ord[CUM_MAXD + 1] = {};
  std::vector<uint8_t> tuples[CUM_MAXD + 1];   // order-k block tuples, k bytes each
  std::vector<double> mult[CUM_MAXD + 1];      // k!/prod(r_l!) per block
  // subrank[s][blk * 2^s + mask]: rank, among the sorted |B|-tuples, of the
  // block tuple restricted to the positions in mask (proper, non-empty B)
  std::vector<int32_t> subrank[CUM_MAXD + 1];
  std::vector<LeftCol> left[CUM_MAXD + 1];
  std::vector<RightCol> right[CUM_MAXD + 1];
  std::vector<Pivot> piv[CUM_MAXD + 1];
};

int64_t binom(int64_t a, int64_t k);
int64_t ipow64(int64_t b, int k);
int build_tables(int n, int b, int d, Tables& T);
std::vector<UpdItem> build_items(const Tables& T, int kmin, int kmax, int tile_rows, int tile_cols);

// The 32 x 32 tiles of build_items in groups of four (one workgroup of the
// four-tile update each), padded with empty tiles (M = N = 0).  A tile costs
// its 16 x 16 fragments inside the pivot GEMM; groups are filled longest
// first, each tile to the open group with the least cost so far, so the
// dearest group (the launch's critical path) stays close to the average.
std::vector<UpdItem> pack_quads(const std::vector<UpdItem>& items);
// Counts how often every stored order-k element is produced by the pivot
// tables; returns the number of (pivot, row, column) triples that land
// outside the pyramid or on an element with different global indices.
int64_t coverage(const Tables& T, int k, std::vector<int32_t>& hits);

}  // namespace cum
