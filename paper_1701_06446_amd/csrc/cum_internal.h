// Internal layout shared by the host-side enumerator and the HIP kernels.
//
// Block structure (Sec. 2.3 / Sec. 4.1 of the paper): an order-k
// super-symmetric tensor over n columns is stored as the blocks whose block
// multi-index j_1 <= ... <= j_k is non-decreasing, listed in lexicographic
// order; each block is a full b^k array, row-major in (a_1..a_k), a_1
// slowest, for global column i_m = j_m*b + a_m.  Columns are zero-padded to
// npad = nbar*b with nbar = ceil(n/b); padded entries are exactly zero.
//
// Update decomposition ("pivot GEMMs").  Split an order-k tuple into a left
// part of order h = ceil(k/2) and a right part of order m = k - h.  For a
// pivot v, the left tuples are the sorted h-tuples whose last index is v and
// the right tuples are the sorted m-tuples whose first index is >= v; every
// stored order-k block is (left ++ right) for exactly one v.  Expanding the
// within-block offsets gives, per pivot, a dense product
//     dS_k[r, c] = sum_rows sign_l * L[l, r] * R[l, c]
// whose row r is a left Khatri-Rao column (product of h entries of one data
// row) and whose column c is a right Khatri-Rao column (m entries).  The
// right tuples with first index >= v are a suffix of all sorted m-tuples in
// lexicographic order, so one right table per order serves every pivot.
#pragma once
#include <stdint.h>

#define CUM_MAXD 6

namespace cum {

// Left Khatri-Rao column of one pivot GEMM row.
struct LeftCol {
  uint16_t c[4];    // data columns (h of them; unused entries 0)
  int64_t base;     // (rank(left ++ v..v) - first_right(v)) * b^k + wL * b^m
};

// Right Khatri-Rao column (shared by every pivot of one order).
struct RightCol {
  uint16_t c[4];    // data columns (m of them)
  int64_t base;     // rank_m(right tuple) * b^k + wR
};

// One workgroup's output tile of one pivot GEMM.
struct UpdItem {
  int k, v;         // order, pivot
  int r0, c0;       // tile origin (rows: left KR columns, cols: right KR columns)
  int M, N;         // extents of this pivot GEMM
  int lrow0;        // index of the pivot's first row in the order-k left table
  int rcol0;        // index of the pivot's first column in the order-k right table
  int ctx;          // batched launches: index of the owning context's descriptor
};

struct OrderInfo {
  int k, h, m;
  int64_t nblocks;  // P_k = C(nbar + k - 1, k)
  int64_t bk;       // b^k
  int64_t nelems;   // nblocks * b^k
};

}  // namespace cum
