// Kernel argument blocks and launch wrappers (host <-> device interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cum_internal.h"

namespace cum {

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };

// Update tile: TM x TN fragments of 16x16 per workgroup (TM, TN in {2, 4});
// the four waves of a workgroup split the rows of every LDS chunk between
// them and are reduced in a fixed order at the end.
constexpr int UPD_X_BYTES = 32768;     // bytes of data rows per LDS chunk
constexpr int UPD_DIRECT_BYTES = 17408; // bytes per buffer of the double-buffered direct path
constexpr int UPD_ZERO_BYTES = 256;     // zeroed device block the direct path reads for padding

struct NormArgs {
  int d;
  int kfirst;               // orders below kfirst already hold their norm in out[] (1: none)
  int64_t nblocks[CUM_MAXD + 1];
  const double* partial[CUM_MAXD + 1];
  double* out;              // [0..d] ||C_k||_F, [d+1 .. 2d+1] nu_k
};

struct UpdArgs {
  const void* xp;           // rows entering the window (+1), row-major np x n
  const void* xm;           // rows leaving the window (-1), row-major nm x n
  int np, nm;
  int n;                    // data columns (LDS rows hold exactly n values)
  int vec;                  // 1: rows and both bases allow 16-byte copies
  int quad;                 // 1: four tiles per workgroup (items padded to groups of four)
  const UpdItem* items;
  const void* zero;         // UPD_ZERO_BYTES of zeros (direct-path padding source)
  const LeftCol* left[CUM_MAXD + 1];
  const RightCol* right[CUM_MAXD + 1];
  void* s_hi[CUM_MAXD + 1]; // running window sums, compensated pair
  void* s_lo[CUM_MAXD + 1];
  // FIFO of batch increments: 0 off; 1 fold the increment and store it in
  // snap; 2 fold the increment, fold out the one stored in snap, store it.
  // 3 (four-tile kernel only): store the increment in s_hi[k], without
  // reading or folding the running sums (k_fold_splits with single = 1
  // folds it in later)
  int fifo;
  void* snap[CUM_MAXD + 1]; // this update's FIFO slot, one value per stored element
  // 1: one extra workgroup (the last) finishes the norms of the previous
  // combine from its block partials, on a CU the tiles leave idle
  int with_norms;
  NormArgs na;
  // 1 when b divides 16: the last factor of a left Khatri-Rao column is then
  // the same for every 16-column fragment of a tile (block v's coordinate
  // picked by the lane), so a tile two fragments high reads it once per row
  int shl;
};

// LDS budget for a combine block's staged lower-order sub-blocks.
constexpr size_t COMB_STAGE_BYTES = 65536;

struct CombArgs {
  int b, nbar;
  int log2b;                // log2(b) when b is a power of two, else -1
  int64_t bs;               // b^s
  const int32_t* subrank;   // per block and subset mask: rank of the sub-tuple
  const void* s_hi;         // order-s running sums (pair)
  const void* s_lo;
  double inv_t;             // 1/t
  const double* C[CUM_MAXD + 1];  // cumulants of orders 1..s-1
  double* Cout;             // order-s cumulants
  const double* mult;       // per-block multiplicity
  double* partial;          // per-block mult * sum(c^2)
  // recursion (rec = 1): c_I = m_I - sum over the proper subsets B holding
  // I's first position of c_B m_{I\B}, with the moments m of the lower
  // orders from their running sums (pairs)
  int rec;
  const void* Shi[CUM_MAXD + 1];
  const void* Slo[CUM_MAXD + 1];
};

// Fused combine of every order (one workgroup per order-d block): the
// block's lattice of proper sub-blocks (one per non-empty proper subset of
// its d index positions) is staged in LDS as moments, their cumulants are
// formed level by level, then the block's own order-d cumulants; each
// lower-order block is written by the one order-d block that extends its
// tuple by repeating the last index (desig bit s: write the prefix-s block).
constexpr size_t LAT_LDS_BYTES = 65536;

struct LatArgs {
  int b, log2b;
  const int32_t* subrank;          // order d: per block and subset mask
  const uint8_t* desig;            // order d: bit s set when the block writes its prefix-s block
  double inv_t;
  const void* s_hi[CUM_MAXD + 1];  // running sums (pair) per order
  const void* s_lo[CUM_MAXD + 1];
  double* C[CUM_MAXD + 1];         // cumulants per order (outputs)
  const double* mult[CUM_MAXD + 1];
  double* partial[CUM_MAXD + 1];   // per-block mult * sum(c^2)
  int off[(1 << CUM_MAXD) + 1];    // LDS element offset of each proper sub-mask's sub-block; off[full] = total
  int rec;                         // batched form: 1 = recursion, 0 = partition sum
};

// LDS bytes the fused combine needs for (d, b): moments and cumulants of the
// (b+1)^d - 1 - b^d elements of the proper sub-blocks.
size_t lattice_lds_bytes(int d, int b);


bool update_tile_supported(int tm, int tn);
bool update_quad_supported(int prec, int n);
// LDS row stride (elements) used for n columns, 0 if n is too large.
int update_lds_stride(int n);
// Rows per LDS chunk for a precision and stride (0: not supported).
int update_chunk_rows(int prec, int str);
// Split contraction: chunks of one contraction run in one batched launch,
// each into its own zeroed copy of the running sums (split s: hi at
// split + 2 s tot, lo at split + (2 s + 1) tot, orders concatenated at
// off[k]); k_fold_splits then folds the copies into the running sums in
// chunk order, the same steps a chunk-by-chunk contraction takes, and
// leaves the copies zeroed for the next split contraction.
struct FoldArgs {
  int d, nsplit;
  int fresh;                         // 1: the running sums start from zero (not read)
  int single;                        // 1: one array of increments (no lo half, not zeroed)
  int64_t tot;                       // state elements of orders 1..d
  int64_t off[CUM_MAXD + 2];         // first element of order k; off[d+1] = tot
  void* s_hi[CUM_MAXD + 1];
  void* s_lo[CUM_MAXD + 1];
  const void* split;
};
hipError_t launch_fold_splits(int prec, const FoldArgs& a, hipStream_t st);

// Zeroes up to ZERO_MAX buffers (sizes in 4-byte words) in one launch: a
// kernel, so the clearing can sit inside a captured graph.
constexpr int ZERO_MAX = 16;
struct ZeroArgs {
  int count;
  void* ptr[ZERO_MAX];
  int64_t words[ZERO_MAX];
};
hipError_t launch_zero(const ZeroArgs& a, hipStream_t st);

// e0/e1 (null: none) record the update kernel's own start and end.
hipError_t launch_update(int prec, int tm, int tn, int kmax, const UpdArgs& a, int nitems, hipStream_t st,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_combine(int prec, int s, const CombArgs& a, int64_t nblocks, hipStream_t st);
// The same per-order combine with every operand in LDS, the partition sum
// grouped on the part holding the first position (orders 5 and 6, b = 4).
bool combine_split_supported(int s, int b);
hipError_t launch_combine_split(int prec, int s, const CombArgs& a, int64_t nblocks, hipStream_t st);
hipError_t launch_norms(const NormArgs& a, hipStream_t st);
// recursion: c_I = m_I - sum over B containing I's first position of c_B m_{I\B}
// (2^(s-1) - 1 terms) instead of the partition sum of Alg. 4 (B(s) - 1 terms)
hipError_t launch_combine_lattice(int prec, int d, bool recursion, const LatArgs& a, int64_t nblocks,
                                  size_t lds_bytes, hipStream_t st);
// b: the block size every member of the launch shares (b in {2, 4, 8} gets
// a kernel with b at compile time)
hipError_t launch_combine_lattice_batch(int prec, int d, int b, const LatArgs* ctxs, const int64_t* items,
                                        int nitems, int grid, size_t lds_bytes, hipStream_t st);

// Batched launches over several contexts (device-resident argument tables).
hipError_t launch_update_batch(int prec, int str, bool vl, int kmax, const UpdArgs* ctxs, const UpdItem* items,
                               int nitems, int grid, hipStream_t st);
// Batched four-tile form: items holds groups of four tiles of one member
// each (pack_quads per member), nitems a multiple of 4; grid workgroups walk
// the groups with a grid-sized stride.
bool update_quad_batch_supported(int prec, int str);
hipError_t launch_update_quad_batch(int prec, int str, int kmax, const UpdArgs* ctxs, const UpdItem* items,
                                    int nitems, int grid, hipStream_t st);
// rec: every listed member uses the recursion (their CombArgs have rec = 1)
hipError_t launch_combine_batch(int prec, int s, const CombArgs* ctxs, const int64_t* items, int nitems,
                                int grid, size_t stage_bytes, bool rec, hipStream_t st);
hipError_t launch_norms_batch(const NormArgs* ctxs, int m, hipStream_t st);

}  // namespace cum
