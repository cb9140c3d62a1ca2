// HIP kernels for gfx950 (CDNA4): sliding-window moment update, moment ->
// cumulant combine, and block-structured norms.
//
//  k_update   Alg. 2 / Eq. (momupdate): for every stored element of orders
//             1..d, dS = sum_{new rows} prod x - sum_{old rows} prod x, computed
//             as one signed pivot GEMM per (order, pivot) on MFMA and folded
//             into the running window sums with a TwoSum (compensated) update.
//  k_combine  Alg. 3 / Alg. 4: C_s = S_s/t - sum over every partition of
//             {1..s} into 2..s parts of the product of lower-order cumulants at
//             the sub-multi-indices, in FP64, one workgroup per stored block.
//  k_norms    Alg. 5 (exponent 2) and Eq. (mef), deterministic fixed-order sums.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <hip/hip_vector_types.h>

#include "cum_internal.h"
#include "kernels.h"
#include "partitions.h"

namespace cum {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void norms_block(const NormArgs& a);

template <int P> struct Tr;
template <> struct Tr<PREC_F64> {
  using X = double; using Acc = f64x4; using A1 = double;
  static constexpr int KS = 4;
};
template <> struct Tr<PREC_F32> {
  using X = float; using Acc = f32x4; using A1 = float;
  static constexpr int KS = 4;
};
template <> struct Tr<PREC_BF16X3> {
  using X = float; using Acc = f32x4; using A1 = float;
  static constexpr int KS = 32;
};

// Row of the 16x16 output fragment that accumulator register r of this lane
// holds (column = lane % 16).  f32/bf16: 4*(lane/16) + r; f64: lane/16 + 4r.
template <int P> __device__ __forceinline__ int frag_row(int lane, int r) {
  return (P == PREC_F64) ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r);
}

__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values v0, v1 (consecutive K indices of one operand) split as
// v = hi + lo, hi = RNE_bf16(v), lo = RNE_bf16(v - hi), each pair packed in
// one register the way the bf16 matrix instruction reads it (element 0 in the
// low half).  One packed conversion per pair for hi and one for lo; hi is
// widened back exactly by placing its bits in the upper half of a float, and
// v - hi is exact in FP32.
__device__ __forceinline__ void split_pair(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v0, v1}, bf16x2));
  const float h0 = __builtin_bit_cast(float, h << 16);
  const float h1 = __builtin_bit_cast(float, h & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v0 - h0, v1 - h1}, bf16x2));
  hi = h;
}

__device__ __forceinline__ bf16x8 as_bf16x8(const uint32_t (&w)[4]) {
  return __builtin_bit_cast(bf16x8, (u32x4){w[0], w[1], w[2], w[3]});
}

// Compensated fold of d into the pair (hi, lo): TwoSum then renormalise.
template <typename T>
__device__ __forceinline__ void fold_val(T& hi, T& lo, T d) {
  const T s = hi + d;
  const T bp = s - hi;
  const T err = (hi - (s - bp)) + (d - bp);
  const T l2 = lo + err;
  const T nh = s + l2;
  lo = l2 - (nh - s);
  hi = nh;
}

template <typename T>
__device__ __forceinline__ void fold(T* hi_p, T* lo_p, T d) {
  T hi = *hi_p, lo = *lo_p;
  fold_val(hi, lo, d);
  *hi_p = hi;
  *lo_p = lo;
}

// Sum over the 64 lanes of a wave by a fixed butterfly (every lane ends with
// the same total, in the same order on every run).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Chunks.  The rows of one contraction are the np rows of xp (sign +1) and
// the nm rows of xm (sign -1).  They are cut into chunks of R rows that never
// mix the two signs: ceil(np/R) plus chunks, then ceil(nm/R) minus chunks, the
// last chunk of each kind zero-filled.  A chunk sits in LDS row-major with a
// compile-time row stride STR >= n + 4, STR = 4 (mod 32): rows stay 16-byte
// aligned for 128-bit stores, every k-step offset is an immediate of the LDS
// read, and four consecutive rows start 4 banks apart.
template <int P, int STR> struct ChunkGeom {
  static constexpr int ES = (P == PREC_F64) ? 8 : 4;
  static constexpr int UB = (P == PREC_BF16X3) ? 128 : 16;     // rows: one k-step for each of 4 waves
  static constexpr int R = (UPD_X_BYTES / ((STR - 4) * ES)) / UB * UB;  // 0: shape not supported
};

// Direct path (f32/f64 with 16-byte rows): every wave copies its own rows
// of each chunk (RW = R/4 rows, the only rows its k-steps read) from global
// memory straight into two private LDS buffers, the next chunk arriving while
// the current one is multiplied; the waves never wait for each other.  R rows
// per chunk (a multiple of 32 when it can be, else 16), row stride STR as in
// ChunkGeom; SU 16-byte units per LDS row; a wave's buffer is rounded up to
// whole 64-lane loads (WU units).  Buffer b of wave w starts at unit
// (4 b + w) WU.
template <int P, int STR> struct DirectGeom {
  static constexpr int ES = (P == PREC_F64) ? 8 : 4;
  static constexpr int X = UPD_DIRECT_BYTES / (STR * ES);
  static constexpr int R = X >= 32 ? X / 32 * 32 : 16;
  static constexpr int RW = R / 4;
  static constexpr int SU = STR * ES / 16;
  static constexpr int WU = (RW * SU + 63) / 64 * 64;
  static constexpr int BUFB = 4 * WU * 16;
  static constexpr int SMEM = 2 * BUFB;
};

template <int V> struct IntC { static constexpr int value = V; };

constexpr int PREF_UNITS = UPD_X_BYTES / 16 / 256;

struct RegChunk {
  uint4 u[PREF_UNITS];
};

// Per-thread LDS byte addresses of the 16-byte units it stores (-1: none);
// the same for every chunk.
template <int P, int STR>
__device__ __forceinline__ void chunk_slots(int (&slot)[PREF_UNITS], int n) {
  using G = ChunkGeom<P, STR>;
  const int upr = n * G::ES / 16;
  const int total = G::R * upr;
  const float inv_upr = 1.0f / (float)upr;
#pragma unroll
  for (int q = 0; q < PREF_UNITS; ++q) {
    const int i = threadIdx.x + 256 * q;
    // exact for i < 2^20: the fractional part of (i + 0.5)/upr is >= 0.5/upr
    const int r = (int)(((float)i + 0.5f) * inv_upr);
    slot[q] = (i < total) ? r * STR * G::ES + (i - r * upr) * 16 : -1;
  }
}

// 16-byte units of chunk `ci` into registers (vector path: n*esize % 16 == 0).
// A full chunk loads without predicates (units past the chunk's last row
// re-read its last unit and are never stored); the last chunk of each sign
// and chunks past the last (ci >= nch) read zeros past their rows.
template <int P, int STR>
__device__ __forceinline__ void fetch_chunk(RegChunk& rc, const UpdArgs& a, int ci, int ncp, int nch) {
  using G = ChunkGeom<P, STR>;
  const int upr = a.n * G::ES / 16;
  const bool plus = ci < ncp;
  const int r0 = (plus ? ci : ci - ncp) * G::R;
  const int rows = ci < nch ? min(G::R, (plus ? a.np : a.nm) - r0) : 0;
  const uint4* src = (const uint4*)(plus ? a.xp : a.xm) + (int64_t)r0 * upr;
  if (rows == G::R) {
    const int last = G::R * upr - 1;
#pragma unroll
    for (int q = 0; q < PREF_UNITS; ++q) rc.u[q] = src[min((int)threadIdx.x + 256 * q, last)];
  } else {
    const int cnt = rows * upr - (int)threadIdx.x;
#pragma unroll
    for (int q = 0; q < PREF_UNITS; ++q)
      rc.u[q] = (256 * q < cnt) ? src[threadIdx.x + 256 * q] : make_uint4(0u, 0u, 0u, 0u);
  }
}

template <int P, int STR>
__device__ __forceinline__ void store_chunk(char* smem, const RegChunk& rc, const int (&slot)[PREF_UNITS]) {
#pragma unroll
  for (int q = 0; q < PREF_UNITS; ++q)
    if (slot[q] >= 0) *(uint4*)(smem + slot[q]) = rc.u[q];
}

// Scalar path (row length not a multiple of 16 bytes, or unaligned bases).
template <int P, int STR>
__device__ __forceinline__ void load_chunk_scalar(char* smem, const UpdArgs& a, int ci, int ncp) {
  using G = ChunkGeom<P, STR>;
  using T = typename Tr<P>::X;
  const bool plus = ci < ncp;
  const int r0 = (plus ? ci : ci - ncp) * G::R;
  const int rows = min(G::R, (plus ? a.np : a.nm) - r0);
  const T* src = (const T*)(plus ? a.xp : a.xm) + (int64_t)r0 * a.n;
  const int cnt = rows * a.n, total = G::R * a.n;
  const float inv_n = 1.0f / (float)a.n;
  T* xs = (T*)smem;
  for (int i = threadIdx.x; i < total; i += 256) {
    const int r = (int)(((float)i + 0.5f) * inv_n);
    xs[r * STR + (i - r * a.n)] = (i < cnt) ? src[i] : T(0);
  }
}

// Direct path: this lane's byte offset, from a wave's first row of a chunk,
// of the 16-byte unit it copies in each load round (the same for every
// chunk).  Unit i of a wave's buffer is row i / SU, column unit i % SU; units
// past a row's data (LDS padding, never read) copy the first unit instead.
template <int P, int STR> struct DirectLanes {
  static constexpr int NQ = DirectGeom<P, STR>::WU / 64;
  uint32_t off[NQ];
};

template <int P, int STR>
__device__ __forceinline__ void direct_lanes(DirectLanes<P, STR>& dl, int n) {
  using G = DirectGeom<P, STR>;
  const int upr = n * G::ES / 16;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < DirectLanes<P, STR>::NQ; ++q) {
    const int i = q * 64 + lane;
    const int r = i / G::SU, c = i - r * G::SU;
    dl.off[q] = (c < upr && r < G::RW) ? (uint32_t)((r * upr + c) * 16) : 0u;
  }
}

// Starts the copy of this wave's rows of chunk `ci` into its buffer at `wbuf`
// (64 consecutive units per load, lane L at unit 64 q + L).  Rows past the
// end of the last chunk of a sign copy a 16-byte block of zeros.
template <int P, int STR>
__device__ __forceinline__ void issue_chunk(char* wbuf, const UpdArgs& a, const DirectLanes<P, STR>& dl, int ci,
                                            int ncp, int wave) {
  using G = DirectGeom<P, STR>;
  const int upr = a.n * G::ES / 16;
  const bool plus = ci < ncp;
  const int r0 = (plus ? ci : ci - ncp) * G::R + wave * G::RW;
  const int rows = (plus ? a.np : a.nm) - r0;
  const char* src = (const char*)(plus ? a.xp : a.xm) + (int64_t)r0 * upr * 16;
  if (rows >= G::RW) {
#pragma unroll
    for (int q = 0; q < DirectLanes<P, STR>::NQ; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src + dl.off[q]),
                                       (__attribute__((address_space(3))) void*)(wbuf + q * 1024), 16, 0, 0);
  } else {
    const uint32_t lim = rows > 0 ? (uint32_t)(rows * upr * 16) : 0u;
#pragma unroll
    for (int q = 0; q < DirectLanes<P, STR>::NQ; ++q) {
      const char* g = dl.off[q] < lim ? src + dl.off[q] : (const char*)a.zero;
      __builtin_amdgcn_global_load_lds((const void*)g,
                                       (__attribute__((address_space(3))) void*)(wbuf + q * 1024), 16, 0, 0);
    }
  }
}

// Row mapping inside a chunk of R rows: wave w owns rows [w R/4, (w+1) R/4).
// f32/f64 (16x16x4), NKS = R/16 k-steps per wave: with NKS even, k-steps 2u
// and 2u+1 of lane group q = lane/16 take the adjacent rows w R/4 + 8u + 2q
// and 8u + 2q + 1 (their two loads merge into one two-address LDS read);
// with NKS odd, k-step s takes row w R/4 + 4s + q.  bf16 (16x16x32): at
// k-step s, K index 8q + j of group q is row w R/4 + 32s + 4j + q.  A and B
// use the same row for the same K index, so the products pair up; the four
// groups always read rows 1 or 2 apart (4 or 8 banks).
template <int NKS, int STR, int ES>
__device__ __forceinline__ constexpr int koff(int s) {
  return (NKS % 2 == 0) ? (8 * (s >> 1) + (s & 1)) * STR * ES : 4 * s * STR * ES;
}

template <int P, int H, int MR, int TM, int TN, int STR, bool VL>
__device__ void upd_body(const UpdArgs& a, const UpdItem& it, char* smem) {
  using T = typename Tr<P>::X;
  using Acc = typename Tr<P>::Acc;
  using A1 = typename Tr<P>::A1;
  using G = ChunkGeom<P, STR>;
  using D = DirectGeom<P, STR>;
  constexpr int KS = Tr<P>::KS;
  constexpr bool DIRECT = (KS == 4 && VL);
  constexpr int ES = G::ES;
  constexpr int R = DIRECT ? D::R : G::R;
  constexpr int RW = R / 4;
  constexpr int NKS = RW / KS;                 // k-steps per wave per chunk
  constexpr int K_ORD = H + MR;
  constexpr int MRC = MR > 0 ? MR : 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const LeftCol* __restrict__ left = a.left[K_ORD];
  const RightCol* __restrict__ right = a.right[K_ORD];
  // this lane's first LDS row: in the direct path inside the wave's own
  // buffer (which starts at byte wave * WU * 16), else inside the chunk
  const int lgrp = (KS == 4 && NKS % 2 == 0) ? 2 * (lane >> 4) : (lane >> 4);
  const int lrow = DIRECT ? lgrp : wave * RW + lgrp;
  const int lbase = DIRECT ? wave * D::WU * 16 : 0;
  const int ncp = (a.np + R - 1) / R;
  const int nch = ncp + (a.nm + R - 1) / R;

  // direct path: the copy of chunk 0 starts before anything else
  DirectLanes<P, STR> dl;
  char* wbuf = smem + (DIRECT ? wave * D::WU * 16 : 0);
  if constexpr (DIRECT) {
    direct_lanes<P, STR>(dl, a.n);
    __syncthreads();  // the previous item's epilogue may still read smem
    issue_chunk<P, STR>(wbuf, a, dl, 0, ncp, wave);
  }

  // Byte addresses of this lane's factor columns at its first row.  Rows past
  // M, columns past N and padded data columns read column 0: their products
  // are computed but never stored, so the inner loop has no masks.
  int ao[TM][H];
  int bo[TN][MRC];
#pragma unroll
  for (int f = 0; f < TM; ++f) {
    const int r = min(it.r0 + 16 * f + (lane & 15), it.M - 1);
    const LeftCol L = left[it.lrow0 + r];
#pragma unroll
    for (int q = 0; q < H; ++q) ao[f][q] = lbase + (lrow * STR + (L.c[q] < a.n ? L.c[q] : 0)) * ES;
  }
#pragma unroll
  for (int g = 0; g < TN; ++g) {
    const int c = min(it.c0 + 16 * g + (lane & 15), it.N - 1);
    const RightCol Rc = right[it.rcol0 + c];
#pragma unroll
    for (int q = 0; q < MRC; ++q) bo[g][q] = lbase + (lrow * STR + ((q < MR && Rc.c[q] < a.n) ? Rc.c[q] : 0)) * ES;
  }
  // (every fragment is multiplied, also those past M or N: branching around
  // MFMAs makes the compiler shuffle the accumulators through VGPRs)
  int slot[PREF_UNITS];
  if constexpr (VL && !DIRECT) chunk_slots<P, STR>(slot, a.n);

  // Epilogue element e = tid + 256 j of the tile (fragment j, row
  // (tid >> 4) & 15, column tid & 15): its stored offset, or -1 past the
  // pivot GEMM or on a padded column.  On the f32 path it is found here and
  // the element's running sums are loaded right after the main loop.
  constexpr int NF = TM * TN;
  constexpr bool EPF = (P == PREC_F32);
  auto elem_offset = [&](int j) __attribute__((always_inline)) -> int64_t {
    const int f = j / TN, g = j - (j / TN) * TN;
    const int r = it.r0 + 16 * f + ((tid >> 4) & 15), c = it.c0 + 16 * g + (tid & 15);
    if (r >= it.M || c >= it.N) return -1;
    const LeftCol L = left[it.lrow0 + r];
    const RightCol Rc = right[it.rcol0 + c];
    bool pad = false;
#pragma unroll
    for (int q = 0; q < H; ++q) pad = pad || L.c[q] >= a.n;
#pragma unroll
    for (int q = 0; q < MR; ++q) pad = pad || Rc.c[q] >= a.n;
    return pad ? -1 : L.base + Rc.base;
  };
  int64_t eoff[NF];
  if constexpr (EPF) {
#pragma unroll
    for (int j = 0; j < NF; ++j) eoff[j] = elem_offset(j);
  }

  Acc acc[TM][TN];
#pragma unroll
  for (int f = 0; f < TM; ++f)
#pragma unroll
    for (int g = 0; g < TN; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[f][g][r] = A1(0);

  // k-steps of one chunk held at byte offset BO of smem (f32/f64 paths)
  auto multiply_chunk = [&](auto bo_c) __attribute__((always_inline)) {
    constexpr int BO = decltype(bo_c)::value;
    // the factor values of k-step s+1 are loaded while k-step s multiplies
    constexpr bool PIPE = (P == PREC_F32 || P == PREC_F64);
    constexpr int NB = PIPE ? 2 : 1;
    T fa[NB][TM][H], fb[NB][TN][MRC];
    auto load_factors = [&](int st, int buf) __attribute__((always_inline)) {
      const int so = koff<NKS, STR, ES>(st) + BO;
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int q = 0; q < H; ++q) fa[buf][f][q] = *(const T*)(smem + ao[f][q] + so);
#pragma unroll
      for (int g = 0; g < TN; ++g)
#pragma unroll
        for (int q = 0; q < MR; ++q) fb[buf][g][q] = *(const T*)(smem + bo[g][q] + so);
    };
    load_factors(0, 0);
#pragma unroll
    for (int st = 0; st < NKS; ++st) {
      const int cur = PIPE ? (st & 1) : 0;
      if (PIPE && st + 1 < NKS) load_factors(st + 1, cur ^ 1);
      if (!PIPE && st > 0) load_factors(st, 0);
      T A[TM], B[TN];
#pragma unroll
      for (int f = 0; f < TM; ++f) {
        T v = fa[cur][f][0];
#pragma unroll
        for (int q = 1; q < H; ++q) v *= fa[cur][f][q];
        A[f] = v;
      }
#pragma unroll
      for (int g = 0; g < TN; ++g) {
        T v = T(1);
        if constexpr (MR > 0) {
          v = fb[cur][g][0];
#pragma unroll
          for (int q = 1; q < MR; ++q) v *= fb[cur][g][q];
        }
        B[g] = v;
      }
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int g = 0; g < TN; ++g) acc[f][g] = mma(A[f], B[g], acc[f][g]);
    }
  };

  if constexpr (DIRECT) {
    // Per wave: wait for this wave's copy of chunk ci (its own loads only),
    // start the copy of chunk ci+1 into the other buffer (whose reads of
    // chunk ci-1 have completed), then run the k-steps of chunk ci.
    auto run_chunk = [&](int ci) __attribute__((always_inline)) {
      __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
      if (ci + 1 < nch) issue_chunk<P, STR>(wbuf + ((ci + 1) & 1) * D::BUFB, a, dl, ci + 1, ncp, wave);
      if (ci & 1) multiply_chunk(IntC<D::BUFB>{});
      else multiply_chunk(IntC<0>{});
    };
    int ci = 0;
    for (; ci < ncp; ++ci) run_chunk(ci);
    if (nch > ncp) {
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int g = 0; g < TN; ++g) acc[f][g] = -acc[f][g];
      for (; ci < nch; ++ci) run_chunk(ci);
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int g = 0; g < TN; ++g) acc[f][g] = -acc[f][g];
    }
  } else {
  RegChunk rc;
  if constexpr (VL) fetch_chunk<P, STR>(rc, a, 0, ncp, nch);

  auto run_chunk = [&](int ci) __attribute__((always_inline)) {
    __syncthreads();
    if constexpr (VL) {
      store_chunk<P, STR>(smem, rc, slot);
      __syncthreads();
      fetch_chunk<P, STR>(rc, a, ci + 1, ncp, nch);
    } else {
      load_chunk_scalar<P, STR>(smem, a, ci, ncp);
      __syncthreads();
    }
    if constexpr (KS == 4) {
      multiply_chunk(IntC<0>{});
    } else {
      // split-BF16x3: v = hi + lo with hi = RNE_bf16(v), lo = RNE_bf16(v - hi);
      // a*b ~ ah*bh + ah*bl + al*bh, accumulated in FP32.
#pragma unroll
      for (int st = 0; st < NKS; ++st) {
        uint32_t Ah[TM][4], Al[TM][4], Bh[TN][4], Bl[TN][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // rows of K indices 2i and 2i + 1
          const int so0 = (32 * st + 8 * i) * STR * ES, so1 = so0 + 4 * STR * ES;
#pragma unroll
          for (int f = 0; f < TM; ++f) {
            float v0 = *(const float*)(smem + ao[f][0] + so0);
            float v1 = *(const float*)(smem + ao[f][0] + so1);
#pragma unroll
            for (int q = 1; q < H; ++q) {
              v0 *= *(const float*)(smem + ao[f][q] + so0);
              v1 *= *(const float*)(smem + ao[f][q] + so1);
            }
            split_pair(v0, v1, Ah[f][i], Al[f][i]);
          }
#pragma unroll
          for (int g = 0; g < TN; ++g) {
            float v0 = 1.0f, v1 = 1.0f;
            if constexpr (MR > 0) {
              v0 = *(const float*)(smem + bo[g][0] + so0);
              v1 = *(const float*)(smem + bo[g][0] + so1);
#pragma unroll
              for (int q = 1; q < MR; ++q) {
                v0 *= *(const float*)(smem + bo[g][q] + so0);
                v1 *= *(const float*)(smem + bo[g][q] + so1);
              }
            }
            split_pair(v0, v1, Bh[g][i], Bl[g][i]);
          }
        }
#pragma unroll
        for (int f = 0; f < TM; ++f)
#pragma unroll
          for (int g = 0; g < TN; ++g) {
            const bf16x8 ah = as_bf16x8(Ah[f]), al = as_bf16x8(Al[f]);
            const bf16x8 bh = as_bf16x8(Bh[g]), bl = as_bf16x8(Bl[g]);
            acc[f][g] = mma16(al, bh, acc[f][g]);
            acc[f][g] = mma16(ah, bl, acc[f][g]);
            acc[f][g] = mma16(ah, bh, acc[f][g]);
          }
      }
    }
  };

  // Sign: the plus chunks run first; the minus chunks then add their
  // products to the negated accumulators, acc <- -(-acc + sum_minus), so no
  // product is negated.
  int ci = 0;
  for (; ci < ncp; ++ci) run_chunk(ci);
  if (nch > ncp) {
#pragma unroll
    for (int f = 0; f < TM; ++f)
#pragma unroll
      for (int g = 0; g < TN; ++g) acc[f][g] = -acc[f][g];
    for (; ci < nch; ++ci) run_chunk(ci);
#pragma unroll
    for (int f = 0; f < TM; ++f)
#pragma unroll
      for (int g = 0; g < TN; ++g) acc[f][g] = -acc[f][g];
  }
  }

  // Reduce the four waves' partial sums in a fixed order (wave 0 + 1 + 2 + 3),
  // GF fragments at a time through LDS, and fold every stored element.
  constexpr int LDSB = DIRECT ? D::SMEM : R * STR * ES;
  constexpr int GMAX = LDSB / (4 * 256 * (int)sizeof(A1));
  constexpr int GF = NF < GMAX ? NF : GMAX;
  static_assert(GF >= 1, "reduction buffer");
  A1* red = (A1*)smem;
  A1* shi = (A1*)a.s_hi[K_ORD];
  A1* slo = (A1*)a.s_lo[K_ORD];
  A1* snp = (A1*)a.snap[K_ORD];
  if constexpr (EPF && GF == NF) {
    // the running sums of this lane's elements load while the partial sums
    // pass through LDS
    A1 ph[NF], pl[NF], ps[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      ph[j] = pl[j] = ps[j] = A1(0);
      if (eoff[j] >= 0) {
        ph[j] = shi[eoff[j]];
        pl[j] = slo[eoff[j]];
        if (a.fifo == 2) ps[j] = snp[eoff[j]];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const int f = q / TN, g = q % TN;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[(wave * NF + q) * 256 + frag_row<P>(lane, r) * 16 + (lane & 15)] = acc[f][g][r];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      if (eoff[j] >= 0) {
        const int e = tid + 256 * j;
        const A1 sum = ((red[e] + red[NF * 256 + e]) + red[2 * NF * 256 + e]) + red[3 * NF * 256 + e];
        fold_val<A1>(ph[j], pl[j], sum);
        // FIFO: the batch leaving the window, its increment exactly as it was added
        if (a.fifo == 2) fold_val<A1>(ph[j], pl[j], -ps[j]);
        shi[eoff[j]] = ph[j];
        slo[eoff[j]] = pl[j];
        if (a.fifo) snp[eoff[j]] = sum;
      }
    }
    return;
  }
#pragma unroll
  for (int f0 = 0; f0 < NF; f0 += GF) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GF; ++q) {
      const int fi = f0 + q;
      if (fi < NF) {
        const int f = fi / TN, g = fi % TN;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[(wave * GF + q) * 256 + frag_row<P>(lane, r) * 16 + (lane & 15)] = acc[f][g][r];
      }
    }
    __syncthreads();
    const int cnt = (NF - f0 < GF ? NF - f0 : GF) * 256;
    for (int e = tid; e < cnt; e += 256) {
      const int fi = f0 + (e >> 8), i = (e >> 4) & 15, j = e & 15;
      const int f = fi / TN, g = fi - f * TN;
      const int r = it.r0 + 16 * f + i, c = it.c0 + 16 * g + j;
      if (r < it.M && c < it.N) {
        const LeftCol L = left[it.lrow0 + r];
        const RightCol Rc = right[it.rcol0 + c];
        bool pad = false;
#pragma unroll
        for (int q = 0; q < H; ++q) pad = pad || L.c[q] >= a.n;
#pragma unroll
        for (int q = 0; q < MR; ++q) pad = pad || Rc.c[q] >= a.n;
        if (!pad) {
          const A1 sum = ((red[e] + red[GF * 256 + e]) + red[2 * GF * 256 + e]) + red[3 * GF * 256 + e];
          const int64_t off = L.base + Rc.base;
          fold<A1>(shi + off, slo + off, sum);
          if (a.fifo) {
            // the batch leaving the window: its increment, exactly as it was added
            A1* sp = (A1*)a.snap[K_ORD] + off;
            if (a.fifo == 2) fold<A1>(shi + off, slo + off, -*sp);
            *sp = sum;
          }
        }
      }
    }
  }
}

// LDS bytes of the update kernels: the two direct-path buffers, or the one
// register-staged chunk.
template <int P, int STR, bool VL>
constexpr int upd_smem_bytes() {
  if constexpr (Tr<P>::KS == 4 && VL) return DirectGeom<P, STR>::SMEM;
  else return ChunkGeom<P, STR>::R * STR * ChunkGeom<P, STR>::ES;
}

// One tile of order k (KMAX: the highest order the launch holds; the
// register allocation follows the largest body compiled in).
template <int P, int TM, int TN, int STR, bool VL, int KMAX>
__device__ __forceinline__ void upd_dispatch(const UpdArgs& a, const UpdItem& it, char* smem) {
  switch (it.k) {
    case 1: upd_body<P, 1, 0, TM, TN, STR, VL>(a, it, smem); break;
    case 2: upd_body<P, 1, 1, TM, TN, STR, VL>(a, it, smem); break;
    case 3: upd_body<P, 2, 1, TM, TN, STR, VL>(a, it, smem); break;
    case 4: upd_body<P, 2, 2, TM, TN, STR, VL>(a, it, smem); break;
    case 5: if constexpr (KMAX >= 5) upd_body<P, 3, 2, TM, TN, STR, VL>(a, it, smem); break;
    case 6: if constexpr (KMAX >= 6) upd_body<P, 3, 3, TM, TN, STR, VL>(a, it, smem); break;
    default: break;
  }
}

template <int P, int TM, int TN, int STR, bool VL, int KMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == PREC_BF16X3 ? 1 : 4))) void k_update(
    UpdArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[upd_smem_bytes<P, STR, VL>()];
  if (a.with_norms && blockIdx.x == gridDim.x - 1) {
    norms_block(a.na);
    return;
  }
  const UpdItem it = a.items[blockIdx.x];
  upd_dispatch<P, TM, TN, STR, VL, KMAX>(a, it, smem);
}

// ---------------------------------------------------------------------------
// Combine (Alg. 3 / Alg. 4).

// One workgroup per stored block of order S.  The lower-order cumulant
// sub-blocks C_|B|(j_B) of the block (every non-empty proper subset B of the
// S positions) are staged in LDS when they fit (STAGE), else gathered from
// global memory.  Each element is c = S_s/t - (sum over partitions of
// {1..S} into 2..S parts of prod_B c_B), Alg. 3/4; or, with REC, c = S_s/t
// - (sum over the proper B holding the first position of c_B m_{rest}),
// where the sub-blocks without the first position hold moments instead.
// The block's weighted sum of squares (Alg. 5) goes to partial[blk].
template <int S, typename St, bool STAGE, bool REC>
__device__ void combine_block(const CombArgs& a, int64_t blk, double* stage) {
  constexpr int NM = 1 << S;
  constexpr int FULL = NM - 1;
  __shared__ int64_t subbase[NM];
  __shared__ int lds_off[NM + 1];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int b = a.b;
  const St* shi = (const St*)a.s_hi;
  const St* slo = (const St*)a.s_lo;

  // the first element's running sums are independent of the prologue
  const int64_t o0 = blk * a.bs + tid;
  const double m0 = tid < a.bs ? ((double)shi[o0] + (double)slo[o0]) * a.inv_t : 0.0;

  if (tid == 0) {
    // LDS offsets of the staged sub-blocks, in mask order
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
  // value of the lower-order sub-block of `mask` at element offset o: its
  // cumulant, or with REC and the first position outside the mask, its
  // moment
  auto sub_value = [&](int mask, int64_t o) __attribute__((always_inline)) -> double {
    const int q = __builtin_popcount(mask);
    if (REC && !(mask & 1))
      return ((double)((const St*)a.Shi[q])[o] + (double)((const St*)a.Slo[q])[o]) * a.inv_t;
    return a.C[q][o];
  };
  if constexpr (STAGE) {
    const int total = lds_off[FULL];
    for (int i = tid; i < total; i += 256) {
      int mask = 1;
      while (mask + 1 < FULL && lds_off[mask + 1] <= i) ++mask;
      stage[i] = sub_value(mask, subbase[mask] + (i - lds_off[mask]));
    }
    __syncthreads();
  }

  double sq = 0.0;
  const int lb = a.log2b;  // >= 0 when b is a power of two
  for (int64_t e = tid; e < a.bs; e += 256) {
    int dig[S];
    if (lb >= 0) {
      const int mb = b - 1;
#pragma unroll
      for (int q = S - 1; q >= 0; --q) dig[q] = (int)(e >> (lb * (S - 1 - q))) & mb;
    } else {
      int64_t rem = e;
#pragma unroll
      for (int q = S - 1; q >= 0; --q) {
        dig[q] = (int)(rem % b);
        rem /= b;
      }
    }
    double cB[NM];
#pragma unroll
    for (int mask = 1; mask < FULL; ++mask) {
      int off = 0;
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (mask & (1 << q)) off = (int)__umul24((unsigned)off, (unsigned)b) + dig[q];
      if constexpr (STAGE) {
        cB[mask] = stage[lds_off[mask] + off];
      } else {
        cB[mask] = sub_value(mask, subbase[mask] + off);
      }
    }
    double A;
    if constexpr (REC) A = recursion_sum<S>(cB);
    else A = partition_sum<S>(cB);
    const int64_t o = blk * a.bs + e;
    const double mval = (e == tid) ? m0 : ((double)shi[o] + (double)slo[o]) * a.inv_t;
    const double c = mval - A;
    a.Cout[o] = c;
    sq += c * c;
  }
  // the same fixed order as the fused combine: wave butterfly, then waves 0..3
  const double w = wave_sum(sq);
  if ((tid & 63) == 0) red[tid >> 6] = w;
  __syncthreads();
  if (tid == 0) a.partial[blk] = a.mult[blk] * (((red[0] + red[1]) + red[2]) + red[3]);
}

template <int S, typename St, bool STAGE, bool REC>
__global__ __launch_bounds__(256) void k_combine(CombArgs a) {
  extern __shared__ __attribute__((aligned(16))) double stage[];
  combine_block<S, St, STAGE, REC>(a, blockIdx.x, stage);
}

// Batched form: items[i] = (context << 40) | block, for one order S (the
// members of one launch share the formula).
template <int S, typename St, bool STAGE, bool REC>
__global__ __launch_bounds__(256) void k_combine_batch(const CombArgs* __restrict__ ctxs,
                                                       const int64_t* __restrict__ items, int nitems) {
  extern __shared__ __attribute__((aligned(16))) double stage[];
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int64_t w = items[i];
    const CombArgs a = ctxs[w >> 40];
    combine_block<S, St, STAGE, REC>(a, w & ((int64_t(1) << 40) - 1), stage);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fused combine over the sub-block lattice of one order-S block.

__host__ __device__ constexpr int popc_c(int x) { return x ? (x & 1) + popc_c(x >> 1) : 0; }

// Mask of the lattice positions picked by local mask q of the positions of m.
__host__ __device__ constexpr int pdep_c(int q, int m) {
  int r = 0, k = 0;
  for (int p = 0; p < 8; ++p)
    if (m & (1 << p)) {
      if (q & (1 << k)) r |= 1 << p;
      ++k;
    }
  return r;
}

// Sub-block element e of a mask with s positions -> its s digits (position
// order, most significant first).
template <int s>
__device__ __forceinline__ void lat_digits(int e, int b, int lb, int (&dig)[s > 0 ? s : 1]) {
  if (lb >= 0) {
#pragma unroll
    for (int q = s - 1; q >= 0; --q) dig[q] = (e >> (lb * (s - 1 - q))) & (b - 1);
  } else {
#pragma unroll
    for (int q = s - 1; q >= 0; --q) {
      dig[q] = e % b;
      e /= b;
    }
  }
}

// The subtracted sum for element `dig` of the sub-block of MASK (s positions):
// Alg. 4's sum over partitions into 2..s parts of products of cumulants, or
// the recursion sum over B containing the first position of c_B * m_{MASK\B}.
// Lattice LDS: moments at off[G], cumulants at tot + off[G] (singletons: the
// moment is the cumulant).
template <int s, int MASK, bool REC>
__device__ __forceinline__ double lat_terms(const LatArgs& a, const double* lat, int tot, const int (&dig)[s > 0 ? s : 1],
                                            int b) {
  constexpr int NQ = 1 << s;
  auto sub = [&](int q) __attribute__((always_inline)) {
    int o = 0;
#pragma unroll
    for (int r = 0; r < s; ++r)
      if (q & (1 << r)) o = (int)__umul24((unsigned)o, (unsigned)b) + dig[r];
    return o;
  };
  if constexpr (REC) {
    double acc = 0.0;
#pragma unroll
    for (int q = 1; q < NQ - 1; q += 2) {
      const int rest = (NQ - 1) & ~q;
      const int G = pdep_c(q, MASK), H = pdep_c(rest, MASK);
      const double cq = popc_c(q) == 1 ? lat[a.off[G] + sub(q)] : lat[tot + a.off[G] + sub(q)];
      acc += cq * lat[a.off[H] + sub(rest)];
    }
    return acc;
  } else {
    double cB[NQ];
#pragma unroll
    for (int q = 1; q < NQ - 1; ++q) {
      const int G = pdep_c(q, MASK);
      cB[q] = popc_c(q) == 1 ? lat[a.off[G] + sub(q)] : lat[tot + a.off[G] + sub(q)];
    }
    cB[0] = 0.0;
    cB[NQ - 1] = 0.0;
    return partition_sum<s>(cB);
  }
}

// Cumulants of the proper sub-block MASK from the staged lattice.
template <int S, bool REC, int MASK>
__device__ __forceinline__ void lat_mask(const LatArgs& a, double* lat, int tot) {
  constexpr int s = popc_c(MASK);
  const int b = a.b;
  int size = 1;
#pragma unroll
  for (int q = 0; q < s; ++q) size *= b;
  for (int e = threadIdx.x; e < size; e += 64) {
    int dig[s];
    lat_digits<s>(e, b, a.log2b, dig);
    lat[tot + a.off[MASK] + e] = lat[a.off[MASK] + e] - lat_terms<s, MASK, REC>(a, lat, tot, dig, b);
  }
}

template <int S, bool REC, int LEVEL, int MASK>
__device__ __forceinline__ void lat_level(const LatArgs& a, double* lat, int tot) {
  if constexpr (MASK < (1 << S) - 1) {
    if constexpr (popc_c(MASK) == LEVEL) lat_mask<S, REC, MASK>(a, lat, tot);
    lat_level<S, REC, LEVEL, MASK + 1>(a, lat, tot);
  }
}

// One order-S block, one wave (64 lanes): stage the moments of the block's
// proper sub-blocks, form their cumulants level by level, then the block's
// own order-S cumulants, write the lower-order blocks this block is
// designated for, and the weighted sums of squares of every block written.
template <int S, typename St, bool REC>
__device__ void lattice_block(const LatArgs& a, int64_t blk, double* lat) {
  constexpr int NM = 1 << S;
  constexpr int FULL = NM - 1;
  constexpr int PRE = 4;  // own-block moments prefetched per lane
  __shared__ int64_t sub_base[NM];
  __shared__ const St* bhi[NM];
  __shared__ const St* blo[NM];
  const int tid = threadIdx.x;
  const int b = a.b;
  const int tot = a.off[FULL];
  int bS = 1;
#pragma unroll
  for (int q = 0; q < S; ++q) bS *= b;

  // the block's own running sums do not depend on the prologue
  const St* shi = (const St*)a.s_hi[S];
  const St* slo = (const St*)a.s_lo[S];
  double mpre[PRE];
#pragma unroll
  for (int u = 0; u < PRE; ++u) {
    const int e = tid + 64 * u;
    const int64_t o = blk * bS + e;
    mpre[u] = e < bS ? ((double)shi[o] + (double)slo[o]) * a.inv_t : 0.0;
  }
  const int des = a.desig[blk];
  if (tid >= 1 && tid < FULL) {
    const int ps = __builtin_popcount(tid);
    int64_t bl = 1;
    for (int q = 0; q < ps; ++q) bl *= b;
    const int64_t sb = (int64_t)a.subrank[blk * NM + tid] * bl;
    sub_base[tid] = sb;
    const St* hi = nullptr;
    const St* lo = nullptr;
#pragma unroll
    for (int k = 1; k < S; ++k)
      if (ps == k) {
        hi = (const St*)a.s_hi[k];
        lo = (const St*)a.s_lo[k];
      }
    bhi[tid] = hi + sb;
    blo[tid] = lo + sb;
  }
  __syncthreads();
  // moments of every proper sub-block, four lattice elements per lane at a
  // time with all their loads in flight together; element i belongs to the
  // last mask whose offset is <= i
  for (int i0 = 0; i0 < tot; i0 += 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + tid + 64 * u;
      v[u] = 0.0;
      if (i < tot) {
        int m = 1, base = 0;
#pragma unroll
        for (int mm = 2; mm < FULL; ++mm)
          if (i >= a.off[mm]) {
            m = mm;
            base = a.off[mm];
          }
        v[u] = ((double)bhi[m][i - base] + (double)blo[m][i - base]) * a.inv_t;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + tid + 64 * u;
      if (i < tot) lat[i] = v[u];
    }
  }
  __syncthreads();
  // cumulants of the proper sub-blocks, one level (subset size) at a time
  if constexpr (S >= 3) { lat_level<S, REC, 2, 1>(a, lat, tot); __syncthreads(); }
  if constexpr (S >= 4) { lat_level<S, REC, 3, 1>(a, lat, tot); __syncthreads(); }
  if constexpr (S >= 5) { lat_level<S, REC, 4, 1>(a, lat, tot); __syncthreads(); }
  if constexpr (S >= 6) { lat_level<S, REC, 5, 1>(a, lat, tot); __syncthreads(); }

  double sq[S + 1];
#pragma unroll
  for (int k = 0; k <= S; ++k) sq[k] = 0.0;
  // the block's own order-S cumulants
  double* Cout = a.C[S];
  for (int e0 = 0; e0 < bS; e0 += 64 * PRE) {
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int e = e0 + tid + 64 * u;
      if (e < bS) {
        int dig[S];
        lat_digits<S>(e, b, a.log2b, dig);
        const int64_t o = blk * bS + e;
        const double m = e0 == 0 ? mpre[u] : ((double)shi[o] + (double)slo[o]) * a.inv_t;
        const double c = m - lat_terms<S, FULL, REC>(a, lat, tot, dig, b);
        Cout[o] = c;
        sq[S] += c * c;
      }
    }
  }
  // the lower-order blocks this block is designated to write
#pragma unroll
  for (int s = 1; s < S; ++s) {
    if (des & (1 << s)) {
      const int mask = (1 << s) - 1;
      const int size = a.off[mask + 1] - a.off[mask];
      const int base = (s == 1 ? 0 : tot) + a.off[mask];
      for (int e = tid; e < size; e += 64) {
        const double c = lat[base + e];
        a.C[s][sub_base[mask] + e] = c;
        sq[s] += c * c;
      }
    }
  }
#pragma unroll
  for (int k = 1; k <= S; ++k) {
    if (k == S || (des & (1 << k))) {
      const double t = wave_sum(sq[k]);
      if (tid == 0) {
        const int64_t kb = (k == S) ? blk : (int64_t)a.subrank[blk * NM + ((1 << k) - 1)];
        a.partial[k][kb] = a.mult[k][kb] * t;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same combine with the block edge b fixed at compile time (2, 4 or 8):
// digits are shifts and masks, every lattice offset is a constant (the LDS
// reads take immediate offsets), the sub-block positions are scalar loads and
// the moments of all sub-blocks are loaded before any is stored.

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(IntC<I>{});
    static_for<I + 1, N>(f);
  }
}

template <int S, int B> struct LatFix {
  static constexpr int NM = 1 << S;
  static constexpr int FULL = NM - 1;
  static constexpr int LB = B == 2 ? 1 : (B == 4 ? 2 : 3);
  static constexpr int size(int m) {
    int r = 1;
    for (int q = 0; q < popc_c(m); ++q) r *= B;
    return r;
  }
  static constexpr int off(int m) {  // lattice offset of proper mask m (off(FULL) = total)
    int o = 0;
    for (int k = 1; k < m; ++k) o += size(k);
    return o;
  }
  static constexpr int TOT = off(FULL);
  static constexpr int BS = size(FULL);
  static constexpr int slots(int m) { return (size(m) + 63) / 64; }
  static constexpr int NSLOT = [] {
    int n = 0;
    for (int m = 1; m < FULL; ++m) n += slots(m);
    return n;
  }();
  static constexpr int slot_mask(int i) {
    for (int m = 1; m < FULL; ++m) {
      if (i < slots(m)) return m;
      i -= slots(m);
    }
    return 0;
  }
  static constexpr int slot_index(int i) {
    for (int m = 1; m < FULL; ++m) {
      if (i < slots(m)) return i;
      i -= slots(m);
    }
    return 0;
  }
};

template <int s, int LB>
__device__ __forceinline__ void fix_digits(int e, int (&dig)[s > 0 ? s : 1]) {
#pragma unroll
  for (int q = 0; q < s; ++q) dig[q] = (e >> (LB * (s - 1 - q))) & ((1 << LB) - 1);
}

// Offset inside the sub-block picked by local mask q of the digits.
template <int q, int s, int LB>
__device__ __forceinline__ int fix_sub(const int (&dig)[s > 0 ? s : 1]) {
  int o = 0;
#pragma unroll
  for (int r = 0; r < s; ++r)
    if (q & (1 << r)) o = (o << LB) | dig[r];
  return o;
}

// lat_terms with every offset a constant (same terms, same order).
template <int S, int B, int s, int MASK, bool REC>
__device__ __forceinline__ double fix_terms(const double* lat, const int (&dig)[s > 0 ? s : 1]) {
  using G = LatFix<S, B>;
  constexpr int NQ = 1 << s;
  if constexpr (REC) {
    double acc = 0.0;
    static_for<0, NQ / 2 - 1>([&](auto ic) __attribute__((always_inline)) {
      constexpr int q = 2 * decltype(ic)::value + 1;
      constexpr int rest = (NQ - 1) & ~q;
      constexpr int OC = (popc_c(q) == 1 ? 0 : G::TOT) + G::off(pdep_c(q, MASK));
      constexpr int OM = G::off(pdep_c(rest, MASK));
      acc += lat[OC + fix_sub<q, s, G::LB>(dig)] * lat[OM + fix_sub<rest, s, G::LB>(dig)];
    });
    return acc;
  } else {
    double cB[NQ];
    static_for<1, NQ - 1>([&](auto ic) __attribute__((always_inline)) {
      constexpr int q = decltype(ic)::value;
      constexpr int OC = (popc_c(q) == 1 ? 0 : G::TOT) + G::off(pdep_c(q, MASK));
      cB[q] = lat[OC + fix_sub<q, s, G::LB>(dig)];
    });
    cB[0] = 0.0;
    cB[NQ - 1] = 0.0;
    return partition_sum<s>(cB);
  }
}

// Cumulants of every proper sub-block of one level (subset size LEVEL).
template <int S, int B, bool REC, int LEVEL>
__device__ __forceinline__ void fix_level(double* lat) {
  using G = LatFix<S, B>;
  static_for<1, G::FULL>([&](auto mc) __attribute__((always_inline)) {
    constexpr int M = decltype(mc)::value;
    if constexpr (popc_c(M) == LEVEL) {
      constexpr int SZ = G::size(M), O = G::off(M);
#pragma unroll
      for (int u = 0; u < G::slots(M); ++u) {
        const int e = (int)threadIdx.x + 64 * u;
        if (SZ % 64 == 0 || e < SZ) {
          int dig[LEVEL];
          fix_digits<LEVEL, G::LB>(e, dig);
          lat[G::TOT + O + e] = lat[O + e] - fix_terms<S, B, LEVEL, M, REC>(lat, dig);
        }
      }
    }
  });
}

template <int S, int B, typename St, bool REC>
__device__ void lattice_fix(const LatArgs& a, int64_t blk, double* lat) {
  using G = LatFix<S, B>;
  constexpr int NM = G::NM, FULL = G::FULL, BS = G::BS, TOT = G::TOT;
  constexpr int NU = (BS + 63) / 64;      // own-block elements per lane
  constexpr int PRE = NU < 4 ? NU : 4;    // of which prefetched
  constexpr int GRP = 16;                 // staged values in flight per lane
  const int tid = threadIdx.x;
  const int32_t* rank = a.subrank + blk * NM;

  const St* shi = (const St*)a.s_hi[S] + blk * BS;
  const St* slo = (const St*)a.s_lo[S] + blk * BS;
  double mpre[PRE];
#pragma unroll
  for (int u = 0; u < PRE; ++u) {
    const int e = min(tid + 64 * u, BS - 1);
    mpre[u] = ((double)shi[e] + (double)slo[e]) * a.inv_t;
  }

  // moments of every proper sub-block, GRP slots of 64 elements at a time
  static_for<0, (G::NSLOT + GRP - 1) / GRP>([&](auto gc) __attribute__((always_inline)) {
    constexpr int g0 = decltype(gc)::value * GRP;
    constexpr int NG = G::NSLOT - g0 < GRP ? G::NSLOT - g0 : GRP;
    double v[NG];
    static_for<0, NG>([&](auto jc) __attribute__((always_inline)) {
      constexpr int j = decltype(jc)::value;
      constexpr int M = G::slot_mask(g0 + j), U = G::slot_index(g0 + j);
      constexpr int s = popc_c(M), SZ = G::size(M);
      const int64_t sb = (int64_t)rank[M] * SZ;
      const int e = SZ % 64 == 0 ? tid + 64 * U : min(tid + 64 * U, SZ - 1);
      v[j] = ((double)((const St*)a.s_hi[s])[sb + e] + (double)((const St*)a.s_lo[s])[sb + e]) * a.inv_t;
    });
    static_for<0, NG>([&](auto jc) __attribute__((always_inline)) {
      constexpr int j = decltype(jc)::value;
      constexpr int M = G::slot_mask(g0 + j), U = G::slot_index(g0 + j);
      constexpr int SZ = G::size(M);
      const int e = tid + 64 * U;
      if (SZ % 64 == 0 || e < SZ) lat[G::off(M) + e] = v[j];
    });
  });
  __syncthreads();
  if constexpr (S >= 3) { fix_level<S, B, REC, 2>(lat); __syncthreads(); }
  if constexpr (S >= 4) { fix_level<S, B, REC, 3>(lat); __syncthreads(); }

  double sq[S + 1];
#pragma unroll
  for (int k = 0; k <= S; ++k) sq[k] = 0.0;
  // the block's own order-S cumulants
  double* Cout = a.C[S] + blk * BS;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = tid + 64 * u;
    if (BS % 64 == 0 || e < BS) {
      int dig[S];
      fix_digits<S, G::LB>(e, dig);
      const double m = u < PRE ? mpre[u < PRE ? u : 0] : ((double)shi[e] + (double)slo[e]) * a.inv_t;
      const double c = m - fix_terms<S, B, S, FULL, REC>(lat, dig);
      Cout[e] = c;
      sq[S] += c * c;
    }
  }
  // the lower-order blocks this block is designated to write
  const int des = a.desig[blk];
  static_for<1, S>([&](auto sc) __attribute__((always_inline)) {
    constexpr int s = decltype(sc)::value;
    constexpr int M = (1 << s) - 1, SZ = G::size(M);
    constexpr int O = (s == 1 ? 0 : TOT) + G::off(M);
    if (des & (1 << s)) {
      double* dst = a.C[s] + (int64_t)rank[M] * SZ;
#pragma unroll
      for (int u = 0; u < G::slots(M); ++u) {
        const int e = tid + 64 * u;
        if (SZ % 64 == 0 || e < SZ) {
          const double c = lat[O + e];
          dst[e] = c;
          sq[s] += c * c;
        }
      }
    }
  });
#pragma unroll
  for (int k = 1; k <= S; ++k) {
    if (k == S || (des & (1 << k))) {
      const int64_t kb = (k == S) ? blk : (int64_t)rank[(1 << k) - 1];
      const double w = a.mult[k][kb] * wave_sum(sq[k]);
      if (tid == 0) a.partial[k][kb] = w;
    }
  }
}

template <int S, int B, typename St, bool REC>
__global__ __launch_bounds__(64) void k_combine_lattice_fix(LatArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lat[];
  lattice_fix<S, B, St, REC>(a, blockIdx.x, lat);
}

// b with a compile-time lattice for order S (its lattice fits the LDS budget).
__host__ __device__ constexpr bool lat_fix_ok(int S, int b) {
  return S >= 2 && S <= 4 && (b == 2 || b == 4 || b == 8);
}

template <int S, typename St, bool REC>
__global__ __launch_bounds__(64) void k_combine_lattice(LatArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lat[];
  lattice_block<S, St, REC>(a, blockIdx.x, lat);
}

// Batched form: items[i] = (context << 40) | order-S block; contexts of one
// order S whose lattices fit, each with its own formula flag.
template <int S, typename St>
__global__ __launch_bounds__(64) void k_combine_lattice_batch(const LatArgs* __restrict__ ctxs,
                                                              const int64_t* __restrict__ items, int nitems) {
  extern __shared__ __attribute__((aligned(16))) double lat[];
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int64_t w = items[i];
    const LatArgs& a = ctxs[w >> 40];
    const int64_t blk = w & ((int64_t(1) << 40) - 1);
    bool done = false;
    if constexpr (lat_fix_ok(S, 2)) {
      static_for<1, 4>([&](auto lc) __attribute__((always_inline)) {
        constexpr int B = 1 << decltype(lc)::value;
        if (a.b == B) {
          if (a.rec) lattice_fix<S, B, St, true>(a, blk, lat);
          else lattice_fix<S, B, St, false>(a, blk, lat);
          done = true;
        }
      });
    }
    if (!done) {
      if (a.rec) lattice_block<S, St, true>(a, blk, lat);
      else lattice_block<S, St, false>(a, blk, lat);
    }
    __syncthreads();
  }
}

// Final norms (Alg. 5 with exponent 2, Eq. (mef)): fro[k] = sqrt(sum of the
// order's block partials); nu[k] = fro[k] / fro[2]^(k/2) for k >= 3 (NaN
// when fro[2] = 0, e.g. a constant window).  One
// workgroup of 1024 threads issues the loads of every order first, then
// reduces all orders together in a fixed order (thread, wave butterfly, then
// the waves in index order): about one memory round trip.  Any block size
// that is a multiple of 64 up to 1024 (the 1024-thread form is the launch of
// its own; an update launch may carry it as one extra workgroup).
__device__ __forceinline__ void norms_block(const NormArgs& a) {
  __shared__ double red[CUM_MAXD + 1][16];
  __shared__ double fro[CUM_MAXD + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nt = blockDim.x, nw = nt >> 6;
  double s[CUM_MAXD + 1];
#pragma unroll
  for (int k = 1; k <= CUM_MAXD; ++k) {
    s[k] = 0.0;
    if (k >= a.kfirst && k <= a.d) {
      const double* p = a.partial[k];
      const int64_t nb = a.nblocks[k];
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = tid + (int64_t)nt * u;
        v[u] = i < nb ? p[i] : 0.0;
      }
      s[k] = (v[0] + v[1]) + (v[2] + v[3]);
      for (int64_t i = tid + 4 * (int64_t)nt; i < nb; i += nt) s[k] += p[i];
    }
  }
#pragma unroll
  for (int k = 1; k <= CUM_MAXD; ++k) {
    const double w = wave_sum(s[k]);
    if (lane == 0) red[k][wv] = w;
  }
  __syncthreads();
  if (tid >= 1 && tid <= a.d) {
    if (tid < a.kfirst) {
      fro[tid] = a.out[tid];  // written by the small-order kernel
    } else {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[tid][w];
      fro[tid] = sqrt(t);
    }
  }
  __syncthreads();
  if (tid <= a.d) {
    a.out[tid] = tid == 0 ? __builtin_nan("") : fro[tid];
    a.out[a.d + 1 + tid] = (tid >= 3 && fro[2] > 0.0) ? fro[tid] / pow(fro[2], 0.5 * tid) : __builtin_nan("");
  }
}

__global__ __launch_bounds__(1024) void k_norms(NormArgs a) { norms_block(a); }

// Batched form: workgroup i finishes the norms of context i.
__global__ __launch_bounds__(1024) void k_norms_batch(const NormArgs* __restrict__ ctxs) {
  const NormArgs a = ctxs[blockIdx.x];
  norms_block(a);
}

// ---------------------------------------------------------------------------
// Launch wrappers.

// Batched form: many contexts in one persistent launch.  ctxs[] holds each
// context's arguments (input pointers and row counts refreshed per update),
// items[] the tiles of all contexts sharing this stride, longest first; every
// workgroup walks the item list with a grid-sized stride.
template <int P, int TM, int TN, int STR, bool VL, int KMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == PREC_BF16X3 ? 1 : 4))) void k_update_batch(
    const UpdArgs* __restrict__ ctxs,
                                                      const UpdItem* __restrict__ items, int nitems) {
  __shared__ __attribute__((aligned(16))) char smem[upd_smem_bytes<P, STR, VL>()];
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const UpdItem it = items[i];
    const UpdArgs a = ctxs[it.ctx];
    upd_dispatch<P, TM, TN, STR, VL, KMAX>(a, it, smem);
    __syncthreads();  // the next item reuses the LDS chunk buffer
  }
}

// ---------------------------------------------------------------------------
// Four tiles per workgroup (f32/f64/split-bf16 rows of 16-byte multiples): 16 waves,
// wave w works on tile w / 4 with row group w % 4 of every chunk.  A row
// group's rows are copied into LDS once (the four waves that use them split
// the copy) and read by all four tiles, so each chunk row crosses a CU's
// load path once per four tiles.  One workgroup-wide barrier per chunk: after
// it the chunk is in its buffer for everyone and nobody reads the other
// buffer any more, so the copy of the next chunk starts before the k-steps.

template <int P, int STR> struct QuadGeom {
  static constexpr int ES = (P == PREC_F64) ? 8 : 4;
  static constexpr int X = UPD_DIRECT_BYTES / (STR * ES);
  static constexpr int RG = X >= 32 ? X / 32 * 32 : 16;      // rows per row group and chunk
  static constexpr int R = 4 * RG;                          // rows per chunk
  static constexpr int SU = STR * ES / 16;                  // 16-byte units per LDS row
  static constexpr int GU = (RG * SU + 63) / 64 * 64;       // units per row-group buffer
  static constexpr int NQ = GU / 64;                        // 64-lane copies per row group
  static constexpr int BUFB = GU * 16;                      // one row group's chunk buffer, bytes
  // row group g's two buffers sit at 2 g BUFB and (2 g + 1) BUFB, so every
  // LDS read offset from a lane's base stays an immediate (< 64 KB)
  static constexpr int REDB = 16 * 4 * 256 * ES;            // cross-wave reduction, bytes
  static constexpr int SMEM = 8 * BUFB > REDB ? 8 * BUFB : REDB;
  static constexpr bool OK = SMEM <= 163840 && (P != PREC_BF16X3 || RG % 32 == 0);
};

template <int P, int STR> struct QuadLanes {
  static constexpr int NQW = (QuadGeom<P, STR>::NQ + 3) / 4;  // copies per wave
  uint32_t off[NQW];
};

// This lane's byte offsets (from its row group's first row) of the units it
// copies: copy i of tile t is the row group's 64-unit slice t + 4 i.
template <int P, int STR>
__device__ __forceinline__ void quad_lanes(QuadLanes<P, STR>& ql, int n, int tile) {
  using G = QuadGeom<P, STR>;
  const int upr = n * G::ES / 16;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < QuadLanes<P, STR>::NQW; ++i) {
    const int u = (tile + 4 * i) * 64 + lane;
    const int r = u / G::SU, c = u - r * G::SU;
    ql.off[i] = (c < upr && r < G::RG) ? (uint32_t)((r * upr + c) * 16) : 0u;
  }
}

template <int P, int STR>
__device__ __forceinline__ void quad_issue(char* gbuf, const UpdArgs& a, const QuadLanes<P, STR>& ql, int ci,
                                           int ncp, int rg, int tile) {
  using G = QuadGeom<P, STR>;
  const int upr = a.n * G::ES / 16;
  const bool plus = ci < ncp;
  const int r0 = (plus ? ci : ci - ncp) * G::R + rg * G::RG;
  const int rows = (plus ? a.np : a.nm) - r0;
  const char* src = (const char*)(plus ? a.xp : a.xm) + (int64_t)r0 * upr * 16;
  const uint32_t lim = rows >= G::RG ? 0xffffffffu : (rows > 0 ? (uint32_t)(rows * upr * 16) : 0u);
#pragma unroll
  for (int i = 0; i < QuadLanes<P, STR>::NQW; ++i) {
    const int q = tile + 4 * i;
    if (q < G::NQ) {
      const char* g = ql.off[i] < lim ? src + ql.off[i] : (const char*)a.zero;
      __builtin_amdgcn_global_load_lds((const void*)g,
                                       (__attribute__((address_space(3))) void*)(gbuf + q * 1024), 16, 0, 0);
    }
  }
}

// TM x TN: the tile's 16 x 16 fragments that lie inside its pivot GEMM (a
// ragged edge tile multiplies only those)
// SHL (a.shl): the tile's fragments share the last factor of their left
// columns, read once per row for all of them.
template <int P, int H, int MR, int STR, int TM, int TN, bool SHL = false>
__device__ void upd_quad_body(const UpdArgs& a, const UpdItem& it, char* smem) {
  constexpr int NF = TM * TN;
  using T = typename Tr<P>::X;
  using Acc = typename Tr<P>::Acc;
  using A1 = typename Tr<P>::A1;
  using G = QuadGeom<P, STR>;
  constexpr int ES = G::ES;
  constexpr int NKS = G::RG / 4;
  constexpr int K_ORD = H + MR;
  constexpr int MRC = MR > 0 ? MR : 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tile = wave >> 2, rg = wave & 3;
  const int ltid = tid & 255;  // thread index inside the tile's four waves
  const LeftCol* __restrict__ left = a.left[K_ORD];
  const RightCol* __restrict__ right = a.right[K_ORD];
  const int R = G::R;
  const int ncp = (a.np + R - 1) / R;
  const int nch = ncp + (a.nm + R - 1) / R;

  char* gbuf = smem + 2 * rg * G::BUFB;

  // k-step s of lane group q = lane / 16 reads row 4 s + q: single-address
  // LDS reads whose k-step offsets all fit the 16-bit immediate, so no
  // address register is spent per k-step
  const int lrow = lane >> 4;
  const int lbase = 2 * rg * G::BUFB;
  // f32: the element offsets are found before the main loop and the
  // running sums are loaded during the last chunk; f64 and split-bf16 find and load them after
  // the loop (held through it they would push the allocation past 128
  // registers into scratch)
  constexpr bool EPF = P == PREC_F32;
  constexpr int NE = EPF ? NF : 1;
  // the tile's table entries are requested before chunk 0's copy, so that
  // waiting for them does not wait for the copy as well; empty tiles (the
  // launch's padding) have M = N = 0 and read row/column 0
  LeftCol La[TM], Le[NE];
  RightCol Rb[TN], Re[NE];
#pragma unroll
  for (int f = 0; f < TM; ++f) La[f] = left[it.lrow0 + max(0, min(it.r0 + 16 * f + (lane & 15), it.M - 1))];
#pragma unroll
  for (int g = 0; g < TN; ++g) Rb[g] = right[it.rcol0 + max(0, min(it.c0 + 16 * g + (lane & 15), it.N - 1))];
  if constexpr (EPF) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int f = j / TN, g = j % TN;
      Le[j] = left[it.lrow0 + max(0, min(it.r0 + 16 * f + ((ltid >> 4) & 15), it.M - 1))];
      Re[j] = right[it.rcol0 + max(0, min(it.c0 + 16 * g + (ltid & 15), it.N - 1))];
    }
  }
  QuadLanes<P, STR> ql;
  quad_lanes<P, STR>(ql, a.n, tile);
  quad_issue<P, STR>(gbuf, a, ql, 0, ncp, rg, tile);

  int ao[TM][H];
  int bo[TN][MRC];
#pragma unroll
  for (int f = 0; f < TM; ++f)
#pragma unroll
    for (int q = 0; q < H; ++q) ao[f][q] = lbase + (lrow * STR + (La[f].c[q] < a.n ? La[f].c[q] : 0)) * ES;
#pragma unroll
  for (int g = 0; g < TN; ++g)
#pragma unroll
    for (int q = 0; q < MRC; ++q)
      bo[g][q] = lbase + (lrow * STR + ((q < MR && Rb[g].c[q] < a.n) ? Rb[g].c[q] : 0)) * ES;
  auto elem_offset = [&](int j) __attribute__((always_inline)) -> int64_t {
    const int f = j / TN, g = j - (j / TN) * TN;
    const int r = it.r0 + 16 * f + ((ltid >> 4) & 15), c = it.c0 + 16 * g + (ltid & 15);
    if (r >= it.M || c >= it.N) return -1;
    const LeftCol L = left[it.lrow0 + r];
    const RightCol Rc = right[it.rcol0 + c];
    bool pad = false;
#pragma unroll
    for (int q = 0; q < H; ++q) pad = pad || L.c[q] >= a.n;
#pragma unroll
    for (int q = 0; q < MR; ++q) pad = pad || Rc.c[q] >= a.n;
    return pad ? -1 : L.base + Rc.base;
  };
  int64_t eoff[NF];
  if constexpr (EPF) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int f = j / TN, g = j % TN;
      const int r = it.r0 + 16 * f + ((ltid >> 4) & 15), c = it.c0 + 16 * g + (ltid & 15);
      bool pad = r >= it.M || c >= it.N;
#pragma unroll
      for (int q = 0; q < H; ++q) pad = pad || Le[j].c[q] >= a.n;
#pragma unroll
      for (int q = 0; q < MR; ++q) pad = pad || Re[j].c[q] >= a.n;
      eoff[j] = pad ? -1 : Le[j].base + Re[j].base;
    }
  }

  Acc acc[TM][TN];
#pragma unroll
  for (int f = 0; f < TM; ++f)
#pragma unroll
    for (int g = 0; g < TN; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[f][g][r] = A1(0);

  // split-BF16x3 k-step: 32 rows, K index 8 q + j of lane group q = lane / 16
  // is row 32 s + 4 j + q (the f32 k-steps 8 s .. 8 s + 7); each product
  // v = hi + lo with hi = RNE_bf16(v), lo = RNE_bf16(v - hi), and
  // a b ~ ah bh + ah bl + al bh, accumulated in FP32
  auto multiply_chunk_bf16 = [&](auto bo_c) __attribute__((always_inline)) {
    constexpr int BO = decltype(bo_c)::value;
    if constexpr (P == PREC_BF16X3) {
#pragma unroll
    for (int st = 0; st < G::RG / 32; ++st) {
      uint32_t Ah[TM][4], Al[TM][4], Bh[TN][4], Bl[TN][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // rows of K indices 2i and 2i + 1
        const int so0 = (32 * st + 8 * i) * STR * ES + BO, so1 = so0 + 4 * STR * ES;
        float l0 = 1.0f, l1 = 1.0f;
        if constexpr (SHL) {
          l0 = *(const float*)(smem + ao[0][H - 1] + so0);
          l1 = *(const float*)(smem + ao[0][H - 1] + so1);
        }
#pragma unroll
        for (int f = 0; f < TM; ++f) {
          float v0 = *(const float*)(smem + ao[f][0] + so0);
          float v1 = *(const float*)(smem + ao[f][0] + so1);
#pragma unroll
          for (int q = 1; q < (SHL ? H - 1 : H); ++q) {
            v0 *= *(const float*)(smem + ao[f][q] + so0);
            v1 *= *(const float*)(smem + ao[f][q] + so1);
          }
          if constexpr (SHL) {
            v0 *= l0;
            v1 *= l1;
          }
          split_pair(v0, v1, Ah[f][i], Al[f][i]);
        }
#pragma unroll
        for (int g = 0; g < TN; ++g) {
          float v0 = 1.0f, v1 = 1.0f;
          if constexpr (MR > 0) {
            v0 = *(const float*)(smem + bo[g][0] + so0);
            v1 = *(const float*)(smem + bo[g][0] + so1);
#pragma unroll
            for (int q = 1; q < MR; ++q) {
              v0 *= *(const float*)(smem + bo[g][q] + so0);
              v1 *= *(const float*)(smem + bo[g][q] + so1);
            }
          }
          split_pair(v0, v1, Bh[g][i], Bl[g][i]);
        }
        // at most two rows' reads in flight (all eight would not fit in
        // registers)
        __builtin_amdgcn_sched_barrier(0);
      }
      // the matrix instructions at raised wave priority, so that a wave whose
      // operands are ready keeps the matrix core busy while the others split
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int g = 0; g < TN; ++g) {
          const bf16x8 ah = as_bf16x8(Ah[f]), al = as_bf16x8(Al[f]);
          const bf16x8 bh = as_bf16x8(Bh[g]), bl = as_bf16x8(Bl[g]);
          acc[f][g] = mma16(al, bh, acc[f][g]);
          acc[f][g] = mma16(ah, bl, acc[f][g]);
          acc[f][g] = mma16(ah, bh, acc[f][g]);
        }
      __builtin_amdgcn_s_setprio(0);
    }
    }
  };

  auto multiply_chunk = [&](auto bo_c) __attribute__((always_inline)) {
    if constexpr (P == PREC_BF16X3) {
      multiply_chunk_bf16(bo_c);
      return;
    }
    constexpr int BO = decltype(bo_c)::value;
    constexpr bool PIPE = (P == PREC_F32 || P == PREC_F64);
    constexpr int NB = PIPE ? 2 : 1;
    T fa[NB][TM][H], fb[NB][TN][MRC];
    auto load_factors = [&](int st, int buf) __attribute__((always_inline)) {
      const int so = 4 * st * STR * ES + BO;
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int q = 0; q < H; ++q)
          if (!SHL || q < H - 1 || f == 0) fa[buf][f][q] = *(const T*)(smem + ao[f][q] + so);
#pragma unroll
      for (int g = 0; g < TN; ++g)
#pragma unroll
        for (int q = 0; q < MR; ++q) fb[buf][g][q] = *(const T*)(smem + bo[g][q] + so);
    };
    load_factors(0, 0);
#pragma unroll
    for (int st = 0; st < NKS; ++st) {
      const int cur = PIPE ? (st & 1) : 0;
      if (PIPE && st + 1 < NKS) load_factors(st + 1, cur ^ 1);
      if (!PIPE && st > 0) load_factors(st, 0);
      // the next k-step's LDS reads stay ahead of this k-step's products
      // (left alone, the scheduler sinks each read to its use)
      if constexpr (PIPE) __builtin_amdgcn_sched_barrier(0);
      T A[TM], B[TN];
#pragma unroll
      for (int f = 0; f < TM; ++f) {
        T v = fa[cur][f][0];
#pragma unroll
        for (int q = 1; q < H; ++q) v *= fa[cur][SHL && q == H - 1 ? 0 : f][q];
        A[f] = v;
      }
#pragma unroll
      for (int g = 0; g < TN; ++g) {
        T v = T(1);
        if constexpr (MR > 0) {
          v = fb[cur][g][0];
#pragma unroll
          for (int q = 1; q < MR; ++q) v *= fb[cur][g][q];
        }
        B[g] = v;
      }
      // the k-step's matrix instructions issue back to back at raised wave
      // priority, the other waves' LDS reads and products fill in around them
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int f = 0; f < TM; ++f)
#pragma unroll
        for (int g = 0; g < TN; ++g) acc[f][g] = mma(A[f], B[g], acc[f][g]);
      __builtin_amdgcn_s_setprio(0);
    }
  };

  A1* shi = (A1*)a.s_hi[K_ORD];
  A1* slo = (A1*)a.s_lo[K_ORD];
  A1* snp = (A1*)a.snap[K_ORD];
  A1 ph[NF], pl[NF], ps[NF];
  auto load_state = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      ph[j] = pl[j] = ps[j] = A1(0);
      if (eoff[j] >= 0 && a.fifo != 3) {
        ph[j] = shi[eoff[j]];
        pl[j] = slo[eoff[j]];
        if (a.fifo == 2) ps[j] = snp[eoff[j]];
      }
    }
  };

  auto run_chunk = [&](int ci) __attribute__((always_inline)) {
    __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();
    if (ci + 1 < nch) quad_issue<P, STR>(gbuf + ((ci + 1) & 1) * G::BUFB, a, ql, ci + 1, ncp, rg, tile);
    if constexpr (EPF)
      if (ci + 1 == nch) load_state();  // arrives during the last chunk's k-steps
    if (ci & 1) multiply_chunk(IntC<G::BUFB>{});
    else multiply_chunk(IntC<0>{});
  };
  // sign: plus chunks, then the minus chunks into the negated accumulators
  int ci = 0;
  for (; ci < ncp; ++ci) run_chunk(ci);
  if (nch > ncp) {
#pragma unroll
    for (int f = 0; f < TM; ++f)
#pragma unroll
      for (int g = 0; g < TN; ++g) acc[f][g] = -acc[f][g];
    for (; ci < nch; ++ci) run_chunk(ci);
#pragma unroll
    for (int f = 0; f < TM; ++f)
#pragma unroll
      for (int g = 0; g < TN; ++g) acc[f][g] = -acc[f][g];
  }

  // each tile's four row-group partials, summed in a fixed order (row group
  // 0 + 1 + 2 + 3), then the compensated fold of every stored element; every
  // wave owns four fragment slots of the buffer whatever its tile's shape
  A1* red = (A1*)smem;
  if constexpr (EPF)
    if (nch == 0) load_state();
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const int f = q / TN, g = q % TN;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      red[((tile * 4 + rg) * 4 + q) * 256 + frag_row<P>(lane, r) * 16 + (lane & 15)] = acc[f][g][r];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    int64_t off;
    if constexpr (EPF) off = eoff[j];
    else off = elem_offset(j);
    if (off >= 0) {
      const int e = j * 256 + ltid;
      const A1* rt = red + tile * 4 * 4 * 256;
      const A1 sum = ((rt[e] + rt[4 * 256 + e]) + rt[2 * 4 * 256 + e]) + rt[3 * 4 * 256 + e];
      if (a.fifo == 3) {  // the increment alone, folded in by a later launch
        shi[off] = sum;
        continue;
      }
      A1 h, l, sn = A1(0);
      if constexpr (EPF) {
        h = ph[j];
        l = pl[j];
        sn = ps[j];
      } else {
        h = shi[off];
        l = slo[off];
        if (a.fifo == 2) sn = snp[off];
      }
      fold_val<A1>(h, l, sum);
      // FIFO: the batch leaving the window, its increment exactly as it was added
      if (a.fifo == 2) fold_val<A1>(h, l, -sn);
      shi[off] = h;
      slo[off] = l;
      if (a.fifo) snp[off] = sum;
    }
  }
}

template <int P, int H, int MR, int STR>
__device__ __forceinline__ void upd_quad_shape(const UpdArgs& a, const UpdItem& it, char* smem) {
  // empty padding tiles (M = N = 0) take the 1 x 1 shape
  const bool m2 = it.M - it.r0 > 16, n2 = it.N - it.c0 > 16;
  if constexpr (H >= 2) {
    if (m2 && a.shl) {
      if (n2) upd_quad_body<P, H, MR, STR, 2, 2, true>(a, it, smem);
      else upd_quad_body<P, H, MR, STR, 2, 1, true>(a, it, smem);
      return;
    }
  }
  if (m2 && n2) upd_quad_body<P, H, MR, STR, 2, 2>(a, it, smem);
  else if (m2) upd_quad_body<P, H, MR, STR, 2, 1>(a, it, smem);
  else if (n2) upd_quad_body<P, H, MR, STR, 1, 2>(a, it, smem);
  else upd_quad_body<P, H, MR, STR, 1, 1>(a, it, smem);
}

// Each tile's waves take the body of its order and shape; every body runs
// the same chunk loop (same barriers), so the tiles of one workgroup may
// differ in both.
// Batched form: every workgroup walks groups of four tiles of one member
// (its arguments from ctxs[]); all tiles of a group share the member's rows,
// so its waves pass the same barriers.
template <int P, int STR, int KMAX>
__global__ __launch_bounds__(1024) void k_update_quad_batch(const UpdArgs* __restrict__ ctxs,
                                                            const UpdItem* __restrict__ items, int ngroups) {
  __shared__ __attribute__((aligned(16))) char smem[QuadGeom<P, STR>::SMEM];
  const int tile = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
  for (int q = blockIdx.x; q < ngroups; q += gridDim.x) {
    const UpdItem it = items[q * 4 + tile];
    const UpdArgs& a = ctxs[it.ctx];
    switch (it.k) {
      case 1: upd_quad_shape<P, 1, 0, STR>(a, it, smem); break;
      case 2: upd_quad_shape<P, 1, 1, STR>(a, it, smem); break;
      case 3: upd_quad_shape<P, 2, 1, STR>(a, it, smem); break;
      case 4: upd_quad_shape<P, 2, 2, STR>(a, it, smem); break;
      case 5: if constexpr (KMAX >= 5) upd_quad_shape<P, 3, 2, STR>(a, it, smem); break;
      case 6: if constexpr (KMAX >= 6) upd_quad_shape<P, 3, 3, STR>(a, it, smem); break;
      default: break;
    }
    __syncthreads();  // the next group's chunk 0 lands on the reduction buffer
  }
}

template <int P, int STR, int KMAX>
__global__ __launch_bounds__(1024) void k_update_quad(UpdArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[QuadGeom<P, STR>::SMEM];
  if (a.with_norms && blockIdx.x == gridDim.x - 1) {
    norms_block(a.na);
    return;
  }
  // the item's address is uniform per wave: a scalar load
  const int tile = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
  const UpdItem it = a.items[blockIdx.x * 4 + tile];
  switch (it.k) {
    case 1: upd_quad_shape<P, 1, 0, STR>(a, it, smem); break;
    case 2: upd_quad_shape<P, 1, 1, STR>(a, it, smem); break;
    case 3: upd_quad_shape<P, 2, 1, STR>(a, it, smem); break;
    case 4: upd_quad_shape<P, 2, 2, STR>(a, it, smem); break;
    case 5: if constexpr (KMAX >= 5) upd_quad_shape<P, 3, 2, STR>(a, it, smem); break;
    case 6: if constexpr (KMAX >= 6) upd_quad_shape<P, 3, 3, STR>(a, it, smem); break;
    default: break;
  }
}

template <int P, int STR, bool VL>
static hipError_t launch_batch_one(int kmax, const UpdArgs* ctxs, const UpdItem* items, int nitems, int grid,
                                   hipStream_t st) {
  if constexpr (ChunkGeom<P, STR>::R >= ChunkGeom<P, STR>::UB) {
    if (kmax <= 4)
      hipLaunchKernelGGL((k_update_batch<P, 2, 2, STR, VL, 4>), dim3(grid), dim3(256), 0, st, ctxs, items, nitems);
    else
      hipLaunchKernelGGL((k_update_batch<P, 2, 2, STR, VL, 6>), dim3(grid), dim3(256), 0, st, ctxs, items, nitems);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t launch_batch_p(int str, bool vl, int kmax, const UpdArgs* ctxs, const UpdItem* items,
                                 int nitems, int grid, hipStream_t st) {
  switch (str) {
    case 36: return vl ? launch_batch_one<P, 36, true>(kmax, ctxs, items, nitems, grid, st)
                       : launch_batch_one<P, 36, false>(kmax, ctxs, items, nitems, grid, st);
    case 68: return vl ? launch_batch_one<P, 68, true>(kmax, ctxs, items, nitems, grid, st)
                       : launch_batch_one<P, 68, false>(kmax, ctxs, items, nitems, grid, st);
    case 132: return vl ? launch_batch_one<P, 132, true>(kmax, ctxs, items, nitems, grid, st)
                        : launch_batch_one<P, 132, false>(kmax, ctxs, items, nitems, grid, st);
    case 260: return vl ? launch_batch_one<P, 260, true>(kmax, ctxs, items, nitems, grid, st)
                        : launch_batch_one<P, 260, false>(kmax, ctxs, items, nitems, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int STR>
static hipError_t launch_quad_batch_s(int kmax, const UpdArgs* ctxs, const UpdItem* items, int nitems, int grid,
                                      hipStream_t st) {
  if constexpr (QuadGeom<P, STR>::OK) {
    if (nitems % 4) return hipErrorInvalidValue;
    if (kmax <= 4)
      hipLaunchKernelGGL((k_update_quad_batch<P, STR, 4>), dim3(grid), dim3(1024), 0, st, ctxs, items, nitems / 4);
    else
      hipLaunchKernelGGL((k_update_quad_batch<P, STR, 6>), dim3(grid), dim3(1024), 0, st, ctxs, items, nitems / 4);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t launch_quad_batch_p(int str, int kmax, const UpdArgs* ctxs, const UpdItem* items, int nitems,
                                      int grid, hipStream_t st) {
  switch (str) {
    case 36: return launch_quad_batch_s<P, 36>(kmax, ctxs, items, nitems, grid, st);
    case 68: return launch_quad_batch_s<P, 68>(kmax, ctxs, items, nitems, grid, st);
    case 132: return launch_quad_batch_s<P, 132>(kmax, ctxs, items, nitems, grid, st);
    case 260: return launch_quad_batch_s<P, 260>(kmax, ctxs, items, nitems, grid, st);
    default: return hipErrorInvalidValue;
  }
}

bool update_quad_batch_supported(int prec, int str) {
  auto ok = [&](auto p) {
    constexpr int PP = decltype(p)::value;
    switch (str) {
      case 36: return QuadGeom<PP, 36>::OK;
      case 68: return QuadGeom<PP, 68>::OK;
      case 132: return QuadGeom<PP, 132>::OK;
      case 260: return QuadGeom<PP, 260>::OK;
      default: return false;
    }
  };
  if (prec == PREC_F32) return ok(IntC<PREC_F32>{});
  if (prec == PREC_F64) return ok(IntC<PREC_F64>{});
  if (prec == PREC_BF16X3) return ok(IntC<PREC_BF16X3>{});
  return false;
}

hipError_t launch_update_quad_batch(int prec, int str, int kmax, const UpdArgs* ctxs, const UpdItem* items,
                                    int nitems, int grid, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (kmax < 1 || kmax > 6) return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return launch_quad_batch_p<PREC_F64>(str, kmax, ctxs, items, nitems, grid, st);
    case PREC_F32: return launch_quad_batch_p<PREC_F32>(str, kmax, ctxs, items, nitems, grid, st);
    case PREC_BF16X3: return launch_quad_batch_p<PREC_BF16X3>(str, kmax, ctxs, items, nitems, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_update_batch(int prec, int str, bool vl, int kmax, const UpdArgs* ctxs, const UpdItem* items,
                               int nitems, int grid, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  switch (prec) {
    case PREC_F64: return launch_batch_p<PREC_F64>(str, vl, kmax, ctxs, items, nitems, grid, st);
    case PREC_F32: return launch_batch_p<PREC_F32>(str, vl, kmax, ctxs, items, nitems, grid, st);
    case PREC_BF16X3: return launch_batch_p<PREC_BF16X3>(str, vl, kmax, ctxs, items, nitems, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fold_splits(FoldArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.tot) return;
  int k = 1;
  for (int q = 2; q <= a.d; ++q)
    if (i >= a.off[q]) k = q;
  const int64_t e = i - a.off[k];
  T* hp = (T*)a.s_hi[1];
  T* lp = (T*)a.s_lo[1];
#pragma unroll
  for (int q = 2; q <= CUM_MAXD; ++q)
    if (k == q) {
      hp = (T*)a.s_hi[q];
      lp = (T*)a.s_lo[q];
    }
  T hi = a.fresh ? T(0) : hp[e], lo = a.fresh ? T(0) : lp[e];
  T* sp = (T*)a.split;
  if (a.single) {
    fold_val(hi, lo, sp[i]);
    hp[e] = hi;
    lp[e] = lo;
    return;
  }
  for (int s = 0; s < a.nsplit; ++s) {
    T* h = sp + (2 * (int64_t)s) * a.tot + i;
    T* l = sp + (2 * (int64_t)s + 1) * a.tot + i;
    fold_val(hi, lo, *h);
    fold_val(hi, lo, *l);
    *h = T(0);
    *l = T(0);
  }
  hp[e] = hi;
  lp[e] = lo;
}

hipError_t launch_fold_splits(int prec, const FoldArgs& a, hipStream_t st) {
  if (a.tot <= 0 || a.nsplit <= 0) return hipSuccess;
  const dim3 grid((unsigned)((a.tot + 255) / 256));
  if (prec == PREC_F64) hipLaunchKernelGGL(k_fold_splits<double>, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_fold_splits<float>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero(ZeroArgs a) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int q = 0; q < a.count; ++q) {
    uint32_t* p = (uint32_t*)a.ptr[q];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.words[q]; i += stride) p[i] = 0u;
  }
}

hipError_t launch_zero(const ZeroArgs& a, hipStream_t st) {
  if (a.count <= 0) return hipSuccess;
  if (a.count > ZERO_MAX) return hipErrorInvalidValue;
  int64_t mx = 0;
  for (int q = 0; q < a.count; ++q) mx = a.words[q] > mx ? a.words[q] : mx;
  const int64_t grid = (mx + 255) / 256 < 2048 ? (mx + 255) / 256 : 2048;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

// e0/e1 (may be null) take the kernel's own start and end timestamps.
template <int P, int STR, bool VL>
static void launch_kmax(int kmax, const UpdArgs& a, int nitems, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (VL && QuadGeom<P, STR>::OK) {
    if (a.quad) {
      // a.items holds nitems rounded up to whole groups of four
      const dim3 grid((unsigned)((nitems + 3) / 4 + (a.with_norms ? 1 : 0)));
      if (kmax <= 4) hipExtLaunchKernelGGL((k_update_quad<P, STR, 4>), grid, dim3(1024), 0, st, e0, e1, 0, a);
      else hipExtLaunchKernelGGL((k_update_quad<P, STR, 6>), grid, dim3(1024), 0, st, e0, e1, 0, a);
      return;
    }
  }
  const dim3 grid((unsigned)(nitems + (a.with_norms ? 1 : 0)));
  if (kmax <= 4) hipExtLaunchKernelGGL((k_update<P, 2, 2, STR, VL, 4>), grid, dim3(256), 0, st, e0, e1, 0, a);
  else hipExtLaunchKernelGGL((k_update<P, 2, 2, STR, VL, 6>), grid, dim3(256), 0, st, e0, e1, 0, a);
}

// Whether launch_update takes the four-tiles-per-workgroup kernel for this
// precision and row length (16-byte rows, and its buffers fit in LDS).
bool update_quad_supported(int prec, int n) {
  const int str = update_lds_stride(n);
  auto ok = [&](auto p) {
    constexpr int PP = decltype(p)::value;
    switch (str) {
      case 36: return QuadGeom<PP, 36>::OK;
      case 68: return QuadGeom<PP, 68>::OK;
      case 132: return QuadGeom<PP, 132>::OK;
      case 260: return QuadGeom<PP, 260>::OK;
      default: return false;
    }
  };
  if (prec == PREC_F32) return ok(IntC<PREC_F32>{});
  if (prec == PREC_F64) return ok(IntC<PREC_F64>{});
  if (prec == PREC_BF16X3) return ok(IntC<PREC_BF16X3>{});
  return false;
}

template <int P, int STR>
static hipError_t launch_one(int kmax, const UpdArgs& a, int nitems, hipStream_t st, hipEvent_t e0,
                             hipEvent_t e1) {
  if constexpr (ChunkGeom<P, STR>::R >= ChunkGeom<P, STR>::UB) {
    if (a.vec) launch_kmax<P, STR, true>(kmax, a, nitems, st, e0, e1);
    else launch_kmax<P, STR, false>(kmax, a, nitems, st, e0, e1);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t launch_update_p(int str, int kmax, const UpdArgs& a, int nitems, hipStream_t st, hipEvent_t e0,
                                  hipEvent_t e1) {
  switch (str) {
    case 36: return launch_one<P, 36>(kmax, a, nitems, st, e0, e1);
    case 68: return launch_one<P, 68>(kmax, a, nitems, st, e0, e1);
    case 132: return launch_one<P, 132>(kmax, a, nitems, st, e0, e1);
    case 260: return launch_one<P, 260>(kmax, a, nitems, st, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

bool update_tile_supported(int tm, int tn) { return tm == 2 && tn == 2; }

int update_lds_stride(int n) {
  return n <= 32 ? 36 : n <= 64 ? 68 : n <= 128 ? 132 : n <= 256 ? 260 : 0;
}

// 0 when the precision cannot use this stride (bf16x3 needs 128-row chunks).
int update_chunk_rows(int prec, int str) {
  switch (prec) {
    case PREC_F64:
      return str == 36 ? ChunkGeom<PREC_F64, 36>::R : str == 68 ? ChunkGeom<PREC_F64, 68>::R
           : str == 132 ? ChunkGeom<PREC_F64, 132>::R : ChunkGeom<PREC_F64, 260>::R;
    case PREC_F32:
      return str == 36 ? ChunkGeom<PREC_F32, 36>::R : str == 68 ? ChunkGeom<PREC_F32, 68>::R
           : str == 132 ? ChunkGeom<PREC_F32, 132>::R : ChunkGeom<PREC_F32, 260>::R;
    default:
      return str == 36 ? ChunkGeom<PREC_BF16X3, 36>::R : str == 68 ? ChunkGeom<PREC_BF16X3, 68>::R
           : str == 132 ? ChunkGeom<PREC_BF16X3, 132>::R : ChunkGeom<PREC_BF16X3, 260>::R;
  }
}

hipError_t launch_update(int prec, int tm, int tn, int kmax, const UpdArgs& a, int nitems, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1) {
  if (nitems <= 0) return hipSuccess;
  if (!update_tile_supported(tm, tn) || kmax < 1 || kmax > 6) return hipErrorInvalidValue;
  const int str = update_lds_stride(a.n);
  switch (prec) {
    case PREC_F64: return launch_update_p<PREC_F64>(str, kmax, a, nitems, st, e0, e1);
    case PREC_F32: return launch_update_p<PREC_F32>(str, kmax, a, nitems, st, e0, e1);
    case PREC_BF16X3: return launch_update_p<PREC_BF16X3>(str, kmax, a, nitems, st, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

template <int S, typename St>
static hipError_t launch_combine_s(const CombArgs& a, int64_t nblocks, hipStream_t st) {
  const dim3 grid((unsigned)nblocks), blk(256);
  // staged sub-blocks: (b+1)^S - 1 - b^S doubles
  int64_t tot = 1, bs = 1;
  for (int q = 0; q < S; ++q) { tot *= (a.b + 1); bs *= a.b; }
  tot = tot - 1 - bs;
  const size_t bytes = (size_t)tot * sizeof(double);
  if (bytes <= COMB_STAGE_BYTES) {
    if (a.rec) hipLaunchKernelGGL((k_combine<S, St, true, true>), grid, blk, bytes, st, a);
    else hipLaunchKernelGGL((k_combine<S, St, true, false>), grid, blk, bytes, st, a);
  } else {
    if (a.rec) hipLaunchKernelGGL((k_combine<S, St, false, true>), grid, blk, 0, st, a);
    else hipLaunchKernelGGL((k_combine<S, St, false, false>), grid, blk, 0, st, a);
  }
  return hipGetLastError();
}

template <typename St>
static hipError_t launch_combine_t(int s, const CombArgs& a, int64_t nblocks, hipStream_t st) {
  switch (s) {
    case 1: return launch_combine_s<1, St>(a, nblocks, st);
    case 2: return launch_combine_s<2, St>(a, nblocks, st);
    case 3: return launch_combine_s<3, St>(a, nblocks, st);
    case 4: return launch_combine_s<4, St>(a, nblocks, st);
    case 5: return launch_combine_s<5, St>(a, nblocks, st);
    case 6: return launch_combine_s<6, St>(a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_combine(int prec, int s, const CombArgs& a, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (prec == PREC_F64) return launch_combine_t<double>(s, a, nblocks, st);
  return launch_combine_t<float>(s, a, nblocks, st);
}

template <int S, typename St>
static hipError_t launch_combine_batch_s(const CombArgs* ctxs, const int64_t* items, int nitems, int grid,
                                         size_t stage_bytes, bool rec, hipStream_t st) {
  if (stage_bytes <= COMB_STAGE_BYTES) {
    if (rec)
      hipLaunchKernelGGL((k_combine_batch<S, St, true, true>), dim3(grid), dim3(256), stage_bytes, st, ctxs, items,
                         nitems);
    else
      hipLaunchKernelGGL((k_combine_batch<S, St, true, false>), dim3(grid), dim3(256), stage_bytes, st, ctxs, items,
                         nitems);
  } else {
    if (rec)
      hipLaunchKernelGGL((k_combine_batch<S, St, false, true>), dim3(grid), dim3(256), 0, st, ctxs, items, nitems);
    else
      hipLaunchKernelGGL((k_combine_batch<S, St, false, false>), dim3(grid), dim3(256), 0, st, ctxs, items, nitems);
  }
  return hipGetLastError();
}

template <typename St>
static hipError_t launch_combine_batch_t(int s, const CombArgs* ctxs, const int64_t* items, int nitems, int grid,
                                         size_t stage_bytes, bool rec, hipStream_t st) {
  switch (s) {
    case 1: return launch_combine_batch_s<1, St>(ctxs, items, nitems, grid, stage_bytes, rec, st);
    case 2: return launch_combine_batch_s<2, St>(ctxs, items, nitems, grid, stage_bytes, rec, st);
    case 3: return launch_combine_batch_s<3, St>(ctxs, items, nitems, grid, stage_bytes, rec, st);
    case 4: return launch_combine_batch_s<4, St>(ctxs, items, nitems, grid, stage_bytes, rec, st);
    case 5: return launch_combine_batch_s<5, St>(ctxs, items, nitems, grid, stage_bytes, rec, st);
    case 6: return launch_combine_batch_s<6, St>(ctxs, items, nitems, grid, stage_bytes, rec, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_combine_batch(int prec, int s, const CombArgs* ctxs, const int64_t* items, int nitems,
                                int grid, size_t stage_bytes, bool rec, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (prec == PREC_F64) return launch_combine_batch_t<double>(s, ctxs, items, nitems, grid, stage_bytes, rec, st);
  return launch_combine_batch_t<float>(s, ctxs, items, nitems, grid, stage_bytes, rec, st);
}

hipError_t launch_norms_batch(const NormArgs* ctxs, int m, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norms_batch, dim3(m), dim3(1024), 0, st, ctxs);
  return hipGetLastError();
}

template <int S, typename St>
static hipError_t launch_lattice_s(bool rec, const LatArgs& a, int64_t nblocks, size_t lds, hipStream_t st) {
  if (rec) hipLaunchKernelGGL((k_combine_lattice<S, St, true>), dim3((unsigned)nblocks), dim3(64), lds, st, a);
  else hipLaunchKernelGGL((k_combine_lattice<S, St, false>), dim3((unsigned)nblocks), dim3(64), lds, st, a);
  return hipGetLastError();
}

template <int S, int B, typename St>
static hipError_t launch_lattice_fix(bool rec, const LatArgs& a, int64_t nblocks, size_t lds, hipStream_t st) {
  if (rec) hipLaunchKernelGGL((k_combine_lattice_fix<S, B, St, true>), dim3((unsigned)nblocks), dim3(64), lds, st, a);
  else hipLaunchKernelGGL((k_combine_lattice_fix<S, B, St, false>), dim3((unsigned)nblocks), dim3(64), lds, st, a);
  return hipGetLastError();
}

template <typename St>
static hipError_t launch_lattice_t(int d, bool rec, const LatArgs& a, int64_t nblocks, size_t lds, hipStream_t st) {
  if (lat_fix_ok(d, a.b)) {
    switch (d * 16 + a.b) {
      case 2 * 16 + 2: return launch_lattice_fix<2, 2, St>(rec, a, nblocks, lds, st);
      case 2 * 16 + 4: return launch_lattice_fix<2, 4, St>(rec, a, nblocks, lds, st);
      case 2 * 16 + 8: return launch_lattice_fix<2, 8, St>(rec, a, nblocks, lds, st);
      case 3 * 16 + 2: return launch_lattice_fix<3, 2, St>(rec, a, nblocks, lds, st);
      case 3 * 16 + 4: return launch_lattice_fix<3, 4, St>(rec, a, nblocks, lds, st);
      case 3 * 16 + 8: return launch_lattice_fix<3, 8, St>(rec, a, nblocks, lds, st);
      case 4 * 16 + 2: return launch_lattice_fix<4, 2, St>(rec, a, nblocks, lds, st);
      case 4 * 16 + 4: return launch_lattice_fix<4, 4, St>(rec, a, nblocks, lds, st);
      case 4 * 16 + 8: return launch_lattice_fix<4, 8, St>(rec, a, nblocks, lds, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (d) {
    case 1: return launch_lattice_s<1, St>(rec, a, nblocks, lds, st);
    case 2: return launch_lattice_s<2, St>(rec, a, nblocks, lds, st);
    case 3: return launch_lattice_s<3, St>(rec, a, nblocks, lds, st);
    case 4: return launch_lattice_s<4, St>(rec, a, nblocks, lds, st);
    case 5: return launch_lattice_s<5, St>(rec, a, nblocks, lds, st);
    case 6: return launch_lattice_s<6, St>(rec, a, nblocks, lds, st);
    default: return hipErrorInvalidValue;
  }
}

// The batched fused combine for members that share one b in {2, 4, 8}: b at
// compile time, and only that b's code in the kernel (the generic batch
// kernel carries every b's variant, and the largest sets its registers).
template <int S, int B, typename St>
__global__ __launch_bounds__(64) void k_combine_lattice_batch_fix(const LatArgs* __restrict__ ctxs,
                                                                  const int64_t* __restrict__ items, int nitems) {
  extern __shared__ __attribute__((aligned(16))) double lat[];
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int64_t w = items[i];
    const LatArgs& a = ctxs[w >> 40];
    const int64_t blk = w & ((int64_t(1) << 40) - 1);
    if (a.rec) lattice_fix<S, B, St, true>(a, blk, lat);
    else lattice_fix<S, B, St, false>(a, blk, lat);
    __syncthreads();
  }
}

template <int S, typename St>
static bool launch_lattice_batch_fix(int b, const LatArgs* ctxs, const int64_t* items, int nitems, dim3 g,
                                     size_t lds, hipStream_t st) {
  if constexpr (lat_fix_ok(S, 2)) {
    const dim3 blk(64);
    switch (b) {
      case 2: hipLaunchKernelGGL((k_combine_lattice_batch_fix<S, 2, St>), g, blk, lds, st, ctxs, items, nitems); return true;
      case 4:
        if constexpr (lat_fix_ok(S, 4)) {
          hipLaunchKernelGGL((k_combine_lattice_batch_fix<S, 4, St>), g, blk, lds, st, ctxs, items, nitems);
          return true;
        }
        return false;
      case 8:
        if constexpr (lat_fix_ok(S, 8)) {
          hipLaunchKernelGGL((k_combine_lattice_batch_fix<S, 8, St>), g, blk, lds, st, ctxs, items, nitems);
          return true;
        }
        return false;
      default: return false;
    }
  }
  return false;
}

template <typename St>
static hipError_t launch_lattice_batch_t(int d, int b, const LatArgs* ctxs, const int64_t* items, int nitems,
                                         int grid, size_t lds, hipStream_t st) {
  const dim3 g((unsigned)grid), blk(64);
  bool done = false;
  switch (d) {
    case 2: done = launch_lattice_batch_fix<2, St>(b, ctxs, items, nitems, g, lds, st); break;
    case 3: done = launch_lattice_batch_fix<3, St>(b, ctxs, items, nitems, g, lds, st); break;
    case 4: done = launch_lattice_batch_fix<4, St>(b, ctxs, items, nitems, g, lds, st); break;
    default: break;
  }
  if (done) return hipGetLastError();
  switch (d) {
    case 1: hipLaunchKernelGGL((k_combine_lattice_batch<1, St>), g, blk, lds, st, ctxs, items, nitems); break;
    case 2: hipLaunchKernelGGL((k_combine_lattice_batch<2, St>), g, blk, lds, st, ctxs, items, nitems); break;
    case 3: hipLaunchKernelGGL((k_combine_lattice_batch<3, St>), g, blk, lds, st, ctxs, items, nitems); break;
    case 4: hipLaunchKernelGGL((k_combine_lattice_batch<4, St>), g, blk, lds, st, ctxs, items, nitems); break;
    case 5: hipLaunchKernelGGL((k_combine_lattice_batch<5, St>), g, blk, lds, st, ctxs, items, nitems); break;
    case 6: hipLaunchKernelGGL((k_combine_lattice_batch<6, St>), g, blk, lds, st, ctxs, items, nitems); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine_lattice_batch(int prec, int d, int b, const LatArgs* ctxs, const int64_t* items,
                                        int nitems, int grid, size_t lds_bytes, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (lds_bytes > LAT_LDS_BYTES) return hipErrorInvalidValue;
  if (prec == PREC_F64) return launch_lattice_batch_t<double>(d, b, ctxs, items, nitems, grid, lds_bytes, st);
  return launch_lattice_batch_t<float>(d, b, ctxs, items, nitems, grid, lds_bytes, st);
}

size_t lattice_lds_bytes(int d, int b) {
  int64_t tot = 1, bd = 1;
  for (int q = 0; q < d; ++q) { tot *= (b + 1); bd *= b; }
  return (size_t)(tot - 1 - bd) * 2 * sizeof(double);
}

hipError_t launch_combine_lattice(int prec, int d, bool recursion, const LatArgs& a, int64_t nblocks,
                                  size_t lds_bytes, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (lds_bytes > LAT_LDS_BYTES) return hipErrorInvalidValue;
  if (prec == PREC_F64) return launch_lattice_t<double>(d, recursion, a, nblocks, lds_bytes, st);
  return launch_lattice_t<float>(d, recursion, a, nblocks, lds_bytes, st);
}

hipError_t launch_norms(const NormArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_norms, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}


}  // namespace cum
