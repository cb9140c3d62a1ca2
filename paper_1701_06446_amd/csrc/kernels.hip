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
#include <hip/hip_runtime.h>

#include "cum_internal.h"
#include "kernels.h"

namespace cum {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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

// Compensated fold of d into the pair (hi, lo): TwoSum then renormalise.
template <typename T>
__device__ __forceinline__ void fold(T* hi_p, T* lo_p, T d) {
  const T hi = *hi_p, lo = *lo_p;
  const T s = hi + d;
  const T bp = s - hi;
  const T err = (hi - (s - bp)) + (d - bp);
  const T l2 = lo + err;
  const T nh = s + l2;
  const T nl = l2 - (nh - s);
  *hi_p = nh;
  *lo_p = nl;
}

// Loads rows [g0, g0 + chunk) of the signed row sequence (plus rows, then
// minus rows) into LDS, row-major with the given stride; rows past the end
// are zero.  Padded columns (>= n) were zeroed once and are never written.
template <typename T>
__device__ __forceinline__ void load_chunk(T* xs, const UpdArgs& a, int g0) {
  const T* xp = (const T*)a.xp;
  const T* xm = (const T*)a.xm;
  const int K = a.np + a.nm;
  const int total = a.chunk * a.n;
  for (int idx = threadIdx.x; idx < total; idx += 256) {
    const int row = idx / a.n;
    const int col = idx - row * a.n;
    const int g = g0 + row;
    T v = T(0);
    if (g < a.np) v = xp[(int64_t)g * a.n + col];
    else if (g < K) v = xm[(int64_t)(g - a.np) * a.n + col];
    xs[row * a.stride + col] = v;
  }
}

template <int P, int H, int MR, int TM, int TN>
__device__ void upd_body(const UpdArgs& a, const UpdItem& it, char* smem) {
  using T = typename Tr<P>::X;
  using Acc = typename Tr<P>::Acc;
  using A1 = typename Tr<P>::A1;
  constexpr int KS = Tr<P>::KS;
  constexpr int K_ORD = H + MR;
  constexpr int MRC = MR > 0 ? MR : 1;
  T* xs = (T*)smem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const LeftCol* __restrict__ left = a.left[K_ORD];
  const RightCol* __restrict__ right = a.right[K_ORD];

  // zero the padded columns once
  for (int idx = tid; idx < a.chunk * (a.npad - a.n); idx += 256) {
    const int row = idx / (a.npad - a.n);
    xs[row * a.stride + a.n + (idx - row * (a.npad - a.n))] = T(0);
  }

  int ac[TM][H];
  bool av[TM];
  int bc[TN][MRC];
  bool bv[TN];
#pragma unroll
  for (int f = 0; f < TM; ++f) {
    const int r = it.r0 + 16 * f + (lane & 15);
    av[f] = r < it.M;
    const LeftCol L = left[it.lrow0 + (av[f] ? r : 0)];
#pragma unroll
    for (int q = 0; q < H; ++q) ac[f][q] = L.c[q];
  }
#pragma unroll
  for (int g = 0; g < TN; ++g) {
    const int c = it.c0 + 16 * g + (lane & 15);
    bv[g] = c < it.N;
    const RightCol R = right[it.rcol0 + (bv[g] ? c : 0)];
#pragma unroll
    for (int q = 0; q < MRC; ++q) bc[g][q] = R.c[q];
  }

  Acc acc[TM][TN];
#pragma unroll
  for (int f = 0; f < TM; ++f)
#pragma unroll
    for (int g = 0; g < TN; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[f][g][r] = A1(0);

  const int K = a.np + a.nm;
  const int nsteps = a.chunk / KS;
  for (int g0 = 0; g0 < K; g0 += a.chunk) {
    __syncthreads();
    load_chunk<T>(xs, a, g0);
    __syncthreads();
    for (int ks = wave; ks < nsteps; ks += 4) {
      if constexpr (KS == 4) {
        const int row = ks * 4 + (lane >> 4);
        const T* xr = xs + row * a.stride;
        const T sgn = (g0 + row < a.np) ? T(1) : T(-1);
        T A[TM], B[TN];
#pragma unroll
        for (int f = 0; f < TM; ++f) {
          T v = xr[ac[f][0]];
#pragma unroll
          for (int q = 1; q < H; ++q) v *= xr[ac[f][q]];
          A[f] = av[f] ? sgn * v : T(0);
        }
#pragma unroll
        for (int g = 0; g < TN; ++g) {
          T v = T(1);
          if constexpr (MR > 0) {
            v = xr[bc[g][0]];
#pragma unroll
            for (int q = 1; q < MR; ++q) v *= xr[bc[g][q]];
          }
          B[g] = bv[g] ? v : T(0);
        }
#pragma unroll
        for (int f = 0; f < TM; ++f)
#pragma unroll
          for (int g = 0; g < TN; ++g) acc[f][g] = mma(A[f], B[g], acc[f][g]);
      } else {
        // split-BF16x3: v = hi + lo with hi = RNE_bf16(v), lo = RNE_bf16(v - hi);
        // a*b ~ ah*bh + ah*bl + al*bh, accumulated in FP32.
        const int rowb = ks * 32 + 8 * (lane >> 4);
        bf16x8 Ah[TM], Al[TM], Bh[TN], Bl[TN];
#pragma unroll
        for (int q8 = 0; q8 < 8; ++q8) {
          const int row = rowb + q8;
          const float* xr = xs + row * a.stride;
          const float sgn = (g0 + row < a.np) ? 1.0f : -1.0f;
#pragma unroll
          for (int f = 0; f < TM; ++f) {
            float v = xr[ac[f][0]];
#pragma unroll
            for (int q = 1; q < H; ++q) v *= xr[ac[f][q]];
            v = av[f] ? sgn * v : 0.0f;
            const __bf16 hi = (__bf16)v;
            Ah[f][q8] = hi;
            Al[f][q8] = (__bf16)(v - (float)hi);
          }
#pragma unroll
          for (int g = 0; g < TN; ++g) {
            float v = 1.0f;
            if constexpr (MR > 0) {
              v = xr[bc[g][0]];
#pragma unroll
              for (int q = 1; q < MR; ++q) v *= xr[bc[g][q]];
            }
            v = bv[g] ? v : 0.0f;
            const __bf16 hi = (__bf16)v;
            Bh[g][q8] = hi;
            Bl[g][q8] = (__bf16)(v - (float)hi);
          }
        }
#pragma unroll
        for (int f = 0; f < TM; ++f)
#pragma unroll
          for (int g = 0; g < TN; ++g) {
            acc[f][g] = mma16(Al[f], Bh[g], acc[f][g]);
            acc[f][g] = mma16(Ah[f], Bl[g], acc[f][g]);
            acc[f][g] = mma16(Ah[f], Bh[g], acc[f][g]);
          }
      }
    }
  }

  // Reduce the four waves' partial sums in a fixed order, then fold.
  __syncthreads();
  A1* red = (A1*)smem;
  constexpr int FR = TM * TN * 256;
#pragma unroll
  for (int f = 0; f < TM; ++f)
#pragma unroll
    for (int g = 0; g < TN; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = frag_row<P>(lane, r), j = lane & 15;
        red[wave * FR + (f * TN + g) * 256 + i * 16 + j] = acc[f][g][r];
      }
  __syncthreads();
  A1* shi = (A1*)a.s_hi[K_ORD];
  A1* slo = (A1*)a.s_lo[K_ORD];
  for (int e = tid; e < FR; e += 256) {
    const int fg = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int f = fg / TN, g = fg - f * TN;
    const int r = it.r0 + 16 * f + i, c = it.c0 + 16 * g + j;
    if (r < it.M && c < it.N) {
      const A1 sum = ((red[e] + red[FR + e]) + red[2 * FR + e]) + red[3 * FR + e];
      const int64_t off = left[it.lrow0 + r].base + right[it.rcol0 + c].base;
      fold<A1>(shi + off, slo + off, sum);
    }
  }
}

template <int P, int TM, int TN>
__global__ __launch_bounds__(256) void k_update(UpdArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[UPD_LDS_BYTES];
  const UpdItem it = a.items[blockIdx.x];
  switch (it.k) {
    case 1: upd_body<P, 1, 0, TM, TN>(a, it, smem); break;
    case 2: upd_body<P, 1, 1, TM, TN>(a, it, smem); break;
    case 3: upd_body<P, 2, 1, TM, TN>(a, it, smem); break;
    case 4: upd_body<P, 2, 2, TM, TN>(a, it, smem); break;
    case 5: upd_body<P, 3, 2, TM, TN>(a, it, smem); break;
    case 6: upd_body<P, 3, 3, TM, TN>(a, it, smem); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Combine (Alg. 3 / Alg. 4).

constexpr int bell_minus_one(int s) {
  return s == 1 ? 0 : s == 2 ? 1 : s == 3 ? 4 : s == 4 ? 14 : s == 5 ? 51 : 202;
}

// Every partition of {0..S-1} into 2..S parts, grouped by the number of parts
// in increasing order (the sigma loop of Alg. 4); each part is a bitmask.
template <int S> struct PartTable {
  static constexpr int CAP = bell_minus_one(S) > 0 ? bell_minus_one(S) : 1;
  int count;
  int nparts[CAP];
  int mask[CAP][S];
};

template <int S> constexpr PartTable<S> make_parts() {
  PartTable<S> t{};
  t.count = 0;
  for (int sigma = 2; sigma <= S; ++sigma) {
    // restricted growth strings: g[0] = 0, g[i] <= 1 + max(g[0..i-1])
    int g[S] = {};
    for (;;) {
      int parts = 0;
      for (int i = 0; i < S; ++i) parts = g[i] + 1 > parts ? g[i] + 1 : parts;
      if (parts == sigma) {
        t.nparts[t.count] = parts;
        for (int q = 0; q < S; ++q) t.mask[t.count][q] = 0;
        for (int i = 0; i < S; ++i) t.mask[t.count][g[i]] |= 1 << i;
        ++t.count;
      }
      int i = S - 1;
      for (; i > 0; --i) {
        int mx = 0;
        for (int q = 0; q < i; ++q) mx = g[q] > mx ? g[q] : mx;
        if (g[i] <= mx) break;
      }
      if (i == 0) break;
      ++g[i];
      for (int q = i + 1; q < S; ++q) g[q] = 0;
    }
  }
  return t;
}

template <int S> __device__ constexpr PartTable<S> kParts = make_parts<S>();

// Lexicographic rank of a non-decreasing m-tuple among all such tuples over
// [0, nbar): sum_i N(m-i+1, j_{i-1}) - N(m-i+1, j_i) with j_0 = 0, where
// N(q, y) counts the sorted q-tuples over [y, nbar).
__device__ __forceinline__ int64_t tuple_rank(const int* j, int m, const int64_t* ntab, int nbar) {
  int64_t r = 0;
  int prev = 0;
  for (int i = 0; i < m; ++i) {
    const int q = m - i;
    r += ntab[q * (nbar + 1) + prev] - ntab[q * (nbar + 1) + j[i]];
    prev = j[i];
  }
  return r;
}

template <int S, typename St>
__global__ __launch_bounds__(256) void k_combine(CombArgs a) {
  constexpr int NM = 1 << S;
  constexpr int FULL = NM - 1;
  __shared__ int64_t subbase[NM];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int b = a.b;

  if (tid > 0 && tid < FULL) {
    int j[CUM_MAXD], len = 0;
    for (int q = 0; q < S; ++q)
      if (tid & (1 << q)) j[len++] = a.tuples[blk * S + q];
    int64_t bl = 1;
    for (int q = 0; q < len; ++q) bl *= b;
    subbase[tid] = tuple_rank(j, len, a.ntab, a.nbar) * bl;
  }
  __syncthreads();

  const St* shi = (const St*)a.s_hi;
  const St* slo = (const St*)a.s_lo;
  double sq = 0.0;
  for (int64_t e = tid; e < a.bs; e += 256) {
    int dig[S];
    int64_t rem = e;
#pragma unroll
    for (int q = S - 1; q >= 0; --q) {
      dig[q] = (int)(rem % b);
      rem /= b;
    }
    double cB[NM];
#pragma unroll
    for (int mask = 1; mask < FULL; ++mask) {
      int64_t off = 0;
      int len = 0;
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (mask & (1 << q)) { off = off * b + dig[q]; ++len; }
      cB[mask] = a.C[len][subbase[mask] + off];
    }
    double A = 0.0;
#pragma unroll
    for (int p = 0; p < kParts<S>.count; ++p) {
      double prod = cB[kParts<S>.mask[p][0]];
#pragma unroll
      for (int q = 1; q < S; ++q)
        if (q < kParts<S>.nparts[p]) prod *= cB[kParts<S>.mask[p][q]];
      A += prod;
    }
    const int64_t o = blk * a.bs + e;
    const double mval = ((double)shi[o] + (double)slo[o]) * a.inv_t;
    const double c = mval - A;
    a.Cout[o] = c;
    sq += c * c;
  }
  red[tid] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) a.partial[blk] = a.mult[blk] * red[0];
}

// Final norms: fro[k] = sqrt(sum of the order's block partials), summed in a
// fixed order; nu[k] = fro[k] / fro[2]^(k/2) for k >= 3 (Eq. (mef)).
__global__ __launch_bounds__(256) void k_norms(NormArgs a) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  for (int k = 1; k <= a.d; ++k) {
    double s = 0.0;
    for (int64_t i = tid; i < a.nblocks[k]; i += 256) s += a.partial[k][i];
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) a.out[k] = sqrt(red[0]);
    __syncthreads();
  }
  if (tid == 0) {
    a.out[0] = __builtin_nan("");
    for (int k = 0; k <= a.d; ++k)
      a.out[a.d + 1 + k] = (k >= 3) ? a.out[k] / pow(a.out[2], 0.5 * k) : __builtin_nan("");
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers.

template <int P>
static hipError_t launch_update_p(const UpdArgs& a, int nitems, hipStream_t st) {
  hipLaunchKernelGGL((k_update<P, UPD_TM, UPD_TN>), dim3(nitems), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_update(int prec, const UpdArgs& a, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  switch (prec) {
    case PREC_F64: return launch_update_p<PREC_F64>(a, nitems, st);
    case PREC_F32: return launch_update_p<PREC_F32>(a, nitems, st);
    case PREC_BF16X3: return launch_update_p<PREC_BF16X3>(a, nitems, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename St>
static hipError_t launch_combine_t(int s, const CombArgs& a, int64_t nblocks, hipStream_t st) {
  const dim3 grid((unsigned)nblocks), blk(256);
  switch (s) {
    case 1: hipLaunchKernelGGL((k_combine<1, St>), grid, blk, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_combine<2, St>), grid, blk, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_combine<3, St>), grid, blk, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_combine<4, St>), grid, blk, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_combine<5, St>), grid, blk, 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_combine<6, St>), grid, blk, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine(int prec, int s, const CombArgs& a, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (prec == PREC_F64) return launch_combine_t<double>(s, a, nblocks, st);
  return launch_combine_t<float>(s, a, nblocks, st);
}

hipError_t launch_norms(const NormArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_norms, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace cum
