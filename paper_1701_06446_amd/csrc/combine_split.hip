// Per-order combine (Alg. 3 / Alg. 4) of one high order S with every operand
// in LDS, evaluated by splitting on the part that holds the block's first
// index position.
//
// Every partition of the S positions into two or more parts has exactly one
// part B0 holding position 1; the other parts form an arbitrary partition of
// the rest R = {1..S} \ B0.  Grouping Alg. 4's partition sum that way,
//
//   c_I = m_I - sum_{B0 holds 1, B0 != I} c_{B0} P_{I \ B0},
//   P_R = sum over all partitions of R of prod c_B,
//
// and P_R is itself the moment of the positions R (the moment-cumulant
// relation of Sec. 2.3 read backwards).  With partitions, P is formed from
// the lower-order cumulants in LDS, lattice level by level, by the same
// grouping (P_R = sum_{B holds min R} c_B P_{R \ B}, P_empty = 1); with the
// recursion it is the moment read from the running sums.  Each element then
// costs 2^(S-1) - 1 fused multiply-adds instead of a product per partition
// (202 at S = 6).
//
// One workgroup per order-S block, one thread per row of the block along its
// last position (the B elements that share every other digit), so operands
// that do not involve the last position are read once per row.  Blocks are
// taken in XCD-contiguous ranges: workgroup i runs on XCD i mod 8, and
// neighbouring blocks share most of their sub-blocks in that XCD's L2.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cum {
namespace {

constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

constexpr int popc(int m) {
  int c = 0;
  for (; m; m &= m - 1) ++c;
  return c;
}

template <int S, int B, bool REC> struct SplitGeom {
  static constexpr int NM = 1 << S;
  static constexpr int FULL = NM - 1;
  static constexpr int LAST = 1 << (S - 1);
  static constexpr int NT = ipow(B, S - 1);  // threads: one per row
  // c_B for the parts B holding position 1 (odd masks below FULL)
  static constexpr int NF = B * ipow(B + 1, S - 1) - ipow(B, S);
  // one value set per non-empty R of the other positions (even masks):
  // c_R (partitions) or m_R (recursion)
  static constexpr int NR = ipow(B + 1, S - 1) - 1;
  static constexpr int NSTAGE = NF + NR;                 // read from global memory
  static constexpr int NLDS = NSTAGE + (REC ? 0 : NR);   // partitions add P_R
  static constexpr int PB = REC ? 0 : NR;                // P_R / m_R = LDS[off[R] + PB + ...]
  static constexpr int NWAVE = NT / 64;
  static constexpr int LB = B == 2 ? 1 : B == 4 ? 2 : 3;  // log2(B)
  static_assert(B == 2 || B == 4 || B == 8, "B must be a power of two");
  static_assert(NT % 64 == 0 && NT <= 1024 && (NT & (NT - 1)) == 0, "whole waves, at most 1024 threads");
};

// LDS offsets: the odd masks (parts holding position 1) in increasing order,
// then the even masks in increasing order; the staged list is exactly this
// range, so a staged item's index is its LDS offset.
template <int S, int B> struct SplitTab {
  int off[1 << S];
  int size[1 << S];
  int order[(1 << S) - 2];   // masks in LDS order
  int start[(1 << S) - 1];   // their offsets, then the end
  // even masks by level: level j (popcount j) at lvl[lstart[j] .. lstart[j+1])
  int lvl[1 << (S - 1)];
  int lstart[S + 1];
  constexpr SplitTab() : off(), size(), order(), start(), lvl(), lstart() {
    constexpr int NM = 1 << S;
    int o = 0, k = 0;
    for (int m = 1; m < NM - 1; m += 2) {
      off[m] = o;
      size[m] = ipow(B, popc(m));
      order[k] = m;
      start[k++] = o;
      o += size[m];
    }
    for (int m = 2; m < NM; m += 2) {
      off[m] = o;
      size[m] = ipow(B, popc(m));
      order[k] = m;
      start[k++] = o;
      o += size[m];
    }
    start[k] = o;
    int q = 0;
    for (int j = 0; j <= S; ++j) {
      lstart[j] = q;
      for (int m = 2; m < NM; m += 2)
        if (popc(m) == j) lvl[q++] = m;
    }
  }
};

template <int S, int B> constexpr SplitTab<S, B> kSplit{};

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int S, int B, typename St, bool REC>
__global__ __launch_bounds__((SplitGeom<S, B, REC>::NT)) void k_combine_split(CombArgs a) {
  using G = SplitGeom<S, B, REC>;
  constexpr auto& T = kSplit<S, B>;
  __shared__ __attribute__((aligned(16))) double lds[G::NLDS];
  __shared__ int64_t sub[G::NM];
  __shared__ double red[G::NWAVE];
  const int tid = threadIdx.x;

  // XCD-contiguous block ranges (a bijection on [0, nblocks))
  const int64_t nb = gridDim.x;
  const int64_t q8 = nb / 8, r8 = nb % 8;
  const int64_t x = blockIdx.x % 8, kx = blockIdx.x / 8;
  const int64_t blk = x * q8 + (x < r8 ? x : r8) + kx;

  // the block's own running sums, requested first
  const St* shi = (const St*)a.s_hi;
  const St* slo = (const St*)a.s_lo;
  const int64_t o = blk * (int64_t)(G::NT * B) + (int64_t)tid * B;
  St mh[B], ml[B];
#pragma unroll
  for (int l = 0; l < B; ++l) {
    mh[l] = shi[o + l];
    ml[l] = slo[o + l];
  }

  if (tid > 0 && tid < G::FULL) sub[tid] = (int64_t)a.subrank[blk * G::NM + tid] * T.size[tid];
  __syncthreads();

  // stage every sub-block: mask by mask (unrolled, so each mask's LDS
  // offset, size and source order are constants), at most one value per
  // thread per mask; the odd masks, then the even ones, each half's loads
  // all issued before its LDS stores
#pragma unroll
  for (int half = 1; half >= 0; --half) {
    double v[G::NM / 2];
#pragma unroll
    for (int k = 0; k < G::NM / 2; ++k) {
      const int m = 2 * k + half;
      v[k] = 0.0;
      if (m == 0 || m == G::FULL) continue;
      if (tid < T.size[m]) {
        const int64_t src = sub[m] + tid;
        if (REC && !(m & 1)) {
          v[k] = ((double)((const St*)a.Shi[__builtin_popcount(m)])[src] +
                  (double)((const St*)a.Slo[__builtin_popcount(m)])[src]) * a.inv_t;
        } else {
          v[k] = a.C[__builtin_popcount(m)][src];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < G::NM / 2; ++k) {
      const int m = 2 * k + half;
      if (m == 0 || m == G::FULL) continue;
      if (tid < T.size[m]) lds[T.off[m] + tid] = v[k];
    }
  }
  __syncthreads();

  if constexpr (!REC) {
    // P_R level by level: P_R[e] = sum over the parts Bm of R holding R's
    // lowest position (the other positions' choice in increasing order) of
    // c_Bm[e_Bm] P_{R \ Bm}[e_{R \ Bm}].  Within a level the masks take
    // consecutive thread ranges of B^j threads each.
#pragma unroll
    for (int j = 1; j < S; ++j) {
      const int bj = ipow(B, j);
      int rank = 0;
#pragma unroll
      for (int R = 2; R < G::NM; R += 2) {
        if (__builtin_popcount(R) != j) continue;
        // this mask's items start at thread rank * B^j (mod NT); B^j <= NT,
        // so a thread has at most one item per mask
        const int e = (tid - rank * bj) & (G::NT - 1);
        ++rank;
        if (e < bj) {
          const int low = R & -R, rem = R ^ low;
          double acc = 0.0;
#pragma unroll
          for (int sm = 0;; sm = (sm - rem) & rem) {
            const int mB = low | sm, mR = rem & ~sm;
            int oB = 0, oR = 0;
#pragma unroll
            for (int p = 1; p < S; ++p) {
              if (R & (1 << p)) {
                // digit of position p: e's digits follow R's positions, the first slowest
                const int t = __builtin_popcount(R & ((1 << p) - 1));
                const int d = (e >> (G::LB * (j - 1 - t))) & (B - 1);
                if (mB & (1 << p)) oB = oB * B + d;
                else oR = oR * B + d;
              }
            }
            const double cb = lds[T.off[mB] + oB];
            const double pr = mR ? lds[T.off[mR] + G::PB + oR] : 1.0;
            acc += cb * pr;
            if (sm == rem) break;
          }
          lds[T.off[R] + G::PB + e] = acc;
        }
      }
      __syncthreads();
    }
  }

  // this row's digits of positions 1 .. S-1 (first = slowest)
  int dig[S - 1];
  {
    int rr = tid;
#pragma unroll
    for (int q = S - 2; q >= 0; --q) {
      dig[q] = rr % B;
      rr /= B;
    }
  }
  double acc[B];
#pragma unroll
  for (int l = 0; l < B; ++l) acc[l] = 0.0;
#pragma unroll
  for (int m0 = 1; m0 < G::FULL; m0 += 2) {
    const int rest = G::FULL & ~m0;
    int o0 = 0, o1 = 0;
#pragma unroll
    for (int q = 0; q < S - 1; ++q) {
      if (m0 & (1 << q)) o0 = o0 * B + dig[q];
      else o1 = o1 * B + dig[q];
    }
    if (m0 & G::LAST) {
      const double p = lds[T.off[rest] + G::PB + o1];
      const double* c = lds + T.off[m0] + o0 * B;
#pragma unroll
      for (int l = 0; l < B; ++l) acc[l] += c[l] * p;
    } else {
      const double c = lds[T.off[m0] + o0];
      const double* p = lds + T.off[rest] + G::PB + o1 * B;
#pragma unroll
      for (int l = 0; l < B; ++l) acc[l] += c * p[l];
    }
  }
  double sq = 0.0;
#pragma unroll
  for (int l = 0; l < B; ++l) {
    const double c = ((double)mh[l] + (double)ml[l]) * a.inv_t - acc[l];
    a.Cout[o + l] = c;
    sq += c * c;
  }
  const double w = wave_sum64(sq);
  if ((tid & 63) == 0) red[tid >> 6] = w;
  __syncthreads();
  if (tid == 0) {
    double s = red[0];
#pragma unroll
    for (int k = 1; k < G::NWAVE; ++k) s += red[k];
    a.partial[blk] = a.mult[blk] * s;
  }
}

template <int S, int B, typename St>
hipError_t launch_sb(const CombArgs& a, int64_t nblocks, hipStream_t st) {
  if (a.rec)
    hipLaunchKernelGGL((k_combine_split<S, B, St, true>), dim3((unsigned)nblocks),
                       dim3(SplitGeom<S, B, true>::NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_combine_split<S, B, St, false>), dim3((unsigned)nblocks),
                       dim3(SplitGeom<S, B, false>::NT), 0, st, a);
  return hipGetLastError();
}

template <typename St>
hipError_t launch_t(int s, const CombArgs& a, int64_t nblocks, hipStream_t st) {
  if (s == 5) return launch_sb<5, 4, St>(a, nblocks, st);
  return launch_sb<6, 4, St>(a, nblocks, st);
}

}  // namespace

bool combine_split_supported(int s, int b) { return (s == 5 || s == 6) && b == 4; }

hipError_t launch_combine_split(int prec, int s, const CombArgs& a, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (!combine_split_supported(s, a.b) || nblocks > 0x7fffffff) return hipErrorInvalidValue;
  if (prec == PREC_F64) return launch_t<double>(s, a, nblocks, st);
  return launch_t<float>(s, a, nblocks, st);
}

}  // namespace cum
