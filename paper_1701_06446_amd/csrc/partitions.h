// Compile-time set-partition tables for the moment -> cumulant combine
// (Alg. 4) and its reverse: every partition of {0..S-1} into 2..S parts,
// grouped by the number of parts in increasing order (the sigma loop of
// Alg. 4), each part a bitmask of positions.
#pragma once
#include <hip/hip_runtime.h>

namespace cum {

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

// Partition sum of Alg. 4 for one element: the sum, over every partition of
// {1..S} into 2..S parts, of the product of the lower-order cumulants c_B.
template <int S>
__device__ __forceinline__ double partition_sum(const double (&cB)[1 << S]) {
  double A = 0.0;
#pragma unroll
  for (int p = 0; p < kParts<S>.count; ++p) {
    double prod = cB[kParts<S>.mask[p][0]];
#pragma unroll
    for (int q = 1; q < S; ++q)
      if (q < kParts<S>.nparts[p]) prod *= cB[kParts<S>.mask[p][q]];
    A += prod;
  }
  return A;
}

// The recursion's subtracted sum for one element: over the proper subsets B
// of {1..S} that hold position 1 (bit 0), the cumulant c_B times the moment
// of the other positions (cm[B] holds c_B when B has bit 0, else m_B).
template <int S>
__device__ __forceinline__ double recursion_sum(const double (&cm)[1 << S]) {
  constexpr int FULL = (1 << S) - 1;
  double A = 0.0;
#pragma unroll
  for (int q = 1; q < FULL; q += 2) A += cm[q] * cm[FULL & ~q];
  return A;
}

}  // namespace cum
