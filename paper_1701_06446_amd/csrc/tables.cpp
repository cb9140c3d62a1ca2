// Host-side block enumerator (integer work only).
//
// Builds, for one (n, b, d): the sorted block tuples of every order in
// lexicographic order (the block structure of Sec. 2.3), their multiplicities
// k!/prod(r_l!) (Alg. 5), the binomial table used by the device-side tuple
// rank, and the pivot Khatri-Rao tables plus the per-workgroup tiles of the
// moment update (Alg. 2 / Eq. (momupdate) as one signed contraction per pivot).
#include "tables.h"

#include <algorithm>
#include <functional>
#include <queue>
#include <unordered_map>

namespace cum {

int64_t binom(int64_t a, int64_t k) {
  if (k < 0 || a < k) return 0;
  if (k == 0) return 1;
  int64_t r = 1;
  for (int64_t i = 1; i <= k; ++i) r = r * (a - k + i) / i;
  return r;
}

int64_t ipow64(int64_t b, int k) {
  int64_t r = 1;
  for (int i = 0; i < k; ++i) r *= b;
  return r;
}

// Sorted (non-decreasing) k-tuples over [lo, hi) in lexicographic order.
static void sorted_tuples(int k, int lo, int hi, std::vector<uint8_t>& out) {
  out.clear();
  if (k == 0) return;
  if (hi <= lo) return;
  std::vector<int> j(k, lo);
  for (;;) {
    for (int m = 0; m < k; ++m) out.push_back((uint8_t)j[m]);
    int m = k - 1;
    while (m >= 0 && j[m] == hi - 1) --m;
    if (m < 0) break;
    ++j[m];
    for (int q = m + 1; q < k; ++q) j[q] = j[m];
  }
}

static uint64_t key_of(const int* j, int k) {
  uint64_t key = 0;
  for (int m = 0; m < k; ++m) key = key * 256u + (uint64_t)j[m];
  return key * 8u + (uint64_t)k;
}

int build_tables(int n, int b, int d, Tables& T) {
  if (n < 1 || b < 1 || d < 1 || d > CUM_MAXD) return -1;
  T.n = n; T.b = b; T.d = d;
  T.nbar = (n + b - 1) / b;
  T.npad = T.nbar * b;
  if (T.nbar > 255 || T.npad > 65535) return -1;
  const int nbar = T.nbar;

  std::unordered_map<uint64_t, int64_t> rank;
  for (int k = 1; k <= d; ++k) {
    OrderInfo& o = T.ord[k];
    o.k = k;
    o.h = (k + 1) / 2;
    o.m = k - o.h;
    sorted_tuples(k, 0, nbar, T.tuples[k]);
    o.nblocks = (int64_t)T.tuples[k].size() / k;
    o.bk = ipow64(b, k);
    o.nelems = o.nblocks * o.bk;
    if (o.nblocks != binom(nbar + k - 1, k)) return -2;
    T.mult[k].resize((size_t)o.nblocks);
    double kf = 1.0;
    for (int q = 2; q <= k; ++q) kf *= q;
    for (int64_t r = 0; r < o.nblocks; ++r) {
      int j[CUM_MAXD];
      for (int m = 0; m < k; ++m) j[m] = T.tuples[k][(size_t)r * k + m];
      rank[key_of(j, k)] = r;
      double den = 1.0;
      int run = 1;
      for (int m = 1; m <= k; ++m) {
        if (m < k && j[m] == j[m - 1]) { ++run; continue; }
        for (int q = 2; q <= run; ++q) den *= q;
        run = 1;
      }
      T.mult[k][(size_t)r] = kf / den;
    }
  }

  // Sub-block ranks for the combine: every proper non-empty subset of the
  // positions of every stored block.
  for (int k = 1; k <= d; ++k) {
    const int nm = 1 << k;
    const int64_t nb = T.ord[k].nblocks;
    T.subrank[k].assign((size_t)nb * nm, 0);
    for (int64_t r = 0; r < nb; ++r) {
      for (int mask = 1; mask < nm - 1; ++mask) {
        int j[CUM_MAXD], len = 0;
        for (int q = 0; q < k; ++q)
          if (mask & (1 << q)) j[len++] = T.tuples[k][(size_t)r * k + q];
        auto it = rank.find(key_of(j, len));
        if (it == rank.end()) return -4;
        T.subrank[k][(size_t)r * nm + mask] = (int32_t)it->second;
      }
    }
  }

  // Pivot Khatri-Rao tables.
  for (int k = 1; k <= d; ++k) {
    const OrderInfo& o = T.ord[k];
    const int h = o.h, m = o.m;
    const int64_t bh = ipow64(b, h), bm = ipow64(b, m), bk = o.bk;
    // right table: every sorted m-tuple (lex) x b^m offsets
    std::vector<uint8_t> rt;
    sorted_tuples(m, 0, nbar, rt);
    const int64_t nr = (m == 0) ? 1 : (int64_t)rt.size() / m;
    T.right[k].clear();
    for (int64_t ri = 0; ri < nr; ++ri) {
      for (int64_t w = 0; w < bm; ++w) {
        RightCol c{};
        int64_t rem = w;
        for (int q = m - 1; q >= 0; --q) {
          c.c[q] = (uint16_t)(rt[(size_t)ri * m + q] * b + (int)(rem % b));
          rem /= b;
        }
        c.base = ri * bk + w;
        T.right[k].push_back(c);
      }
    }
    // left table and pivot extents
    T.piv[k].clear();
    T.left[k].clear();
    for (int v = 0; v < nbar; ++v) {
      Pivot P{};
      P.lrow0 = (int)T.left[k].size();
      // first sorted m-tuple whose first index is >= v: (v, ..., v)
      // rank of (v, ..., v) among sorted m-tuples = number of tuples whose
      // first index x < v, i.e. sum_x N(m-1, x)
      int64_t first = 0;
      if (m > 0)
        for (int x = 0; x < v; ++x) first += binom(nbar - x + m - 2, m - 1);
      P.rcol0 = (int)(first * bm);
      P.ncols = (int)(((m == 0) ? 1 : binom(nbar - v + m - 1, m)) * bm);
      std::vector<uint8_t> pre;
      sorted_tuples(h - 1, 0, v + 1, pre);
      const int64_t npre = (h == 1) ? 1 : (int64_t)pre.size() / (h - 1);
      for (int64_t pi = 0; pi < npre; ++pi) {
        int full[CUM_MAXD];
        for (int q = 0; q < h - 1; ++q) full[q] = pre[(size_t)pi * (h - 1) + q];
        for (int q = h - 1; q < k; ++q) full[q] = v;
        auto it = rank.find(key_of(full, k));
        if (it == rank.end()) return -3;
        const int64_t rbase = it->second;
        for (int64_t w = 0; w < bh; ++w) {
          LeftCol c{};
          int64_t rem = w;
          for (int q = h - 1; q >= 0; --q) {
            c.c[q] = (uint16_t)(full[q] * b + (int)(rem % b));
            rem /= b;
          }
          c.base = (rbase - first) * bk + w * bm;
          T.left[k].push_back(c);
        }
      }
      P.nrows = (int)(T.left[k].size() - (size_t)P.lrow0);
      T.piv[k].push_back(P);
    }
  }
  return 0;
}

std::vector<UpdItem> build_items(const Tables& T, int kmin, int kmax, int tile_rows, int tile_cols) {
  std::vector<UpdItem> items;
  for (int k = kmax; k >= kmin; --k) {
    for (int v = 0; v < T.nbar; ++v) {
      const Pivot& P = T.piv[k][(size_t)v];
      for (int r0 = 0; r0 < P.nrows; r0 += tile_rows)
        for (int c0 = 0; c0 < P.ncols; c0 += tile_cols) {
          UpdItem it{};
          it.k = k; it.v = v; it.r0 = r0; it.c0 = c0;
          it.M = P.nrows; it.N = P.ncols;
          it.lrow0 = P.lrow0; it.rcol0 = P.rcol0;
          items.push_back(it);
        }
    }
  }
  return items;
}

std::vector<UpdItem> pack_quads(const std::vector<UpdItem>& items) {
  if (items.empty()) return {};
  auto cost = [](const UpdItem& it) {
    const int fm = it.M - it.r0 > 16 ? 2 : 1, fn = it.N - it.c0 > 16 ? 2 : 1;
    return fm * fn;
  };
  std::vector<size_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return cost(items[x]) > cost(items[y]); });
  const size_t ng = (items.size() + 3) / 4;
  std::vector<int> load(ng, 0), fill(ng, 0);
  std::vector<UpdItem> out(ng * 4);
  UpdItem empty = items[0];
  empty.M = 0;
  empty.N = 0;
  for (size_t g = 0; g < ng; ++g)
    for (int j = 0; j < 4; ++j) out[g * 4 + (size_t)j] = empty;
  // open groups in a min-heap of (cost so far, index): the least loaded,
  // lowest index first
  using Slot = std::pair<int, size_t>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> open;
  for (size_t g = 0; g < ng; ++g) open.push({0, g});
  for (size_t i : order) {
    const size_t best = open.top().second;
    open.pop();
    out[best * 4 + (size_t)fill[best]] = items[i];
    ++fill[best];
    load[best] += cost(items[i]);
    if (fill[best] < 4) open.push({load[best], best});
  }
  return out;
}

int64_t coverage(const Tables& T, int k, std::vector<int32_t>& hits) {
  const OrderInfo& o = T.ord[k];
  hits.assign((size_t)o.nelems, 0);
  int64_t bad = 0;
  for (int v = 0; v < T.nbar; ++v) {
    const Pivot& P = T.piv[k][(size_t)v];
    for (int r = 0; r < P.nrows; ++r)
      for (int c = 0; c < P.ncols; ++c) {
        const LeftCol& L = T.left[k][(size_t)P.lrow0 + r];
        const RightCol& R = T.right[k][(size_t)P.rcol0 + c];
        const int64_t off = L.base + R.base;
        if (off < 0 || off >= o.nelems) { ++bad; continue; }
        // the element's own global indices must be the product's columns
        const int64_t blk = off / o.bk;
        int64_t rem = off % o.bk;
        int idx[CUM_MAXD];
        for (int q = k - 1; q >= 0; --q) {
          idx[q] = T.tuples[k][(size_t)blk * k + q] * T.b + (int)(rem % T.b);
          rem /= T.b;
        }
        bool same = true;
        for (int q = 0; q < o.h; ++q) same = same && (idx[q] == L.c[q]);
        for (int q = 0; q < o.m; ++q) same = same && (idx[o.h + q] == R.c[q]);
        if (!same) { ++bad; continue; }
        hits[(size_t)off] += 1;
      }
  }
  return bad;
}

}  // namespace cum
