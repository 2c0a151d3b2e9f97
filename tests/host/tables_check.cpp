// Host-side checks of the library's table builders (Bessel zeros, index
// sets, band tables of the Wigner recurrence, work splits, ball voxels, the
// union of launch intervals),
// built with the address and undefined-behaviour sanitizers and bounds-
// checked standard containers by tests/test_host_sanitize.py.  Prints one
// line per failed invariant and exits non-zero if any failed.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <set>
#include <utility>
#include <vector>

#include "bh_tables.h"

using namespace bh;

static int failures = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      ++failures;                               \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);                 \
      std::printf("\n");                        \
    }                                           \
  } while (0)

static void check_index_set(int L) {
  const IndexSet& s = index_set(L);
  CHECK(s.L == L, "index_set(%d).L = %d", L, s.L);
  int64_t off = 0;
  double prev = 0.0;
  for (const Radial& r : s.rad) {
    CHECK(r.l >= 0 && r.l <= L, "L=%d: radial degree %d", L, r.l);
    CHECK(r.lam > prev || (r.lam == prev && off > 0), "L=%d: lambda not ascending", L);
    CHECK(r.lam < s.cutoff, "L=%d: lambda %g above cutoff %g", L, r.lam, s.cutoff);
    CHECK(r.offset == off, "L=%d: offset %d != %lld", L, r.offset, (long long)off);
    CHECK(std::isfinite(r.c) && r.c > 0.0, "L=%d: c = %g", L, r.c);
    off += 2 * r.l + 1;
    prev = r.lam;
  }
  CHECK(off == s.C, "L=%d: C = %lld, sum 2l+1 = %lld", L, (long long)s.C, (long long)off);
  // every degree up to L has its first zero below the cutoff (lambda_{l,1}
  // increases with l and the cutoff is lambda_{L+1,1})
  std::set<int> degs;
  for (const Radial& r : s.rad) degs.insert(r.l);
  CHECK((int)degs.size() == L + 1, "L=%d: %zu degrees present", L, degs.size());
}

static void check_band(int L, int Lmax) {
  const BandTables t = band_tables(L, Lmax);
  // (2m + 1) classes of L - m + 1 chain entries each, stored padded to an
  // even number
  int64_t entries = 0;
  for (int m = 0; m <= L; ++m) entries += (int64_t)(2 * m + 1) * class_span(L - m + 1);
  CHECK(t.n_entries == entries, "band %d: %lld entries, expected %lld", L, (long long)t.n_entries,
        (long long)entries);
  CHECK(t.n_classes == (L + 1) * (L + 1), "band %d: %d classes", L, t.n_classes);
  CHECK((int64_t)t.rec.size() == 2 * t.n_entries && (int64_t)t.wt.size() == 2 * t.n_entries &&
            (int64_t)t.sel.size() == 4 * t.n_entries,
        "band %d: table sizes", L);
  CHECK((int)t.p_first.size() == 2 * L + 2 && t.p_first[0] == 0 &&
            t.p_first[2 * L + 1] == t.n_entries,
        "band %d: p_first ends", L);
  for (int p = 0; p <= 2 * L; ++p) {
    // classes of p: q = p mod 2, ..., 2L - p; class (m, n) holds l = m..L
    int64_t want = 0;
    for (int q = p % 2; q <= 2 * L - p; q += 2) {
      const int n = L - (p + q) / 2 + 1;
      const int64_t e0 = t.p_first[p] + want;
      CHECK(e0 % 2 == 0, "band %d: class (p %d, q %d) starts at entry %lld", L, p, q, (long long)e0);
      // the chain's entries run l = m .. L, then padding with zero weights
      for (int i = 0; i < class_span(n) && e0 + i < t.n_entries; ++i) {
        const int64_t e = e0 + i;
        if (i < n) {
          CHECK(t.sel[4 * e] == (p + q) / 2 + i, "band %d: entry %lld degree", L, (long long)e);
          CHECK(t.wt[2 * e] != 0.0, "band %d: entry %lld zero weight", L, (long long)e);
        } else {
          CHECK(t.wt[2 * e] == 0.0 && t.wt[2 * e + 1] == 0.0 && t.rec[2 * e] == 0.0 &&
                    t.rec[2 * e + 1] == 0.0,
                "band %d: padding entry %lld not zero", L, (long long)e);
        }
      }
      want += class_span(n);
    }
    CHECK(t.p_first[p + 1] - t.p_first[p] == want, "band %d: p-group %d size", L, p);
  }
  for (int64_t e = 0; e < t.n_entries; ++e) {
    const int l = t.sel[4 * e], m = t.sel[4 * e + 1], n = t.sel[4 * e + 2];
    CHECK(m >= 0 && m <= L && n >= -m && n <= m && l >= m && l <= L,
          "band %d: entry %lld has (l, m, n) = (%d, %d, %d)", L, (long long)e, l, m, n);
    CHECK(std::isfinite(t.rec[2 * e]) && std::isfinite(t.rec[2 * e + 1]) &&
              std::isfinite(t.wt[2 * e]) && std::isfinite(t.wt[2 * e + 1]),
          "band %d: entry %lld not finite", L, (long long)e);
  }
  // every wave split covers each p-group exactly once
  const int row = 2 * L + 2;
  for (int wi = 0; wi < kNumWaveChoices; ++wi) {
    const int W = kWaveChoices[wi];
    const int64_t o = wave_block_offset(L, W);
    CHECK(o >= 0 && o + (int64_t)W * row <= (int64_t)t.wave_p.size(), "band %d: W=%d block", L, W);
    if (o < 0) continue;
    std::vector<int> seen(2 * L + 1, 0);
    for (int w = 0; w < W; ++w) {
      const int32_t* r = &t.wave_p[o + (int64_t)w * row];
      CHECK(r[0] >= 0 && r[0] <= 2 * L + 1, "band %d: W=%d wave %d count %d", L, W, w, r[0]);
      for (int i = 0; i < r[0] && i < 2 * L + 1; ++i) {
        CHECK(r[1 + i] >= 0 && r[1 + i] <= 2 * L, "band %d: W=%d p = %d", L, W, r[1 + i]);
        if (r[1 + i] >= 0 && r[1 + i] <= 2 * L) ++seen[r[1 + i]];
      }
    }
    for (int p = 0; p <= 2 * L; ++p)
      CHECK(seen[p] == 1, "band %d: W=%d p-group %d assigned %d times", L, W, p, seen[p]);
  }
  // degree groups of the radial entries, as offsets in the Lmax layout
  const IndexSet& big = index_set(Lmax);
  CHECK((int)t.deg_start.size() == L + 2 && t.deg_start[L + 1] == (int32_t)t.deg_off.size(),
        "band %d: deg_start", L);
  for (int l = 0; l <= L; ++l) {
    CHECK(t.deg_start[l] <= t.deg_start[l + 1], "band %d: deg_start not monotone", L);
    for (int i = t.deg_start[l]; i < t.deg_start[l + 1]; ++i)
      CHECK(t.deg_off[i] >= 0 && t.deg_off[i] + 2 * l + 1 <= big.C, "band %d (Lmax %d): offset", L,
            Lmax);
  }
  CHECK((int64_t)t.deg_off.size() == (int64_t)index_set(L).rad.size(),
        "band %d: %zu radial entries, index set has %zu", L, t.deg_off.size(),
        index_set(L).rad.size());
}

static void check_voxels(int N) {
  const std::vector<int32_t> ball = ball_voxels(N);
  int64_t brute = 0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) {
        const long long a = 2LL * i - (N - 1), b = 2LL * j - (N - 1), c = 2LL * k - (N - 1);
        if (a * a + b * b + c * c < (long long)N * N) ++brute;
      }
  CHECK((int64_t)ball.size() == brute, "N=%d: %zu ball voxels, brute force %lld", N, ball.size(),
        (long long)brute);
  const std::set<int32_t> in(ball.begin(), ball.end());
  const std::vector<int32_t> rep = orbit_representatives(N);
  for (int32_t v : rep) CHECK(in.count(v) == 1, "N=%d: representative %d outside the ball", N, v);
}

// interval_union against its definition: exact sums for disjoint, nested,
// touching and reversed intervals, and a brute-force count on a grid for
// random intervals with endpoints on that grid.
static void check_interval_union() {
  using V = std::vector<std::pair<double, double>>;
  CHECK(interval_union(V{}) == 0.0, "empty union");
  CHECK(interval_union(V{{1, 2}, {3, 5}}) == 3.0, "disjoint");
  CHECK(interval_union(V{{3, 5}, {1, 2}}) == 3.0, "disjoint, unsorted");
  CHECK(interval_union(V{{0, 10}, {2, 3}, {4, 9}}) == 10.0, "nested");
  CHECK(interval_union(V{{0, 2}, {2, 4}}) == 4.0, "touching");
  CHECK(interval_union(V{{0, 3}, {1, 4}, {2, 5}}) == 5.0, "overlapping chain");
  CHECK(interval_union(V{{1, 1}, {2, 2}}) == 0.0, "points");
  CHECK(interval_union(V{{5, 4}, {0, 1}}) == 1.0, "reversed interval");
  uint64_t z = 88172645463325252ull;
  auto next = [&](int m) {
    z ^= z << 13;
    z ^= z >> 7;
    z ^= z << 17;
    return (int)(z % (uint64_t)m);
  };
  for (int t = 0; t < 200; ++t) {
    const int n = next(12), G = 64;
    V iv;
    std::vector<char> cover(G, 0);   // cell [g, g + 1) covered
    for (int i = 0; i < n; ++i) {
      int a = next(G + 1), b = next(G + 1);
      if (a > b) std::swap(a, b);
      iv.push_back({a / 8.0, b / 8.0});
      for (int g = a; g < b; ++g) cover[g] = 1;
    }
    int cells = 0;
    for (char c : cover) cells += c;
    CHECK(interval_union(iv) == cells / 8.0, "random case %d: %g against %g", t,
          interval_union(iv), cells / 8.0);
  }
}

int main() {
  check_interval_union();
  for (int L = 0; L <= 64; ++L) check_index_set(L);
  for (int L : {0, 1, 2, 3, 4, 7, 8, 11, 16, 24, 32, 40, 41, 42, 64}) check_band(L, L);
  check_band(8, 32);
  check_band(16, 40);
  for (int N : {1, 2, 3, 8, 9, 16, 17, 32}) check_voxels(N);
  for (int l = 0; l <= 8; ++l)
    for (int j = 0; j <= 2 * l; ++j) {
      const int c = column_parity_class(l, j);
      CHECK(c >= 0 && c < 8, "parity class of (%d, %d) = %d", l, j, c);
    }
  std::printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
