// Host tables: Bessel zeros, index set, Wigner-recurrence band tables.
#include "bh_tables.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

#include "bh_special.h"

namespace bh {

namespace {

// Refine a bracketed sign change of j_l on [lo, hi] by bisection until the
// bracket is a few ulps wide.
double bisect_zero(int l, double lo, double hi) {
  double flo = bh_sph_jn(l, lo);
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double fm = bh_sph_jn(l, mid);
    if (fm == 0.0) return mid;
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

constexpr double kScanStep = 0.1;  // zeros of j_l are more than pi apart

}  // namespace

std::vector<double> bessel_zeros_below(int l, double x_max) {
  std::vector<double> out;
  double x = std::max((double)l, 0.05);
  double f = bh_sph_jn(l, x);
  while (x < x_max) {
    const double xn = x + kScanStep;
    const double fn = bh_sph_jn(l, xn);
    if (f == 0.0) {
      out.push_back(x);
    } else if ((f < 0) != (fn < 0) && fn != 0.0) {
      out.push_back(bisect_zero(l, x, xn));
    }
    x = xn;
    f = fn;
  }
  while (!out.empty() && out.back() >= x_max) out.pop_back();
  return out;
}

double bessel_zero(int l, int k) {
  double x_max = l + 4.0 * k + 8.0;
  for (;;) {
    auto z = bessel_zeros_below(l, x_max);
    if ((int)z.size() >= k) return z[k - 1];
    x_max *= 1.5;
  }
}

const IndexSet& index_set(int L) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<IndexSet>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(L);
  if (it != cache.end()) return *it->second;
  auto s = std::make_unique<IndexSet>();
  s->L = L;
  s->cutoff = bessel_zero(L + 1, 1);
  for (int l = 0; l <= L; ++l) {
    auto z = bessel_zeros_below(l, s->cutoff);
    for (size_t i = 0; i < z.size(); ++i) {
      if (z[i] >= s->cutoff) continue;
      Radial r;
      r.l = l;
      r.k = (int)i + 1;
      r.lam = z[i];
      r.c = std::sqrt(2.0) / std::fabs(bh_sph_jn(l + 1, z[i]));
      r.offset = 0;
      s->rad.push_back(r);
    }
  }
  std::sort(s->rad.begin(), s->rad.end(), [](const Radial& a, const Radial& b) {
    if (a.lam != b.lam) return a.lam < b.lam;
    if (a.l != b.l) return a.l < b.l;
    return a.k < b.k;
  });
  int64_t off = 0;
  for (auto& r : s->rad) {
    r.offset = (int)off;
    off += 2 * r.l + 1;
  }
  s->C = off;
  auto& ref = *s;
  cache[L] = std::move(s);
  return ref;
}

std::vector<int32_t> ball_voxels(int N) {
  std::vector<int32_t> v;
  const long long N2 = (long long)N * N;
  for (int i = 0; i < N; ++i) {
    const long long a = 2LL * i - (N - 1);
    for (int j = 0; j < N; ++j) {
      const long long b = 2LL * j - (N - 1);
      for (int k = 0; k < N; ++k) {
        const long long c = 2LL * k - (N - 1);
        if (a * a + b * b + c * c < N2) v.push_back((int32_t)(((long long)i * N + j) * N + k));
      }
    }
  }
  return v;
}

std::vector<int32_t> orbit_representatives(int N) {
  std::vector<int32_t> v;
  const long long N2 = (long long)N * N;
  for (int i = N / 2; i < N; ++i) {
    const long long a = 2LL * i - (N - 1);
    for (int j = N / 2; j < N; ++j) {
      const long long b = 2LL * j - (N - 1);
      for (int k = N / 2; k < N; ++k) {
        const long long c = 2LL * k - (N - 1);
        if (a * a + b * b + c * c < N2) v.push_back((int32_t)(((long long)i * N + j) * N + k));
      }
    }
  }
  return v;
}

// x -> -x maps phi to pi - phi: cos m phi keeps the sign (-1)^m, sin m phi
// takes (-1)^(m+1); y -> -y maps phi to -phi (sin odd); z -> -z maps
// cos theta to -cos theta, and P_l^m(-t) = (-1)^(l+m) P_l^m(t).
int column_parity_class(int l, int j) {
  const int m = (j + 1) / 2;
  const bool sine = j > 0 && (j % 2 == 0);
  const int cx = sine ? (m + 1) & 1 : m & 1;
  const int cy = sine ? 1 : 0;
  const int cz = (l + m) & 1;
  return cx | (cy << 1) | (cz << 2);
}

int64_t wave_block_offset(int L, int W) {
  int64_t off = 0;
  for (int wi = 0; wi < kNumWaveChoices; ++wi) {
    if (kWaveChoices[wi] == W) return off;
    off += (int64_t)kWaveChoices[wi] * (2 * L + 2);
  }
  return -1;
}

BandTables band_tables(int L, int Lmax) {
  BandTables t;
  t.L = L;
  t.p_first.assign(2 * L + 2, 0);
  for (int p = 0; p <= 2 * L; ++p) {
    t.p_first[p] = (int32_t)t.n_entries;
    for (int q = p % 2; q <= 2 * L - p; q += 2) {
      const int m = (p + q) / 2, n = (p - q) / 2;
      double w1, w2;
      if (q == 0 && p == 0) {
        w1 = 1.0; w2 = 0.0;
      } else if (q == 0) {
        w1 = 2.0; w2 = 0.0;
      } else if (p == 0) {
        w1 = 1.0; w2 = 1.0;
      } else {
        w1 = 2.0; w2 = 2.0;
      }
      const double sgn_swap = ((m - n) % 2 == 0) ? 1.0 : -1.0;
      // seed scale (-1)^q sqrt(binom(2m, p))
      long double bin = 1.0L;
      for (int i = 1; i <= p; ++i) bin = bin * (long double)(2 * m - p + i) / (long double)i;
      const double nu0 = ((q % 2) ? -1.0 : 1.0) * std::sqrt((double)bin);
      auto wfun = [&](int l) {
        return std::sqrt(((double)l * l - (double)m * m) * ((double)l * l - (double)n * n));
      };
      const int len = L - m + 1;
      std::vector<double> nu(len + 1), ap(len, 0.0), bq(len, 0.0);
      nu[0] = nu0;                  // l = m
      if (len >= 2) nu[1] = nu0;    // l = m + 1
      for (int l = m; l < L; ++l) {
        const int i = l - m;
        const double wl1 = wfun(l + 1);
        const double A = (2.0 * l + 1.0) * (l + 1.0) / wl1;
        const double B = (l > 0) ? (double)m * n / ((double)l * (l + 1.0)) : 0.0;
        const double Cc = (l > 0) ? (l + 1.0) * wfun(l) / ((double)l * wl1) : 0.0;
        if (i >= 1) nu[i + 1] = Cc * nu[i - 1];
        ap[i] = A * nu[i] / nu[i + 1];
        bq[i] = B;
      }
      for (int i = 0; i < class_span(len); ++i) {
        const bool pad = i >= len;
        const int l = pad ? L : m + i;
        t.rec.push_back(pad ? 0.0 : ap[i]);
        t.rec.push_back(pad ? 0.0 : bq[i]);
        t.sel.push_back(l);
        t.sel.push_back(m);
        t.sel.push_back(n);
        t.sel.push_back(0);
        t.wt.push_back(pad ? 0.0 : w1 * nu[i]);
        t.wt.push_back(pad ? 0.0 : w2 * sgn_swap * nu[i]);
      }
      t.n_entries += class_span(len);
      t.n_classes += 1;
    }
  }
  t.p_first[2 * L + 1] = (int32_t)t.n_entries;

  // Longest-first assignment of p-groups to waves.  Cost of a group: its
  // recurrence entries and class epilogues, in instructions of the kernel.
  std::vector<std::pair<int64_t, int>> cost;
  for (int p = 0; p <= 2 * L; ++p) {
    int64_t entries = 0;   // chain entries, padding not counted
    for (int q = p % 2; q <= 2 * L - p; q += 2) entries += L - (p + q) / 2 + 1;
    const int64_t classes = (2 * L - p) / 2 + 1;
    cost.push_back({13 * entries + 32 * classes, p});
  }
  std::sort(cost.begin(), cost.end(), [](const std::pair<int64_t, int>& a,
                                         const std::pair<int64_t, int>& b) {
    return a.first != b.first ? a.first > b.first : a.second < b.second;
  });
  const int row = 2 * L + 2;
  for (int wi = 0; wi < kNumWaveChoices; ++wi) {
    const int W = kWaveChoices[wi];
    std::vector<int64_t> load(W, 0);
    std::vector<std::vector<int>> lists(W);
    for (const auto& c : cost) {
      int best = 0;
      for (int w = 1; w < W; ++w)
        if (load[w] < load[best]) best = w;
      load[best] += c.first;
      lists[best].push_back(c.second);
    }
    for (int w = 0; w < W; ++w) {
      std::sort(lists[w].begin(), lists[w].end());
      t.wave_p.push_back((int32_t)lists[w].size());
      for (int i = 0; i < row - 1; ++i)
        t.wave_p.push_back(i < (int)lists[w].size() ? lists[w][i] : 0);
    }
  }

  // radial entries of band L grouped by degree, as offsets in the Lmax layout
  const IndexSet& big = index_set(Lmax);
  const double cut = index_set(L).cutoff;
  t.deg_start.assign(L + 2, 0);
  std::vector<std::vector<int32_t>> by_l(L + 1);
  for (const auto& r : big.rad)
    if (r.lam < cut && r.l <= L) by_l[r.l].push_back(r.offset);
  for (int l = 0; l <= L; ++l) {
    t.deg_start[l] = (int32_t)t.deg_off.size();
    for (int32_t o : by_l[l]) t.deg_off.push_back(o);
  }
  t.deg_start[L + 1] = (int32_t)t.deg_off.size();
  return t;
}

double interval_union(std::vector<std::pair<double, double>> iv) {
  std::sort(iv.begin(), iv.end());
  double busy = 0.0, lo = 0.0, hi = 0.0;
  bool open = false;
  for (const auto& x : iv) {
    if (x.second < x.first) continue;
    if (!open || x.first > hi) {
      if (open) busy += hi - lo;
      lo = x.first;
      hi = x.second;
      open = true;
    } else if (x.second > hi) {
      hi = x.second;
    }
  }
  if (open) busy += hi - lo;
  return busy;
}

}  // namespace bh
