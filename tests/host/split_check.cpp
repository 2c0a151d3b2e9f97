// Host checks of the expansion GEMM's split-K rule and slice ranges
// (bh_internal.h: expand_split, split_range).  Prints "ok: 0 failures".
#include <cstdio>
#include <map>

#include "bh_internal.h"

static int failures = 0;
#define CHECK(c, ...)                  \
  do {                                 \
    if (!(c)) {                        \
      ++failures;                      \
      std::printf("FAIL: " __VA_ARGS__); \
      std::printf("\n");               \
    }                                  \
  } while (0)

int main() {
  using bh::expand_split;
  using bh::split_range;
  // slices: consecutive, covering [0, nk) exactly, lengths differing by at
  // most one, equal where the factor divides nk
  for (int64_t nk = 1; nk <= 2000; nk += (nk < 64 ? 1 : 37)) {
    for (int64_t ns = 1; ns <= bh::kMaxSplit && ns <= nk; ++ns) {
      int64_t next = 0, lo = nk, hi = 0;
      for (int64_t s = 0; s < ns; ++s) {
        int64_t k0, n;
        split_range(s, ns, nk, k0, n);
        CHECK(k0 == next, "slice %lld of %lld over %lld starts at %lld", (long long)s,
              (long long)ns, (long long)nk, (long long)k0);
        next = k0 + n;
        lo = n < lo ? n : lo;
        hi = n > hi ? n : hi;
      }
      CHECK(next == nk, "slices of %lld over %lld end at %lld", (long long)ns, (long long)nk,
            (long long)next);
      CHECK(hi - lo <= 1 && lo >= 1, "slice lengths %lld..%lld", (long long)lo, (long long)hi);
      if (nk % ns == 0) CHECK(lo == nk / ns && hi == nk / ns, "unequal slices of a divisor");
    }
  }
  const int64_t slots = 512;
  for (int64_t nt : {4, 10, 36, 70}) {
    for (int64_t nk : {32, 96, 544, 1088}) {
      const int inv = expand_split(8, nt, nk, true);
      for (int64_t mt = 1; mt <= 100; ++mt) {
        // batch-invariant: the same factor for every batch size
        CHECK(expand_split(mt, nt, nk, true, nullptr, slots, 4) == inv,
              "batch-invariant factor depends on the batch (nt %lld nk %lld mt %lld)",
              (long long)nt, (long long)nk, (long long)mt);
        for (int64_t q : {4, 18}) {
          const int ns = expand_split(mt, nt, nk, false, nullptr, slots, q);
          CHECK(ns >= 1 && ns <= bh::kMaxSplit, "factor %d out of range", ns);
          CHECK(ns == 1 || nk / ns >= 8, "split of fewer than 8 K-steps (ns %d nk %lld)", ns,
                (long long)nk);
          // the model's factor only where its grid fits in two rounds of
          // the resident workgroups, else the fixed rule of the batch
          const int64_t rounds = (mt * nt * ns + slots - 1) / slots;
          CHECK(rounds <= 2 || ns == expand_split(mt, nt, nk, false, nullptr, 0),
                "grid of %lld rounds from the model", (long long)rounds);
        }
        // no slot count: the fixed rule of the actual batch
        const int f = expand_split(mt, nt, nk, false, nullptr, 0);
        CHECK(f >= 1 && f <= bh::kMaxSplit && (f & (f - 1)) == 0, "fixed rule factor %d", f);
      }
    }
  }
  // the factors measured best at 64^3, L = 32 (36 coefficient tiles, 544
  // K-steps, 512 resident workgroups): FP32 (q = 4) and split BF16 (q = 18)
  const struct { int64_t mt, q; int want; } meas[] = {
      {1, 4, 14}, {2, 4, 7}, {4, 4, 7}, {8, 4, 8}, {16, 4, 4},
      {2, 18, 7}, {4, 18, 7}, {8, 18, 8}, {16, 18, 4}};
  for (const auto& m : meas) {
    const int ns = expand_split(m.mt, 36, 544, false, nullptr, slots, m.q);
    CHECK(ns == m.want, "64^3 L32: %lld particle tiles, q %lld -> %d splits, want %d",
          (long long)m.mt, (long long)m.q, ns, m.want);
  }
  CHECK(expand_split(3, 36, 544, true) == 8, "batch-invariant factor at 64^3 L32 is not 8");
  // a tuned factor wins over the rule, except for batch-invariant calls
  std::map<int64_t, int> tuned{{8, 5}};
  CHECK(expand_split(8, 36, 544, false, &tuned, slots, 4) == 5, "tuned factor ignored");
  CHECK(expand_split(8, 36, 544, true, &tuned, slots, 4) == 8, "tuned factor used when invariant");
  CHECK(expand_split(9, 36, 544, false, &tuned, slots, 4) ==
            expand_split(9, 36, 544, false, nullptr, slots, 4),
        "tuned factor of another tile count used");
  std::printf("ok: %d failures\n", failures);
  return failures ? 1 : 0;
}
