// Host-side tables: Bessel zeros and the frequency-ordered index set
// (Sec. II-A), and the per-band tables of the Wigner small-d recurrence used
// by the score kernels (Eq. (2)).
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

namespace bh {

// One radial entry (l, k) of the index set, in ascending lambda_lk.
struct Radial {
  int l, k;
  double lam;    // k-th positive zero of j_l
  double c;      // sqrt(2) / |j_{l+1}(lam)|
  int offset;    // first coefficient of this entry; m = -l..l follow
};

struct IndexSet {
  int L = -1;
  double cutoff = 0;            // lambda_{L+1,1}
  std::vector<Radial> rad;      // ascending lambda, ties by (l, k)
  int64_t C = 0;                // number of complex coefficients
};

// k-th positive zero of j_l (k >= 1), by sign-change bracketing + bisection.
double bessel_zero(int l, int k);
// All positive zeros of j_l below x_max.
std::vector<double> bessel_zeros_below(int l, double x_max);
// Index set of band L (cached; thread-safe).
const IndexSet& index_set(int L);

// Number of ball voxels of the N^3 cell-centred grid and their linear indices.
std::vector<int32_t> ball_voxels(int N);

// Ball voxels with all three coordinates >= 0: one voxel of each orbit of
// the three coordinate-plane reflections (linear indices, k fastest).  On
// an odd grid an orbit touching a mirror plane has fewer than 8 members.
std::vector<int32_t> orbit_representatives(int N);

// Parity class 0..7 of real basis column j (0: m = 0; 2m-1: cos m phi;
// 2m: sin m phi) of degree l under the reflections x -> -x (bit 0),
// y -> -y (bit 1), z -> -z (bit 2): a set bit means the column changes sign.
int column_parity_class(int l, int j);

// ---------------------------------------------------------------------------
// Score tables of one band L.
//
// The score sum over (l, m, n) is reorganised into "classes": ordered pairs
// (m, n) modulo the swap (m, n) -> (n, m) (d^l_{nm} = (-1)^{m-n} d^l_{mn})
// and the real-input conjugation (m, n) -> (-m, -n).  Canonical member:
// m >= |n|.  Classes are enumerated by p = m + n in 0..2L and, inside,
// q = m - n = p mod 2, p mod 2 + 2, ..., <= 2L - p.  Class (m, n) owns the
// chain l = m..L.  Along the chain d^l_{mn}(beta) = nu_l e_l with
//   e_{m-1} = 0, e_m = cos(beta/2)^p sin(beta/2)^q,
//   e_{l+1} = ap_l (cos(beta) - bq_l) e_l - e_{l-1},
// which is the three-term recurrence in l rescaled so that the coefficient
// of e_{l-1} is one; nu_l carries the scale, the sign (-1)^q and
// sqrt(binom(2m, p)) of the closed-form seed d^m_{mn}.
//
// Entry e (class, l) holds, for the kernels:
//   rec[e]   = {ap_l, bq_l}
//   sel[e]   = {l, m, n, flags}
//   wt[e]    = {w1 nu_l, w2 (-1)^{m-n} nu_l}: weights of xi^l_{mn} and
//              xi^l_{nm}.  w1 = w2 = 2 for m > |n| (the swapped pair and the
//              conjugate pairs), w1 = 2, w2 = 0 for n = m > 0, w1 = w2 = 1 for
//              n = -m < 0, w1 = 1, w2 = 0 for (0, 0).
// Per class: a contiguous run of entries (L - m + 1 of them), followed by a
// zero-weight padding entry if that number is odd (class_span), so that
// every chain starts on a 64-byte boundary of the per-particle weights: the
// score kernels read a chain in rounds of four entries with 64-byte scalar
// loads, and an aligned round's weights then span two cache lines rather
// than three.  (Padding to four entries, which also aligns rec, measured the
// same for the ascent kernel and cost the Newton bands, which stream the
// weights from HBM, 13 % more bytes instead of 6 %.)  Padding entries repeat
// the class's last (l, m, n) with zero weights and zero recurrence
// coefficients; no kernel uses their values.
// ---------------------------------------------------------------------------
// Stored entries of a chain of n entries (n rounded up to even).
constexpr int class_span(int n) { return (n + 1) & ~1; }

struct BandTables {
  int L = -1;
  int n_classes = 0;
  int64_t n_entries = 0;
  std::vector<double> rec;        // [n_entries][2]
  std::vector<int32_t> sel;       // [n_entries][4]
  std::vector<double> wt;         // [n_entries][2]
  std::vector<int32_t> p_first;   // [2L+2] first entry of the classes with this p
  // Work split of the classes over the W waves of a workgroup, for each W in
  // kWaveChoices: the p-groups are assigned longest first to the least
  // loaded wave.  Block of W rows of (2L+2) ints: [count, p_1, ..., p_count].
  std::vector<int32_t> wave_p;
  // radial entries of the band grouped by degree (for the cross-power sums)
  std::vector<int32_t> deg_start; // [L+2]
  std::vector<int32_t> deg_off;   // coefficient offsets of (l, k) with lambda < cutoff(L)
};

// Wave counts per workgroup for which band_tables prepares a work split.
constexpr int kWaveChoices[] = {4, 5, 6, 8, 10, 12, 16};
constexpr int kNumWaveChoices = 7;
// Offset of the block of W (one of kWaveChoices) in BandTables::wave_p.
int64_t wave_block_offset(int L, int W);

// Tables of band L; coefficient offsets refer to the layout of index_set(Lmax).
BandTables band_tables(int L, int Lmax);

// Total length of the union of closed intervals [first, second] (in any
// order; intervals that touch or overlap count once; second < first counts
// as empty).  The busy time of kernel launches that overlap on two streams.
double interval_union(std::vector<std::pair<double, double>> iv);

}  // namespace bh
