// Internal declarations of the bh library: plan state, error reporting and
// the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bh.h"
#include "bh_tables.h"

namespace bh {

// ----------------------------------------------------------------- errors --
int set_error(int code, const std::string& msg);

#define BH_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::bh::set_error(BH_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// -------------------------------------------------------------- GEMM shape --
// Expansion GEMM a[b][c] = sum_v F[b][v] Psi[v][c] on MFMA f32 32x32x2.
//
// The cell-centred ball is symmetric under the reflections x, y, z -> -x,
// -y, -z, and every real basis column is even or odd under each of them
// (its parity class P, 3 bits).  With g_P(v) = sum over the 8 reflections R
// of chi_P(R) f(R v) at one representative v per orbit (chi_P(R) = -1 when
// R flips an odd number of the axes P marks), the column's coefficient is
// sum_v g_P(v) Psi(v) / |orbit stabiliser| over the representatives only:
// the GEMM runs over an eighth of the voxels, class by class.  Columns are
// stored class after class, each class padded to whole column tiles.
constexpr int kGemmBM = 128;     // particles per tile
constexpr int kGemmBN = 128;     // coefficients per tile
constexpr int kGemmBK = 32;      // voxels per K step
constexpr int kGemmKAlign = kGemmBK * 16;   // VR padded to this, split-K <= 16
constexpr int kParityClasses = 8;

// Column tiles [first[P], first[P+1]) hold parity class P; passed by value.
struct ClassTiles {
  int32_t first[kParityClasses + 1];
};
__host__ __device__ inline int class_of_tile(const ClassTiles& ct, int64_t tn) {
  int c = 0;
  while (c < kParityClasses - 1 && tn >= ct.first[c + 1]) ++c;
  return c;
}

// Placement of the expansion GEMM's tiles.  Workgroups are dispatched
// round-robin over the 8 XCDs (linear id mod 8), each with its own L2.  The
// tiles are ordered (split, coefficient tile, particle tile), particle tiles
// fastest, and XCD x takes the x-th contiguous eighth of that order (the
// first total % 8 XCDs one tile more).  Co-resident workgroups of an XCD then
// work on one K-slice: those of one coefficient tile share its basis slice,
// those of neighbouring coefficient tiles (mostly one parity class) the
// folded-volume slice, and each slice is fetched by one XCD (two where a
// boundary falls) instead of by all eight.
__device__ inline void gemm_tile(int64_t bid, int64_t mt, int64_t nt, int64_t ns, int64_t& m,
                                 int64_t& n, int64_t& sp) {
  const int64_t total = mt * nt * ns, q = total / 8, rem = total % 8;
  const int64_t xcd = bid % 8, local = bid / 8;
  const int64_t g = xcd * q + (xcd < rem ? xcd : rem) + local;
  m = g % mt;
  const int64_t u = g / mt;
  n = u % nt;
  sp = u / nt;
}

// The 8 mirror images of voxel (i, j, k): image s (bit 0: i -> N-1-i,
// bit 1: j, bit 2: k) at linear offset off[s].
__device__ inline void mirror_offsets(int32_t lin, int N, int32_t off[8]) {
  const int i = lin / (N * N), j = (lin / N) % N, k = lin % N;
  const int32_t I[2] = {i * N * N, (N - 1 - i) * N * N};
  const int32_t J[2] = {j * N, (N - 1 - j) * N};
  const int32_t K[2] = {k, N - 1 - k};
#pragma unroll
  for (int s = 0; s < 8; ++s) off[s] = I[s & 1] + J[(s >> 1) & 1] + K[s >> 2];
}

// The volume row that expansion particle b reads: rows[b] with a row table,
// else b; -1 for the padding particles b >= B; -2 (and the error word `bad`
// raised, when given) for a table entry outside [0, n_rows).
__device__ inline int64_t volume_row(const int64_t* __restrict__ rows, int64_t n_rows, int64_t B,
                                     int64_t b, int* bad) {
  if (b >= B) return -1;
  if (!rows) return b;
  const int64_t r = rows[b];
  if (r >= 0 && r < n_rows) return r;
  if (bad) *reinterpret_cast<volatile int*>(bad) = 1;
  return -2;
}

// In place: f[P] = sum_s (-1)^popcount(P & s) f[s] (size-8 Walsh-Hadamard),
// the mirror sum g_P of parity class P from the 8 image values.
__device__ inline void parity_fold(float f[8]) {
#pragma unroll
  for (int h = 1; h < 8; h <<= 1) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (s & h) continue;
      const float a = f[s], b = f[s | h];
      f[s] = a + b;
      f[s | h] = a - b;
    }
  }
}

// The score loop loads whole rounds of four table entries, up to three
// past a chain's end; the recurrence tables and the per-particle cross-power
// buffers carry this many entries past their end for the last chain (the
// values read there are never used).
constexpr int kTablePad = 4;

// Largest restart count for which candidates can be pruned after the first
// band (the pruning kernel ranks the restarts of a particle in LDS).
constexpr int kPruneMaxP = 1024;

// Device copy of one band's score tables (see BandTables).
struct DevBand {
  int L = -1;
  int n_classes = 0;
  int64_t n_entries = 0;
  double* rec = nullptr;        // [n_entries][2]
  int32_t* sel = nullptr;       // [n_entries][4]
  double* wt = nullptr;         // [n_entries][2]
  int32_t* p_first = nullptr;   // [2L+2]
  int32_t* wave_p = nullptr;    // work split per wave count (BandTables::wave_p)
  int32_t* deg_start = nullptr; // [L+2]
  int32_t* deg_off = nullptr;   // [n_deg]
  int n_deg = 0;                // (l, k) pairs of the band
};

struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Opt-in per-launch timing: a pair of HIP events recorded on the launch
// stream around each kernel while enabled.
struct Profiler {
  bool on = false;
  struct Rec {
    std::string name;
    hipEvent_t start, stop;
    int64_t work;      // caller-defined work units of the launch (for reporting)
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t take();
  void clear();
  void destroy();
};

}  // namespace bh

struct bh_plan {
  int N = 0, L_max = 0, device = 0;
  const bh::IndexSet* idx = nullptr;
  int64_t V = 0;                 // ball voxels
  int64_t VR = 0, VR_pad = 0;    // orbit representatives, padded to kGemmKAlign
  int64_t C = 0, C_pad = 0;      // complex coefficients of L_max; real columns with class padding
  bh::ClassTiles ctiles = {};    // column tiles of each parity class
  float* psi = nullptr;          // [VR_pad][C_pad] h^3 / |stabiliser| * real columns of conj(psi)
  uint16_t* psi_h = nullptr;     // [C_pad][VR_pad] BF16 of psi (built on first BF16 use)
  uint16_t* psi_l = nullptr;     // [C_pad][VR_pad] BF16 of psi - psi_h
  int32_t* vrep = nullptr;       // [VR] linear voxel index of each orbit representative
  int32_t* csrc = nullptr;       // [C][2] real column feeding re/im of each complex coefficient
  float* csgn = nullptr;         // [C][2] sign applied to it
  std::vector<int64_t> band_size;   // C(L) for L = 0..L_max
  // error word raised by kernels that meet a template index outside the
  // table: pinned, mapped host memory (err_host) and its device address
  int* err_host = nullptr;
  int* err_dev = nullptr;
  // scratch (grown on demand, owned by the plan)
  bh::Buffer gathered, partial, xi_scr, state_scr, misc_scr, prune_scr, shift_scr, newton_scr,
      energy_scr;
  std::map<int, bh::DevBand> bands;
  bh::Profiler prof;
  // autotuned launch shapes (0 / absent: the built-in rules)
  int tuned_waves[BH_MAX_L + 1] = {};
  int tuned_persist[BH_MAX_L + 1] = {};   // 1: ascent launches as resident workgroups only
  std::map<int64_t, int> tuned_split[2];   // particle tiles -> split-K (FP32, BF16 GEMM)
  // a march split into two halves on two streams (launch_align): the
  // second half's scratch, its stream (default priority) and the fork and
  // join events, created on first use; march_streams 1 never splits
  bh::Buffer xi_scr2, state_scr2, misc_scr2;
  hipStream_t aux_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int march_streams = 2;
};

namespace bh {

// Records start/stop events around the launches made during its lifetime
// (when the plan's profiler is on).
class ProfScope {
 public:
  ProfScope(bh_plan* p, const std::string& name, hipStream_t s, int64_t work = 0);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  bh_plan* p_;
  hipStream_t s_;
  int idx_ = -1;
};

int grow(Buffer& b, size_t bytes);
int get_band(bh_plan* p, int L, const DevBand** out);

// launchers (return BH_OK or an error code)
int build_basis(bh_plan* p);
// Split-K factor of the expansion GEMM.
//
// Fixed rule: doubled while the grid has fewer than 2048 tiles and each
// split keeps at least 8 K-steps.  With batch_invariant it is applied with
// the particle-tile count taken as 8 (1024 particles) whatever the batch, so
// a particle's sums never depend on the batch size.
//
// Otherwise a tuned factor if there is one.  Else, for grids of at most two
// rounds of the `slots` resident workgroups, the factor ns (1..16, at least
// 8 K-steps per split) with the smallest modelled cost in units of one
// workgroup's K-step,
//   ceil(tiles ns / slots) slots ceil(nk_total / ns) + ns tiles q,
// the rounds (each as long as its longest split) plus the partial sums, q
// being the HBM time of one tile's partial sums (written by the GEMM, read
// back by the reduction) over the chip-wide time of one workgroup K-step
// (ties to fewer splits).  Small batches gain most: at 64^3, L = 32 the fixed
// rule's 16 splits of one or two particle tiles overflow one round by a few
// workgroups.  Where the model's grid needs more rounds the fixed rule is
// kept: its factors 4, 8 and 16 give each XCD whole K-slices (tiles are
// placed split-major, XCD by XCD), which measured faster than the model's
// fuller last round.  Splits need not divide nk_total: split s takes K-steps
// [s nk_total / ns, (s + 1) nk_total / ns), the equal slices of the fixed
// rule where ns divides nk_total.  Without a slot count (slots <= 0) the
// fixed rule is used.
constexpr int kMaxSplit = 16;   // split-K factors 1..16 (the reductions hold one value per split)
inline int expand_split(int64_t mt, int64_t nt, int64_t nk_total, bool batch_invariant,
                        const std::map<int64_t, int>* tuned = nullptr, int64_t slots = 0,
                        int64_t q = 0) {
  if (!batch_invariant && tuned) {
    const auto it = tuned->find(mt);
    if (it != tuned->end()) return it->second;
  }
  if (!batch_invariant && slots > 0) {
    const int64_t tiles = mt * nt;
    int best = 1;
    int64_t best_cost = -1, best_rounds = 0;
    for (int ns = 1; ns <= kMaxSplit && (ns == 1 || nk_total / ns >= 8); ++ns) {
      const int64_t rounds = (tiles * ns + slots - 1) / slots;
      const int64_t cost = rounds * slots * ((nk_total + ns - 1) / ns) + ns * tiles * q;
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        best = ns;
        best_rounds = rounds;
      }
    }
    if (best_rounds <= 2) return best;
  }
  if (batch_invariant) mt = 8;
  int nsplit = 1;
  while (nsplit < kMaxSplit && mt * nt * nsplit < 2048 && (nk_total / (nsplit * 2)) >= 8)
    nsplit *= 2;
  return nsplit;
}
// K-steps [k0, k0 + nk) of split ts of nsplit over nk_total steps.
__host__ __device__ inline void split_range(int64_t ts, int64_t nsplit, int64_t nk_total,
                                            int64_t& k0, int64_t& nk) {
  k0 = ts * nk_total / nsplit;
  nk = (ts + 1) * nk_total / nsplit - k0;
}
// Workgroups of a kernel that fit on the current device at once (0 if
// unknown), cached per kernel.
template <typename K>
int64_t resident_workgroups(K kernel, int threads) {
  static std::mutex mu;
  static std::map<const void*, int64_t> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find((const void*)kernel);
  if (it != cache.end()) return it->second;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cache[(const void*)kernel] = (int64_t)per_cu * cus;
}
// The split-K factors the FP32 and split-BF16 expansions use for B particles
// (each GEMM's resident workgroups on the current device as the slots;
// refine: the split-BF16 GEMM with the correction products).
int expand_split_f32(const bh_plan* p, int64_t B, bool batch_invariant);
int expand_split_bf16(const bh_plan* p, int64_t B, bool batch_invariant, bool refine = true);
// Integer voxel shifts, passed to kernels by value.
constexpr int kMaxShifts = 125;
struct ShiftTable {
  int32_t d[kMaxShifts][3];
};
// With `shifts` the rows are the B*S shifted volumes (particle-major) of
// the S integer voxel shifts.
// ldc: complex stride between particles' coefficient rows (0: C(L_max)).
// rows: device table of B volume rows (particle b is vols[rows[b]], vols
// holding n_rows volumes), or NULL (particle b is vols[b]); not with shifts.
int launch_expand(bh_plan* p, const float* vols, int64_t B, float* coeffs, hipStream_t s,
                  bool batch_invariant = false, const ShiftTable* shifts = nullptr, int S = 1,
                  int64_t ldc = 0, const int64_t* rows = nullptr, int64_t n_rows = 0);
// Allocation-free expansion: resolve this device's copy of the static
// scratch (once per device, with the device current; called at plan
// creation), how many 128-particle tiles one pass holds (returns the split-K
// factor), and the launcher.
int noalloc_scratch_init(int device);
int noalloc_expand_pass(const bh_plan* p, int64_t* tiles_per_pass);
int launch_expand_noalloc(bh_plan* p, const float* vols, int64_t B, float* coeffs, hipStream_t s);
int launch_expand_bf16(bh_plan* p, const float* vols, int64_t B, bool refine, float* coeffs,
                       float* coarse_out, hipStream_t s, bool batch_invariant = false,
                       int64_t ldc = 0, const int64_t* rows = nullptr, int64_t n_rows = 0);
int launch_cross_power_dense(bh_plan* p, const DevBand& band, const float* a, const float* b,
                             int64_t B, double* xi, hipStream_t s);
int launch_correlate(bh_plan* p, const DevBand& band, const float* a, const float* b, int64_t B,
                     const double* euler, int R, double* score, double* grad, double* hess,
                     hipStream_t s);
int launch_degree_energy(bh_plan* p, const DevBand& band, const float* a, const float* b,
                         const int32_t* tmpl, int n_tmpl, int64_t B, double* energy,
                         hipStream_t s);
// Milliseconds of `launch` on stream s (HIP events), summed over `reps` runs
// after one warm-up run; `prepare` is enqueued before each run, untimed.
template <typename Prep, typename Launch>
int time_on_stream(hipStream_t s, int reps, Prep&& prepare, Launch&& launch, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_error(BH_EDEVICE, "hipEventCreate failed");
  }
  float total = 0.0f;
  hipError_t e = hipSuccess;
  for (int rep = 0; rep <= reps && e == hipSuccess; ++rep) {
    prepare();
    if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
    launch();
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
      break;
    float t = 0.0f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
    if (rep > 0) total += t;
    e = hipGetLastError();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_error(BH_EDEVICE, std::string("timing: ") + hipGetErrorString(e));
  *ms = total;
  return BH_OK;
}

// Autotuning (see bh_plan_autotune): time the candidate shapes on random
// data of B particles and record the fastest in the plan.
int tune_march(bh_plan* p, int64_t B, int P, const int32_t* bands, int n_bands, hipStream_t s);
int tune_expand_f32(bh_plan* p, int64_t B, hipStream_t s);
int tune_expand_bf16(bh_plan* p, int64_t B, hipStream_t s);
// Thresholds of the energy-ratio band selection, passed by value.
constexpr int kMaxBandThresholds = 16;
struct BandThresholds {
  double t[kMaxBandThresholds];
};
int launch_select_bands(bh_plan* p, const DevBand& band, const float* a, const float* templates,
                        const int32_t* tmpl, int n_tmpl, int64_t B, const BandThresholds& th,
                        int n_tau, int32_t* bands, int32_t* common, double* ratio, hipStream_t s);
int launch_prune(bh_plan* p, const double* euler, const double* score, int64_t B, int P, int K,
                 double min_sep, double* euler_out, double* score_out, hipStream_t s);
int launch_align_shifts(bh_plan* p, const float* vols, int64_t B, const int32_t* shifts_host,
                        int S, const float* b, const bh_align_opts& o, const double* starts,
                        double* euler_out, double* score_out, int32_t* shift_out, hipStream_t s);
// lda / ldt: complex strides of the particle and template rows (0: C(L_max));
// active: particles taking each band (a prefix of the batch; NULL: all B).
int launch_align(bh_plan* p, const float* a, const float* b, const int32_t* tmpl, int n_tmpl,
                 int64_t B, const bh_align_opts& o,
                 const double* starts, double* euler_out, double* score_out, double* all_euler,
                 double* all_score, hipStream_t s, int64_t lda = 0, int64_t ldt = 0,
                 const int64_t* active = nullptr);

}  // namespace bh
