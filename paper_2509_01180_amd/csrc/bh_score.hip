// Rotational correlation of Eq. (2), its Euler gradient, and frequency
// marching with multi-start gradient ascent (Sec. II-B, II-C).
//
// Score at a rotation g = (alpha, beta, gamma):
//   S = Re sum_l sum_{m,n} xi^l_{mn} e^{-i m alpha} d^l_{mn}(beta) e^{-i n gamma}.
// The (m, n) pairs are grouped in classes (see bh_tables.h): class (m, n),
// m >= |n|, carries the pairs (m, n) and (n, m) (which share d^l up to the
// sign folded into its weights) and, for real inputs, their conjugates
// (-m, -n), (-n, -m).  For each class the kernel runs the rescaled
// three-term recurrence of d^l_{mn}(beta) and of its beta-derivative along
// l = m..L in FP64, accumulating
//   T1 = sum_l X1_l e_l, T2 = sum_l X2_l e_l, R1 = sum_l X1_l r_l, R2 = ...,
// with X1_l = w1 nu_l xi^l_{mn}, X2_l = w2 (-1)^{m-n} nu_l xi^l_{nm} prepared
// per particle by k_xi_classes.  The class then contributes, with
// W1 = e^{-i(m alpha + n gamma)}, W2 = e^{-i(n alpha + m gamma)}:
//   S += Re(W1 T1 + W2 T2),       dS/dbeta  += Re(W1 R1 + W2 R2),
//   dS/dalpha += m Im(W1 T1) + n Im(W2 T2),
//   dS/dgamma += n Im(W1 T1) + m Im(W2 T2).
//
// Mapping: one lane per rotation (a restart), one workgroup per
// (particle, 64 rotations); the W waves of a workgroup split the classes by
// p = m + n (p = wave, wave + W, ...).  All class data are wave-uniform, so
// they are read with scalar loads and every lane runs the same instruction
// stream.  Partial sums are reduced across waves through LDS in a fixed
// order, so every wave holds the same totals.
#include "bh_eval.h"
#include "bh_internal.h"

#include <cmath>
#include <string>

namespace bh {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kSin2Floor = 1e-6;

// Occupancy target of the score kernels (waves per SIMD; 0 = compiler's
// choice) and an optional fixed wave count per workgroup (0 = automatic);
// build-time tuning parameters.
#ifndef BH_SCORE_WAVES_PER_EU
#define BH_SCORE_WAVES_PER_EU 6
#endif
#ifndef BH_SCORE_FIXED_W
#define BH_SCORE_FIXED_W 0
#endif
#if BH_SCORE_WAVES_PER_EU > 0
#define BH_SCORE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(BH_SCORE_WAVES_PER_EU)))
#else
#define BH_SCORE_OCCUPANCY
#endif

// ------------------------------------------------------------ cross-power --

// Dense xi^l_{mn} for the ABI: thread per (particle, entry of E(L)).
__global__ void k_xi_dense(const float* __restrict__ a, const float* __restrict__ b, int64_t C,
                           int L, const int32_t* __restrict__ deg_start,
                           const int32_t* __restrict__ deg_off, int64_t E, double* __restrict__ xi) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pb = blockIdx.y;
  if (t >= E) return;
  // find l: block l starts at l(4l^2-1)/3
  int l = 0;
  while (l < L && (int64_t)(l + 1) * (4LL * (l + 1) * (l + 1) - 1) / 3 <= t) ++l;
  const int64_t r = t - (int64_t)l * (4LL * l * l - 1) / 3;
  const int w = 2 * l + 1;
  const int m = (int)(r / w) - l, n = (int)(r % w) - l;
  const float* ap = a + pb * 2 * C;
  double sre = 0.0, sim = 0.0;
  for (int i = deg_start[l]; i < deg_start[l + 1]; ++i) {
    const int o = deg_off[i];
    const double br = b[2 * (o + l + m)], bi = b[2 * (o + l + m) + 1];
    const double ar = ap[2 * (o + l + n)], ai = ap[2 * (o + l + n) + 1];
    sre += br * ar + bi * ai;   // conj(b) * a
    sim += br * ai - bi * ar;
  }
  xi[(pb * E + t) * 2] = sre;
  xi[(pb * E + t) * 2 + 1] = sim;
}

// Template of particle pb: tmpl[pb] clamped to [0, n_tmpl) (template 0 without a table).
__device__ inline int64_t template_of(const int32_t* __restrict__ tmpl, int n_tmpl, int64_t pb) {
  if (!tmpl) return 0;
  const int t = tmpl[pb];
  return t < 0 ? 0 : (t >= n_tmpl ? n_tmpl - 1 : t);
}

// Class-major weighted cross-power of one band: X[pb][e] = {X1re, X1im, X2re, X2im}.
__global__ void k_xi_classes(const float* __restrict__ a, const float* __restrict__ btab, int64_t C,
                             const int32_t* __restrict__ tmpl, int n_tmpl,
                             int64_t n_entries, const int32_t* __restrict__ sel,
                             const double* __restrict__ wt, const int32_t* __restrict__ deg_start,
                             const int32_t* __restrict__ deg_off, double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pb = blockIdx.y;
  if (e >= n_entries) return;
  const int l = sel[4 * e], m = sel[4 * e + 1], n = sel[4 * e + 2];
  const double w1 = wt[2 * e], w2 = wt[2 * e + 1];
  const float* ap = a + pb * 2 * C;
  const float* b = btab + template_of(tmpl, n_tmpl, pb) * 2 * C;
  double x1r = 0, x1i = 0, x2r = 0, x2i = 0;
  for (int i = deg_start[l]; i < deg_start[l + 1]; ++i) {
    const int o = deg_off[i];
    const double bmr = b[2 * (o + l + m)], bmi = b[2 * (o + l + m) + 1];
    const double bnr = b[2 * (o + l + n)], bni = b[2 * (o + l + n) + 1];
    const double amr = ap[2 * (o + l + m)], ami = ap[2 * (o + l + m) + 1];
    const double anr = ap[2 * (o + l + n)], ani = ap[2 * (o + l + n) + 1];
    x1r += bmr * anr + bmi * ani;      // conj(b_m) a_n
    x1i += bmr * ani - bmi * anr;
    x2r += bnr * amr + bni * ami;      // conj(b_n) a_m
    x2i += bnr * ami - bni * amr;
  }
  double* out = X + (pb * n_entries + e) * 4;
  out[0] = w1 * x1r;
  out[1] = w1 * x1i;
  out[2] = w2 * x2r;
  out[3] = w2 * x2i;
}

// W_b = sum_l l(l+1) ||a_l|| ||b_l|| over the band; one block per particle.
__global__ void k_band_weight(const float* __restrict__ a, const float* __restrict__ btab, int64_t C,
                              const int32_t* __restrict__ tmpl, int n_tmpl,
                              int L, const int32_t* __restrict__ deg_start,
                              const int32_t* __restrict__ deg_off, double* __restrict__ Wb) {
  __shared__ double part[BH_MAX_L + 1];
  const int64_t pb = blockIdx.x;
  const float* ap = a + pb * 2 * C;
  const float* b = btab + template_of(tmpl, n_tmpl, pb) * 2 * C;
  for (int l = threadIdx.x; l <= L; l += blockDim.x) {
    double na = 0.0, nb = 0.0;
    for (int i = deg_start[l]; i < deg_start[l + 1]; ++i) {
      const int o = deg_off[i];
      for (int m = -l; m <= l; ++m) {
        const double ar = ap[2 * (o + l + m)], ai = ap[2 * (o + l + m) + 1];
        const double br = b[2 * (o + l + m)], bi = b[2 * (o + l + m) + 1];
        na += ar * ar + ai * ai;
        nb += br * br + bi * bi;
      }
    }
    part[l] = (double)l * (l + 1) * sqrt(na) * sqrt(nb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int l = 0; l <= L; ++l) s += part[l];
    Wb[pb] = s;
  }
}

// Sum the W wave partials (fixed order) through LDS buffer `buf`.
__device__ inline Acc reduce_waves(Acc mine, double* buf, int wave, int lane, int W) {
  buf[(wave * 4 + 0) * 64 + lane] = mine.S;
  buf[(wave * 4 + 1) * 64 + lane] = mine.ga;
  buf[(wave * 4 + 2) * 64 + lane] = mine.gb;
  buf[(wave * 4 + 3) * 64 + lane] = mine.gg;
  __syncthreads();
  Acc t = {0.0, 0.0, 0.0, 0.0};
  for (int w = 0; w < W; ++w) {
    t.S += buf[(w * 4 + 0) * 64 + lane];
    t.ga += buf[(w * 4 + 1) * 64 + lane];
    t.gb += buf[(w * 4 + 2) * 64 + lane];
    t.gg += buf[(w * 4 + 3) * 64 + lane];
  }
  return t;
}

__device__ inline double wrap_pi(double t) { return t - kTwoPi * floor((t + kPi) / kTwoPi); }

__device__ inline void wrap_euler(double& a, double& b, double& g) {
  b = b - kTwoPi * floor(b / kTwoPi);
  if (b > kPi) {
    b = kTwoPi - b;
    a += kPi;
    g += kPi;
  }
  a = wrap_pi(a);
  g = wrap_pi(g);
}

template <int W>
__global__ __launch_bounds__(64 * W) BH_SCORE_OCCUPANCY void k_correlate(
    const int32_t* __restrict__ p_first, const int32_t* __restrict__ wave_p,
                                                      const double* __restrict__ rec,
                                                      const double* __restrict__ X, int64_t n_entries,
                                                      int L, const double* __restrict__ euler, int R,
                                                      double* __restrict__ score,
                                                      double* __restrict__ grad) {
  __shared__ double buf[W * 4 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t pb = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const bool active = r < R;
  double al = 0.0, be = 0.0, ga = 0.0;
  if (active) {
    const double* eu = euler + (pb * R + r) * 3;
    al = eu[0];
    be = eu[1];
    ga = eu[2];
  }
  const Angles A = prep(al, be, ga);
  const Acc mine = eval_wave(A, wave_p + wave * (2 * L + 2), L, p_first, rec, X + pb * n_entries * 4);
  const Acc t = reduce_waves(mine, buf, wave, lane, W);
  if (wave == 0 && active) {
    score[pb * R + r] = t.S;
    if (grad) {
      grad[(pb * R + r) * 3 + 0] = t.ga;
      grad[(pb * R + r) * 3 + 1] = t.gb;
      grad[(pb * R + r) * 3 + 2] = t.gg;
    }
  }
}

// One band of the ascent for 64 restarts of one particle (see bh.h).
//
// Every evaluation is split over the W waves; the ascent state of the 64
// lanes lives in LDS and is updated by wave 0 between two barriers, so the
// other waves carry no optimiser state through the evaluation.
enum { ST_XA, ST_XB, ST_XG, ST_S, ST_GA, ST_GB, ST_GG, ST_ETA, ST_TA, ST_TB, ST_TG, ST_N };

template <int W>
__global__ __launch_bounds__(64 * W) BH_SCORE_OCCUPANCY void k_march(
    const int32_t* __restrict__ p_first, const int32_t* __restrict__ wave_p,
                                                  const double* __restrict__ rec,
                                                  const double* __restrict__ X, int64_t n_entries,
                                                  int L, const double* __restrict__ Wb, int P,
                                                  int steps, double step_init, double grow,
                                                  double shrink, double* __restrict__ state,
                                                  double* __restrict__ sscore) {
  __shared__ double red[W * 4 * 64];
  __shared__ double st[ST_N * 64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t pb = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const bool active = r < P;
  const double* Xp = X + pb * n_entries * 4;
  if (wave == 0) {
    double xa = 0.0, xb = 0.0, xg = 0.0;
    if (active) {
      const double* s0 = state + (pb * P + r) * 3;
      xa = s0[0];
      xb = s0[1];
      xg = s0[2];
    }
    wrap_euler(xa, xb, xg);
    const double wb = Wb[pb];
    st[ST_TA * 64 + lane] = xa;
    st[ST_TB * 64 + lane] = xb;
    st[ST_TG * 64 + lane] = xg;
    st[ST_ETA * 64 + lane] = (wb > 0.0) ? step_init / wb : 0.0;
  }
  __syncthreads();
  for (int t = 0; t <= steps; ++t) {
    const Angles A = prep(st[ST_TA * 64 + lane], st[ST_TB * 64 + lane], st[ST_TG * 64 + lane]);
    const Acc mine = eval_wave(A, wave_p + wave * (2 * L + 2), L, p_first, rec, Xp);
    red[(wave * 4 + 0) * 64 + lane] = mine.S;
    red[(wave * 4 + 1) * 64 + lane] = mine.ga;
    red[(wave * 4 + 2) * 64 + lane] = mine.gb;
    red[(wave * 4 + 3) * 64 + lane] = mine.gg;
    __syncthreads();
    if (wave == 0) {
      Acc tr = {0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < W; ++w) {
        tr.S += red[(w * 4 + 0) * 64 + lane];
        tr.ga += red[(w * 4 + 1) * 64 + lane];
        tr.gb += red[(w * 4 + 2) * 64 + lane];
        tr.gg += red[(w * 4 + 3) * 64 + lane];
      }
      double eta = st[ST_ETA * 64 + lane];
      // t == 0: the carried point itself; later: accept if not worse
      const bool take = (t == 0) || (tr.S >= st[ST_S * 64 + lane]);
      if (take) {
        st[ST_XA * 64 + lane] = st[ST_TA * 64 + lane];
        st[ST_XB * 64 + lane] = st[ST_TB * 64 + lane];
        st[ST_XG * 64 + lane] = st[ST_TG * 64 + lane];
        st[ST_S * 64 + lane] = tr.S;
        st[ST_GA * 64 + lane] = tr.ga;
        st[ST_GB * 64 + lane] = tr.gb;
        st[ST_GG * 64 + lane] = tr.gg;
      }
      if (t > 0) eta *= take ? grow : shrink;
      st[ST_ETA * 64 + lane] = eta;
      if (t < steps) {
        // natural-gradient step from the current point
        const double xa = st[ST_XA * 64 + lane], xb = st[ST_XB * 64 + lane],
                     xg = st[ST_XG * 64 + lane];
        const double ga = st[ST_GA * 64 + lane], gb = st[ST_GB * 64 + lane],
                     gg = st[ST_GG * 64 + lane];
        const double cb = cos(xb);
        double s2 = 1.0 - cb * cb;
        s2 = s2 > kSin2Floor ? s2 : kSin2Floor;
        double ta = xa + eta * ((ga - cb * gg) / s2);
        double tb = xb + eta * gb;
        double tg = xg + eta * ((gg - cb * ga) / s2);
        wrap_euler(ta, tb, tg);
        st[ST_TA * 64 + lane] = ta;
        st[ST_TB * 64 + lane] = tb;
        st[ST_TG * 64 + lane] = tg;
      }
    }
    __syncthreads();
  }
  if (wave == 0 && active) {
    double* so = state + (pb * P + r) * 3;
    so[0] = st[ST_XA * 64 + lane];
    so[1] = st[ST_XB * 64 + lane];
    so[2] = st[ST_XG * 64 + lane];
    sscore[pb * P + r] = st[ST_S * 64 + lane];
  }
}

// Best restart per particle (highest score, lowest index on ties).
__global__ __launch_bounds__(64) void k_select(const double* __restrict__ state,
                                               const double* __restrict__ sscore, int P,
                                               double* __restrict__ euler_out,
                                               double* __restrict__ score_out) {
  const int64_t pb = blockIdx.x;
  const int lane = threadIdx.x;
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int r = lane; r < P; r += 64) {
    const double v = sscore[pb * P + r];
    if (v > best) {           // r increases, so ties keep the lower index
      best = v;
      bi = r;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_down(best, off, 64);
    const int oi = __shfl_down(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    if (bi >= P) bi = 0;
    euler_out[pb * 3 + 0] = state[(pb * P + bi) * 3 + 0];
    euler_out[pb * 3 + 1] = state[(pb * P + bi) * 3 + 1];
    euler_out[pb * 3 + 2] = state[(pb * P + bi) * 3 + 2];
    score_out[pb] = sscore[pb * P + bi];
  }
}

int pick_waves(int64_t groups, int L, bool batch_invariant = false) {
  if (BH_SCORE_FIXED_W > 0) return BH_SCORE_FIXED_W;
  // Measured on MI355X (1000 particles x 64 restarts, bands 8..32): 12 waves
  // per workgroup at 6 waves per SIMD (two workgroups per CU) is fastest for
  // L > 8, 4 waves for L <= 8; small batches spread one particle over 16
  // waves unless the split must not depend on the batch.  More than 2L+1
  // waves would have no p-group to work on.
  int W = (L <= 8) ? 4 : 12;
  if (groups < 256 && !batch_invariant) W = 16;
  while (W > 2 * L + 1 && W > 4) W = (W == 16) ? 12 : (W == 12 ? 8 : (W == 8 ? 6 : W - 1));
  return W;
}

template <int W>
void launch_correlate_w(bh_plan* p, dim3 grid, hipStream_t s, const DevBand& band, const double* X,
                        int L, const double* euler, int R, double* score, double* grad) {
  ProfScope ps(p, "correlate_L" + std::to_string(L), s,
               (int64_t)grid.y * R * band.n_entries);
  hipLaunchKernelGGL(k_correlate<W>, grid, dim3(64 * W), 0, s, band.p_first,
                     band.wave_p + wave_block_offset(L, W), band.rec, X,
                     band.n_entries, L, euler, R, score, grad);
}

template <int W>
void launch_march_w(bh_plan* p, dim3 grid, hipStream_t s, const DevBand& band, const double* X,
                    int L, const double* Wb, int P, const bh_align_opts& o, double* state,
                    double* sscore) {
  ProfScope ps(p, "march_L" + std::to_string(L), s,
               (int64_t)grid.y * P * (o.steps_per_band + 1) * band.n_entries);
  hipLaunchKernelGGL(k_march<W>, grid, dim3(64 * W), 0, s, band.p_first,
                     band.wave_p + wave_block_offset(L, W), band.rec, X,
                     band.n_entries, L, Wb, P, o.steps_per_band, o.step_init, o.step_grow,
                     o.step_shrink, state, sscore);
}

int prepare_band(bh_plan* p, const DevBand& band, const float* a, const float* b,
                 const int32_t* tmpl, int n_tmpl, int64_t B, double** X, hipStream_t s) {
  // + kTablePad entries: the score loop reads up to three entries ahead
  int rc = grow(p->xi_scr, ((size_t)B * band.n_entries + kTablePad) * 4 * sizeof(double));
  if (rc != BH_OK) return rc;
  *X = (double*)p->xi_scr.ptr;
  ProfScope ps(p, "xi_classes", s, B);
  hipLaunchKernelGGL(k_xi_classes, dim3((unsigned)((band.n_entries + 127) / 128), (unsigned)B),
                     dim3(128), 0, s, a, b, p->C, tmpl, n_tmpl, band.n_entries, band.sel, band.wt,
                     band.deg_start, band.deg_off, *X);
  BH_HIP(hipGetLastError());
  return BH_OK;
}

}  // namespace

int launch_cross_power_dense(bh_plan* p, const DevBand& band, const float* a, const float* b,
                             int64_t B, double* xi, hipStream_t s) {
  const int L = band.L;
  const int64_t E = (int64_t)(L + 1) * (4LL * (L + 1) * (L + 1) - 1) / 3;
  ProfScope ps(p, "xi_dense", s, B);
  hipLaunchKernelGGL(k_xi_dense, dim3((unsigned)((E + 255) / 256), (unsigned)B), dim3(256), 0, s, a,
                     b, p->C, L, band.deg_start, band.deg_off, E, xi);
  BH_HIP(hipGetLastError());
  return BH_OK;
}

int launch_correlate(bh_plan* p, const DevBand& band, const float* a, const float* b, int64_t B,
                     const double* euler, int R, double* score, double* grad, hipStream_t s) {
  double* X = nullptr;
  int rc = prepare_band(p, band, a, b, nullptr, 1, B, &X, s);
  if (rc != BH_OK) return rc;
  const int64_t chunks = (R + 63) / 64;
  const dim3 grid((unsigned)chunks, (unsigned)B);
  const int W = pick_waves(chunks * B, band.L);
  switch (W) {
    case 16: launch_correlate_w<16>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
    case 12: launch_correlate_w<12>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
    case 10: launch_correlate_w<10>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
    case 8: launch_correlate_w<8>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
    case 6: launch_correlate_w<6>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
    case 5: launch_correlate_w<5>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
    default: launch_correlate_w<4>(p, grid, s, band, X, band.L, euler, R, score, grad); break;
  }
  BH_HIP(hipGetLastError());
  return BH_OK;
}

int launch_align(bh_plan* p, const float* a, const float* b, const int32_t* tmpl, int n_tmpl,
                 int64_t B, const bh_align_opts& o,
                 const double* starts, double* euler_out, double* score_out, double* all_euler,
                 double* all_score, hipStream_t s) {
  const int P = o.n_restarts;
  int rc;
  if ((rc = grow(p->state_scr, (size_t)B * P * 4 * sizeof(double))) != BH_OK) return rc;
  if ((rc = grow(p->misc_scr, (size_t)B * sizeof(double))) != BH_OK) return rc;
  double* state = (double*)p->state_scr.ptr;
  double* sscore = state + (size_t)B * P * 3;
  double* Wb = (double*)p->misc_scr.ptr;
  BH_HIP(hipMemcpyAsync(state, starts, (size_t)B * P * 3 * sizeof(double),
                        hipMemcpyDeviceToDevice, s));
  // bands are prepared first (host tables, uploads) so the loop only launches
  std::vector<const DevBand*> bands;
  for (int i = 0; i < o.n_bands; ++i) {
    const DevBand* band = nullptr;
    if ((rc = get_band(p, o.bands[i], &band)) != BH_OK) return rc;
    bands.push_back(band);
  }
  const int64_t chunks = (P + 63) / 64;
  const dim3 grid((unsigned)chunks, (unsigned)B);
  for (const DevBand* band : bands) {
    double* X = nullptr;
    if ((rc = prepare_band(p, *band, a, b, tmpl, n_tmpl, B, &X, s)) != BH_OK) return rc;
    {
      ProfScope ps(p, "band_weight", s, B);
      hipLaunchKernelGGL(k_band_weight, dim3((unsigned)B), dim3(64), 0, s, a, b, p->C, tmpl,
                         n_tmpl, band->L,
                         band->deg_start, band->deg_off, Wb);
    }
    BH_HIP(hipGetLastError());
    const int W = pick_waves(chunks * B, band->L, o.batch_invariant != 0);
    switch (W) {
      case 16: launch_march_w<16>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
      case 12: launch_march_w<12>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
      case 10: launch_march_w<10>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
      case 8: launch_march_w<8>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
      case 6: launch_march_w<6>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
      case 5: launch_march_w<5>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
      default: launch_march_w<4>(p, grid, s, *band, X, band->L, Wb, P, o, state, sscore); break;
    }
    BH_HIP(hipGetLastError());
  }
  {
  ProfScope ps(p, "select", s, B);
  hipLaunchKernelGGL(k_select, dim3((unsigned)B), dim3(64), 0, s, state, sscore, P, euler_out,
                     score_out);
  }
  BH_HIP(hipGetLastError());
  if (all_euler)
    BH_HIP(hipMemcpyAsync(all_euler, state, (size_t)B * P * 3 * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  if (all_score)
    BH_HIP(hipMemcpyAsync(all_score, sscore, (size_t)B * P * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  return BH_OK;
}

}  // namespace bh
