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
#include <map>
#include <mutex>
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
// The Hessian evaluators (four more chain sums, a longer epilogue) and the
// packed march (weights in vector registers) are given up to 128 registers
// (4 waves per SIMD) instead.
// Both together get up to 168 (3 waves per SIMD).
#define BH_HESS_OCCUPANCY(H) __attribute__((amdgpu_waves_per_eu((H) ? 4 : BH_SCORE_WAVES_PER_EU)))
#define BH_MARCH_OCCUPANCY(NEWTON, PACKED)                                              \
  __attribute__((amdgpu_waves_per_eu(((NEWTON) && (PACKED)) ? 3                          \
                                     : (((NEWTON) || (PACKED)) ? 4 : BH_SCORE_WAVES_PER_EU))))

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

// Template of particle pb (template 0 without a table), or -1 when tmpl[pb]
// lies outside [0, n_tmpl).  For such a particle the kernels read template 0
// in its place (no access outside the table), write NaN results and raise
// the plan's error word `bad` (a mapped host word; any writer stores 1).
__device__ inline int64_t template_of(const int32_t* __restrict__ tmpl, int n_tmpl, int64_t pb) {
  if (!tmpl) return 0;
  const int t = tmpl[pb];
  return (t < 0 || t >= n_tmpl) ? -1 : t;
}

__device__ inline void raise_bad(int* bad) {
  if (bad) *reinterpret_cast<volatile int*>(bad) = 1;
}

// Class-major weighted cross-power of one band: X[pb][e] = {X1re, X1im, X2re, X2im}.
__global__ void k_xi_classes(const float* __restrict__ a, int64_t lda,
                             const float* __restrict__ btab, int64_t ldt,
                             const int32_t* __restrict__ tmpl, int n_tmpl,
                             int64_t n_entries, const int32_t* __restrict__ sel,
                             const double* __restrict__ wt, const int32_t* __restrict__ deg_start,
                             const int32_t* __restrict__ deg_off, double* __restrict__ X,
                             int* bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pb = blockIdx.y;
  if (e >= n_entries) return;
  const int64_t ti = template_of(tmpl, n_tmpl, pb);
  if (ti < 0 && e == 0) raise_bad(bad);
  const int l = sel[4 * e], m = sel[4 * e + 1], n = sel[4 * e + 2];
  const double w1 = wt[2 * e], w2 = wt[2 * e + 1];
  const float2* ap = reinterpret_cast<const float2*>(a + pb * 2 * lda);
  const float2* b = reinterpret_cast<const float2*>(btab + (ti < 0 ? 0 : ti) * 2 * ldt);
  double x1r = 0, x1i = 0, x2r = 0, x2i = 0;
  for (int i = deg_start[l]; i < deg_start[l + 1]; ++i) {
    const int o = deg_off[i];
    const float2 bm = b[o + l + m], bn = b[o + l + n], am = ap[o + l + m], an = ap[o + l + n];
    const double bmr = bm.x, bmi = bm.y, bnr = bn.x, bni = bn.y;
    const double amr = am.x, ami = am.y, anr = an.x, ani = an.y;
    x1r += bmr * anr + bmi * ani;      // conj(b_m) a_n
    x1i += bmr * ani - bmi * anr;
    x2r += bnr * amr + bni * ami;      // conj(b_n) a_m
    x2i += bnr * ami - bni * amr;
  }
  double* out = X + (pb * n_entries + e) * 4;
  const double nan = __builtin_nan("");
  out[0] = ti < 0 ? nan : w1 * x1r;
  out[1] = ti < 0 ? nan : w1 * x1i;
  out[2] = ti < 0 ? nan : w2 * x2r;
  out[3] = ti < 0 ? nan : w2 * x2i;
}

// W_b = sum_l l(l+1) ||a_l|| ||b_l|| over the band; one block per particle.
__global__ void k_band_weight(const float* __restrict__ a, int64_t lda,
                              const float* __restrict__ btab, int64_t ldt,
                              const int32_t* __restrict__ tmpl, int n_tmpl,
                              int L, const int32_t* __restrict__ deg_start,
                              const int32_t* __restrict__ deg_off, double* __restrict__ Wb,
                              int* bad) {
  __shared__ double part[BH_MAX_L + 1];
  const int64_t pb = blockIdx.x;
  const int64_t ti = template_of(tmpl, n_tmpl, pb);
  const float* ap = a + pb * 2 * lda;
  const float* b = btab + (ti < 0 ? 0 : ti) * 2 * ldt;
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
    Wb[pb] = ti < 0 ? __builtin_nan("") : s;
    if (ti < 0) raise_bad(bad);
  }
}

// k_xi_classes and k_band_weight in one pass, one block per particle: the
// band's particle and template coefficients (the first C(L) of each, at most
// kXiLdsCoeffs) and the degree tables are staged in LDS, so an entry's sum
// reads only LDS after its table entry; a thread keeps two entries in flight
// and writes each entry's four weights as one 32-byte store.  Same sums in
// the same order as the two kernels above.
constexpr int64_t kSplitMinHalf = 256;   // particles per half of a split march
constexpr int kXiLdsCoeffs = 7680;   // (re, im) pairs of each operand (L <= 40)
constexpr int kXiLdsDeg = 512;       // (l, k) pairs staged (279 at L = 40)

// X1 = conj(b_m) a_n and X2 = conj(b_n) a_m summed over the entry's degree
// terms, the products in FP64 from the FP32 coefficients.
__device__ inline void xi_entry(const float2* sa, const float2* sb, const int32_t* sdeg_start,
                                const int32_t* sdeg_off, int l, int m, int n, double& x1r,
                                double& x1i, double& x2r, double& x2i) {
  x1r = 0.0;
  x1i = 0.0;
  x2r = 0.0;
  x2i = 0.0;
  for (int i = sdeg_start[l]; i < sdeg_start[l + 1]; ++i) {
    const int o = sdeg_off[i];
    const float2 bm = sb[o + l + m], bn = sb[o + l + n], am = sa[o + l + m], an = sa[o + l + n];
    const double bmr = bm.x, bmi = bm.y, bnr = bn.x, bni = bn.y;
    const double amr = am.x, ami = am.y, anr = an.x, ani = an.y;
    x1r += bmr * anr + bmi * ani;      // conj(b_m) a_n
    x1i += bmr * ani - bmi * anr;
    x2r += bnr * amr + bni * ami;      // conj(b_n) a_m
    x2i += bnr * ami - bni * amr;
  }
}

__global__ __launch_bounds__(512) void k_xi_band(
    const float* __restrict__ a, int64_t lda, const float* __restrict__ btab, int64_t ldt,
    const int32_t* __restrict__ tmpl, int n_tmpl, int64_t n_entries,
    const int32_t* __restrict__ sel, const double* __restrict__ wt,
    const int32_t* __restrict__ deg_start, const int32_t* __restrict__ deg_off, int n_deg, int L,
    int CL, double* __restrict__ X, double* __restrict__ Wb, int* bad) {
  extern __shared__ float2 sa[];   // [2 CL]: the particle's coefficients, then the template's
  __shared__ double part[BH_MAX_L + 1];
  __shared__ int32_t sdeg_start[BH_MAX_L + 2];
  __shared__ int32_t sdeg_off[kXiLdsDeg];
  float2* sb = sa + CL;
  const int tid = threadIdx.x;
  const int64_t pb = blockIdx.x;
  const int64_t ti = template_of(tmpl, n_tmpl, pb);
  const double nan = __builtin_nan("");
  const float2* ap = reinterpret_cast<const float2*>(a + pb * 2 * lda);
  const float2* b = reinterpret_cast<const float2*>(btab + (ti < 0 ? 0 : ti) * 2 * ldt);
  for (int i = tid; i < CL; i += blockDim.x) {
    sa[i] = ap[i];
    sb[i] = b[i];
  }
  for (int i = tid; i <= L + 1; i += blockDim.x) sdeg_start[i] = deg_start[i];
  for (int i = tid; i < n_deg; i += blockDim.x) sdeg_off[i] = deg_off[i];
  __syncthreads();
  double4* Xp = reinterpret_cast<double4*>(X + pb * n_entries * 4);
  const int stride = blockDim.x;
  for (int64_t e0 = tid; e0 < n_entries; e0 += 2 * stride) {
    const int64_t e1 = e0 + stride;
    const bool has1 = e1 < n_entries;
    const int4 s0 = reinterpret_cast<const int4*>(sel)[e0];
    const int4 s1 = has1 ? reinterpret_cast<const int4*>(sel)[e1] : s0;
    const double2 w0 = reinterpret_cast<const double2*>(wt)[e0];
    const double2 w1 = has1 ? reinterpret_cast<const double2*>(wt)[e1] : w0;
    // a chain's padding entries (zero weights) are never read: not written
    const bool live0 = w0.x != 0.0 || w0.y != 0.0;
    const bool live1 = has1 && (w1.x != 0.0 || w1.y != 0.0);
    double a0r, a0i, c0r, c0i, a1r, a1i, c1r, c1i;
    xi_entry(sa, sb, sdeg_start, sdeg_off, s0.x, s0.y, s0.z, a0r, a0i, c0r, c0i);
    xi_entry(sa, sb, sdeg_start, sdeg_off, s1.x, s1.y, s1.z, a1r, a1i, c1r, c1i);
    if (live0)
      Xp[e0] = ti < 0 ? double4{nan, nan, nan, nan}
                      : double4{w0.x * a0r, w0.x * a0i, w0.y * c0r, w0.y * c0i};
    if (live1)
      Xp[e1] = ti < 0 ? double4{nan, nan, nan, nan}
                      : double4{w1.x * a1r, w1.x * a1i, w1.y * c1r, w1.y * c1i};
  }
  for (int l = tid; l <= L; l += blockDim.x) {
    double na = 0.0, nb = 0.0;
    for (int i = sdeg_start[l]; i < sdeg_start[l + 1]; ++i) {
      const int o = sdeg_off[i];
      for (int m = -l; m <= l; ++m) {
        const float2 av = sa[o + l + m], bv = sb[o + l + m];
        const double ar = av.x, ai = av.y, br = bv.x, bi = bv.y;
        na += ar * ar + ai * ai;
        nb += br * br + bi * bi;
      }
    }
    part[l] = (double)l * (l + 1) * sqrt(na) * sqrt(nb);
  }
  __syncthreads();
  if (tid == 0) {
    double w = 0.0;
    for (int l = 0; l <= L; ++l) w += part[l];
    Wb[pb] = ti < 0 ? nan : w;
    if (ti < 0) raise_bad(bad);
  }
}

// Sum the W wave partials (fixed order) through LDS buffer `buf`
// ([W][NV][64]); NV = 4 (score, gradient) or 10 (and the Hessian).
template <int NV>
__device__ inline void store_partials(const Acc& mine, double* buf, int wave, int lane) {
  const double v[10] = {mine.S, mine.ga, mine.gb, mine.gg, mine.haa,
                        mine.hab, mine.hag, mine.hbb, mine.hbg, mine.hgg};
#pragma unroll
  for (int k = 0; k < NV; ++k) buf[(wave * NV + k) * 64 + lane] = v[k];
}

template <int NV>
__device__ inline Acc sum_partials(const double* buf, int lane, int W) {
  double v[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int w = 0; w < W; ++w) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += buf[(w * NV + k) * 64 + lane];
  }
  return Acc{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9]};
}

// This lane's index in its wave, computed where it is called from the lane
// masks (v_mbcnt): the compiler cannot hoist it, so values derived from it
// are not held through loops (and spilled) either.
__device__ inline int lane_index() {
  int v;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
  return v;
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

// Score, gradient and (HESS) Hessian at R rotations per particle; hess
// holds (aa, ab, ag, bb, bg, gg) per rotation.
template <int W, bool HESS>
__global__ __launch_bounds__(64 * W) BH_HESS_OCCUPANCY(HESS) void k_correlate(
    const int32_t* __restrict__ p_first, const int32_t* __restrict__ wave_p,
    const double* __restrict__ rec, const double* __restrict__ X, int64_t n_entries, int L,
    const double* __restrict__ euler, int R, double* __restrict__ score,
    double* __restrict__ grad, double* __restrict__ hess) {
  constexpr int NV = HESS ? 10 : 4;
  __shared__ double buf[W * NV * 64];
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
  const Acc mine =
      eval_wave<HESS>(A, wave_p + wave * (2 * L + 2), L, p_first, rec, X + pb * n_entries * 4);
  store_partials<NV>(mine, buf, wave, lane);
  __syncthreads();
  if (wave == 0 && active) {
    const Acc t = sum_partials<NV>(buf, lane, W);
    score[pb * R + r] = t.S;
    if (grad) {
      grad[(pb * R + r) * 3 + 0] = t.ga;
      grad[(pb * R + r) * 3 + 1] = t.gb;
      grad[(pb * R + r) * 3 + 2] = t.gg;
    }
    if constexpr (HESS) {
      double* h = hess + (pb * R + r) * 6;
      h[0] = t.haa;
      h[1] = t.hab;
      h[2] = t.hag;
      h[3] = t.hbb;
      h[4] = t.hbg;
      h[5] = t.hgg;
    }
  }
}

// Natural-gradient direction g^{-1} grad S in ZYZ Euler coordinates, with
// sin^2(beta) floored (the metric is singular at the poles).
__device__ inline void natural_gradient(double xb, double ga, double gb, double gg, double& da,
                                        double& db, double& dg) {
  const double cb = cos(xb);
  double s2 = 1.0 - cb * cb;
  s2 = s2 > kSin2Floor ? s2 : kSin2Floor;
  da = (ga - cb * gg) / s2;
  db = gb;
  dg = (gg - cb * ga) / s2;
}

// Step of a Newton band: (-H)^{-1} grad S where -H is positive definite
// (leading principal minors positive; solved with the adjugate), else
// eta0 times the natural gradient; scaled to a largest component of at most
// kNewtonMaxStep radians.  h = (aa, ab, ag, bb, bg, gg).
constexpr double kNewtonMaxStep = 0.5;

__device__ inline void newton_direction(double xb, double ga, double gb, double gg,
                                        const double* h, double eta0, double& da, double& db,
                                        double& dg) {
  const double n11 = -h[0], n12 = -h[1], n13 = -h[2], n22 = -h[3], n23 = -h[4], n33 = -h[5];
  const double m2 = n11 * n22 - n12 * n12;
  const double c11 = n22 * n33 - n23 * n23;
  const double c12 = n13 * n23 - n12 * n33;
  const double c13 = n12 * n23 - n13 * n22;
  const double det = n11 * c11 + n12 * c12 + n13 * c13;
  if (n11 > 0.0 && m2 > 0.0 && det > 0.0) {
    const double c22 = n11 * n33 - n13 * n13;
    const double c23 = n12 * n13 - n11 * n23;
    const double c33 = m2;
    da = (c11 * ga + c12 * gb + c13 * gg) / det;
    db = (c12 * ga + c22 * gb + c23 * gg) / det;
    dg = (c13 * ga + c23 * gb + c33 * gg) / det;
  } else {
    natural_gradient(xb, ga, gb, gg, da, db, dg);
    da *= eta0;
    db *= eta0;
    dg *= eta0;
  }
  const double big = fmax(fabs(da), fmax(fabs(db), fabs(dg)));
  if (big > kNewtonMaxStep) {
    const double f = kNewtonMaxStep / big;
    da *= f;
    db *= f;
    dg *= f;
  }
}

// One band of the ascent for 64 restarts of one particle (see bh.h).
//
// Every evaluation is split over the W waves; the ascent state of the 64
// lanes lives in LDS and is updated by wave 0 between two barriers, so the
// other waves carry no optimiser state through the evaluation.  Wave 0 also
// prepares the trial rotation's half-angle and phase factors once for all
// waves (LDS `ang`).  NEWTON:
// Newton steps from the Hessian (ST_ETA holds the damping mu <= 1).
enum {
  ST_XA, ST_XB, ST_XG, ST_S, ST_GA, ST_GB, ST_GG, ST_ETA, ST_TA, ST_TB, ST_TG,
  ST_HAA, ST_HAB, ST_HAG, ST_HBB, ST_HBG, ST_HGG, ST_ETA0, ST_N
};

//
// G < 64 packs 64 / G particles into a workgroup, G lanes (restarts) each
// (P <= G): the restarts that survive candidate pruning fill the waves.
// The weights X then differ between lane groups and are read with vector
// loads; the recurrence tables stay wave-uniform.
template <int W, bool NEWTON, int G>
__global__ __launch_bounds__(64 * W) BH_MARCH_OCCUPANCY(NEWTON, G < 64) void k_march(
    const int32_t* __restrict__ p_first, const int32_t* __restrict__ wave_p,
    const double* __restrict__ rec, const double* __restrict__ X, int64_t n_entries, int L,
    const double* __restrict__ Wb, int64_t B, int P, int steps, double step_init, double grow,
    double shrink, double* __restrict__ state, double* __restrict__ sscore) {
  constexpr int NV = NEWTON ? 10 : 4;
  constexpr int NS = NEWTON ? ST_N : ST_HAA;
  __shared__ double red[W * NV * 64];
  __shared__ double st[NS * 64];
  __shared__ double ang[kAngleWords * 64];   // the trial rotation's Angles, set by wave 0
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Particles are taken in a grid-stride loop over blockIdx.y: one pass when
  // the grid covers the batch, persistent workgroups when it is smaller.
  constexpr int64_t PER = (G == 64) ? 1 : 64 / G;
  for (int64_t base = blockIdx.y; base * PER < B; base += gridDim.y) {
    // The index arithmetic of the per-particle state I/O derives from an
    // opaque copy of the lane index (recomputed from the lane masks, not
    // kept from the kernel's start), so the compiler keeps it inside the
    // particle loop: hoisted out of it, it would be held in scratch memory
    // (written by each of the launch's waves).
    const int lane_o = lane_index();
    int64_t pb;
    int r;                            // restart (P <= 65536)
    if constexpr (G == 64) {
      pb = base;
      r = (int)blockIdx.x * 64 + lane_o;
    } else {
      pb = base * PER + lane_o / G;
      r = lane_o % G;
    }
    const bool active = pb < B && r < P;
    if (pb >= B) pb = B - 1;          // idle lanes read a valid particle
    const double* Xp = X + pb * n_entries * 4;
    const double wb = Wb[pb];
    const double eta0 = (wb > 0.0) ? step_init / wb : 0.0;
    if (wave == 0) {
      double xa = 0.0, xb = 0.0, xg = 0.0;
      if (active) {
        const double* s0 = state + (pb * P + r) * 3;
        xa = s0[0];
        xb = s0[1];
        xg = s0[2];
      }
      wrap_euler(xa, xb, xg);
      st[ST_TA * 64 + lane] = xa;
      st[ST_TB * 64 + lane] = xb;
      st[ST_TG * 64 + lane] = xg;
      st[ST_ETA * 64 + lane] = NEWTON ? 1.0 : eta0;
      store_angles(prep(xa, xb, xg), ang + lane, 64);
    }
    __syncthreads();
    for (int t = 0; t <= steps; ++t) {
      const Angles A = load_angles(ang + lane, 64);
      Acc mine =
          eval_wave<NEWTON, G == 64, NEWTON>(A, wave_p + wave * (2 * L + 2), L, p_first, rec, Xp);
      if constexpr (!NEWTON) mine.gb *= ang[kAngleMsb * 64 + lane];   // -sin(beta), trial point
      store_partials<NV>(mine, red, wave, lane);
      __syncthreads();
      if (wave == 0) {
        const Acc tr = sum_partials<NV>(red, lane, W);
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
          if constexpr (NEWTON) {
            st[ST_HAA * 64 + lane] = tr.haa;
            st[ST_HAB * 64 + lane] = tr.hab;
            st[ST_HAG * 64 + lane] = tr.hag;
            st[ST_HBB * 64 + lane] = tr.hbb;
            st[ST_HBG * 64 + lane] = tr.hbg;
            st[ST_HGG * 64 + lane] = tr.hgg;
          }
        }
        if (t > 0) {
          if (NEWTON)
            eta = take ? fmin(1.0, eta * grow) : eta * shrink;
          else
            eta *= take ? grow : shrink;
        }
        st[ST_ETA * 64 + lane] = eta;
        if (t < steps) {
          const double xa = st[ST_XA * 64 + lane], xb = st[ST_XB * 64 + lane],
                       xg = st[ST_XG * 64 + lane];
          const double ga = st[ST_GA * 64 + lane], gb = st[ST_GB * 64 + lane],
                       gg = st[ST_GG * 64 + lane];
          double da, db, dg;
          if constexpr (NEWTON) {
            const double h[6] = {st[ST_HAA * 64 + lane], st[ST_HAB * 64 + lane],
                                 st[ST_HAG * 64 + lane], st[ST_HBB * 64 + lane],
                                 st[ST_HBG * 64 + lane], st[ST_HGG * 64 + lane]};
            newton_direction(xb, ga, gb, gg, h, eta0, da, db, dg);
          } else {
            natural_gradient(xb, ga, gb, gg, da, db, dg);
          }
          double ta = xa + eta * da;
          double tb = xb + eta * db;
          double tg = xg + eta * dg;
          wrap_euler(ta, tb, tg);
          st[ST_TA * 64 + lane] = ta;
          st[ST_TB * 64 + lane] = tb;
          st[ST_TG * 64 + lane] = tg;
          store_angles(prep(ta, tb, tg), ang + lane, 64);
        }
      }
      __syncthreads();
    }
    if (wave == 0) {
      // indices re-derived from a fresh opaque lane copy (see above)
      const int lane_e = lane_index();
      if constexpr (G == 64) {
        // the wave's end points [64][3] leave as three contiguous 512-byte
        // runs read across the LDS state (whole cache lines, not three
        // strided 8-byte stores per lane)
        const int r0 = (int)blockIdx.x * 64;
        const int n = 3 * min(64, P - r0);
        double* so = state + (base * P + r0) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int idx = k * 64 + lane_e;
          if (idx < n) so[idx] = st[(ST_XA + idx % 3) * 64 + idx / 3];
        }
        if (r0 + lane_e < P) sscore[base * P + r0 + lane_e] = st[ST_S * 64 + lane_e];
      } else {
        const int64_t pe = base * PER + lane_e / G;
        const int re = lane_e % G;
        if (pe < B && re < P) {
          double* so = state + (pe * P + re) * 3;
          so[0] = st[ST_XA * 64 + lane_e];
          so[1] = st[ST_XB * 64 + lane_e];
          so[2] = st[ST_XG * 64 + lane_e];
          sscore[pe * P + re] = st[ST_S * 64 + lane_e];
        }
      }
    }
    __syncthreads();   // the next particle's set-up overwrites the ascent state
  }
}

// Newton bands of packed restarts (at most 32 per particle), one launch per
// evaluation: the classes of each group of 64 / G particles are split over
// kNewtonParts workgroups of kNewtonWaves waves (the work split of
// kNewtonParts * kNewtonWaves waves), so a group occupies several CUs; a
// step kernel adds the parts in a fixed order and makes the Newton update.
// The per-lane rule is the ascent kernel's (NEWTON).
constexpr int kNewtonParts = 4, kNewtonWaves = 4;
static_assert(kNewtonParts * kNewtonWaves == 16, "the work split of 16 waves is used");

// trial[b][r] = the wrapped carried rotation (the first evaluation point).
template <int G>
__global__ __launch_bounds__(64) void k_newton_init(const double* __restrict__ state, int64_t B,
                                                    int P, double* __restrict__ trial) {
  constexpr int PER = 64 / G;
  const int lane = threadIdx.x;
  const int64_t pb = (int64_t)blockIdx.x * PER + lane / G;
  const int r = lane % G;
  if (pb >= B || r >= P) return;
  const int64_t i = pb * P + r;
  double a = state[i * 3], b = state[i * 3 + 1], g = state[i * 3 + 2];
  wrap_euler(a, b, g);
  trial[i * 3] = a;
  trial[i * 3 + 1] = b;
  trial[i * 3 + 2] = g;
}

// part[group][sp][k][lane]: score, gradient and Hessian sums of part sp of
// the classes at the trial rotations, the weights staged through an LDS
// ring per wave (XRing).  Two waves per SIMD leave the Hessian evaluator
// its ~190 registers (at three it spilled 72 bytes per lane and ran 4 %
// longer).
template <int G>
__global__ __launch_bounds__(64 * kNewtonWaves) __attribute__((amdgpu_waves_per_eu(2))) void k_newton_part(
    const int32_t* __restrict__ p_first, const int32_t* __restrict__ wave_p,
    const double* __restrict__ rec, const double* __restrict__ X, int64_t n_entries, int L,
    int64_t B, int P, const double* __restrict__ trial, double* __restrict__ part) {
  constexpr int W = kNewtonWaves, NV = 10, PER = 64 / G;
  __shared__ double red[W * NV * 64];
  __shared__ __attribute__((aligned(1024))) char xring[W][XRing<G>::kBlocks * XRing<G>::kBlockBytes];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sp = blockIdx.x;
  const int64_t grp = blockIdx.y;
  int64_t pb = grp * PER + lane / G;
  const int r = lane % G;
  const bool active = pb < B && r < P;
  if (pb >= B) pb = B - 1;          // idle lanes read a valid particle
  double al = 0.0, be = 0.0, ga = 0.0;
  if (active) {
    const double* t = trial + (pb * P + r) * 3;
    al = t[0];
    be = t[1];
    ga = t[2];
  }
  const Angles A = prep(al, be, ga);
  const int32_t* plist = wave_p + (sp * W + wave) * (2 * L + 2);
  XRing<G> xr;
  xr.start(xring[wave], X, n_entries, grp * PER, B, plist, p_first, L);
  const Acc mine = eval_wave_staged<G>(A, plist, L, p_first, rec, xr);
  store_partials<NV>(mine, red, wave, lane);
  __syncthreads();
  if (wave == 0) {
    const Acc t = sum_partials<NV>(red, lane, W);
    const double v[NV] = {t.S, t.ga, t.gb, t.gg, t.haa, t.hab, t.hag, t.hbb, t.hbg, t.hgg};
    double* o = part + (grp * kNewtonParts + sp) * NV * 64 + lane;
#pragma unroll
    for (int k = 0; k < NV; ++k) o[k * 64] = v[k];
  }
}

// Evaluation t of a Newton band (t = 0: the carried point): accept the trial
// point if not worse (t = 0: always), adapt the damping mu <= 1, and (t <
// steps) place the next trial point.  nst[b][r] = (gradient, Hessian, mu).
template <int G>
__global__ __launch_bounds__(64) void k_newton_step(
    const double* __restrict__ part, const double* __restrict__ Wb, int64_t B, int P, int t,
    int steps, double step_init, double grow, double shrink, double* __restrict__ state,
    double* __restrict__ sscore, double* __restrict__ trial, double* __restrict__ nst) {
  constexpr int NV = 10, PER = 64 / G;
  const int lane = threadIdx.x;
  const int64_t grp = blockIdx.x;
  const int64_t pb = grp * PER + lane / G;
  const int r = lane % G;
  if (pb >= B || r >= P) return;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double acc = 0.0;
    for (int sp = 0; sp < kNewtonParts; ++sp)
      acc += part[((grp * kNewtonParts + sp) * NV + k) * 64 + lane];
    v[k] = acc;
  }
  const int64_t i = pb * P + r;
  double* x = state + i * 3;
  double* tr = trial + i * 3;
  double* ns = nst + i * 10;
  double eta = (t == 0) ? 1.0 : ns[9];
  const bool take = (t == 0) || (v[0] >= sscore[i]);
  if (take) {
    x[0] = tr[0];
    x[1] = tr[1];
    x[2] = tr[2];
    sscore[i] = v[0];
#pragma unroll
    for (int k = 0; k < 9; ++k) ns[k] = v[k + 1];
  }
  if (t > 0) eta = take ? fmin(1.0, eta * grow) : eta * shrink;
  ns[9] = eta;
  if (t < steps) {
    const double wb = Wb[pb];
    const double eta0 = (wb > 0.0) ? step_init / wb : 0.0;
    double da, db, dg;
    newton_direction(x[1], ns[0], ns[1], ns[2], ns + 3, eta0, da, db, dg);
    double ta = x[0] + eta * da;
    double tb = x[1] + eta * db;
    double tg = x[2] + eta * dg;
    wrap_euler(ta, tb, tg);
    tr[0] = ta;
    tr[1] = tb;
    tr[2] = tg;
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

// Rotation matrix R_z(a) R_y(b) R_z(g), row-major.
__device__ inline void euler_matrix(double a, double b, double g, double* R) {
  double sa, ca, sb, cb, sg, cg;
  sincos(a, &sa, &ca);
  sincos(b, &sb, &cb);
  sincos(g, &sg, &cg);
  R[0] = ca * cb * cg - sa * sg;
  R[1] = -ca * cb * sg - sa * cg;
  R[2] = ca * sb;
  R[3] = sa * cb * cg + ca * sg;
  R[4] = -sa * cb * sg + ca * cg;
  R[5] = sa * sb;
  R[6] = -sb * cg;
  R[7] = sb * sg;
  R[8] = cb;
}

// Candidates after the first band: visit the restarts by decreasing score
// (lower index first on ties) and take one if 3 - tr(Rc^T Rj) > thr for
// every taken j (thr = 4 sin^2(min_sep / 2): farther than min_sep), until K
// are taken; fill any remaining slots with the skipped restarts in the same
// order.  One wave per particle; lane j holds the matrix of the j-th taken
// restart (K <= 64).
__global__ __launch_bounds__(64) void k_prune(const double* __restrict__ state,
                                              const double* __restrict__ sscore, int P, int K,
                                              double thr, double* __restrict__ out_state,
                                              double* __restrict__ out_score) {
  __shared__ int order[kPruneMaxP];
  __shared__ int chosen[64];
  __shared__ unsigned char taken[kPruneMaxP];
  const int64_t pb = blockIdx.x;
  const int lane = threadIdx.x;
  const double* S = sscore + pb * P;
  const double* x = state + pb * P * 3;
  // a NaN score ranks as -infinity, so the ranks are a permutation
  for (int i = lane; i < P; i += 64) {
    const double si = isnan(S[i]) ? -INFINITY : S[i];
    int rank = 0;
    for (int j = 0; j < P; ++j) {
      const double sj = isnan(S[j]) ? -INFINITY : S[j];
      rank += (sj > si || (sj == si && j < i)) ? 1 : 0;
    }
    order[rank] = i;
    taken[i] = 0;
  }
  __syncthreads();
  double Rm[9];                 // this lane's taken restart (lane < n)
  int n = 0;
  for (int s = 0; s < P && n < K; ++s) {
    const int c = order[s];
    double Rc[9];
    euler_matrix(x[c * 3], x[c * 3 + 1], x[c * 3 + 2], Rc);
    bool close = false;
    if (lane < n) {
      double tr = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) tr += Rc[k] * Rm[k];
      close = !(3.0 - tr > thr);
    }
    if (!__any(close)) {
      if (lane == n) {
#pragma unroll
        for (int k = 0; k < 9; ++k) Rm[k] = Rc[k];
        chosen[n] = c;
        taken[c] = 1;
      }
      ++n;
    }
    __syncthreads();
  }
  for (int s = 0; s < P && n < K; ++s) {
    const int c = order[s];
    if (!taken[c]) {
      if (lane == 0) chosen[n] = c;
      ++n;
    }
  }
  __syncthreads();
  for (int k = lane; k < K; k += 64) {
    const int c = chosen[k];
    out_state[(pb * K + k) * 3 + 0] = x[c * 3 + 0];
    out_state[(pb * K + k) * 3 + 1] = x[c * 3 + 1];
    out_state[(pb * K + k) * 3 + 2] = x[c * 3 + 2];
    out_score[pb * K + k] = S[c];
  }
}

// ||xi^l||_F^2 of the band-L cross-power for l = 0..L; one block per particle.
__global__ __launch_bounds__(256) void k_degree_energy(
    const float* __restrict__ a, const float* __restrict__ btab, int64_t C,
    const int32_t* __restrict__ tmpl, int n_tmpl, int L, const int32_t* __restrict__ deg_start,
    const int32_t* __restrict__ deg_off, double* __restrict__ energy, int* bad) {
  __shared__ double part[256];
  const int64_t pb = blockIdx.x;
  const int64_t ti = template_of(tmpl, n_tmpl, pb);
  if (ti < 0 && threadIdx.x == 0) raise_bad(bad);
  const float* ap = a + pb * 2 * C;
  const float* b = btab + (ti < 0 ? 0 : ti) * 2 * C;
  for (int l = 0; l <= L; ++l) {
    const int w = 2 * l + 1;
    double acc = 0.0;
    for (int t = threadIdx.x; t < w * w; t += 256) {
      const int m = t / w - l, n = t % w - l;
      double sre = 0.0, sim = 0.0;
      for (int i = deg_start[l]; i < deg_start[l + 1]; ++i) {
        const int o = deg_off[i];
        const double br = b[2 * (o + l + m)], bi = b[2 * (o + l + m) + 1];
        const double ar = ap[2 * (o + l + n)], ai = ap[2 * (o + l + n) + 1];
        sre += br * ar + bi * ai;
        sim += br * ai - bi * ar;
      }
      acc += sre * sre + sim * sim;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) energy[pb * (L + 1) + l] = ti < 0 ? __builtin_nan("") : part[0];
    __syncthreads();
  }
}

// Energy ratio of each particle's band-L cross-power and, per threshold,
// the smallest L' with Ratio(L') <= tau (one thread per particle):
// Ratio(L') = sum_{l > L'} E_l / sum_l E_l, the tails summed from the top
// degree down (no cancellation for small tails); 0 when every E_l is 0.  A
// NaN energy (template index outside the table) gives NaN ratios and the
// band L for every threshold.
__global__ void k_select_bands(const double* __restrict__ energy, int64_t B, int L,
                               BandThresholds th, int n_tau, int32_t* __restrict__ bands,
                               double* __restrict__ ratio) {
  const int64_t pb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pb >= B) return;
  const double* E = energy + pb * (L + 1);
  double tot = 0.0;
  for (int l = L; l >= 0; --l) tot += E[l];
  int32_t pick[kMaxBandThresholds];
  for (int j = 0; j < n_tau; ++j) pick[j] = L;
  // walk L' downwards: the last L' that satisfies a threshold is the smallest
  double tail = 0.0;
  for (int Lq = L; Lq >= 0; --Lq) {
    const double r = tot == 0.0 ? 0.0 : tail / tot;
    if (ratio) ratio[pb * (L + 1) + Lq] = r;
    for (int j = 0; j < n_tau; ++j)
      if (r <= th.t[j]) pick[j] = Lq;
    tail += E[Lq];
  }
  for (int j = 0; j < n_tau; ++j) bands[pb * n_tau + j] = pick[j];
}

// Batch choice per threshold j: the smallest L' whose per-particle choices
// are <= L' for at least ceil(B/2) particles (the lower median of the
// choices; the same as the smallest L' whose ratio is <= tau for at least
// half the particles, Ratio being non-increasing in L').  One block per
// threshold, an integer histogram in LDS.
__global__ __launch_bounds__(256) void k_common_bands(const int32_t* __restrict__ bands,
                                                      int64_t B, int L, int n_tau,
                                                      int32_t* __restrict__ common) {
  __shared__ int64_t hist[BH_MAX_L + 1];
  const int j = blockIdx.x;
  for (int l = threadIdx.x; l <= L; l += blockDim.x) hist[l] = 0;
  __syncthreads();
  for (int64_t b = threadIdx.x; b < B; b += blockDim.x) {
    const int v = bands[b * n_tau + j];
    atomicAdd(reinterpret_cast<unsigned long long*>(&hist[v < 0 ? 0 : (v > L ? L : v)]), 1ull);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t need = (B + 1) / 2;
    int64_t cum = 0;
    int pick = L;
    for (int l = 0; l <= L; ++l) {
      cum += hist[l];
      if (cum >= need) {
        pick = l;
        break;
      }
    }
    common[j] = pick;
  }
}

// starts of particle b for each of its S shifted copies: out[b*S + s] = in[b].
__global__ void k_repeat_starts(const double* __restrict__ in, int64_t B, int S, int P,
                                double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)P * 3;
  if (t >= B * S * per) return;
  const int64_t row = t / per, k = t % per;
  out[t] = in[(row / S) * per + k];
}

// Best shift per particle: highest score over its S rows (lowest shift
// index on ties).
__global__ void k_select_shift(const double* __restrict__ eu, const double* __restrict__ sc,
                               int64_t B, int S, double* __restrict__ euler_out,
                               double* __restrict__ score_out, int32_t* __restrict__ shift_out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  int best = 0;
  double bs = sc[b * S];
  for (int s = 1; s < S; ++s) {
    const double v = sc[b * S + s];
    if (v > bs || (isnan(bs) && !isnan(v))) {
      bs = v;
      best = s;
    }
  }
  euler_out[b * 3 + 0] = eu[(b * S + best) * 3 + 0];
  euler_out[b * 3 + 1] = eu[(b * S + best) * 3 + 1];
  euler_out[b * 3 + 2] = eu[(b * S + best) * 3 + 2];
  score_out[b] = bs;
  shift_out[b] = best;
}

int pick_waves(const bh_plan* p, int64_t groups, int L, bool batch_invariant = false) {
  if (BH_SCORE_FIXED_W > 0) return BH_SCORE_FIXED_W;
  if (p->tuned_waves[L] > 0) return p->tuned_waves[L];
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

template <int W, bool HESS>
void launch_correlate_w(bh_plan* p, dim3 grid, hipStream_t s, const DevBand& band, const double* X,
                        int L, const double* euler, int R, double* score, double* grad,
                        double* hess) {
  ProfScope ps(p, (HESS ? "correlate_hess_L" : "correlate_L") + std::to_string(L), s,
               (int64_t)grid.y * R * band.n_entries);
  hipLaunchKernelGGL((k_correlate<W, HESS>), grid, dim3(64 * W), 0, s, band.p_first,
                     band.wave_p + wave_block_offset(L, W), band.rec, X, band.n_entries, L, euler,
                     R, score, grad, hess);
}

template <bool HESS>
void launch_correlate_any(int W, bh_plan* p, dim3 grid, hipStream_t s, const DevBand& band,
                          const double* X, const double* euler, int R, double* score,
                          double* grad, double* hess) {
  const int L = band.L;
  switch (W) {
    case 16: launch_correlate_w<16, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
    case 12: launch_correlate_w<12, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
    case 10: launch_correlate_w<10, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
    case 8: launch_correlate_w<8, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
    case 6: launch_correlate_w<6, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
    case 5: launch_correlate_w<5, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
    default: launch_correlate_w<4, HESS>(p, grid, s, band, X, L, euler, R, score, grad, hess); break;
  }
}

template <int W, bool NEWTON, int G>
void launch_march_w(bh_plan* p, int64_t B, hipStream_t s, const DevBand& band, const double* X,
                    const double* Wb, int P, int steps, const bh_align_opts& o, double* state,
                    double* sscore) {
  const int L = band.L;
  int64_t ny = (G == 64) ? B : (B + 64 / G - 1) / (64 / G);
  const int64_t nx = (G == 64) ? (P + 63) / 64 : 1;
  if (p->tuned_persist[L]) {   // persistent: only as many workgroups as are resident
    const int64_t cap = resident_workgroups(k_march<W, NEWTON, G>, 64 * W) / nx;
    if (cap > 0 && cap < ny) ny = cap;
  }
  const dim3 grid((unsigned)nx, (unsigned)ny);
  ProfScope ps(p, (NEWTON ? "newton_L" : "march_L") + std::to_string(L), s,
               B * P * (int64_t)(steps + 1) * band.n_entries);
  hipLaunchKernelGGL((k_march<W, NEWTON, G>), grid, dim3(64 * W), 0, s, band.p_first,
                     band.wave_p + wave_block_offset(L, W), band.rec, X, band.n_entries, L, Wb, B,
                     P, steps, o.step_init, o.step_grow, o.step_shrink, state, sscore);
}

// G: lanes per particle (64, or 32 / 16 / 8 when P <= G, packed).
template <bool NEWTON>
void launch_march_any(int W, int G, bh_plan* p, int64_t B, hipStream_t s, const DevBand& band,
                      const double* X, const double* Wb, int P, int steps,
                      const bh_align_opts& o, double* state, double* sscore) {
  if (G < 64) {
    // packed launches use 12 waves (4 for bands up to 8)
    const bool small = W <= 6;
#define BH_PACKED(GG)                                                                         \
  if (small)                                                                                  \
    launch_march_w<4, NEWTON, GG>(p, B, s, band, X, Wb, P, steps, o, state, sscore);          \
  else                                                                                        \
    launch_march_w<12, NEWTON, GG>(p, B, s, band, X, Wb, P, steps, o, state, sscore);
    if (G == 8) {
      BH_PACKED(8)
    } else if (G == 16) {
      BH_PACKED(16)
    } else {
      BH_PACKED(32)
    }
#undef BH_PACKED
    return;
  }
  switch (W) {
    case 16: launch_march_w<16, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
    case 12: launch_march_w<12, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
    case 10: launch_march_w<10, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
    case 8: launch_march_w<8, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
    case 6: launch_march_w<6, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
    case 5: launch_march_w<5, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
    default: launch_march_w<4, NEWTON, 64>(p, B, s, band, X, Wb, P, steps, o, state, sscore); break;
  }
}

template <int G>
int launch_newton_split_g(bh_plan* p, int64_t B, hipStream_t s, const DevBand& band,
                          const double* X, const double* Wb, int P, int steps,
                          const bh_align_opts& o, double* state, double* sscore) {
  constexpr int PER = 64 / G;
  const int64_t groups = (B + PER - 1) / PER;
  const size_t n_lane = (size_t)B * P;
  const size_t n_part = (size_t)groups * kNewtonParts * 10 * 64;
  int rc = grow(p->newton_scr, (n_lane * 13 + n_part) * sizeof(double));
  if (rc != BH_OK) return rc;
  double* trial = (double*)p->newton_scr.ptr;
  double* nst = trial + n_lane * 3;
  double* part = nst + n_lane * 10;
  const int L = band.L;
  ProfScope ps(p, "newton_L" + std::to_string(L), s, groups * PER * P * band.n_entries);
  const int32_t* wp = band.wave_p + wave_block_offset(L, kNewtonParts * kNewtonWaves);
  hipLaunchKernelGGL(k_newton_init<G>, dim3((unsigned)groups), dim3(64), 0, s, state, B, P, trial);
  for (int t = 0; t <= steps; ++t) {
    hipLaunchKernelGGL(k_newton_part<G>, dim3(kNewtonParts, (unsigned)groups),
                       dim3(64 * kNewtonWaves), 0, s, band.p_first, wp, band.rec, X,
                       band.n_entries, L, B, P, trial, part);
    hipLaunchKernelGGL(k_newton_step<G>, dim3((unsigned)groups), dim3(64), 0, s, part, Wb, B, P, t,
                       steps, o.step_init, o.step_grow, o.step_shrink, state, sscore, trial, nst);
  }
  BH_HIP(hipGetLastError());
  return BH_OK;
}

int launch_newton_split(int G, bh_plan* p, int64_t B, hipStream_t s, const DevBand& band,
                        const double* X, const double* Wb, int P, int steps,
                        const bh_align_opts& o, double* state, double* sscore) {
  if (G == 8) return launch_newton_split_g<8>(p, B, s, band, X, Wb, P, steps, o, state, sscore);
  if (G == 16) return launch_newton_split_g<16>(p, B, s, band, X, Wb, P, steps, o, state, sscore);
  return launch_newton_split_g<32>(p, B, s, band, X, Wb, P, steps, o, state, sscore);
}

// Class weights X of the band for B particles, and (Wb != NULL) the step
// scale W_b of each.
// k_xi_band stages two operands of up to kXiLdsCoeffs pairs in dynamic LDS
// (120 KB at L = 40), above the default dynamic-LDS limit of a launch: the
// limit is raised once per process (and device), else the two-kernel path
// runs instead.
bool xi_band_lds_ok() {
  static thread_local int dev_ok[64] = {};   // 0 unknown, 1 ok, -1 refused
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  if (dev_ok[dev] == 0) {
    const int bytes = 2 * kXiLdsCoeffs * (int)sizeof(float2);
    const hipError_t e = hipFuncSetAttribute((const void*)k_xi_band,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    dev_ok[dev] = (e == hipSuccess) ? 1 : -1;
    if (e != hipSuccess) (void)hipGetLastError();
  }
  return dev_ok[dev] > 0;
}

int prepare_band(bh_plan* p, const DevBand& band, const float* a, const float* b,
                 const int32_t* tmpl, int n_tmpl, int64_t B, double** X, hipStream_t s,
                 int64_t lda = 0, int64_t ldt = 0, double* Wb = nullptr, Buffer* xbuf = nullptr) {
  if (lda <= 0) lda = p->C;
  if (ldt <= 0) ldt = p->C;
  if (!xbuf) xbuf = &p->xi_scr;
  // + kTablePad entries: the score loop reads up to three entries ahead
  int rc = grow(*xbuf, ((size_t)B * band.n_entries + kTablePad) * 4 * sizeof(double));
  if (rc != BH_OK) return rc;
  *X = (double*)xbuf->ptr;
  const int64_t CL = p->band_size[band.L];
  if (Wb && CL <= kXiLdsCoeffs && band.n_deg <= kXiLdsDeg && xi_band_lds_ok()) {
    ProfScope ps(p, "xi_classes", s, B);
    hipLaunchKernelGGL(k_xi_band, dim3((unsigned)B), dim3(512), (size_t)2 * CL * sizeof(float2), s,
                       a, lda, b, ldt, tmpl, n_tmpl, band.n_entries, band.sel, band.wt,
                       band.deg_start, band.deg_off, band.n_deg, band.L, (int)CL, *X, Wb,
                       p->err_dev);
    BH_HIP(hipGetLastError());
    return BH_OK;
  }
  {
    ProfScope ps(p, "xi_classes", s, B);
    hipLaunchKernelGGL(k_xi_classes, dim3((unsigned)((band.n_entries + 127) / 128), (unsigned)B),
                       dim3(128), 0, s, a, lda, b, ldt, tmpl, n_tmpl, band.n_entries, band.sel,
                       band.wt, band.deg_start, band.deg_off, *X, p->err_dev);
  }
  BH_HIP(hipGetLastError());
  if (Wb) {
    ProfScope ps(p, "band_weight", s, B);
    hipLaunchKernelGGL(k_band_weight, dim3((unsigned)B), dim3(64), 0, s, a, lda, b, ldt, tmpl,
                       n_tmpl, band.L, band.deg_start, band.deg_off, Wb, p->err_dev);
    BH_HIP(hipGetLastError());
  }
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

int launch_degree_energy(bh_plan* p, const DevBand& band, const float* a, const float* b,
                         const int32_t* tmpl, int n_tmpl, int64_t B, double* energy,
                         hipStream_t s) {
  ProfScope ps(p, "degree_energy", s, B);
  hipLaunchKernelGGL(k_degree_energy, dim3((unsigned)B), dim3(256), 0, s, a, b, p->C, tmpl, n_tmpl,
                     band.L, band.deg_start, band.deg_off, energy, p->err_dev);
  BH_HIP(hipGetLastError());
  return BH_OK;
}

int launch_select_bands(bh_plan* p, const DevBand& band, const float* a, const float* templates,
                        const int32_t* tmpl, int n_tmpl, int64_t B, const BandThresholds& th,
                        int n_tau, int32_t* bands, int32_t* common, double* ratio,
                        hipStream_t s) {
  const int L = band.L;
  int rc = grow(p->energy_scr, (size_t)B * (L + 1) * sizeof(double));
  if (rc != BH_OK) return rc;
  double* E = (double*)p->energy_scr.ptr;
  if ((rc = launch_degree_energy(p, band, a, templates, tmpl, n_tmpl, B, E, s)) != BH_OK) return rc;
  {
    ProfScope ps(p, "select_bands", s, B);
    hipLaunchKernelGGL(k_select_bands, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, E, B, L,
                       th, n_tau, bands, ratio);
  }
  BH_HIP(hipGetLastError());
  if (common) {
    hipLaunchKernelGGL(k_common_bands, dim3((unsigned)n_tau), dim3(256), 0, s, bands, B, L, n_tau,
                       common);
    BH_HIP(hipGetLastError());
  }
  return BH_OK;
}

int launch_correlate(bh_plan* p, const DevBand& band, const float* a, const float* b, int64_t B,
                     const double* euler, int R, double* score, double* grad, double* hess,
                     hipStream_t s) {
  double* X = nullptr;
  int rc = prepare_band(p, band, a, b, nullptr, 1, B, &X, s);
  if (rc != BH_OK) return rc;
  const int64_t chunks = (R + 63) / 64;
  const dim3 grid((unsigned)chunks, (unsigned)B);
  const int W = pick_waves(p, chunks * B, band.L);
  if (hess)
    launch_correlate_any<true>(W, p, grid, s, band, X, euler, R, score, grad, hess);
  else
    launch_correlate_any<false>(W, p, grid, s, band, X, euler, R, score, grad, nullptr);
  BH_HIP(hipGetLastError());
  return BH_OK;
}

namespace {
// The march of launch_align for particles [0, B) of the given arrays, on
// stream s with the given scratch (cross-power, restart state, step scales).
int align_part(bh_plan* p, const float* a, const float* b, const int32_t* tmpl, int n_tmpl,
               int64_t B, const bh_align_opts& o, const double* starts, double* euler_out,
               double* score_out, double* all_euler, double* all_score, hipStream_t s,
               int64_t lda, int64_t ldt, const int64_t* active, Buffer& xi_buf, Buffer& st_buf,
               Buffer& misc_buf) {
  int P = o.n_restarts;
  const bool prune = o.n_keep > 0 && o.n_keep < P;
  const int K = prune ? o.n_keep : P;
  int rc;
  if ((rc = grow(st_buf, (size_t)B * P * 4 * sizeof(double))) != BH_OK) return rc;
  if ((rc = grow(misc_buf, (size_t)B * sizeof(double))) != BH_OK) return rc;
  if (prune && (rc = grow(p->prune_scr, (size_t)B * K * 4 * sizeof(double))) != BH_OK) return rc;
  double* state = (double*)st_buf.ptr;
  double* sscore = state + (size_t)B * P * 3;
  double* Wb = (double*)misc_buf.ptr;
  BH_HIP(hipMemcpyAsync(state, starts, (size_t)B * P * 3 * sizeof(double),
                        hipMemcpyDeviceToDevice, s));
  // bands are prepared first (host tables, uploads) so the loop only launches
  std::vector<const DevBand*> bands;
  for (int i = 0; i < o.n_bands; ++i) {
    const DevBand* band = nullptr;
    if ((rc = get_band(p, o.bands[i], &band)) != BH_OK) return rc;
    bands.push_back(band);
  }
  const int64_t B_all = B;
  for (int bi = 0; bi < o.n_bands; ++bi) {
    const DevBand* band = bands[bi];
    B = active ? active[bi] : B_all;     // the particles that take this band
    if (B == 0) continue;
    double* X = nullptr;
    if ((rc = prepare_band(p, *band, a, b, tmpl, n_tmpl, B, &X, s, lda, ldt, Wb, &xi_buf)) !=
        BH_OK)
      return rc;
    // lanes per particle: 64, or fewer when the (pruned) restarts fit
    const int G = P <= 8 ? 8 : (P <= 16 ? 16 : (P <= 32 ? 32 : 64));
    const int64_t groups = (G == 64) ? (P + 63) / 64 * B : (B + 64 / G - 1) / (64 / G);
    const int W = pick_waves(p, groups, band->L, o.batch_invariant != 0);
    const bool newton = bi >= o.n_bands - o.newton_bands;
    if (newton) {
      const int steps = o.newton_steps > 0 ? o.newton_steps : o.steps_per_band;
      if (G < 64) {
        if ((rc = launch_newton_split(G, p, B, s, *band, X, Wb, P, steps, o, state, sscore)) !=
            BH_OK)
          return rc;
      } else {
        launch_march_any<true>(W, G, p, B, s, *band, X, Wb, P, steps, o, state, sscore);
      }
    } else {
      launch_march_any<false>(W, G, p, B, s, *band, X, Wb, P, o.steps_per_band, o, state,
                              sscore);
    }
    BH_HIP(hipGetLastError());
    if (bi == 0 && prune) {
      double* kst = (double*)p->prune_scr.ptr;
      double* ksc = kst + (size_t)B * K * 3;
      const double half = 0.5 * o.keep_min_sep;
      const double thr = 4.0 * sin(half) * sin(half);
      {
        ProfScope ps(p, "prune", s, B);
        hipLaunchKernelGGL(k_prune, dim3((unsigned)B), dim3(64), 0, s, state, sscore, P, K, thr,
                           kst, ksc);
      }
      BH_HIP(hipGetLastError());
      state = kst;
      sscore = ksc;
      P = K;
    }
  }
  B = B_all;
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
}  // namespace

// A batch's march is split into two halves marched on two streams (the
// caller's and the plan's own, joined back to the caller's) when every
// particle's result stays the same bits: the plain gradient march (no
// pruning, Newton bands or per-band particle counts), 64 lanes per
// particle, at least 256 particles in each half (the wave split does not
// change), and the caller's stream not being captured into a graph.  A
// band launch of a few hundred workgroups spends a good part of its time
// in its first and last rounds; with two independent halves one half's
// last round overlaps the other's middle.
int launch_align(bh_plan* p, const float* a, const float* b, const int32_t* tmpl, int n_tmpl,
                 int64_t B, const bh_align_opts& o, const double* starts, double* euler_out,
                 double* score_out, double* all_euler, double* all_score, hipStream_t s,
                 int64_t lda, int64_t ldt, const int64_t* active) {
  if (lda <= 0) lda = p->C;
  if (ldt <= 0) ldt = p->C;
  const int P = o.n_restarts;
  bool split = p->march_streams > 1 && !active && !(o.n_keep > 0 && o.n_keep < P) &&
               o.newton_bands == 0 && P > 32 && B >= 2 * kSplitMinHalf;
  if (split) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    BH_HIP(hipStreamIsCapturing(s, &cs));
    split = cs == hipStreamCaptureStatusNone;
  }
  if (!split)
    return align_part(p, a, b, tmpl, n_tmpl, B, o, starts, euler_out, score_out, all_euler,
                      all_score, s, lda, ldt, active, p->xi_scr, p->state_scr, p->misc_scr);
  if (!p->aux_stream) {
    BH_HIP(hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking));
    BH_HIP(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
    BH_HIP(hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming));
  }
  const int64_t h = B / 2;
  hipStream_t s2 = p->aux_stream;
  BH_HIP(hipEventRecord(p->fork_ev, s));
  BH_HIP(hipStreamWaitEvent(s2, p->fork_ev, 0));
  int rc = align_part(p, a, b, tmpl, n_tmpl, h, o, starts, euler_out, score_out, all_euler,
                      all_score, s, lda, ldt, nullptr, p->xi_scr, p->state_scr, p->misc_scr);
  if (rc == BH_OK)
    rc = align_part(p, a + (size_t)h * 2 * lda, b, tmpl ? tmpl + h : nullptr, n_tmpl, B - h, o,
                    starts + (size_t)h * P * 3, euler_out + (size_t)h * 3, score_out + h,
                    all_euler ? all_euler + (size_t)h * P * 3 : nullptr,
                    all_score ? all_score + (size_t)h * P : nullptr, s2, lda, ldt, nullptr,
                    p->xi_scr2, p->state_scr2, p->misc_scr2);
  // the caller's stream waits for the second half whatever happened above
  BH_HIP(hipEventRecord(p->join_ev, s2));
  BH_HIP(hipStreamWaitEvent(s, p->join_ev, 0));
  return rc;
}

namespace {
// x[i] = uniform in [-1, 1) from a counter hash of (i, seed) (timing data only).
__global__ void k_fill_random(float* __restrict__ x, int64_t n, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (float)((double)(z >> 11) * (1.0 / 4503599627370496.0) - 1.0);
}

__global__ void k_widen(const float* __restrict__ x, int64_t n, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 3.14159265358979 * (double)x[i];
}
}  // namespace

int tune_march(bh_plan* p, int64_t B, int P, const int32_t* bands, int n_bands, hipStream_t s) {
  const int64_t na = B * p->C * 2, nb = p->C * 2, ns = B * P * 3;
  float* buf = nullptr;
  double* starts = nullptr;
  if (hipMalloc((void**)&buf, (size_t)(na + nb + ns) * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&starts, (size_t)ns * sizeof(double)) != hipSuccess) {
    (void)hipFree(buf);
    return set_error(BH_ENOMEM, "autotune buffers");
  }
  float* a = buf;
  float* b = buf + na;
  hipLaunchKernelGGL(k_fill_random, dim3((unsigned)((na + nb + ns + 255) / 256)), dim3(256), 0, s,
                     buf, na + nb + ns, 12345u);
  hipLaunchKernelGGL(k_widen, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, buf + na + nb,
                     ns, starts);
  int rc = BH_OK;
  if ((rc = grow(p->state_scr, (size_t)B * P * 4 * sizeof(double))) != BH_OK ||
      (rc = grow(p->misc_scr, (size_t)B * sizeof(double))) != BH_OK) {
    (void)hipFree(buf);
    (void)hipFree(starts);
    return rc;
  }
  double* state = (double*)p->state_scr.ptr;
  double* sscore = state + (size_t)B * P * 3;
  double* Wb = (double*)p->misc_scr.ptr;
  bh_align_opts o = {};
  o.step_init = 1.0;
  o.step_grow = 1.25;
  o.step_shrink = 0.5;
  auto reset = [&] {
    (void)hipMemcpyAsync(state, starts, (size_t)ns * sizeof(double), hipMemcpyDeviceToDevice, s);
  };
  for (int bi = 0; bi < n_bands && rc == BH_OK; ++bi) {
    const DevBand* band = nullptr;
    if ((rc = get_band(p, bands[bi], &band)) != BH_OK) break;
    double* X = nullptr;
    if ((rc = prepare_band(p, *band, a, b, nullptr, 1, B, &X, s, 0, 0, Wb)) != BH_OK) break;
    float best_ms = 1e30f;
    int best_w = 0;
    p->tuned_persist[band->L] = 0;
    for (int W : {4, 5, 6, 8, 10, 12, 16}) {
      if (W > 2 * band->L + 1 && W > 4) continue;
      float ms = 0.0f;
      rc = time_on_stream(
          s, 2, reset,
          [&] { launch_march_any<false>(W, 64, p, B, s, *band, X, Wb, P, 2, o, state, sscore); },
          &ms);
      if (rc != BH_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best_w = W;
      }
    }
    if (rc != BH_OK) break;
    // the best wave count again with persistent workgroups
    p->tuned_persist[band->L] = 1;
    float pms = 0.0f;
    rc = time_on_stream(
        s, 2, reset,
        [&] { launch_march_any<false>(best_w, 64, p, B, s, *band, X, Wb, P, 2, o, state, sscore); },
        &pms);
    if (rc != BH_OK) break;
    p->tuned_persist[band->L] = (pms < 0.99f * best_ms) ? 1 : 0;
    p->tuned_waves[band->L] = best_w;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  (void)hipFree(starts);
  return rc;
}

int launch_prune(bh_plan* p, const double* euler, const double* score, int64_t B, int P, int K,
                 double min_sep, double* euler_out, double* score_out, hipStream_t s) {
  const double half = 0.5 * min_sep;
  const double thr = 4.0 * sin(half) * sin(half);
  ProfScope ps(p, "prune", s, B);
  hipLaunchKernelGGL(k_prune, dim3((unsigned)B), dim3(64), 0, s, euler, score, P, K, thr,
                     euler_out, score_out);
  BH_HIP(hipGetLastError());
  return BH_OK;
}

int launch_align_shifts(bh_plan* p, const float* vols, int64_t B, const int32_t* shifts_host,
                        int S, const float* b, const bh_align_opts& o, const double* starts,
                        double* euler_out, double* score_out, int32_t* shift_out,
                        hipStream_t s) {
  const int64_t rows = B * S;
  const int P = o.n_restarts;
  // scratch: coefficients [rows][C][2] | starts [rows][P][3] | best per row
  ShiftTable tab = {};
  for (int i = 0; i < S; ++i)
    for (int k = 0; k < 3; ++k) tab.d[i][k] = shifts_host[3 * i + k];
  const size_t sh_bytes = 0;
  const size_t co_bytes = ((size_t)rows * p->C * 2 * sizeof(float) + 255) / 256 * 256;
  const size_t st_bytes = (size_t)rows * P * 3 * sizeof(double);
  const size_t eu_bytes = (size_t)rows * 3 * sizeof(double);
  const size_t sc_bytes = (size_t)rows * sizeof(double);
  int rc = grow(p->shift_scr, sh_bytes + co_bytes + st_bytes + eu_bytes + sc_bytes);
  if (rc != BH_OK) return rc;
  char* base = (char*)p->shift_scr.ptr;
  float* coeffs = (float*)(base + sh_bytes);
  double* st = (double*)(base + sh_bytes + co_bytes);
  double* eu = (double*)(base + sh_bytes + co_bytes + st_bytes);
  double* sc = (double*)(base + sh_bytes + co_bytes + st_bytes + eu_bytes);
  if ((rc = launch_expand(p, vols, B, coeffs, s, false, &tab, S)) != BH_OK) return rc;
  const int64_t n = rows * P * 3;
  hipLaunchKernelGGL(k_repeat_starts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, starts,
                     B, S, P, st);
  BH_HIP(hipGetLastError());
  if ((rc = launch_align(p, coeffs, b, nullptr, 1, rows, o, st, eu, sc, nullptr, nullptr, s)) !=
      BH_OK)
    return rc;
  hipLaunchKernelGGL(k_select_shift, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, eu, sc, B,
                     S, euler_out, score_out, shift_out);
  BH_HIP(hipGetLastError());
  return BH_OK;
}

}  // namespace bh
