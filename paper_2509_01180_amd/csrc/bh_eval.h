// Score evaluator of Eq. (2) and its Euler gradient for one wave's share of
// the (m, n) classes; included by the score kernels (and usable from host
// code, which runs the same arithmetic lane by lane).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bh_special.h"

// Phases e^{-i p sigma} by FP64 sincos per p-group (1) or by a running
// product along the wave's ascending p-list (0); build-time parameter.
#ifndef BH_SCORE_PHASE_SINCOS
#define BH_SCORE_PHASE_SINCOS 0
#endif

namespace bh {

struct cplx {
  double re, im;
};

BH_HD inline cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
BH_HD inline cplx cmulc(cplx a, cplx b) {   // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// ------------------------------------------------------------- evaluation --

struct Angles {
  double x, sb;          // cos(beta), sin(beta)
  double c, s, s2;       // cos(beta/2), sin(beta/2), sin^2(beta/2)
  double sigma;          // (alpha + gamma) / 2
  cplx th1, th2;         // e^{-i delta}, e^{-2 i delta}, delta = (alpha - gamma) / 2
};

BH_HD inline Angles prep(double al, double be, double ga) {
  Angles A;
  sincos(be, &A.sb, &A.x);
  sincos(0.5 * be, &A.s, &A.c);
  A.s2 = A.s * A.s;
  A.sigma = 0.5 * (al + ga);
  const double delta = 0.5 * (al - ga);
  double sd, cd, s2d, c2d;
  sincos(delta, &sd, &cd);
  sincos(2.0 * delta, &s2d, &c2d);
  A.th1 = {cd, -sd};
  A.th2 = {c2d, -s2d};
  return A;
}

struct Acc {
  double S, ga, gb, gg;
};

// One step of the rescaled recurrence for chain entry x/c (see below).
#define BH_CHAIN_STEP(X4, C2, EA, RA, EB, RB)                                 \
  do {                                                                        \
    t1r = fma((X4).x, EA, t1r);                                               \
    t1i = fma((X4).y, EA, t1i);                                               \
    t2r = fma((X4).z, EA, t2r);                                               \
    t2i = fma((X4).w, EA, t2i);                                               \
    r1r = fma((X4).x, RA, r1r);                                               \
    r1i = fma((X4).y, RA, r1i);                                               \
    r2r = fma((X4).z, RA, r2r);                                               \
    r2i = fma((X4).w, RA, r2i);                                               \
    const double u_ = (C2).x * (A.x - (C2).y);                                \
    const double msa_ = (C2).x * msb;                                         \
    EB = fma(u_, EA, -EB);                                                    \
    RB = fma(msa_, EA, fma(u_, RA, -RB));                                     \
  } while (0)

// Partial sums of one wave over the classes of its p-groups: plist holds
// [count, p_1, ..., p_count] (a wave's share of the longest-first split).
//
// Chain loop: four entries per round.  The four X and rec entries of a
// round are wave-uniform and fetched together with scalar loads (one wait
// per round: scalar loads return out of order, so a wait drains them all);
// (ea, ra) and (eb, rb) hold e, de/dbeta of two consecutive degrees and each
// step overwrites the older pair, so no register moves are needed.
BH_HD inline Acc eval_wave(const Angles& A, const int32_t* __restrict__ plist, int L,
                           const int32_t* __restrict__ p_first,
                           const double* __restrict__ rec, const double* __restrict__ X) {
  Acc acc = {0.0, 0.0, 0.0, 0.0};
  const double msb = -A.sb;
  const int np = plist[0];
#if !BH_SCORE_PHASE_SINCOS
  // Phi = e^{-i pc sigma} and cpm1 = c^{max(pc-1,0)}, advanced along the
  // ascending p-list one degree at a time.
  double s1, c1;
  sincos(A.sigma, &s1, &c1);
  const cplx E1 = {c1, -s1};
  cplx Phi = {1.0, 0.0};
  double cpm1 = 1.0;
  int pc = 0;
#endif
  for (int j = 0; j < np; ++j) {
    const int p = plist[1 + j];
#if BH_SCORE_PHASE_SINCOS
    double sp, cpp;
    sincos((double)p * A.sigma, &sp, &cpp);
    const cplx Phi = {cpp, -sp};          // e^{-i p sigma}
    double cpm1 = 1.0;                    // c^{max(p-1,0)}
    for (int i = 1; i < p; ++i) cpm1 *= A.c;
#else
    for (; pc < p; ++pc) {
      Phi = cmul(Phi, E1);
      cpm1 = (pc >= 1) ? cpm1 * A.c : 1.0;
    }
#endif
    const double cp = (p > 0) ? cpm1 * A.c : 1.0;
    const double cpp1 = cp * A.c;
    int off = p_first[p];
    const int q0 = p & 1;
    cplx Th = q0 ? A.th1 : cplx{1.0, 0.0};
    double sq = q0 ? A.s : 1.0;       // s^q
    double sqm1 = q0 ? 1.0 : 0.0;     // s^{q-1} (0 stands in for q = 0)
    for (int q = q0; q <= 2 * L - p; q += 2) {
      const int m = (p + q) >> 1, n = (p - q) >> 1;
      const int len = L - m + 1;
      // seeds: e_m = c^p s^q, r_m = d/dbeta e_m = (q c^{p+1} s^{q-1} - p c^{p-1} s^{q+1}) / 2
      double ea = cp * sq;
      double ra = 0.5 * ((double)q * cpp1 * sqm1 - (double)p * cpm1 * (sq * A.s));
      double eb = 0.0, rb = 0.0;
      double t1r = 0, t1i = 0, t2r = 0, t2i = 0, r1r = 0, r1i = 0, r2r = 0, r2i = 0;
      const double4* Xc = reinterpret_cast<const double4*>(X) + off;
      const double2* Rc = reinterpret_cast<const double2*>(rec) + off;
      // Full rounds of four entries: straight-line code, one load batch and
      // one wait per round.  Then a tail of two and/or one entries.
      const int n4 = len & ~3;
      int i = 0;
      for (; i < n4; i += 4) {
        const double4 x0 = Xc[i], x1 = Xc[i + 1], x2 = Xc[i + 2], x3 = Xc[i + 3];
        const double2 c0_ = Rc[i], c1 = Rc[i + 1], c2 = Rc[i + 2], c3 = Rc[i + 3];
        BH_CHAIN_STEP(x0, c0_, ea, ra, eb, rb);
        BH_CHAIN_STEP(x1, c1, eb, rb, ea, ra);
        BH_CHAIN_STEP(x2, c2, ea, ra, eb, rb);
        BH_CHAIN_STEP(x3, c3, eb, rb, ea, ra);
      }
      if (len & 2) {
        const double4 x0 = Xc[i], x1 = Xc[i + 1];
        const double2 c0_ = Rc[i], c1 = Rc[i + 1];
        BH_CHAIN_STEP(x0, c0_, ea, ra, eb, rb);
        BH_CHAIN_STEP(x1, c1, eb, rb, ea, ra);
        i += 2;
      }
      if (len & 1) {
        const double4 x0 = Xc[i];
        const double2 c0_ = Rc[i];
        BH_CHAIN_STEP(x0, c0_, ea, ra, eb, rb);
      }
      const cplx W1 = cmul(Phi, Th);
      const cplx W2 = cmulc(Phi, Th);
      const cplx z1 = cmul(W1, {t1r, t1i});
      const cplx z2 = cmul(W2, {t2r, t2i});
      acc.S += z1.re + z2.re;
      acc.ga += (double)m * z1.im + (double)n * z2.im;
      acc.gg += (double)n * z1.im + (double)m * z2.im;
      acc.gb += (W1.re * r1r - W1.im * r1i) + (W2.re * r2r - W2.im * r2i);
      off += len;
      Th = cmul(Th, A.th2);
      sqm1 = (q == 0) ? A.s : sqm1 * A.s2;
      sq *= A.s2;
    }
  }
  return acc;
}
#undef BH_CHAIN_STEP

}  // namespace bh
