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
  double x;              // cos(beta)
  double c, s;           // cos(beta/2), sin(beta/2), magnitudes floored at kPoleFloor
  double ic2, is2;       // 1 / (4 c^2), 1 / (4 s^2)
  double msb;            // -sin(beta) = -2 s c (with the floored c, s)
  double sigma;          // (alpha + gamma) / 2
  cplx th1, th2;         // e^{-i delta}, e^{-2 i delta}, delta = (alpha - gamma) / 2
};

// Half-angle sines and cosines are kept at least this large in magnitude
// (sign preserved) so that the x-derivative seeds below stay finite at the
// poles beta = 0, pi; the change to any score is far below rounding.
constexpr double kPoleFloor = 1e-100;

BH_HD inline Angles prep(double al, double be, double ga) {
  Angles A;
  double sb;
  sincos(be, &sb, &A.x);
  sincos(0.5 * be, &A.s, &A.c);
  A.s = copysign(fmax(fabs(A.s), kPoleFloor), A.s);
  A.c = copysign(fmax(fabs(A.c), kPoleFloor), A.c);
  A.ic2 = 0.25 / (A.c * A.c);
  A.is2 = 0.25 / (A.s * A.s);
  A.msb = -2.0 * A.s * A.c;
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

// One step of the rescaled recurrence for chain entry x/c (see below):
// e' = u e - e_prev and its x-derivative r' = u r - r_prev + ap e, with
// u = ap (x - bq) from the table entry {ap, bq}.  (Written as a subtraction
// and a product, each instruction reads one table value: a vector
// instruction can take only one scalar-register operand.)
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
    EB = fma(u_, EA, -EB);                                                    \
    RB = fma((C2).x, EA, fma(u_, RA, -RB));                                   \
  } while (0)

// Partial sums of one wave over the classes of its p-groups: plist holds
// [count, p_1, ..., p_count] (a wave's share of the longest-first split).
//
// The chains carry de/dx (x = cos beta) rather than de/dbeta: the
// recurrence for de/dx needs no per-step sin(beta) factor, and the beta
// derivative is -sin(beta) times the accumulated x-derivative sums, applied
// once at the end.
//
// Chain loop: the first entry (e_{m-1} = 0) is peeled, which also starts
// the accumulators; then four entries per round.  The four X and rec
// entries of a round are wave-uniform and fetched together with scalar
// loads (one wait per round: scalar loads return out of order, so a wait
// drains them all); (ea, ra) and (eb, rb) hold e, de/dx of two consecutive
// degrees and each step overwrites the older pair, so no register moves are
// needed.
//
// Class epilogue: with W1 = e^{-i p sigma} e^{-i q delta} and W2 =
// e^{-i p sigma} e^{+i q delta} (advanced by e^{-+2i delta} per class), the
// class adds Re(W1 t1 + W2 t2) to S and Re(W1 r1 + W2 r2) to the x-gradient;
// the alpha and gamma derivatives m I1 + n I2 and n I1 + m I2 (I = Im(W t))
// are accumulated as (p SP +- SQ) / 2 with SP = sum (I1 + I2) and
// SQ = sum q (I1 - I2) over the p-group.
BH_HD inline Acc eval_wave(const Angles& A, const int32_t* __restrict__ plist, int L,
                           const int32_t* __restrict__ p_first,
                           const double* __restrict__ rec, const double* __restrict__ X) {
  Acc acc = {0.0, 0.0, 0.0, 0.0};
  const int np = plist[0];
#if !BH_SCORE_PHASE_SINCOS
  // Phi = e^{-i pc sigma} and cp = c^pc, advanced along the ascending
  // p-list one degree at a time.
  double s1, c1;
  sincos(A.sigma, &s1, &c1);
  const cplx E1 = {c1, -s1};
  cplx Phi = {1.0, 0.0};
  double cp = 1.0;
  int pc = 0;
#endif
  const double s2 = A.s * A.s;
  const cplx th2c = {A.th2.re, -A.th2.im};
  for (int j = 0; j < np; ++j) {
    const int p = plist[1 + j];
#if BH_SCORE_PHASE_SINCOS
    double sp, cpp;
    sincos((double)p * A.sigma, &sp, &cpp);
    const cplx Phi = {cpp, -sp};          // e^{-i p sigma}
    double cp = 1.0;                      // c^p
    for (int i = 0; i < p; ++i) cp *= A.c;
#else
    for (; pc < p; ++pc) {
      Phi = cmul(Phi, E1);
      cp *= A.c;
    }
#endif
    const double pic2 = (double)p * A.ic2;
    int off = p_first[p];
    const int q0 = p & 1;
    cplx W1 = q0 ? cmul(Phi, A.th1) : Phi;
    cplx W2 = q0 ? cmulc(Phi, A.th1) : Phi;
    double sq = q0 ? A.s : 1.0;       // s^q
    double qd = (double)q0;
    double SP = 0.0, SQ = 0.0;
    for (int q = q0; q <= 2 * L - p; q += 2) {
      const int m = (p + q) >> 1;
      const int rem = L - m;          // chain entries after the first
      const double4* Xc = reinterpret_cast<const double4*>(X) + off;
      const double2* Rc = reinterpret_cast<const double2*>(rec) + off;
      // seeds: e_m = c^p s^q and de_m/dx = e_m (p / (4 c^2) - q / (4 s^2));
      // the peeled first step starts the sums and yields e_{m+1}.
      double eb = cp * sq;
      double rb = eb * fma(-qd, A.is2, pic2);
      double t1r, t1i, t2r, t2i, r1r, r1i, r2r, r2i, ea, ra;
      {
        const double4 x0 = Xc[0];
        const double2 c0_ = Rc[0];
        t1r = x0.x * eb;
        t1i = x0.y * eb;
        t2r = x0.z * eb;
        t2i = x0.w * eb;
        r1r = x0.x * rb;
        r1i = x0.y * rb;
        r2r = x0.z * rb;
        r2i = x0.w * rb;
        const double u_ = c0_.x * (A.x - c0_.y);
        ea = u_ * eb;
        ra = fma(c0_.x, eb, u_ * rb);
      }
      // Full rounds of four entries: straight-line code, one load batch and
      // one wait per round.  Then a tail of two and/or one entries.
      const int n4 = rem & ~3;
      int i = 1;
      for (; i <= n4; i += 4) {
        const double4 x0 = Xc[i], x1 = Xc[i + 1], x2 = Xc[i + 2], x3 = Xc[i + 3];
        const double2 c0_ = Rc[i], c1 = Rc[i + 1], c2 = Rc[i + 2], c3 = Rc[i + 3];
        BH_CHAIN_STEP(x0, c0_, ea, ra, eb, rb);
        BH_CHAIN_STEP(x1, c1, eb, rb, ea, ra);
        BH_CHAIN_STEP(x2, c2, ea, ra, eb, rb);
        BH_CHAIN_STEP(x3, c3, eb, rb, ea, ra);
      }
      if (rem & 2) {
        const double4 x0 = Xc[i], x1 = Xc[i + 1];
        const double2 c0_ = Rc[i], c1 = Rc[i + 1];
        BH_CHAIN_STEP(x0, c0_, ea, ra, eb, rb);
        BH_CHAIN_STEP(x1, c1, eb, rb, ea, ra);
        i += 2;
      }
      if (rem & 1) {
        const double4 x0 = Xc[i];
        const double2 c0_ = Rc[i];
        BH_CHAIN_STEP(x0, c0_, ea, ra, eb, rb);
      }
      acc.S = fma(W1.re, t1r, acc.S);
      acc.S = fma(-W1.im, t1i, acc.S);
      acc.S = fma(W2.re, t2r, acc.S);
      acc.S = fma(-W2.im, t2i, acc.S);
      SP = fma(W1.re, t1i, SP);
      SP = fma(W1.im, t1r, SP);
      SP = fma(W2.re, t2i, SP);
      SP = fma(W2.im, t2r, SP);
      double D = W1.re * t1i;
      D = fma(W1.im, t1r, D);
      D = fma(-W2.re, t2i, D);
      D = fma(-W2.im, t2r, D);
      SQ = fma(qd, D, SQ);
      acc.gb = fma(W1.re, r1r, acc.gb);
      acc.gb = fma(-W1.im, r1i, acc.gb);
      acc.gb = fma(W2.re, r2r, acc.gb);
      acc.gb = fma(-W2.im, r2i, acc.gb);
      off += rem + 1;
      W1 = cmul(W1, A.th2);
      W2 = cmul(W2, th2c);
      sq *= s2;
      qd += 2.0;
    }
    const double pSP = (double)p * SP;
    acc.ga += 0.5 * (pSP + SQ);
    acc.gg += 0.5 * (pSP - SQ);
  }
  acc.gb *= A.msb;
  return acc;
}
#undef BH_CHAIN_STEP

}  // namespace bh
