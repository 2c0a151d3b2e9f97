// Score evaluator of Eq. (2) and its Euler gradient for one wave's share of
// the (m, n) classes; included by the score kernels (and usable from host
// code, which runs the same arithmetic lane by lane).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bh_special.h"

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

// Partial sums of one wave over its classes p = wave, wave + W, ...
BH_HD inline Acc eval_wave(const Angles& A, int wave, int W, int L,
                                const int32_t* __restrict__ p_first,
                                const double* __restrict__ rec, const double* __restrict__ X) {
  Acc acc = {0.0, 0.0, 0.0, 0.0};
  // c^p, c^{max(p-1,0)}, c^{p+1} for the first p of this wave, and c^W, c^{W-1}
  double cW = 1.0, cW1 = 1.0;
  for (int i = 0; i < W; ++i) cW *= A.c;
  for (int i = 0; i < W - 1; ++i) cW1 *= A.c;
  double cp = 1.0;
  for (int i = 0; i < wave; ++i) cp *= A.c;
  double cpm1 = 1.0;
  for (int i = 0; i < wave - 1; ++i) cpm1 *= A.c;
  double cpp1 = cp * A.c;
  const double msb = -A.sb;
  for (int p = wave; p <= 2 * L; p += W) {
    double sp, cpp;
    sincos((double)p * A.sigma, &sp, &cpp);
    const cplx Phi = {cpp, -sp};
    int off = p_first[p];
    const int q0 = p & 1;
    cplx Th = q0 ? A.th1 : cplx{1.0, 0.0};
    double sq = q0 ? A.s : 1.0;       // s^q
    double sqm1 = q0 ? 1.0 : 0.0;     // s^{q-1} (0 stands in for q = 0)
    for (int q = q0; q <= 2 * L - p; q += 2) {
      const int m = (p + q) >> 1, n = (p - q) >> 1;
      const int len = L - m + 1;
      // seeds: e_m = c^p s^q, r_m = d/dbeta e_m = (q c^{p+1} s^{q-1} - p c^{p-1} s^{q+1}) / 2
      double e = cp * sq;
      double r = 0.5 * ((double)q * cpp1 * sqm1 - (double)p * cpm1 * (sq * A.s));
      double t1r = 0, t1i = 0, t2r = 0, t2i = 0, r1r = 0, r1i = 0, r2r = 0, r2i = 0;
      const double* Xc = X + 4 * (int64_t)off;
      const double* Rc = rec + 2 * (int64_t)off;
      // Two chain entries per iteration: (ea, ra) hold e_i, r_i and (eb, rb)
      // hold e_{i-1}, r_{i-1}; each step overwrites the older pair, so no
      // register moves are needed.  The next pair's table entries are loaded
      // one iteration ahead (buffers are padded past their last entry).
      double ea = e, ra = r, eb = 0.0, rb = 0.0;
      double4 xa = *reinterpret_cast<const double4*>(Xc);
      double4 xb = *reinterpret_cast<const double4*>(Xc + 4);
      double2 ca = *reinterpret_cast<const double2*>(Rc);
      double2 cb = *reinterpret_cast<const double2*>(Rc + 2);
      for (int i = 0; i < len; i += 2) {
        const double4 nxa = *reinterpret_cast<const double4*>(Xc + 4 * (i + 2));
        const double4 nxb = *reinterpret_cast<const double4*>(Xc + 4 * (i + 3));
        const double2 nca = *reinterpret_cast<const double2*>(Rc + 2 * (i + 2));
        const double2 ncb = *reinterpret_cast<const double2*>(Rc + 2 * (i + 3));
        // entry i: accumulate with e_i, then e_{i+1} -> (eb, rb)
        t1r = fma(xa.x, ea, t1r);
        t1i = fma(xa.y, ea, t1i);
        t2r = fma(xa.z, ea, t2r);
        t2i = fma(xa.w, ea, t2i);
        r1r = fma(xa.x, ra, r1r);
        r1i = fma(xa.y, ra, r1i);
        r2r = fma(xa.z, ra, r2r);
        r2i = fma(xa.w, ra, r2i);
        {
          const double u = ca.x * (A.x - ca.y);
          const double msa = ca.x * msb;
          eb = fma(u, ea, -eb);
          rb = fma(msa, ea, fma(u, ra, -rb));
        }
        if (i + 1 < len) {
          // entry i+1: accumulate with e_{i+1}, then e_{i+2} -> (ea, ra)
          t1r = fma(xb.x, eb, t1r);
          t1i = fma(xb.y, eb, t1i);
          t2r = fma(xb.z, eb, t2r);
          t2i = fma(xb.w, eb, t2i);
          r1r = fma(xb.x, rb, r1r);
          r1i = fma(xb.y, rb, r1i);
          r2r = fma(xb.z, rb, r2r);
          r2i = fma(xb.w, rb, r2i);
          const double u = cb.x * (A.x - cb.y);
          const double msa = cb.x * msb;
          ea = fma(u, eb, -ea);
          ra = fma(msa, eb, fma(u, rb, -ra));
        }
        xa = nxa;
        xb = nxb;
        ca = nca;
        cb = ncb;
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
    if (p == 0) {
      cpm1 = cW1;
    } else {
      cpm1 *= cW;
    }
    cp *= cW;
    cpp1 *= cW;
  }
  return acc;
}

}  // namespace bh
