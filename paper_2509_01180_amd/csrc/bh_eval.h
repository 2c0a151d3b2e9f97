// Score evaluator of Eq. (2) and its Euler gradient for one wave's share of
// the (m, n) classes; included by the score kernels (and usable from host
// code, which runs the same arithmetic lane by lane).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bh_special.h"
#include "bh_tables.h"

// Phases e^{-i p sigma} by FP64 sincos per p-group (1) or by a running
// product along the wave's ascending p-list (0); build-time parameter.  The
// sincos form holds three fewer values through the class loop (the running
// phase, its step and c^p are recomputed per p-group), which keeps the
// ascent kernel within 80 registers without spills, for about one sincos
// per p-group of a wave (under 1 % of the evaluation).
#ifndef BH_SCORE_PHASE_SINCOS
#define BH_SCORE_PHASE_SINCOS 1
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
  cplx e1;               // e^{-i sigma}
  cplx th1, th2;         // e^{-i delta}, e^{-2 i delta}, delta = (alpha - gamma) / 2
};
constexpr int kAngleWords = 13;   // doubles in Angles
constexpr int kAngleMsb = 5;      // position of msb among them (store_angles)

// Half-angle sines and cosines are kept at least this large in magnitude
// (sign preserved) so that the x-derivative seeds below (up to 1 / s^4 for
// the second derivative) stay finite at the poles beta = 0, pi; the change
// to any score is far below rounding.
constexpr double kPoleFloor = 1e-30;

// Three sincos per rotation: cos(beta) = 1 - 2 sin^2(beta/2) and
// e^{-2 i delta} = (e^{-i delta})^2 follow from the half angles.
BH_HD inline Angles prep(double al, double be, double ga) {
  Angles A;
  double s, c;
  sincos(0.5 * be, &s, &c);
  A.x = fma(-2.0 * s, s, 1.0);
  A.s = copysign(fmax(fabs(s), kPoleFloor), s);
  A.c = copysign(fmax(fabs(c), kPoleFloor), c);
  A.ic2 = 0.25 / (A.c * A.c);
  A.is2 = 0.25 / (A.s * A.s);
  A.msb = -2.0 * A.s * A.c;
  A.sigma = 0.5 * (al + ga);
  double ss, cs;
  sincos(A.sigma, &ss, &cs);
  A.e1 = {cs, -ss};
  double sd, cd;
  sincos(0.5 * (al - ga), &sd, &cd);
  A.th1 = {cd, -sd};
  A.th2 = cmul(A.th1, A.th1);
  return A;
}

// Angles <-> kAngleWords doubles at stride `ld` (lane-major LDS rows).
BH_HD inline void store_angles(const Angles& A, double* p, int ld) {
  const double v[kAngleWords] = {A.x,     A.c,      A.s,      A.ic2,    A.is2,
                                 A.msb,   A.sigma,  A.e1.re,  A.e1.im,  A.th1.re,
                                 A.th1.im, A.th2.re, A.th2.im};
  for (int k = 0; k < kAngleWords; ++k) p[k * ld] = v[k];
}
BH_HD inline Angles load_angles(const double* p, int ld) {
  Angles A;
  A.x = p[0];
  A.c = p[ld];
  A.s = p[2 * ld];
  A.ic2 = p[3 * ld];
  A.is2 = p[4 * ld];
  A.msb = p[5 * ld];
  A.sigma = p[6 * ld];
  A.e1 = {p[7 * ld], p[8 * ld]};
  A.th1 = {p[9 * ld], p[10 * ld]};
  A.th2 = {p[11 * ld], p[12 * ld]};
  return A;
}

struct Acc {
  double S, ga, gb, gg;
  double haa, hab, hag, hbb, hbg, hgg;   // Hessian (evaluators with HESS only)
};

// One step of the rescaled recurrence for chain entry x/c (see below):
// e' = u e - e_prev and its x-derivative r' = u r - r_prev + ap e, with
// u = ap (x - bq) from the table entry {ap, bq}.  (Written as a subtraction
// and a product, each instruction reads one table value: a vector
// instruction can take only one scalar-register operand.)
// With HESS the chains carry beta-derivatives instead (no pole
// singularity in second derivatives): with u = ap (x - bq), u' = -ap
// sin(beta) and u'' = -ap cos(beta),
//   r' = u r - r_prev + u' e,   q' = u q - q_prev + 2 u' r + u'' e
// for r = de/dbeta and q = d^2e/dbeta^2.
#define BH_CHAIN_STEP(X4, C2, EA, RA, QA, EB, RB, QB)                         \
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
    if constexpr (HESS) {                                                     \
      q1r = fma((X4).x, QA, q1r);                                             \
      q1i = fma((X4).y, QA, q1i);                                             \
      q2r = fma((X4).z, QA, q2r);                                             \
      q2i = fma((X4).w, QA, q2i);                                             \
      const double du_ = (C2).x * A.msb;                                      \
      const double dd_ = (C2).x * mx;                                         \
      QB = fma(dd_, EA, fma(du_ + du_, RA, fma(u_, QA, -QB)));                \
      RB = fma(du_, EA, fma(u_, RA, -RB));                                    \
    } else {                                                                  \
      RB = fma((C2).x, EA, fma(u_, RA, -RB));                                 \
    }                                                                         \
    EB = fma(u_, EA, -EB);                                                    \
  } while (0)

#if defined(__HIP_DEVICE_COMPILE__)
// The chain sums of one class for wave-uniform weights, as one asm block:
// t = sum_l X_l e_l and r = sum_l X_l de_l/dx over the chain's n entries,
// from the seeds (e_m, de_m/dx) = (eb, rb), in rounds of four entries.
// Each round fetches its four X entries (32 B each) and recurrence entries
// {ap, bq} (16 B each) with three 64-byte scalar loads into s36..s83 and
// waits once; the first round also does the peeled first entry, so a chain
// of n entries waits ceil(n / 4) times (against one wait for the peeled
// entry, one per full round and one per tail of two or one entries in the
// compiled loop, where the compiler also moves each load into the branch
// that first uses it).  The last entry adds to the sums only.  Loads read
// up to three entries past the chain (the next class's, or the tables'
// padding); every load is waited for inside the block.  The arithmetic
// and its order per value are those of the compiled loop: u = ap (x - bq),
// r' = fma(ap, e, fma(u, r, -r_prev)), e' = fma(u, e, -e_prev), sums by
// fma, the first entry's terms by products.
#define BH_CA_ACC(XA, XB, XC, XD, EA, RA)      \
  "v_fmac_f64 %[t1r], " XA ", %[" EA "]\n"     \
  "v_fmac_f64 %[t1i], " XB ", %[" EA "]\n"     \
  "v_fmac_f64 %[t2r], " XC ", %[" EA "]\n"     \
  "v_fmac_f64 %[t2i], " XD ", %[" EA "]\n"     \
  "v_fmac_f64 %[r1r], " XA ", %[" RA "]\n"     \
  "v_fmac_f64 %[r1i], " XB ", %[" RA "]\n"     \
  "v_fmac_f64 %[r2r], " XC ", %[" RA "]\n"     \
  "v_fmac_f64 %[r2i], " XD ", %[" RA "]\n"
#define BH_CA_STEP(XA, XB, XC, XD, AP, BQ, EA, RA, EB, RB)  \
  "v_add_f64 %[u], %[x], -" BQ "\n"                         \
  "v_mul_f64 %[u], " AP ", %[u]\n"                          \
  BH_CA_ACC(XA, XB, XC, XD, EA, RA)                         \
  "v_fma_f64 %[" RB "], %[u], %[" RA "], -%[" RB "]\n"      \
  "v_fmac_f64 %[" RB "], " AP ", %[" EA "]\n"               \
  "v_fma_f64 %[" EB "], %[u], %[" EA "], -%[" EB "]\n"
#define BH_CA_ACC_(...) BH_CA_ACC(__VA_ARGS__)
#define BH_CA_STEP_(...) BH_CA_STEP(__VA_ARGS__)
// round entry j: X at s[36 + 8j ...], {ap, bq} at s[68 + 4j ...]
#define BH_CA_X0 "s[36:37]", "s[38:39]", "s[40:41]", "s[42:43]"
#define BH_CA_X1 "s[44:45]", "s[46:47]", "s[48:49]", "s[50:51]"
#define BH_CA_X2 "s[52:53]", "s[54:55]", "s[56:57]", "s[58:59]"
#define BH_CA_X3 "s[60:61]", "s[62:63]", "s[64:65]", "s[66:67]"
#define BH_CA_E0 BH_CA_X0, "s[68:69]", "s[70:71]"
#define BH_CA_E1 BH_CA_X1, "s[72:73]", "s[74:75]"
#define BH_CA_E2 BH_CA_X2, "s[76:77]", "s[78:79]"
#define BH_CA_E3 BH_CA_X3, "s[80:81]", "s[82:83]"
#define BH_CA_LOAD                                  \
  "s_add_u32 s85, s84, 0x40\n"                      \
  "s_load_dwordx16 s[36:51], %[xc], s84\n"          \
  "s_load_dwordx16 s[52:67], %[xc], s85\n"          \
  "s_load_dwordx16 s[68:83], %[rc], s86\n"          \
  "s_waitcnt lgkmcnt(0)\n"

// Chain text shared by the asm blocks below: the first round (peeled
// entry, loaded by the block's own first loads) and the later rounds.
#define BH_CA_CHAIN \
  "v_mul_f64 %[t1r], s[36:37], %[eb]\n" \
  "v_mul_f64 %[t1i], s[38:39], %[eb]\n" \
  "v_mul_f64 %[t2r], s[40:41], %[eb]\n" \
  "v_mul_f64 %[t2i], s[42:43], %[eb]\n" \
  "v_mul_f64 %[r1r], s[36:37], %[rb]\n" \
  "v_mul_f64 %[r1i], s[38:39], %[rb]\n" \
  "v_mul_f64 %[r2r], s[40:41], %[rb]\n" \
  "v_mul_f64 %[r2i], s[42:43], %[rb]\n" \
  "s_cmp_eq_u32 %[n], 1\n" \
  "s_cbranch_scc1 .Lbhc_end%=\n" \
  "v_add_f64 %[u], %[x], -s[70:71]\n" \
  "v_mul_f64 %[u], s[68:69], %[u]\n" \
  "v_mul_f64 %[ea], %[u], %[eb]\n" \
  "v_mul_f64 %[ra], %[u], %[rb]\n" \
  "v_fmac_f64 %[ra], s[68:69], %[eb]\n" \
  "s_cmp_eq_u32 %[n], 2\n" \
  "s_cbranch_scc1 .Lbhc_f2%=\n" \
  BH_CA_STEP_(BH_CA_E1, "ea", "ra", "eb", "rb") \
  "s_cmp_eq_u32 %[n], 3\n" \
  "s_cbranch_scc1 .Lbhc_f3%=\n" \
  BH_CA_STEP_(BH_CA_E2, "eb", "rb", "ea", "ra") \
  "s_cmp_eq_u32 %[n], 4\n" \
  "s_cbranch_scc1 .Lbhc_f4%=\n" \
  BH_CA_STEP_(BH_CA_E3, "ea", "ra", "eb", "rb") \
  "s_sub_u32 %[n], %[n], 4\n" \
  ".Lbhc_loop%=:\n" \
  "s_add_u32 s84, s84, 0x80\n" \
  "s_add_u32 s86, s86, 0x40\n" \
  BH_CA_LOAD \
  "s_cmp_le_i32 %[n], 4\n" \
  "s_cbranch_scc1 .Lbhc_last%=\n" \
  BH_CA_STEP_(BH_CA_E0, "eb", "rb", "ea", "ra") \
  BH_CA_STEP_(BH_CA_E1, "ea", "ra", "eb", "rb") \
  BH_CA_STEP_(BH_CA_E2, "eb", "rb", "ea", "ra") \
  BH_CA_STEP_(BH_CA_E3, "ea", "ra", "eb", "rb") \
  "s_sub_u32 %[n], %[n], 4\n" \
  "s_branch .Lbhc_loop%=\n" \
  ".Lbhc_last%=:\n" \
  "s_cmp_eq_u32 %[n], 1\n" \
  "s_cbranch_scc1 .Lbhc_l1%=\n" \
  BH_CA_STEP_(BH_CA_E0, "eb", "rb", "ea", "ra") \
  "s_cmp_eq_u32 %[n], 2\n" \
  "s_cbranch_scc1 .Lbhc_l2%=\n" \
  BH_CA_STEP_(BH_CA_E1, "ea", "ra", "eb", "rb") \
  "s_cmp_eq_u32 %[n], 3\n" \
  "s_cbranch_scc1 .Lbhc_l3%=\n" \
  BH_CA_STEP_(BH_CA_E2, "eb", "rb", "ea", "ra") \
  BH_CA_ACC_(BH_CA_X3, "ea", "ra") \
  "s_branch .Lbhc_end%=\n" \
  ".Lbhc_f2%=:\n" \
  BH_CA_ACC_(BH_CA_X1, "ea", "ra") \
  "s_branch .Lbhc_end%=\n" \
  ".Lbhc_f3%=:\n" \
  BH_CA_ACC_(BH_CA_X2, "eb", "rb") \
  "s_branch .Lbhc_end%=\n" \
  ".Lbhc_f4%=:\n" \
  BH_CA_ACC_(BH_CA_X3, "ea", "ra") \
  "s_branch .Lbhc_end%=\n" \
  ".Lbhc_l1%=:\n" \
  BH_CA_ACC_(BH_CA_X0, "eb", "rb") \
  "s_branch .Lbhc_end%=\n" \
  ".Lbhc_l2%=:\n" \
  BH_CA_ACC_(BH_CA_X1, "ea", "ra") \
  "s_branch .Lbhc_end%=\n" \
  ".Lbhc_l3%=:\n" \
  BH_CA_ACC_(BH_CA_X2, "eb", "rb") \
  ".Lbhc_end%=:\n"

// Class epilogue: the class's chain sums into the score, the alpha/gamma
// sums SP, SQ of its p-group and the x-gradient, with the phase weights
// W1, W2 of the class (the same fma sequence as the compiled epilogue).
#define BH_CA_EPI_(D)                                \
  "v_fmac_f64 %[S], %[w1r], %[t1r]\n"                \
  "v_fma_f64 %[S], -%[w1i], %[t1i], %[S]\n"          \
  "v_fmac_f64 %[S], %[w2r], %[t2r]\n"                \
  "v_fma_f64 %[S], -%[w2i], %[t2i], %[S]\n"          \
  "v_fmac_f64 %[SP], %[w1r], %[t1i]\n"               \
  "v_fmac_f64 %[SP], %[w1i], %[t1r]\n"               \
  "v_fmac_f64 %[SP], %[w2r], %[t2i]\n"               \
  "v_fmac_f64 %[SP], %[w2i], %[t2r]\n"               \
  "v_mul_f64 %[" D "], %[w1r], %[t1i]\n"                 \
  "v_fmac_f64 %[" D "], %[w1i], %[t1r]\n"                \
  "v_fma_f64 %[" D "], -%[w2r], %[t2i], %[" D "]\n"          \
  "v_fma_f64 %[" D "], -%[w2i], %[t2r], %[" D "]\n"          \
  "v_fmac_f64 %[SQ], %[qd], %[" D "]\n"                  \
  "v_fmac_f64 %[gb], %[w1r], %[r1r]\n"               \
  "v_fma_f64 %[gb], -%[w1i], %[r1i], %[gb]\n"        \
  "v_fmac_f64 %[gb], %[w2r], %[r2r]\n"               \
  "v_fma_f64 %[gb], -%[w2i], %[r2i], %[gb]\n"
// The next class's W1 *= e^{-2i delta}, W2 *= e^{+2i delta}, s^q, q.
#define BH_CA_ROT_(D)                                \
  "v_mul_f64 %[" D "], %[w1i], %[th2i]\n"                \
  "v_mul_f64 %[u], %[w1r], %[th2i]\n"                \
  "v_fma_f64 %[w1r], %[w1r], %[th2r], -%[" D "]\n"       \
  "v_fma_f64 %[w1i], %[w1i], %[th2r], %[u]\n"        \
  "v_mul_f64 %[" D "], %[w2r], %[th2r]\n"                \
  "v_mul_f64 %[u], %[w2r], %[th2i]\n"                \
  "v_fma_f64 %[w2r], %[w2i], %[th2i], %[" D "]\n"        \
  "v_fma_f64 %[w2i], %[w2i], %[th2r], -%[u]\n"       \
  "v_mul_f64 %[sq], %[sq], %[s2]\n"                  \
  "v_add_f64 %[qd], %[qd], 2.0\n"
#define BH_CA_CLOBBERS                                                                     \
  "s36", "s37", "s38", "s39", "s40", "s41", "s42", "s43", "s44", "s45", "s46", "s47", "s48", \
      "s49", "s50", "s51", "s52", "s53", "s54", "s55", "s56", "s57", "s58", "s59", "s60",    \
      "s61", "s62", "s63", "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "s72",    \
      "s73", "s74", "s75", "s76", "s77", "s78", "s79", "s80", "s81", "s82", "s83", "s84",    \
      "s85", "s86", "scc", "memory"

// One class of a p-group as one asm block: the class's first-round loads
// are issued first, and while they are in flight the previous class's
// epilogue (if `prev`) and phase rotation run and this class's seeds
// e_m = c^p s^q, de_m/dx = e_m (p / 4c^2 - q / 4s^2) are formed; then the
// chain.  (t1r .. r2i): in, the previous class's chain sums; out, this
// class's.  S, SP, SQ, gb accumulate; W1, W2, sq, qd advance to this class.
__device__ inline void class_step_asm(int prev, const void* xc, const void* rc, int n, double x,
                                      double th2r, double th2i, double s2, double is2,
                                      double pic2, double cp, double& t1r, double& t1i,
                                      double& t2r, double& t2i, double& r1r, double& r1i,
                                      double& r2r, double& r2i, double& S, double& SP,
                                      double& SQ, double& gb, double& w1r, double& w1i,
                                      double& w2r, double& w2i, double& sq, double& qd) {
  double ea, ra, u, eb, rb;   // ea also serves the epilogue
  asm volatile(
      "s_mov_b32 s84, 0\n"
      "s_mov_b32 s86, 0\n"
      "s_add_u32 s85, s84, 0x40\n"
      "s_load_dwordx16 s[36:51], %[xc], s84\n"
      "s_load_dwordx16 s[52:67], %[xc], s85\n"
      "s_load_dwordx16 s[68:83], %[rc], s86\n"
      "s_cmp_eq_u32 %[prev], 0\n"
      "s_cbranch_scc1 .Lbhc_seed%=\n"
      BH_CA_EPI_("ea")
      BH_CA_ROT_("ea")
      ".Lbhc_seed%=:\n"
      "v_mul_f64 %[eb], %[cp], %[sq]\n"
      "v_fma_f64 %[rb], -%[qd], %[is2], %[pic2]\n"
      "v_mul_f64 %[rb], %[eb], %[rb]\n"
      "s_waitcnt lgkmcnt(0)\n"
      BH_CA_CHAIN
      : [t1r] "+v"(t1r), [t1i] "+v"(t1i), [t2r] "+v"(t2r), [t2i] "+v"(t2i), [r1r] "+v"(r1r),
        [r1i] "+v"(r1i), [r2r] "+v"(r2r), [r2i] "+v"(r2i), [S] "+v"(S), [SP] "+v"(SP),
        [SQ] "+v"(SQ), [gb] "+v"(gb), [w1r] "+v"(w1r), [w1i] "+v"(w1i), [w2r] "+v"(w2r),
        [w2i] "+v"(w2i), [sq] "+v"(sq), [qd] "+v"(qd), [ea] "=&v"(ea), [ra] "=&v"(ra),
        [u] "=&v"(u), [eb] "=&v"(eb), [rb] "=&v"(rb), [n] "+s"(n)
      : [x] "v"(x), [th2r] "v"(th2r), [th2i] "v"(th2i), [s2] "v"(s2), [is2] "v"(is2),
        [pic2] "v"(pic2), [cp] "v"(cp), [xc] "s"(xc), [rc] "s"(rc), [prev] "s"(prev)
      : BH_CA_CLOBBERS);
}

// The last class's epilogue of a p-group.
__device__ inline void class_epilogue_asm(double t1r, double t1i, double t2r, double t2i,
                                          double r1r, double r1i, double r2r, double r2i,
                                          double w1r, double w1i, double w2r, double w2i,
                                          double qd, double& S, double& SP, double& SQ,
                                          double& gb) {
  double d;
  asm volatile(BH_CA_EPI_("d")
               : [S] "+v"(S), [SP] "+v"(SP), [SQ] "+v"(SQ), [gb] "+v"(gb), [d] "=&v"(d)
               : [t1r] "v"(t1r), [t1i] "v"(t1i), [t2r] "v"(t2r), [t2i] "v"(t2i),
                 [r1r] "v"(r1r), [r1i] "v"(r1i), [r2r] "v"(r2r), [r2i] "v"(r2i),
                 [w1r] "v"(w1r), [w1i] "v"(w1i), [w2r] "v"(w2r), [w2i] "v"(w2i), [qd] "v"(qd));
}
#undef BH_CA_ACC_
#undef BH_CA_STEP_
#endif

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
// needed.  Without Hessian terms and with wave-uniform weights the chain
// runs as one asm block (chain_sums_asm) that also takes the peeled entry
// into the first round and the tail into one last round.
//
// Class epilogue: with W1 = e^{-i p sigma} e^{-i q delta} and W2 =
// e^{-i p sigma} e^{+i q delta} (advanced by e^{-+2i delta} per class), the
// class adds Re(W1 t1 + W2 t2) to S and Re(W1 r1 + W2 r2) to the x-gradient;
// the alpha and gamma derivatives m I1 + n I2 and n I1 + m I2 (I = Im(W t))
// are accumulated as (p SP +- SQ) / 2 with SP = sum (I1 + I2) and
// SQ = sum q (I1 - I2) over the p-group.
//
// HESS (second derivatives, m = (p+q)/2, n = (p-q)/2; chains in beta):
//   d2/dalpha2  = -sum m^2 Re z1 + n^2 Re z2,  d2/dgamma2 with m, n swapped,
//   d2/dalpha dgamma = -sum mn (Re z1 + Re z2)   (z = W t),
// written with the per-p sums A0 = sum (Re z1 + Re z2), A2 = sum q^2 (...),
// B1 = sum q (Re z1 - Re z2); the mixed beta terms m Im(W1 r1) + n Im(W2 r2)
// (and swapped) through ZP, ZQ as SP, SQ; d2/dbeta2 = Re(W1 q1 + W2 q2).
// Without MSB (and HESS) the x-gradient sum is returned unscaled, for a
// caller that applies -sin(beta) itself (from memory it reads afterwards,
// rather than holding it in a register through the evaluation).
template <bool HESS, bool XU = true, bool MSB = true>
BH_HD inline Acc eval_wave(const Angles& A, const int32_t* __restrict__ plist, int L,
                           const int32_t* __restrict__ p_first,
                           const double* __restrict__ rec, const double* __restrict__ X) {
  Acc acc = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int np = plist[0];
#if !BH_SCORE_PHASE_SINCOS
  // Phi = e^{-i pc sigma} and cp = c^pc, advanced along the ascending
  // p-list one degree at a time.
  const cplx E1 = A.e1;
  cplx Phi = {1.0, 0.0};
  double cp = 1.0;
  int pc = 0;
#endif
  const double s2 = A.s * A.s;
  const cplx th2c = {A.th2.re, -A.th2.im};
  double qsum = 0.0, zpx = 0.0, zgx = 0.0;     // HESS: sum Re(W q), mixed-beta sums
  const double mx = -A.x;
  // HESS: c^{p-2} .. c^{p+2} (negative powers stand as 0: their
  // coefficients vanish), advanced with p
  double cw[5] = {0.0, 0.0, 1.0, A.c, A.c * A.c};
  int pw = 0;
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
    if constexpr (HESS) {
      for (; pw < p; ++pw) {
        cw[0] = cw[1];
        cw[1] = cw[2];
        cw[2] = cw[3];
        cw[3] = cw[4];
        cw[4] *= A.c;
      }
    }
    int off = p_first[p];
    const int q0 = p & 1;
    cplx W1 = q0 ? cmul(Phi, A.th1) : Phi;
    cplx W2 = q0 ? cmulc(Phi, A.th1) : Phi;
    double sq = q0 ? A.s : 1.0;       // s^q
    double qd = (double)q0;
    double SP = 0.0, SQ = 0.0;
    double A0 = 0.0, A2 = 0.0, B1 = 0.0, ZP = 0.0, ZQ = 0.0;
    // HESS: s^{q-2} .. s^{q+2} (as cw), advanced by two per class
    double sw[5] = {0.0, q0 ? 1.0 : 0.0, q0 ? A.s : 1.0, q0 ? s2 : A.s, q0 ? s2 * A.s : s2};
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (!HESS && XU) {
      // the classes of the p-group as asm blocks, each running the previous
      // class's epilogue while its own first loads are in flight
      double t1r = 0.0, t1i = 0.0, t2r = 0.0, t2i = 0.0, r1r = 0.0, r1i = 0.0, r2r = 0.0,
             r2i = 0.0;
      double w1r = W1.re, w1i = W1.im, w2r = W2.re, w2i = W2.im;
      int prev = 0;
      for (int q = q0; q <= 2 * L - p; q += 2) {
        const int n = L - ((p + q) >> 1) + 1;
        class_step_asm(prev, reinterpret_cast<const double4*>(X) + off,
                       reinterpret_cast<const double2*>(rec) + off, n, A.x, A.th2.re, A.th2.im,
                       s2, A.is2, pic2, cp, t1r, t1i, t2r, t2i, r1r, r1i, r2r, r2i, acc.S, SP,
                       SQ, acc.gb, w1r, w1i, w2r, w2i, sq, qd);
        prev = 1;
        off += class_span(n);
      }
      class_epilogue_asm(t1r, t1i, t2r, t2i, r1r, r1i, r2r, r2i, w1r, w1i, w2r, w2i, qd, acc.S,
                         SP, SQ, acc.gb);
    } else
#endif
    for (int q = q0; q <= 2 * L - p; q += 2) {
      const int m = (p + q) >> 1;
      const int rem = L - m;          // chain entries after the first
      const double4* Xc = reinterpret_cast<const double4*>(X) + off;
      const double2* Rc = reinterpret_cast<const double2*>(rec) + off;
      // seeds: e_m = c^p s^q and de_m/dx = e_m (p / (4c^2) - q / (4s^2)); with
      // HESS de_m/dbeta = (q c^{p+1} s^{q-1} - p c^{p-1} s^{q+1}) / 2 and
      // d2e_m/dbeta2 = (q(q-1) c^{p+2} s^{q-2} + p(p-1) c^{p-2} s^{q+2}
      //                 - (q(p+1) + p(q+1)) c^p s^q) / 4.
      // The peeled first step starts the sums and yields e_{m+1}.
      double eb, rb, qb = 0.0;
      if constexpr (HESS) {
        const double pd = (double)p;
        eb = cw[2] * sw[2];
        rb = 0.5 * (qd * cw[3] * sw[1] - pd * cw[1] * sw[3]);
        qb = 0.25 * (qd * (qd - 1.0) * cw[4] * sw[0] + pd * (pd - 1.0) * cw[0] * sw[4] -
                     (qd * (pd + 1.0) + pd * (qd + 1.0)) * eb);
      } else {
        eb = cp * sq;
        rb = eb * fma(-qd, A.is2, pic2);
      }
      double t1r, t1i, t2r, t2i, r1r, r1i, r2r, r2i;
      double q1r = 0.0, q1i = 0.0, q2r = 0.0, q2i = 0.0;
      {
        double ea, ra, qa = 0.0;
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
          if constexpr (HESS) {
            q1r = x0.x * qb;
            q1i = x0.y * qb;
            q2r = x0.z * qb;
            q2i = x0.w * qb;
            const double du_ = c0_.x * A.msb;
            qa = fma(c0_.x * mx, eb, fma(du_ + du_, rb, u_ * qb));
            ra = fma(du_, eb, u_ * rb);
          } else {
            ra = fma(c0_.x, eb, u_ * rb);
          }
        }
        // Full rounds of four entries: straight-line code, one load batch and
        // one wait per round.  Then a tail of two and/or one entries.
        const int n4 = rem & ~3;
        int i = 1;
        for (; i <= n4; i += 4) {
          const double4 x0 = Xc[i], x1 = Xc[i + 1], x2 = Xc[i + 2], x3 = Xc[i + 3];
          const double2 c0_ = Rc[i], c1 = Rc[i + 1], c2 = Rc[i + 2], c3 = Rc[i + 3];
          BH_CHAIN_STEP(x0, c0_, ea, ra, qa, eb, rb, qb);
          BH_CHAIN_STEP(x1, c1, eb, rb, qb, ea, ra, qa);
          BH_CHAIN_STEP(x2, c2, ea, ra, qa, eb, rb, qb);
          BH_CHAIN_STEP(x3, c3, eb, rb, qb, ea, ra, qa);
        }
        if (rem & 2) {
          const double4 x0 = Xc[i], x1 = Xc[i + 1];
          const double2 c0_ = Rc[i], c1 = Rc[i + 1];
          BH_CHAIN_STEP(x0, c0_, ea, ra, qa, eb, rb, qb);
          BH_CHAIN_STEP(x1, c1, eb, rb, qb, ea, ra, qa);
          i += 2;
        }
        if (rem & 1) {
          const double4 x0 = Xc[i];
          const double2 c0_ = Rc[i];
          BH_CHAIN_STEP(x0, c0_, ea, ra, qa, eb, rb, qb);
        }
      }
      if constexpr (HESS) {
        const double z1 = fma(W1.re, t1r, -W1.im * t1i);
        const double z2 = fma(W2.re, t2r, -W2.im * t2i);
        const double zs = z1 + z2;
        acc.S += zs;
        A0 += zs;
        A2 = fma(qd * qd, zs, A2);
        B1 = fma(qd, z1 - z2, B1);
        const double y1 = fma(W1.re, r1i, W1.im * r1r);
        const double y2 = fma(W2.re, r2i, W2.im * r2r);
        ZP += y1 + y2;
        ZQ = fma(qd, y1 - y2, ZQ);
        qsum = fma(W1.re, q1r, qsum);
        qsum = fma(-W1.im, q1i, qsum);
        qsum = fma(W2.re, q2r, qsum);
        qsum = fma(-W2.im, q2i, qsum);
      } else {
        acc.S = fma(W1.re, t1r, acc.S);
        acc.S = fma(-W1.im, t1i, acc.S);
        acc.S = fma(W2.re, t2r, acc.S);
        acc.S = fma(-W2.im, t2i, acc.S);
      }
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
      off += class_span(rem + 1);
      W1 = cmul(W1, A.th2);
      W2 = cmul(W2, th2c);
      sq *= s2;
      qd += 2.0;
      if constexpr (HESS) {
        sw[0] = sw[2];
        sw[1] = sw[3];
        sw[2] = sw[4];
        sw[3] *= s2;
        sw[4] *= s2;
      }
    }
    const double pd = (double)p;
    const double pSP = pd * SP;
    acc.ga += 0.5 * (pSP + SQ);
    acc.gg += 0.5 * (pSP - SQ);
    if constexpr (HESS) {
      const double pp = pd * pd * A0;
      acc.haa -= 0.25 * (pp + A2 + 2.0 * pd * B1);
      acc.hgg -= 0.25 * (pp + A2 - 2.0 * pd * B1);
      acc.hag -= 0.25 * (pp - A2);
      zpx += 0.5 * (pd * ZP + ZQ);
      zgx += 0.5 * (pd * ZP - ZQ);
    }
  }
  if constexpr (HESS) {
    acc.hab = zpx;
    acc.hbg = zgx;
    acc.hbb = qsum;
  } else if constexpr (MSB) {
    acc.gb *= A.msb;
  }
  return acc;
}

// ------------------------------------------------- staged packed Hessian --
//
// The packed Newton evaluator (64 / G particles per wave, G lanes each)
// reads its weights X from an LDS ring that LDS-DMA loads fill several
// blocks ahead.  A block is four chain entries of every particle of the
// wave (64 / G x 128 bytes, one DMA instruction); blocks follow the wave's
// classes in evaluation order, each class starting a new block.  In a
// block, particle g's 16-byte chunk j sits at g * 128 + (j ^ g) * 16, so the
// reads of one entry by the wave's particles hit distinct bank groups.
// Vector loads return in order, so "this block has landed" is a wait for
// the number of blocks issued after it.
template <int G>
struct XRing {
  static constexpr int PER = 64 / G;
  static constexpr int kBlocks = 8, kAhead = kBlocks - 1, kBlockBytes = 1024;
  char* ring;                 // this wave's kBlocks blocks of LDS
  const char* src;            // DMA source of this lane (lanes < 8 PER): its particle and chunk
  bool dma_lane;
  const int32_t* plist;
  const int32_t* p_first;
  int L, np;
  int ij, ip, iq, ioff, in, ik;   // issue position: p-list index, p, q, class offset and size, block
  int issued, consumed;

  __device__ void start(char* ring_, const double* X, int64_t n_entries, int64_t pb0, int64_t B,
                        const int32_t* plist_, const int32_t* p_first_, int L_) {
    ring = ring_;
    plist = plist_;
    p_first = p_first_;
    L = L_;
    np = plist[0];
    const int lane = (int)(threadIdx.x & 63);
    const int g = lane >> 3, j = (lane & 7) ^ (g & 7);
    dma_lane = g < PER;
    int64_t pd = pb0 + (dma_lane ? g : 0);
    if (pd > B - 1) pd = B - 1;
    src = reinterpret_cast<const char*>(X + pd * n_entries * 4) + 16 * j;
    issued = consumed = 0;
    ij = 0;
    if (np > 0) {
      ip = plist[1];
      iq = ip & 1;
      ioff = p_first[ip];
      in = L - ((ip + iq) >> 1) + 1;
      ik = 0;
    }
    while (issued < kAhead && ij < np) issue();
  }
  __device__ void issue() {
    typedef __attribute__((address_space(1))) void global_void;
    typedef __attribute__((address_space(3))) void lds_void;
    char* dst = ring + (issued % kBlocks) * kBlockBytes;
    if (dma_lane)
      __builtin_amdgcn_global_load_lds((global_void*)(src + (int64_t)(ioff + 4 * ik) * 32),
                                       (lds_void*)dst, 16, 0, 0);
    ++issued;
    if (4 * ++ik < in) return;
    ik = 0;
    ioff += class_span(in);
    iq += 2;
    if (iq > 2 * L - ip) {
      if (++ij >= np) return;
      ip = plist[1 + ij];
      iq = ip & 1;
      ioff = p_first[ip];
    }
    in = L - ((ip + iq) >> 1) + 1;
  }
  // The next block in evaluation order, landed; first tops up the ring
  // (the slot refilled is the block consumed last, whose reads returned
  // before ring_block finished).
  __device__ const char* next() {
    if (ij < np) issue();
    const int younger = issued - consumed - 1;
    switch (younger) {   // kAhead == 7
      case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
      case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
      case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
      case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
      case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
      case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
      case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
      default: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
    }
    const char* b = ring + (consumed % kBlocks) * kBlockBytes;
    ++consumed;
    return b;
  }
};
static_assert(XRing<8>::kAhead == 7, "the wait table covers 0..7 younger blocks");

// The four entries of a block for particle gq of the wave.  The reads are
// written out, with their wait, because the compiler would otherwise wait
// for every LDS-DMA load in flight before any read of the ring.  Every
// output is early-clobber: a read's result may land while later reads of
// the block still need their addresses.
struct Block4 {
  double4 x[4];
};
__device__ inline Block4 ring_block(const char* blk, int gq) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(3))) const char lds_char;
  const uint32_t base = (uint32_t)(uintptr_t)(lds_char*)(blk + gq * 128);
  uint32_t a[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) a[c] = base + (uint32_t)((c ^ gq) * 16);
  d2 v0, v1, v2, v3, v4, v5, v6, v7;
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %9\n\t"
      "ds_read_b128 %2, %10\n\t"
      "ds_read_b128 %3, %11\n\t"
      "ds_read_b128 %4, %12\n\t"
      "ds_read_b128 %5, %13\n\t"
      "ds_read_b128 %6, %14\n\t"
      "ds_read_b128 %7, %15\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3), "=&v"(v4), "=&v"(v5), "=&v"(v6), "=&v"(v7)
      : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7])
      : "memory");
  Block4 b;
  b.x[0] = {v0.x, v0.y, v1.x, v1.y};
  b.x[1] = {v2.x, v2.y, v3.x, v3.y};
  b.x[2] = {v4.x, v4.y, v5.x, v5.y};
  b.x[3] = {v6.x, v6.y, v7.x, v7.y};
  return b;
}

// eval_wave<true> with the weights from the ring (same arithmetic, same order).
template <int G>
__device__ inline Acc eval_wave_staged(const Angles& A, const int32_t* __restrict__ plist, int L,
                                       const int32_t* __restrict__ p_first,
                                       const double* __restrict__ rec, XRing<G>& xr) {
  constexpr bool HESS = true;
  Acc acc = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int np = plist[0];
  const int gq = (int)(threadIdx.x & 63) / G;
  const cplx E1 = A.e1;
  cplx Phi = {1.0, 0.0};
  int pc = 0;
  const double s2 = A.s * A.s;
  const cplx th2c = {A.th2.re, -A.th2.im};
  double qsum = 0.0, zpx = 0.0, zgx = 0.0;
  const double mx = -A.x;
  double cw[5] = {0.0, 0.0, 1.0, A.c, A.c * A.c};
  int pw = 0;
  for (int j = 0; j < np; ++j) {
    const int p = plist[1 + j];
    for (; pc < p; ++pc) Phi = cmul(Phi, E1);
    for (; pw < p; ++pw) {
      cw[0] = cw[1];
      cw[1] = cw[2];
      cw[2] = cw[3];
      cw[3] = cw[4];
      cw[4] *= A.c;
    }
    int off = p_first[p];
    const int q0 = p & 1;
    cplx W1 = q0 ? cmul(Phi, A.th1) : Phi;
    cplx W2 = q0 ? cmulc(Phi, A.th1) : Phi;
    double qd = (double)q0;
    double SP = 0.0, SQ = 0.0;
    double A0 = 0.0, A2 = 0.0, B1 = 0.0, ZP = 0.0, ZQ = 0.0;
    double sw[5] = {0.0, q0 ? 1.0 : 0.0, q0 ? A.s : 1.0, q0 ? s2 : A.s, q0 ? s2 * A.s : s2};
    for (int q = q0; q <= 2 * L - p; q += 2) {
      const int m = (p + q) >> 1;
      const int n = L - m + 1;        // chain entries
      const double2* Rc = reinterpret_cast<const double2*>(rec) + off;
      const double pd = (double)p;
      double eb = cw[2] * sw[2];
      double rb = 0.5 * (qd * cw[3] * sw[1] - pd * cw[1] * sw[3]);
      double qb = 0.25 * (qd * (qd - 1.0) * cw[4] * sw[0] + pd * (pd - 1.0) * cw[0] * sw[4] -
                          (qd * (pd + 1.0) + pd * (qd + 1.0)) * eb);
      double t1r, t1i, t2r, t2i, r1r, r1i, r2r, r2i, ea, ra, qa;
      double q1r, q1i, q2r, q2i;
      // A block's four recurrence entries are loaded before its ring reads,
      // whose wait then covers them too (one wait per block, not one per
      // entry); the last block's loads may read past the chain (padding).
      double2 rc0 = Rc[0], rc1 = Rc[1], rc2 = Rc[2], rc3 = Rc[3];
      Block4 xb = ring_block(xr.next(), gq);
      {
        const double4 x0 = xb.x[0];
        const double2 c0_ = rc0;
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
        q1r = x0.x * qb;
        q1i = x0.y * qb;
        q2r = x0.z * qb;
        q2i = x0.w * qb;
        const double du_ = c0_.x * A.msb;
        qa = fma(c0_.x * mx, eb, fma(du_ + du_, rb, u_ * qb));
        ra = fma(du_, eb, u_ * rb);
      }
      for (int i0 = 0; i0 < n; i0 += 4) {
        if (i0 > 0) {
          rc0 = Rc[i0];
          rc1 = Rc[i0 + 1];
          rc2 = Rc[i0 + 2];
          rc3 = Rc[i0 + 3];
          xb = ring_block(xr.next(), gq);
          const double4 x0 = xb.x[0];
          BH_CHAIN_STEP(x0, rc0, eb, rb, qb, ea, ra, qa);
        }
        if (i0 + 1 < n) {
          const double4 x1 = xb.x[1];
          BH_CHAIN_STEP(x1, rc1, ea, ra, qa, eb, rb, qb);
        }
        if (i0 + 2 < n) {
          const double4 x2 = xb.x[2];
          BH_CHAIN_STEP(x2, rc2, eb, rb, qb, ea, ra, qa);
        }
        if (i0 + 3 < n) {
          const double4 x3 = xb.x[3];
          BH_CHAIN_STEP(x3, rc3, ea, ra, qa, eb, rb, qb);
        }
      }
      const double z1 = fma(W1.re, t1r, -W1.im * t1i);
      const double z2 = fma(W2.re, t2r, -W2.im * t2i);
      const double zs = z1 + z2;
      acc.S += zs;
      A0 += zs;
      A2 = fma(qd * qd, zs, A2);
      B1 = fma(qd, z1 - z2, B1);
      const double y1 = fma(W1.re, r1i, W1.im * r1r);
      const double y2 = fma(W2.re, r2i, W2.im * r2r);
      ZP += y1 + y2;
      ZQ = fma(qd, y1 - y2, ZQ);
      qsum = fma(W1.re, q1r, qsum);
      qsum = fma(-W1.im, q1i, qsum);
      qsum = fma(W2.re, q2r, qsum);
      qsum = fma(-W2.im, q2i, qsum);
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
      off += class_span(n);
      W1 = cmul(W1, A.th2);
      W2 = cmul(W2, th2c);
      qd += 2.0;
      sw[0] = sw[2];
      sw[1] = sw[3];
      sw[2] = sw[4];
      sw[3] *= s2;
      sw[4] *= s2;
    }
    const double pd = (double)p;
    const double pSP = pd * SP;
    acc.ga += 0.5 * (pSP + SQ);
    acc.gg += 0.5 * (pSP - SQ);
    const double pp = pd * pd * A0;
    acc.haa -= 0.25 * (pp + A2 + 2.0 * pd * B1);
    acc.hgg -= 0.25 * (pp + A2 - 2.0 * pd * B1);
    acc.hag -= 0.25 * (pp - A2);
    zpx += 0.5 * (pd * ZP + ZQ);
    zgx += 0.5 * (pd * ZP - ZQ);
  }
  acc.hab = zpx;
  acc.hbg = zgx;
  acc.hbb = qsum;
  return acc;
}

#undef BH_CHAIN_STEP

}  // namespace bh
