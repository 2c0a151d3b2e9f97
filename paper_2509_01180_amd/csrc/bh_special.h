// Special functions shared by the host tables and the device basis build.
//
// Spherical Bessel functions of the first kind j_l(x) (Sec. II-A: radial
// factor of psi_klm, and the zeros lambda_lk).  For l < x the three-term
// recurrence j_{n+1} = (2n+1)/x j_n - j_{n-1} is run upward from the closed
// forms of j_0, j_1 (both solutions oscillate there, so it is stable); for
// l >= x it is run downward from n = l + 60 (Miller's method), rescaled to
// stay in range, and normalised by whichever of j_0, j_1 is larger.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define BH_HD __host__ __device__
#else
#define BH_HD
#endif

BH_HD inline double bh_sph_jn(int l, double x) {
  if (x < 0.0) x = -x;
  if (x == 0.0) return l == 0 ? 1.0 : 0.0;
  const double s = sin(x), c = cos(x);
  const double j0 = s / x;
  if (l == 0) return j0;
  // Closed form of j_1; it cancels for small x, where Miller is used instead.
  const double j1 = s / (x * x) - c / x;
  if ((double)l < x) {
    double jm = j0, jc = j1;
    for (int n = 1; n < l; ++n) {
      const double jn = (2.0 * n + 1.0) / x * jc - jm;
      jm = jc;
      jc = jn;
    }
    return jc;
  }
  // Miller: downward from n0 with f_{n0+1} = 0, f_{n0} = tiny.
  const int n0 = l + 60;
  double fp = 0.0, fc = 1e-250, fl = 0.0, f1 = 0.0, f0 = 0.0;
  for (int n = n0; n >= 1; --n) {
    const double fm = (2.0 * n + 1.0) / x * fc - fp;   // f_{n-1}
    fp = fc;
    fc = fm;
    if (n == l + 1) fl = fc;                          // f_l
    if (fabs(fc) > 1e200) {                           // rescale everything kept
      fp *= 1e-200;
      fc *= 1e-200;
      fl *= 1e-200;
      f1 *= 1e-200;
    }
    if (n == 2) f1 = fc;                              // f_1
  }
  f0 = fc;
  // For x <= l the larger of j_0, j_1 is j_0 whenever x < 1, so the
  // cancelling closed form of j_1 is only used where it is accurate.
  return (fabs(j0) >= fabs(j1)) ? fl * (j0 / f0) : fl * (j1 / f1);
}
