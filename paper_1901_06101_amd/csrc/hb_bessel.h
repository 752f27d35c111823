// Bessel functions J_0 and Y_0 of a positive real argument, for the EFIE2D
// kernel H_0^(2)(x) = J_0(x) - i Y_0(x) (Section "Numerical Results",
// kernel 2), to full double precision.
//
//  * x < 25: Miller's backward recurrence J_{n-1} = (2n / x) J_n - J_{n+1}
//    started far above x with arbitrary values, normalised by
//    J_0 + 2 (J_2 + J_4 + ...) = 1 (Abramowitz and Stegun 9.1.46); Y_0 from
//    Neumann's series Y_0 = (2/pi) (ln(x/2) + gamma) J_0
//    - (4/pi) sum_k (-1)^k J_{2k} / k (Abramowitz and Stegun 9.1.88) over
//    the same recurrence values.  The recurrence is stable downwards; values
//    are rescaled before they can overflow.
//  * x >= 25: Hankel's asymptotic expansion (Abramowitz and Stegun 9.2.5,
//    9.2.6, 9.2.9, 9.2.10 with nu = 0): J_0 = sqrt(2/(pi x)) (P cos chi -
//    Q sin chi), Y_0 = sqrt(2/(pi x)) (P sin chi + Q cos chi), chi =
//    x - pi/4, summed until the terms fall below 1e-17 (the smallest term
//    near 2x is about exp(-2x) < 1e-21 here).
//
// The functions compile for the device and, for the host tests of this
// code, for the host.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define HB_BESSEL_FN __host__ __device__ inline
#else
#define HB_BESSEL_FN inline
#endif

HB_BESSEL_FN void hb_bessel_j0y0(double x, double* j0v, double* y0v) {
  const double kPi = 3.14159265358979323846;
  const double kGamma = 0.57721566490153286061;  // Euler's constant
  if (x < 25.0) {
    // start index: even, well above x so that J_N is negligible
    int n0 = (int)(x + 20.0 + 10.0 * cbrt(x));
    n0 += n0 & 1;
    double jp = 0.0;      // J_{n+1}
    double jc = 1e-300;   // J_n (arbitrary start)
    double norm = 0.0;    // J_0 + 2 sum J_{2k}
    double neu = 0.0;     // sum_{k>=1} (-1)^k J_{2k} / k
    const double ix = 1.0 / x;
    for (int n = n0; n >= 1; --n) {
      // at even n the current value is J_n: add it to the sums
      if ((n & 1) == 0) {
        norm += 2.0 * jc;
        const int k = n / 2;
        neu += ((k & 1) ? -jc : jc) / (double)k;
      }
      const double jm = 2.0 * n * ix * jc - jp;  // J_{n-1}
      jp = jc;
      jc = jm;
      if (fabs(jc) > 1e250) {  // rescale everything carried so far
        jc *= 1e-250;
        jp *= 1e-250;
        norm *= 1e-250;
        neu *= 1e-250;
      }
    }
    norm += jc;  // J_0
    const double j0 = jc / norm;
    *j0v = j0;
    *y0v = (2.0 / kPi) * ((log(0.5 * x) + kGamma) * j0 - 2.0 * neu / norm);
    return;
  }
  // Hankel's expansion with mu = 4 nu^2 = 0: b_m = prod_{j<=m} (2j-1)^2 /
  // (m! (8x)^m); P = sum_k (-1)^k b_{2k}, Q = sum_k (-1)^(k+1) b_{2k+1}
  double P = 1.0, Q = 0.0, b = 1.0;
  const double i8x = 1.0 / (8.0 * x);
  for (int m = 1; m <= 60; ++m) {
    b *= (double)(2 * m - 1) * (double)(2 * m - 1) / (double)m * i8x;
    const int k = m / 2;
    if (m & 1) Q += (k & 1) ? b : -b;
    else P += (k & 1) ? -b : b;
    if (b < 1e-17) break;
  }
  // cos and sin of chi = x - pi/4 from those of x (no rounding of pi/4 into x)
  double s, c;
  sincos(x, &s, &c);
  const double r2 = 0.70710678118654752440;
  const double cchi = (c + s) * r2, schi = (s - c) * r2;
  const double a = sqrt(2.0 / (kPi * x));
  *j0v = a * (P * cchi - Q * schi);
  *y0v = a * (P * schi + Q * cchi);
}
