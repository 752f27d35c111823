// Host build of the kernel library's J_0 / Y_0 (hb_bessel.h), for the CPU
// test that compares it with SciPy's Bessel routines.
#include "../../paper_1901_06101_amd/csrc/hb_bessel.h"

extern "C" void hb_host_j0y0(const double* x, double* j0, double* y0, long n) {
  for (long i = 0; i < n; ++i) hb_bessel_j0y0(x[i], j0 + i, y0 + i);
}
