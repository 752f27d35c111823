// On-the-fly matrix entries (device side).
//
// The method assumes every entry A(i, j) can be computed in O(1) (Abstract;
// the kernels are listed in Section "Numerical Results").  Points are held
// structure-of-arrays: coordinate c of row point i is X[c * ldx + i].
#pragma once

#include "hb_bessel.h"
#include "hb_common.h"

enum hb_kind_dev {
  HBK_GAUSS = 1,          // exp(-|x - y|^2 / (c h^2))
  HBK_LAPLACE = 2,        // 1 / |x - y|
  HBK_HELMHOLTZ = 3,      // exp(i k |x - y|) / (4 pi |x - y|)  (complex)
  HBK_LOWRANK_SPIKES = 4, // (G1 G2)(i, j) + spike(i, j)
  HBK_EFIE2D = 5,         // H_0^(2)(k |x - y|) = J_0 - i Y_0  (complex)
  HBK_POLYNOMIAL = 6      // (x^T y + h)^2
};

#define HB_MAXDIM 8

struct EntryDev {
  int kind;
  int dim;
  const double* X;  // SoA rows: X[c * ldx + i]
  const double* Y;  // SoA columns
  int64_t ldx, ldy;
  double neg_inv_ch2;  // -1 / (c h^2)
  double wavenumber;
  // low rank + spikes
  const double* G1;  // m x r0 row-major
  const double* G2;  // r0 x n row-major
  int r0;
  int64_t n_glob;
  const int64_t* spike_lin;  // sorted i * n + j
  const double* spike_val;
  int nspk;
  // polynomial kernel: the coordinates are read from X, Y by global index
  // (pdim of them; dim is 0 so nothing is preloaded into registers)
  int pdim;
  double poly_h;
};

__device__ inline double kernel_r2(const double* x, const double* y, int dim) {
  double r2 = 0.0;
#pragma unroll
  for (int c = 0; c < HB_MAXDIM; ++c) {
    if (c < dim) {
      double dlt = x[c] - y[c];
      r2 = fma(dlt, dlt, r2);
    }
  }
  return r2;
}

__device__ inline double spike_lookup(const EntryDev& P, int64_t i, int64_t j) {
  if (P.nspk == 0) return 0.0;
  int64_t key = i * P.n_glob + j;
  int lo = 0, hi = P.nspk - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (P.spike_lin[mid] < key) lo = mid + 1; else hi = mid;
  }
  return P.spike_lin[lo] == key ? P.spike_val[lo] : 0.0;
}

// (x_i^T y_j + h) for the polynomial kernel, SoA coordinates by global index
__device__ inline double poly_base(const EntryDev& P, int64_t i, int64_t j) {
  double s = P.poly_h;
  for (int c = 0; c < P.pdim; ++c) s = fma(P.X[(int64_t)c * P.ldx + i], P.Y[(int64_t)c * P.ldy + j], s);
  return s;
}

// Entry for global row i / column j with their coordinates already loaded.
template <typename T>
__device__ inline T eval_entry(const EntryDev& P, int64_t i, int64_t j, const double* x,
                               const double* y);

template <>
__device__ inline double eval_entry<double>(const EntryDev& P, int64_t i, int64_t j,
                                            const double* x, const double* y) {
  if (P.kind == HBK_GAUSS) {
    return exp(kernel_r2(x, y, P.dim) * P.neg_inv_ch2);
  } else if (P.kind == HBK_LAPLACE) {
    return 1.0 / sqrt(kernel_r2(x, y, P.dim));
  } else if (P.kind == HBK_POLYNOMIAL) {
    const double b = poly_base(P, i, j);
    return b * b;
  } else {  // HBK_LOWRANK_SPIKES
    double s = 0.0;
    const double* g1 = P.G1 + i * P.r0;
    const double* g2 = P.G2 + j;
    for (int t = 0; t < P.r0; ++t) s = fma(g1[t], g2[(int64_t)t * P.n_glob], s);
    return s + spike_lookup(P, i, j);
  }
}

template <>
__device__ inline float eval_entry<float>(const EntryDev& P, int64_t i, int64_t j,
                                          const double* x, const double* y) {
  // single-precision entries: distance in FP64 (cheap, avoids cancellation
  // between nearby coordinates), transcendental in FP32
  if (P.kind == HBK_GAUSS) {
    return expf((float)(kernel_r2(x, y, P.dim) * P.neg_inv_ch2));
  } else if (P.kind == HBK_LAPLACE) {
    return 1.0f / sqrtf((float)kernel_r2(x, y, P.dim));
  } else if (P.kind == HBK_POLYNOMIAL) {
    const float b = (float)poly_base(P, i, j);
    return b * b;
  } else {
    double s = 0.0;
    const double* g1 = P.G1 + i * P.r0;
    const double* g2 = P.G2 + j;
    for (int t = 0; t < P.r0; ++t) s = fma(g1[t], g2[(int64_t)t * P.n_glob], s);
    return (float)(s + spike_lookup(P, i, j));
  }
}

template <>
__device__ inline hb_cplx eval_entry<hb_cplx>(const EntryDev& P, int64_t /*i*/, int64_t /*j*/,
                                              const double* x, const double* y) {
  double r = sqrt(kernel_r2(x, y, P.dim));
  if (P.kind == HBK_EFIE2D) {
    // Hankel function of the second kind, order 0: J_0 - i Y_0
    double jv, yv;
    hb_bessel_j0y0(P.wavenumber * r, &jv, &yv);
    return hb_cplx{jv, -yv};
  }
  // Helmholtz free-space Green's function
  double s, c;
  sincos(P.wavenumber * r, &s, &c);
  double a = 1.0 / (4.0 * M_PI * r);
  return hb_cplx{c * a, s * a};
}
