// Shared device helpers for the H-BACA HIP kernels (gfx950, wave64).
//
// Scalars: double (real FP64), hb_cplx (complex FP64, interleaved re/im) and
// float (the single-precision residual path).  Every kernel is templated on
// the scalar and uses the helpers below, so one body serves all of them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HB_WAVE 64

struct hb_cplx {
  double re, im;
};

// ---------------------------------------------------------------- scalars --
template <typename T> struct hb_traits;
template <> struct hb_traits<double> {
  using real = double;
  static constexpr bool is_complex = false;
  static constexpr int words = 1;
};
template <> struct hb_traits<float> {
  using real = float;
  static constexpr bool is_complex = false;
  static constexpr int words = 1;
};
template <> struct hb_traits<hb_cplx> {
  using real = double;
  static constexpr bool is_complex = true;
  static constexpr int words = 2;
};

__device__ __host__ inline hb_cplx mk_c(double r, double i) { return hb_cplx{r, i}; }

// zero / conversions
template <typename T> __device__ __host__ inline T sc_zero();
template <> __device__ __host__ inline double sc_zero<double>() { return 0.0; }
template <> __device__ __host__ inline float sc_zero<float>() { return 0.0f; }
template <> __device__ __host__ inline hb_cplx sc_zero<hb_cplx>() { return hb_cplx{0.0, 0.0}; }

template <typename T> __device__ __host__ inline T sc_real(double r);
template <> __device__ __host__ inline double sc_real<double>(double r) { return r; }
template <> __device__ __host__ inline float sc_real<float>(double r) { return (float)r; }
template <> __device__ __host__ inline hb_cplx sc_real<hb_cplx>(double r) { return hb_cplx{r, 0.0}; }

__device__ __host__ inline double sc_conj(double a) { return a; }
__device__ __host__ inline float sc_conj(float a) { return a; }
__device__ __host__ inline hb_cplx sc_conj(hb_cplx a) { return hb_cplx{a.re, -a.im}; }

__device__ __host__ inline double sc_abs2(double a) { return a * a; }
__device__ __host__ inline double sc_abs2(float a) { return (double)a * (double)a; }
__device__ __host__ inline double sc_abs2(hb_cplx a) { return a.re * a.re + a.im * a.im; }

__device__ __host__ inline double sc_re(double a) { return a; }
__device__ __host__ inline double sc_re(float a) { return a; }
__device__ __host__ inline double sc_re(hb_cplx a) { return a.re; }

__device__ __host__ inline double sc_add(double a, double b) { return a + b; }
__device__ __host__ inline float sc_add(float a, float b) { return a + b; }
__device__ __host__ inline hb_cplx sc_add(hb_cplx a, hb_cplx b) { return hb_cplx{a.re + b.re, a.im + b.im}; }
__device__ __host__ inline double sc_sub(double a, double b) { return a - b; }
__device__ __host__ inline float sc_sub(float a, float b) { return a - b; }
__device__ __host__ inline hb_cplx sc_sub(hb_cplx a, hb_cplx b) { return hb_cplx{a.re - b.re, a.im - b.im}; }
__device__ __host__ inline double sc_mul(double a, double b) { return a * b; }
__device__ __host__ inline float sc_mul(float a, float b) { return a * b; }
__device__ __host__ inline hb_cplx sc_mul(hb_cplx a, hb_cplx b) {
  return hb_cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
__device__ __host__ inline double sc_mulc(double a, double b) { return a * b; }
__device__ __host__ inline float sc_mulc(float a, float b) { return a * b; }
__device__ __host__ inline hb_cplx sc_mulc(hb_cplx a, hb_cplx b) {
  return hb_cplx{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
__device__ __host__ inline double sc_cmul(double a, double b) { return a * b; }
__device__ __host__ inline float sc_cmul(float a, float b) { return a * b; }
__device__ __host__ inline hb_cplx sc_cmul(hb_cplx a, hb_cplx b) {
  return hb_cplx{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ __host__ inline double sc_scale(double a, double s) { return a * s; }
__device__ __host__ inline float sc_scale(float a, double s) { return (float)((double)a * s); }
__device__ __host__ inline hb_cplx sc_scale(hb_cplx a, double s) { return hb_cplx{a.re * s, a.im * s}; }
__device__ __host__ inline double sc_div(double a, double b) { return a / b; }
__device__ __host__ inline float sc_div(float a, float b) { return a / b; }
__device__ __host__ inline hb_cplx sc_div(hb_cplx a, hb_cplx b) {
  // Smith's algorithm (Smith 1962) keeps the quotient free of needless overflow
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return hb_cplx{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    double r = b.re / b.im, den = b.re * r + b.im;
    return hb_cplx{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}
// Accumulation type of a storage scalar: FP32 data accumulate in FP64.
template <typename T> struct acc_type { using type = T; };
template <> struct acc_type<float> { using type = double; };
__device__ __host__ inline double sc_to_acc(float a) { return (double)a; }
__device__ __host__ inline double sc_to_acc(double a) { return a; }
__device__ __host__ inline hb_cplx sc_to_acc(hb_cplx a) { return a; }
template <typename T> __device__ __host__ inline T sc_from_acc(typename acc_type<T>::type a);
template <> __device__ __host__ inline float sc_from_acc<float>(double a) { return (float)a; }
template <> __device__ __host__ inline double sc_from_acc<double>(double a) { return a; }
template <> __device__ __host__ inline hb_cplx sc_from_acc<hb_cplx>(hb_cplx a) { return a; }

// acc += a * b ; acc += conj(a) * b ; acc += a * conj(b)
__device__ inline void sc_fma(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ inline void sc_fma(float& acc, float a, float b) { acc = fmaf(a, b, acc); }
__device__ inline void sc_fma(hb_cplx& acc, hb_cplx a, hb_cplx b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
__device__ inline void sc_cfma(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ inline void sc_cfma(float& acc, float a, float b) { acc = fmaf(a, b, acc); }
__device__ inline void sc_cfma(hb_cplx& acc, hb_cplx a, hb_cplx b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// acc -= s * v * w  (s real)
__device__ inline void sc_axpy_neg(double& x, double s, double v, double w) { x = fma(-s * v, w, x); }
// FP32 data: the product is formed in FP64 (a reflector's s can exceed the
// FP32 range when v is tiny)
__device__ inline void sc_axpy_neg(float& x, double s, float v, float w) {
  x = (float)fma(-s * (double)v, (double)w, (double)x);
}
__device__ inline void sc_axpy_neg(hb_cplx& x, double s, hb_cplx v, hb_cplx w) {
  hb_cplx p = sc_mul(v, w);
  x.re = fma(-s, p.re, x.re);
  x.im = fma(-s, p.im, x.im);
}

// unit-modulus phase of x (1 for x == 0)
__device__ inline double sc_phase(double x) { return x < 0.0 ? -1.0 : 1.0; }
__device__ inline float sc_phase(float x) { return x < 0.0f ? -1.0f : 1.0f; }
__device__ inline hb_cplx sc_phase(hb_cplx x) {
  double a = sqrt(x.re * x.re + x.im * x.im);
  if (a == 0.0) return hb_cplx{1.0, 0.0};
  return hb_cplx{x.re / a, x.im / a};
}

// ------------------------------------------------------------ shuffles -----
__device__ inline double shfl_xor_d(double v, int mask) { return __shfl_xor(v, mask, HB_WAVE); }
__device__ inline float shfl_xor_d(float v, int mask) { return __shfl_xor(v, mask, HB_WAVE); }
__device__ inline int shfl_xor_i(int v, int mask) { return __shfl_xor(v, mask, HB_WAVE); }
__device__ inline double shfl_d(double v, int src) { return __shfl(v, src, HB_WAVE); }
__device__ inline float shfl_d(float v, int src) { return __shfl(v, src, HB_WAVE); }

__device__ inline double sc_shfl(double v, int src) { return __shfl(v, src, HB_WAVE); }
__device__ inline float sc_shfl(float v, int src) { return __shfl(v, src, HB_WAVE); }
__device__ inline hb_cplx sc_shfl(hb_cplx v, int src) {
  return hb_cplx{__shfl(v.re, src, HB_WAVE), __shfl(v.im, src, HB_WAVE)};
}
__device__ inline double sc_shfl_xor(double v, int m) { return __shfl_xor(v, m, HB_WAVE); }
__device__ inline float sc_shfl_xor(float v, int m) { return __shfl_xor(v, m, HB_WAVE); }
__device__ inline hb_cplx sc_shfl_xor(hb_cplx v, int m) {
  return hb_cplx{__shfl_xor(v.re, m, HB_WAVE), __shfl_xor(v.im, m, HB_WAVE)};
}

// Butterfly partner exchange inside a wave.  Steps 1 and 2 swap lanes
// inside a quad, step 4 mirrors each half-row of 8 lanes and step 8 mirrors
// each row of 16 lanes: all four are DPP moves (no LDS round trip).  Applied
// in ascending order, each step pairs a lane with one holding the partial sum
// of the other half of its group, so a butterfly sum ends with the same
// value in every lane.  Steps 16 and 32 cross rows and use a shuffle.
template <int CTRL> __device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int M, typename R> __device__ inline R bfly(R v) {
  if constexpr (M == 1) return dpp_move<0xB1>(v);        // quad_perm(1,0,3,2)
  else if constexpr (M == 2) return dpp_move<0x4E>(v);   // quad_perm(2,3,0,1)
  else if constexpr (M == 4) return dpp_move<0x141>(v);  // row_half_mirror
  else if constexpr (M == 8) return dpp_move<0x140>(v);  // row_mirror
  else return __shfl_xor(v, M, HB_WAVE);
}
template <int M> __device__ inline hb_cplx bfly_sc(hb_cplx v) {
  return hb_cplx{bfly<M>(v.re), bfly<M>(v.im)};
}
template <int M> __device__ inline double bfly_sc(double v) { return bfly<M>(v); }
template <int M> __device__ inline float bfly_sc(float v) { return bfly<M>(v); }

template <int G, int M = 1> __device__ inline double group_sum_step(double v) {
  if constexpr (M >= G) return v;
  else return group_sum_step<G, 2 * M>(v + bfly<M>(v));
}
template <int G, typename T, int M = 1> __device__ inline T group_sum_sc_step(T v) {
  if constexpr (M >= G) return v;
  else return group_sum_sc_step<G, T, 2 * M>(sc_add(v, bfly_sc<M>(v)));
}

// Sum over groups of G adjacent lanes (G a power of two <= 64); all lanes of
// a group must be active, and all receive the same value.
template <int G> __device__ inline double group_sum(double v) { return group_sum_step<G>(v); }
template <int G, typename T> __device__ inline T group_sum_sc(T v) {
  return group_sum_sc_step<G, T>(v);
}

template <int M> __device__ inline void argmax_step(double& val, int& idx) {
  const double ov = bfly<M>(val);
  int oi;
  if constexpr (M <= 8) oi = __builtin_amdgcn_mov_dpp(idx, M == 1 ? 0xB1 : M == 2 ? 0x4E : M == 4 ? 0x141 : 0x140, 0xF, 0xF, false);
  else oi = __shfl_xor(idx, M, HB_WAVE);
  if (ov > val || (ov == val && oi < idx)) {
    val = ov;
    idx = oi;
  }
}

// Wave-wide argmax of (val, idx): larger value wins, equal values go to the
// lower index.  Every lane gets the winner.
__device__ inline void wave_argmax(double& val, int& idx) {
  argmax_step<1>(val, idx);
  argmax_step<2>(val, idx);
  argmax_step<4>(val, idx);
  argmax_step<8>(val, idx);
  argmax_step<16>(val, idx);
  argmax_step<32>(val, idx);
}

__device__ inline double wave_sum(double v) { return group_sum<64>(v); }

// Block-wide sum of one double; every thread receives the result.  `red`
// holds NW doubles of LDS; the call contains one barrier on entry-to-exit
// and one before return so consecutive calls may reuse `red`.
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  constexpr int NW = NT / HB_WAVE;
  v = wave_sum(v);
  const int w = threadIdx.x / HB_WAVE;
  if ((threadIdx.x & (HB_WAVE - 1)) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  __syncthreads();
  return s;
}

template <typename T> __device__ inline T ldg(const T* p) { return *p; }
