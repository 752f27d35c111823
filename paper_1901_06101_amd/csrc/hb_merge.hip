// Tall-skinny Householder QR (TSQR), one-sided Jacobi SVD and block
// products used by the SVD re-compression of BACA leaves and the
// hierarchical merges (Algorithm 3, eqs. (14)-(15)).
//
// TSQR: B (rows x k) is cut into chunks of MC = 256 rows; each chunk is
// factored by one workgroup with the chunk held in registers (thread (j, q)
// owns column j, rows q, q + NQ, ...; the NQ threads of a column are adjacent
// lanes, so column norms and reflector dot products reduce with shuffles and
// each Householder step needs a single barrier).  The R factors of up to
// MC / k chunks are stacked and factored again, up to one root R.  Q is kept
// implicitly as the reflectors of every node; Q Z is applied top-down.
#include "hb_common.h"
#include "hb_merge.h"

#include <hip/hip_cooperative_groups.h>

#include <vector>

#include <algorithm>

namespace {

constexpr int MC_ALL = 256;
// reflector entries read from LDS per batch in the TSQR inner products (the
// entries below the diagonal step are stored as zeros, so every lane runs the
// same straight-line code)
constexpr int TQ_CH = 8;

template <typename T>
__device__ __forceinline__ T node_R(const T* store, const T* alpha, const QRNodeDev& N, int i, int j) {
  // R(i, j) of a factored node (i < steps, j < k)
  if (i < j) return store[N.store + (int64_t)j * MC_ALL + i];
  if (i == j) return alpha[N.ab + j];
  return sc_zero<T>();
}

template <typename T, int KMAX, int NQ, int SEG>
__global__ __launch_bounds__(KMAX* NQ) __attribute__((amdgpu_waves_per_eu(1, 2))) void tsqr_factor_kernel(const QRNodeDev* __restrict__ nodes,
                                                              const QRNodeDev* __restrict__ below,
                                                              T* __restrict__ store,
                                                              T* __restrict__ alpha,
                                                              double* __restrict__ beta) {
  static_assert(NQ * SEG == MC_ALL, "chunk height");
  static_assert(SEG % TQ_CH == 0, "register segments are read in chunks of TQ_CH");
  constexpr int MC = MC_ALL;
  const QRNodeDev N = nodes[blockIdx.x];
  const int tid = threadIdx.x;
  const int q = tid % NQ, j = tid / NQ;
  const int k = N.k, rows = N.rows, steps = N.steps;
  __shared__ T sV[2][MC];
  __shared__ double sB[2];

  T x[SEG];
#pragma unroll
  for (int s = 0; s < SEG; ++s) x[s] = sc_zero<T>();
  if (N.level0) {
    if (j < k) {
      const T* P;
      int64_t ld;
      int jj;
      const double* S;
      if (j < N.n1) {
        P = (const T*)N.P1; ld = N.ld1; jj = j; S = N.S1;
      } else {
        P = (const T*)N.P2; ld = N.ld2; jj = j - N.n1; S = N.S2;
      }
      const double sc = S ? S[jj] : 1.0;
#pragma unroll
      for (int s = 0; s < SEG; ++s) {
        const int rho = s * NQ + q;
        if (rho < rows) x[s] = sc_scale(P[(int64_t)jj * ld + N.row0 + rho], sc);
      }
    }
  } else if (j < k) {
    int off = 0;
    for (int c = 0; c < N.nchild; ++c) {
      const QRNodeDev Cn = below[N.child0 + c];
      const int pc = Cn.steps;
#pragma unroll
      for (int s = 0; s < SEG; ++s) {
        const int rho = s * NQ + q;
        if (rho >= off && rho < off + pc) x[s] = node_R<T>(store, alpha, Cn, rho - off, j);
      }
      off += pc;
    }
  }

  int buf = 0;
  for (int st = 0; st < steps; ++st) {
    if (j == st) {
      double part = 0.0;
      T xs0 = sc_zero<T>();
#pragma unroll
      for (int s = 0; s < SEG; ++s) {
        const int rho = s * NQ + q;
        if (rho >= st) part += sc_abs2(x[s]);
        if (rho == st) xs0 = x[s];
      }
      const double sig2 = group_sum<NQ>(part);
      const T x0 = group_sum_sc<NQ>(xs0);
      const double sigma = sqrt(sig2);
      T al = sc_zero<T>();
      double be = 0.0;
      if (sigma > 0.0) {
        al = sc_scale(sc_phase(x0), -sigma);
        be = 1.0 / (sigma * (sigma + sqrt(sc_abs2(x0))));
      }
      const T v0 = sc_sub(x0, al);
#pragma unroll
      for (int s = 0; s < SEG; ++s) {
        const int rho = s * NQ + q;
        if (rho == st) x[s] = v0;
        sV[buf][rho] = rho >= st ? x[s] : sc_zero<T>();
      }
      if (q == 0) {
        sB[buf] = be;
        alpha[N.ab + st] = al;
        beta[N.ab + st] = be;
      }
    }
    __syncthreads();
    if (j > st && j < k) {
      const double be = sB[buf];
      if (be != 0.0) {
        T w = sc_zero<T>();
#pragma unroll
        for (int s0 = 0; s0 < SEG; s0 += TQ_CH) {
          T vv[TQ_CH];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) vv[u] = sV[buf][(s0 + u) * NQ + q];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) sc_cfma(w, vv[u], x[s0 + u]);
          __builtin_amdgcn_sched_barrier(0);
        }
        w = group_sum_sc<NQ>(w);
#pragma unroll
        for (int s0 = 0; s0 < SEG; s0 += TQ_CH) {
          T vv[TQ_CH];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) vv[u] = sV[buf][(s0 + u) * NQ + q];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) sc_axpy_neg(x[s0 + u], be, vv[u], w);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    buf ^= 1;
  }
  if (j < k) {
#pragma unroll
    for (int s = 0; s < SEG; ++s) store[N.store + (int64_t)j * MC + s * NQ + q] = x[s];
  }
}

template <typename T, int KMAX, int NQ, int SEG>
__global__ __launch_bounds__(KMAX* NQ) __attribute__((amdgpu_waves_per_eu(1, 2))) void tsqr_apply_kernel(const QRApplyDev* __restrict__ jobs,
                                                             const T* __restrict__ store,
                                                             const double* __restrict__ beta) {
  constexpr int MC = MC_ALL;
  constexpr int NTH = KMAX * NQ;
  const QRApplyDev J = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int q = tid % NQ, j = tid / NQ;
  const int rows = J.rows, steps = J.steps, r = J.r;
  const T* Zin = (const T*)J.Zin;
  T* Zout = (T*)J.Zout;
  __shared__ T sV[2][MC];
  __shared__ double sB[2];
  const T* Ztr = (const T*)J.Ztr;
  T z[SEG];
#pragma unroll
  for (int s = 0; s < SEG; ++s) {
    const int rho = s * NQ + q;
    T v = sc_zero<T>();
    if (j < r) {
      if (rho < steps) v = Zin[(int64_t)j * J.ldin + rho];
      else if (Ztr && rho < rows) v = Ztr[(int64_t)j * J.ldtr + (rho - steps)];
    }
    z[s] = v;
  }
  // reflector st is read from HBM one step ahead of its use (one element
  // per thread, MC <= NTH), so the load latency overlaps the previous step
  static_assert(MC <= NTH, "one reflector element per thread");
  static_assert(SEG % TQ_CH == 0 && NQ * SEG == MC_ALL, "register segments of TQ_CH");
  auto vload = [&](int st) -> T {
    return (st >= 0 && tid >= st && tid < rows) ? store[J.store + (int64_t)st * MC + tid]
                                                : sc_zero<T>();
  };
  T vnext = vload(steps - 1);
  double bnext = steps > 0 ? beta[J.ab + steps - 1] : 0.0;
  int buf = 0;
  for (int st = steps - 1; st >= 0; --st) {
    if (tid < MC) sV[buf][tid] = vnext;
    if (tid == 0) sB[buf] = bnext;
    __syncthreads();
    vnext = vload(st - 1);
    if (st > 0) bnext = beta[J.ab + st - 1];
    if (j < r) {
      const double be = sB[buf];
      if (be != 0.0) {
        T w = sc_zero<T>();
#pragma unroll
        for (int s0 = 0; s0 < SEG; s0 += TQ_CH) {
          T vv[TQ_CH];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) vv[u] = sV[buf][(s0 + u) * NQ + q];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) sc_cfma(w, vv[u], z[s0 + u]);
          __builtin_amdgcn_sched_barrier(0);
        }
        w = group_sum_sc<NQ>(w);
#pragma unroll
        for (int s0 = 0; s0 < SEG; s0 += TQ_CH) {
          T vv[TQ_CH];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) vv[u] = sV[buf][(s0 + u) * NQ + q];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) sc_axpy_neg(z[s0 + u], be, vv[u], w);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    buf ^= 1;
  }
  if (j < r) {
#pragma unroll
    for (int s = 0; s < SEG; ++s) {
      const int rho = s * NQ + q;
      if (rho < rows) Zout[(int64_t)j * J.ldout + rho] = z[s];
    }
  }
}


template <typename T, int KMAX, int NQ, int SEG>
__global__ __launch_bounds__(KMAX* NQ) __attribute__((amdgpu_waves_per_eu(1, 2))) void tsqr_applyh_kernel(const QRApplyHDev* __restrict__ jobs,
                                                              const T* __restrict__ store,
                                                              const double* __restrict__ beta) {
  constexpr int MC = MC_ALL;
  constexpr int NTH = KMAX * NQ;
  const QRApplyHDev J = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int q = tid % NQ, j = tid / NQ;
  const int rows = J.rows, steps = J.steps, r = J.r;
  const T* Zin = (const T*)J.Zin;
  __shared__ T sV[2][MC];
  __shared__ double sB[2];
  T z[SEG];
#pragma unroll
  for (int s = 0; s < SEG; ++s) {
    const int rho = s * NQ + q;
    z[s] = (j < r && rho < rows) ? Zin[(int64_t)j * J.ldin + rho] : sc_zero<T>();
  }
  // reflector st is read from HBM one step ahead of its use
  static_assert(MC <= NTH, "one reflector element per thread");
  static_assert(SEG % TQ_CH == 0 && NQ * SEG == MC_ALL, "register segments of TQ_CH");
  auto vload = [&](int st) -> T {
    return (st < steps && tid >= st && tid < rows) ? store[J.store + (int64_t)st * MC + tid]
                                                   : sc_zero<T>();
  };
  T vnext = vload(0);
  double bnext = steps > 0 ? beta[J.ab] : 0.0;
  int buf = 0;
  for (int st = 0; st < steps; ++st) {
    if (tid < MC) sV[buf][tid] = vnext;
    if (tid == 0) sB[buf] = bnext;
    __syncthreads();
    vnext = vload(st + 1);
    if (st + 1 < steps) bnext = beta[J.ab + st + 1];
    if (j < r) {
      const double be = sB[buf];
      if (be != 0.0) {
        T w = sc_zero<T>();
#pragma unroll
        for (int s0 = 0; s0 < SEG; s0 += TQ_CH) {
          T vv[TQ_CH];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) vv[u] = sV[buf][(s0 + u) * NQ + q];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) sc_cfma(w, vv[u], z[s0 + u]);
          __builtin_amdgcn_sched_barrier(0);
        }
        w = group_sum_sc<NQ>(w);
#pragma unroll
        for (int s0 = 0; s0 < SEG; s0 += TQ_CH) {
          T vv[TQ_CH];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) vv[u] = sV[buf][(s0 + u) * NQ + q];
#pragma unroll
          for (int u = 0; u < TQ_CH; ++u) sc_axpy_neg(z[s0 + u], be, vv[u], w);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    buf ^= 1;
  }
  if (j < r) {
    T* Zup = (T*)J.Zup;
    T* Ztr = (T*)J.Ztr;
#pragma unroll
    for (int s = 0; s < SEG; ++s) {
      const int rho = s * NQ + q;
      if (rho < steps) Zup[(int64_t)j * J.ldup + rho] = z[s];
      else if (rho < rows) Ztr[(int64_t)j * J.ldtr + (rho - steps)] = z[s];
    }
  }
}

template <typename T>
__global__ void concat_kernel(const ConcatDev* __restrict__ jobs) {
  const ConcatDev J = jobs[blockIdx.y];
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= J.m) return;
  const T* P1 = (const T*)J.P1;
  const T* P2 = (const T*)J.P2;
  T* B = (T*)J.B;
  for (int j = 0; j < J.n1; ++j)
    B[(int64_t)j * J.m + row] = sc_scale(P1[(int64_t)j * J.m + row], J.S1 ? J.S1[j] : 1.0);
  for (int j = 0; j < J.n2; ++j)
    B[(int64_t)(J.n1 + j) * J.m + row] = sc_scale(P2[(int64_t)j * J.m + row], J.S2 ? J.S2[j] : 1.0);
}


template <typename T>
__global__ void rcopy_kernel(const RCopyDev* __restrict__ jobs, const T* __restrict__ store,
                             const T* __restrict__ alpha) {
  const RCopyDev J = jobs[blockIdx.x];
  QRNodeDev N;
  N.store = J.store;
  N.ab = J.ab;
  T* dst = (T*)J.dst;
  for (int e = threadIdx.x; e < J.p * J.k; e += blockDim.x) {
    const int i = e % J.p, j = e / J.p;
    dst[(int64_t)j * J.ld + i] = node_R<T>(store, alpha, N, i, j);
  }
}

template <typename T>
__global__ void rcompact_kernel(const RCompactDev* __restrict__ jobs) {
  const RCompactDev J = jobs[blockIdx.x];
  const T* src = (const T*)J.src;
  T* dst = (T*)J.dst;
  for (int e = threadIdx.x; e < J.P * J.k; e += blockDim.x) {
    const int i = e % J.P, j = e / J.P;
    dst[e] = src[(int64_t)j * J.ld_src + i];
  }
}

// One thread per entry of M = A B^H; the sum starts at max(i, j) since
// both factors vanish left of their diagonal.
template <typename T>
__global__ void rrh_explicit_kernel(const RRhDev* __restrict__ jobs) {
  const RRhDev J = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)J.pa * J.pb) return;
  const int i = (int)(e % J.pa), j = (int)(e / J.pa);
  const T* A = (const T*)J.A;
  const T* B = (const T*)J.B;
  T acc = sc_zero<T>();
  for (int t = max(i, j); t < J.k; ++t)
    sc_fma(acc, A[(int64_t)t * J.pa + i], sc_conj(B[(int64_t)t * J.pb + j]));
  ((T*)J.M)[e] = acc;
}

__global__ void zero_fill_kernel(uint64_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}


__global__ void copy_list_kernel(const CopyDev* __restrict__ jobs) {
  const CopyDev J = jobs[blockIdx.x];
  const int64_t n = J.bytes / 8;
  const uint64_t* src = (const uint64_t*)J.src;
  uint64_t* dst = (uint64_t*)J.dst;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------- Jacobi SVD --
// One-sided (Hestenes) Jacobi on the columns of R (p x k) with the classic
// round-robin pairing: k/2 disjoint column pairs per round, each rotated by
// a group of G lanes.  Column norms are recomputed at the start of every
// sweep and updated in closed form after each rotation (recomputed when the
// update would cancel).  Sweeps end when no pair has
// |a_i^H a_j| > tol |a_i| |a_j|; a column whose norm is below the rounding
// level of R (1e-16 sqrt(p) ||R||_F) takes no part.  The rotation tangent is
// evaluated without overflow for large zeta.  R lives in LDS when it fits,
// otherwise in the HBM workspace.  The rotations are not accumulated: the
// normalised final columns are the left singular vectors X (orthonormal to
// the sweep tolerance) and the kept right vectors follow as R^H X_r / S_r.
constexpr int SVD_NT = 512;
// A sweep whose rotations all had |a_i^H a_j| <= JAC_QUAD |a_i| |a_j| leaves
// the columns orthogonal to about JAC_QUAD^2 (one-sided Jacobi converges
// quadratically), far inside the sweep tolerance: the sweeps end there
// instead of running one more sweep that would rotate nothing.
constexpr double JAC_QUAD = 1.0e-8;

template <typename T, int G>
__device__ __forceinline__ int jacobi_rounds(T* A, int lda, int p, int k, int K, double tol, double negl,
                             double* nrm, int* sRot) {
  const int tid = threadIdx.x;
  const int grp = tid / G, gl = tid % G;
  constexpr int ngrp = SVD_NT / G;
  // elements per lane loaded together before use (LDS latency is paid once
  // per chunk, not per element); indexes past p are clamped and masked
  constexpr int CH = 8;
  const int npairs = K / 2;
  const double tol2 = tol * tol;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    // fresh column norms
    for (int j = grp; j < k; j += ngrp) {
      const T* x = A + (int64_t)j * lda;
      double s2 = 0.0;
      for (int i0 = gl; i0 < p; i0 += CH * G) {
        T u[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) u[c] = x[min(i0 + c * G, p - 1)];
#pragma unroll
        for (int c = 0; c < CH; ++c)
          if (i0 + c * G < p) s2 += sc_abs2(u[c]);
      }
      s2 = group_sum<G>(s2);
      if (gl == 0) nrm[j] = s2;
    }
    if (tid == 0) {
      sRot[0] = 0;
      sRot[1] = 0;
    }
    __syncthreads();
    for (int t = 0; t < K - 1; ++t) {
      for (int pi = grp; pi < npairs; pi += ngrp) {
        int a, b;
        if (pi == 0) {
          a = 0;
          b = 1 + (t % (K - 1));
        } else {
          a = 1 + (t + pi) % (K - 1);
          b = 1 + (t - pi + (K - 1)) % (K - 1);
        }
        if (a > b) {
          const int tmp = a; a = b; b = tmp;
        }
        if (b >= k) continue;  // padding column of an odd k (uniform in the group)
        const double al = nrm[a], bt = nrm[b];
        // a column below the rounding level of R cannot move any singular
        // value that a truncation can see: leave it alone
        if (al <= negl || bt <= negl) continue;
        T* xa = A + (int64_t)a * lda;
        T* xb = A + (int64_t)b * lda;
        T g = sc_zero<T>();
        for (int i0 = gl; i0 < p; i0 += CH * G) {
          T u[CH], v[CH];
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            const int i = min(i0 + c * G, p - 1);
            u[c] = xa[i];
            v[c] = xb[i];
          }
#pragma unroll
          for (int c = 0; c < CH; ++c)
            if (i0 + c * G < p) sc_cfma(g, u[c], v[c]);
        }
        g = group_sum_sc<G, T>(g);
        const double g2 = sc_abs2(g);
        if (g2 > tol2 * al * bt) {
          const double ag = sqrt(g2);
          const double iag = 1.0 / ag;
          const T ph = sc_scale(g, iag);
          const double zeta = 0.5 * (bt - al) * iag;
          const double az = fabs(zeta);
          // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), without overflow
          double tt = az > 1.0e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
          if (zeta < 0.0) tt = -tt;
          const double c = rsqrt(1.0 + tt * tt), s = c * tt;
          for (int i0 = gl; i0 < p; i0 += CH * G) {
            T u[CH], v[CH];
#pragma unroll
            for (int e = 0; e < CH; ++e) {
              const int i = min(i0 + e * G, p - 1);
              u[e] = xa[i];
              v[e] = xb[i];
            }
#pragma unroll
            for (int e = 0; e < CH; ++e) {
              const int i = i0 + e * G;
              if (i < p) {
                const T vv = sc_mulc(v[e], ph);  // y * conj(phase)
                xa[i] = sc_sub(sc_scale(u[e], c), sc_scale(vv, s));
                xb[i] = sc_add(sc_scale(u[e], s), sc_scale(vv, c));
              }
            }
          }
          // squared norms after the rotation: |a'|^2 = |a|^2 - t |g|,
          // |b'|^2 = |b|^2 + t |g|; a norm that shrinks below a quarter of its
          // old value is recomputed, as the update then cancels
          double na = al - tt * ag, nb = bt + tt * ag;
          if (na < 0.25 * al || nb < 0.25 * bt) {
            na = 0.0;
            nb = 0.0;
            for (int i = gl; i < p; i += G) {
              na += sc_abs2(xa[i]);
              nb += sc_abs2(xb[i]);
            }
            na = group_sum<G>(na);
            nb = group_sum<G>(nb);
          }
          if (gl == 0) {
            nrm[a] = na;
            nrm[b] = nb;
            sRot[0] = 1;
            if (g2 > JAC_QUAD * JAC_QUAD * al * bt) sRot[1] = 1;
          }
        }
      }
      __syncthreads();
    }
    const int rot = sRot[0], big = sRot[1];
    __syncthreads();
    if (!rot || !big) break;
  }
  return sweep + 1;
}

// The same rounds with each pair's two columns held in registers for the
// whole round: G lanes own elements gl, gl + G, ... (EPL per lane) of both
// columns, load them once, form the dot product and both squared norms in
// one pass, rotate in registers, and store back only when they rotated.
// This halves the LDS traffic of a round (the columns are read once, not
// once for the dot product and again for the update) and needs no norm
// bookkeeping across rounds.  Used when a column fits in G * EPL elements;
// a group takes the pairs grp, grp + SVD_NT / G, ... of a round in turn.
template <typename T, int G, int EPL>
__device__ __forceinline__ int jacobi_rounds_reg(T* A, int lda, int p, int k, int K, double tol,
                                                 double negl, int* sRot) {
  const int tid = threadIdx.x;
  const int grp = tid / G, gl = tid % G;
  constexpr int ngrp = SVD_NT / G;
  const int npairs = K / 2;
  const double tol2 = tol * tol;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (tid == 0) {
      sRot[0] = 0;
      sRot[1] = 0;
    }
    __syncthreads();
    for (int t = 0; t < K - 1; ++t) {
      for (int pi = grp; pi < npairs; pi += ngrp) {
        int a, b;
        if (pi == 0) {
          a = 0;
          b = 1 + (t % (K - 1));
        } else {
          a = 1 + (t + pi) % (K - 1);
          b = 1 + (t - pi + (K - 1)) % (K - 1);
        }
        if (a > b) {
          const int tmp = a; a = b; b = tmp;
        }
        if (b < k) {  // b == k is the padding column of an odd k
          T* xa = A + (int64_t)a * lda;
          T* xb = A + (int64_t)b * lda;
          T u[EPL], v[EPL];
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            const int i = gl + e * G;
            const int ic = i < p ? i : p - 1;
            const T uu = xa[ic], vv = xb[ic];
            u[e] = i < p ? uu : sc_zero<T>();
            v[e] = i < p ? vv : sc_zero<T>();
          }
          T g = sc_zero<T>();
          double al = 0.0, bt = 0.0;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            sc_cfma(g, u[e], v[e]);
            al += sc_abs2(u[e]);
            bt += sc_abs2(v[e]);
          }
          g = group_sum_sc<G, T>(g);
          al = group_sum<G>(al);
          bt = group_sum<G>(bt);
          // a column below the rounding level of R cannot move any singular
          // value that a truncation can see: leave it alone
          const double g2 = sc_abs2(g);
          if (al > negl && bt > negl && g2 > tol2 * al * bt) {
            const double ag = sqrt(g2);
            const double iag = 1.0 / ag;
            const T ph = sc_scale(g, iag);
            const double zeta = 0.5 * (bt - al) * iag;
            const double az = fabs(zeta);
            double tt = az > 1.0e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
            if (zeta < 0.0) tt = -tt;
            const double c = rsqrt(1.0 + tt * tt), sn = c * tt;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
              const int i = gl + e * G;
              const T vv = sc_mulc(v[e], ph);  // y * conj(phase)
              const T na = sc_sub(sc_scale(u[e], c), sc_scale(vv, sn));
              const T nb = sc_add(sc_scale(u[e], sn), sc_scale(vv, c));
              if (i < p) {
                xa[i] = na;
                xb[i] = nb;
              }
            }
            if (gl == 0) {
              sRot[0] = 1;
              if (g2 > JAC_QUAD * JAC_QUAD * al * bt) sRot[1] = 1;
            }
          }
        }
      }
      __syncthreads();
    }
    const int rot = sRot[0], big = sRot[1];
    __syncthreads();
    if (!rot || !big) break;
  }
  return sweep + 1;
}

// Small SVD of R (p x k), preconditioned as in the one-sided Jacobi SVD of
// Drmac and Veselic (2008): a QR factorisation with column pivoting of R^H,
//   R^H P = Q2 R2   (R2 upper trapezoidal, q = min(p, k) rows),
// followed by one-sided Jacobi on the columns of W = R2^H (p x q).  The rows
// of R2 are strongly graded, so the Jacobi sweeps converge in a few passes.
// With W V = U Sigma, R = (P U) Sigma (Q2 V)^H: the left singular vectors of
// R are the rows of U permuted by P (orthonormal to the sweep tolerance) and
// the kept right vectors follow as Y_r = R^H X_r / S_r.
//
// QRCP picks, at every step, the candidate column with the largest trailing
// norm (recomputed exactly during the previous step's update) and leaves the
// columns in place: a logical-to-physical column map is permuted instead.
// The transposition R2 -> R2^H goes through the HBM workspace W.
constexpr int SVD_G = 8;  // lanes per column in the QRCP updates

__host__ __device__ __forceinline__ int svd_odd(int n) { return n | 1; }

template <typename T>
struct SvdSmem {
  T* mat;        // LDS matrix region (INLDS only)
  double* nrm2;  // 2 x nm
  int* cp;       // 2 x p
  double* sN;    // k
  int* sPerm;    // k
};

// bytes of dynamic LDS for a job: [matrix | aux]; the matrix part only when
// the matrices are held in LDS
__host__ __device__ inline size_t svd_mat_bytes(int p, int k, size_t sb) {
  const int q = p < k ? p : k;
  const size_t b1 = (size_t)svd_odd(k) * p, b2 = (size_t)svd_odd(p) * q;
  return ((b1 > b2 ? b1 : b2) * sb + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t svd_aux_bytes(int p, int k) {
  const int nm = p > k ? p : k;
  return (size_t)2 * nm * 8 + (size_t)k * 8 + (((size_t)2 * p * 4 + (size_t)k * 4 + 15) & ~(size_t)15);
}

template <typename T, bool INLDS>
__global__ __launch_bounds__(SVD_NT) void svd_kernel(const SVDJobDev* __restrict__ jobs,
                                                     const T* __restrict__ store,
                                                     const T* __restrict__ alpha, double eps,
                                                     int precond_only) {
  const SVDJobDev Jb = jobs[blockIdx.x];
  const int p = Jb.p, k = Jb.k, tid = threadIdx.x;
  const int q = p < k ? p : k;
  const int lane = tid & 63, wid = tid >> 6;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int sRot[2];
  __shared__ int sR;
  __shared__ double sWv[SVD_NT / 64];
  __shared__ int sWi[SVD_NT / 64];
  // dynamic LDS layout
  unsigned char* sp = smem_raw;
  T* Lmat = (T*)sp;
  if (INLDS) sp += svd_mat_bytes(p, k, sizeof(T));
  const int nm = p > k ? p : k;
  double* nrm2 = (double*)sp;
  double* sN = nrm2 + 2 * nm;
  int* cp = (int*)(sN + k);
  int* sPerm = cp + 2 * p;
  // B = R^H (k x p, ld ldb), W = R2^H (p x q, ld ldw); in LDS both share the
  // matrix region, in HBM they are the A and W workspaces
  const int ldb = INLDS ? svd_odd(k) : k;
  const int ldw = INLDS ? svd_odd(p) : p;
  T* B = INLDS ? Lmat : (T*)Jb.A;
  T* W = INLDS ? Lmat : (T*)Jb.W;
  T* Wg = (T*)Jb.W;
  QRNodeDev N;
  N.store = Jb.store;
  N.ab = Jb.ab;
  auto Rat = [&](int i, int j) -> T {
    return Jb.from_node ? node_R<T>(store, alpha, N, i, j) : ((const T*)Jb.R)[(int64_t)j * p + i];
  };
  constexpr int G = SVD_G;
  constexpr int NGRP = SVD_NT / G;
  constexpr int CH = 8;
  const int grp = tid / G, gl = tid % G;

  // ---- load B = R^H and the initial column norms
  for (int e = tid; e < p * k; e += SVD_NT) {
    const int i = e % k, j = e / k;  // B(i, j) = conj(R(j, i))
    B[(int64_t)j * ldb + i] = sc_conj(Rat(j, i));
  }
  if (tid < p) {
    cp[tid] = tid;
    cp[p + tid] = tid;
  }
  __syncthreads();
  for (int j = grp; j < p; j += NGRP) {
    const T* col = B + (int64_t)j * ldb;
    double s2 = 0.0;
    for (int i = gl; i < k; i += G) s2 += sc_abs2(col[i]);
    s2 = group_sum<G>(s2);
    if (gl == 0) nrm2[j] = s2;
  }
  __syncthreads();

  // ---- QRCP of B: q steps, two barriers each
  int cur = 0;
  for (int s = 0; s < q; ++s) {
    const int nxt = cur ^ 1;
    double* n_cur = nrm2 + cur * nm;
    double* n_nxt = nrm2 + nxt * nm;
    int* c_cur = cp + cur * p;
    int* c_nxt = cp + nxt * p;
    {
      double v = -1.0;
      int idx = 0x7fffffff;
      if (tid >= s && tid < p) {
        v = n_cur[tid];
        if (!(v == v)) v = 0.0;  // non-finite data still yield a valid pivot
        idx = tid;
      }
      wave_argmax(v, idx);
      if (lane == 0) {
        sWv[wid] = v;
        sWi[wid] = idx;
      }
    }
    __syncthreads();
    double bv = sWv[0];
    int piv = sWi[0];
    for (int w = 1; w < SVD_NT / 64; ++w)
      if (sWv[w] > bv || (sWv[w] == bv && sWi[w] < piv)) {
        bv = sWv[w];
        piv = sWi[w];
      }
    // a candidate always exists (s < p); the clamp keeps LDS indexing in
    // range even if non-finite data left no winner
    if (piv < s || piv >= p) piv = s;
    const int cs = c_cur[s], cpv = c_cur[piv];
    if (tid < p) c_nxt[tid] = tid == s ? cpv : (tid == piv ? cs : c_cur[tid]);
    const T* vcol = B + (int64_t)cpv * ldb;
    const T x0 = vcol[s];
    const double sig = sqrt(n_cur[piv]);
    T al = sc_zero<T>();
    double be = 0.0;
    if (sig > 0.0) {
      al = sc_scale(sc_phase(x0), -sig);
      be = 1.0 / (sig * (sig + sqrt(sc_abs2(x0))));
    }
    const T v0 = sc_sub(x0, al);
    for (int j = s + 1 + grp; j < p; j += NGRP) {
      T* col = B + (int64_t)(j == piv ? cs : c_cur[j]) * ldb;
      T w = sc_zero<T>();
      for (int i0 = s + gl; i0 < k; i0 += CH * G) {
        T u[CH], v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int i = min(i0 + c * G, k - 1);
          u[c] = vcol[i];
          v[c] = col[i];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int i = i0 + c * G;
          if (i < k) sc_cfma(w, i == s ? v0 : u[c], v[c]);
        }
      }
      w = group_sum_sc<G, T>(w);
      double n2 = 0.0;
      for (int i0 = s + gl; i0 < k; i0 += CH * G) {
        T u[CH], v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int i = min(i0 + c * G, k - 1);
          u[c] = vcol[i];
          v[c] = col[i];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int i = i0 + c * G;
          if (i < k) {
            T x = v[c];
            if (be != 0.0) sc_axpy_neg(x, be, i == s ? v0 : u[c], w);
            col[i] = x;
            if (i > s) n2 += sc_abs2(x);
          }
        }
      }
      n2 = group_sum<G>(n2);
      if (gl == 0) n_nxt[j] = n2;
    }
    __syncthreads();
    // the pivot column is not touched after its step: its entry s becomes
    // the diagonal of R2 (every read of x0 happened before the barrier)
    if (tid == 0) B[(int64_t)cpv * ldb + s] = al;
    cur = nxt;
  }
  __syncthreads();
  const int* cfin = cp + cur * p;  // logical -> physical (= row of R)

  // ---- W = R2^H (p x q) through the HBM workspace
  for (int e = tid; e < p * q; e += SVD_NT) {
    const int i = e % p, a = e / p;
    Wg[e] = i >= a ? sc_conj(B[(int64_t)cfin[i] * ldb + a]) : sc_zero<T>();
  }
  if (precond_only) {
    // the multi-workgroup Jacobi takes over from W and the permutation
    for (int i = tid; i < p; i += SVD_NT) Jb.cperm[i] = cfin[i];
    return;
  }
  __syncthreads();
  if (INLDS) {
    for (int e = tid; e < p * q; e += SVD_NT) W[(int64_t)(e / p) * ldw + (e % p)] = Wg[e];
    __syncthreads();
  }

  // ---- one-sided Jacobi on the columns of W
  const int Q = q + (q & 1);
  const double tol = 4.0e-16 * (p > 4 ? (double)p : 4.0);
  double f2 = 0.0;
  for (int e = tid; e < p * q; e += SVD_NT) f2 += sc_abs2(W[(int64_t)(e / p) * ldw + (e % p)]);
  f2 = wave_sum(f2);
  if (lane == 0) sWv[wid] = f2;
  __syncthreads();
  f2 = 0.0;
  for (int w = 0; w < SVD_NT / 64; ++w) f2 += sWv[w];
  const double negl = 1.0e-32 * (double)(p > 1 ? p : 1) * f2;
  double* jn = nrm2;  // Jacobi column norms (q)
  int sweeps = 0;
  if (q >= 2) {
    const int npairs = Q / 2;
    // register-resident rounds whenever a column fits in a group's
    // registers: 8 lanes per pair up to 128 rows, 16 up to 256, 32 up to 512
    if (p <= 8 * 4) {
      sweeps = jacobi_rounds_reg<T, 8, 4>(W, ldw, p, q, Q, tol, negl, sRot);
    } else if (p <= 8 * 8) {
      sweeps = jacobi_rounds_reg<T, 8, 8>(W, ldw, p, q, Q, tol, negl, sRot);
    } else if (p <= 8 * 16) {
      sweeps = jacobi_rounds_reg<T, 8, 16>(W, ldw, p, q, Q, tol, negl, sRot);
    } else if (p <= 16 * 16) {
      sweeps = jacobi_rounds_reg<T, 16, 16>(W, ldw, p, q, Q, tol, negl, sRot);
    } else if (p <= 32 * 16) {
      sweeps = jacobi_rounds_reg<T, 32, 16>(W, ldw, p, q, Q, tol, negl, sRot);
    } else {
      const int gp = p <= 16 ? 2 : (p <= 32 ? 4 : 8);
      const int gk = npairs * 8 <= SVD_NT ? 8 : (npairs * 4 <= SVD_NT ? 4 : 2);
      const int g = gp < gk ? gp : gk;
      if (g == 8) sweeps = jacobi_rounds<T, 8>(W, ldw, p, q, Q, tol, negl, jn, sRot);
      else if (g == 4) sweeps = jacobi_rounds<T, 4>(W, ldw, p, q, Q, tol, negl, jn, sRot);
      else sweeps = jacobi_rounds<T, 2>(W, ldw, p, q, Q, tol, negl, jn, sRot);
    }
  }
  __syncthreads();
  // ---- singular values: column norms, sorted descending (ties by index)
  double* sS = nrm2 + nm;
  for (int j = grp; j < q; j += NGRP) {
    const T* x = W + (int64_t)j * ldw;
    double s2 = 0.0;
    for (int i = gl; i < p; i += G) s2 += sc_abs2(x[i]);
    s2 = group_sum<G>(s2);
    // a non-finite column (non-finite input) sorts as zero, so the sort
    // below still yields a permutation
    if (gl == 0) sS[j] = (s2 == s2 && s2 <= 1.0e300) ? sqrt(s2) : 0.0;
  }
  __syncthreads();
  for (int j = tid; j < k; j += SVD_NT) {
    if (j < q) {
      const double sj = sS[j];
      int pos = 0;
      for (int i = 0; i < q; ++i) {
        const double si = sS[i];
        if (si > sj || (si == sj && i < j)) ++pos;
      }
      sPerm[pos] = j;
      sN[pos] = sj;
    } else {
      sPerm[j] = -1;
      sN[j] = 0.0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const double s1 = q > 0 ? sN[0] : 0.0;
    int r = 0;
    if (s1 > 0.0)
      while (r < q && sN[r] >= eps * s1) ++r;
    sR = r;
    Jb.rank[0] = r;
    Jb.rank[1] = sweeps;
  }
  for (int j = tid; j < k; j += SVD_NT) {
    Jb.S[j] = sN[j];
    Jb.perm[j] = sPerm[j];
  }
  __syncthreads();
  const int r = sR;
  // ---- X = P U: X(cfin[i], pos) = W(i, sPerm[pos]) / S(pos); zero columns
  // beyond q
  T* Xr = (T*)Jb.Xr;
  for (int e = tid; e < p * k; e += SVD_NT) {
    const int i = e % p, pos = e / p;
    T v = sc_zero<T>();
    if (pos < q && sN[pos] > 0.0) v = sc_scale(W[(int64_t)sPerm[pos] * ldw + i], 1.0 / sN[pos]);
    Xr[(int64_t)pos * p + cfin[i]] = v;
  }
  __syncthreads();
  // ---- Y_r = R^H X_r diag(1 / S_r); G lanes per output, R upper trapezoidal
  // when it comes from a TSQR node
  T* Yr = (T*)Jb.Yr;
  for (int o = grp; o < k * r; o += NGRP) {
    const int i = o % k, pos = o / k;
    const T* x = Xr + (int64_t)pos * p;
    const int tmax = Jb.from_node ? (i < p - 1 ? i : p - 1) : p - 1;
    T acc = sc_zero<T>();
    for (int t = gl; t <= tmax; t += G) sc_cfma(acc, Rat(t, i), x[t]);
    acc = group_sum_sc<G, T>(acc);
    if (gl == 0) Yr[(int64_t)pos * k + i] = sc_scale(acc, 1.0 / sN[pos]);
  }
}

// ------------------------------------------- multi-workgroup Jacobi SVD ---
// The same SVD for a few large R (the top merge levels), with the Jacobi
// sweeps spread over B workgroups per matrix in one cooperative launch.  The
// single-workgroup kernel first computes the preconditioned W = R2^H (the
// QRCP of R^H, p x q with q = k here since p >= k) and its row permutation;
// this kernel runs one-sided Jacobi on the k columns of W, cut into 2B
// blocks of NB columns.  A sweep is 2B - 1 rounds of the round-robin
// tournament over the blocks; in a round each workgroup loads its two blocks
// into LDS, rotates the column pairs across them (in round 0 also the pairs
// inside each block), writes them back, and the grid synchronises.  Every
// column pair meets once per sweep; sweeps end when a whole sweep rotated
// nothing.  The rotation rule, tolerance and rounding-level cut-off are those
// of the single-workgroup rounds, and so are the outputs: X = P U from the
// normalised columns, Y_r = R^H X_r / S_r.
constexpr int WS_NT = 512;

template <typename T> struct WideCfg;
template <> struct WideCfg<double> { static constexpr int NB = 16; };   // 32 lanes per pair
template <> struct WideCfg<hb_cplx> { static constexpr int NB = 8; };   // 64 lanes per pair
constexpr int WS_PMAX = 512;

// Rotates the column pair (ca, cb) of the LDS block L (column stride ldl)
// with G lanes, each holding EPL entries in registers.  Returns (in every
// lane of the group) 0 when the pair was not rotated, 1 when it was, 2 when
// it was and its cosine exceeded JAC_QUAD.
template <typename T, int G, int EPL>
__device__ __forceinline__ int wide_pair(T* L, int ldl, int p, int ca, int cb, int gl, double tol2,
                                         double negl) {
  T* xa = L + (int64_t)ca * ldl;
  T* xb = L + (int64_t)cb * ldl;
  T u[EPL], v[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int i = gl + e * G;
    const int ic = i < p ? i : p - 1;
    const T uu = xa[ic], vv = xb[ic];
    u[e] = i < p ? uu : sc_zero<T>();
    v[e] = i < p ? vv : sc_zero<T>();
  }
  T g = sc_zero<T>();
  double al = 0.0, bt = 0.0;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    sc_cfma(g, u[e], v[e]);
    al += sc_abs2(u[e]);
    bt += sc_abs2(v[e]);
  }
  g = group_sum_sc<G, T>(g);
  al = group_sum<G>(al);
  bt = group_sum<G>(bt);
  const double g2 = sc_abs2(g);
  if (!(al > negl && bt > negl && g2 > tol2 * al * bt)) return 0;
  const double ag = sqrt(g2);
  const double iag = 1.0 / ag;
  const T ph = sc_scale(g, iag);
  const double zeta = 0.5 * (bt - al) * iag;
  const double az = fabs(zeta);
  double tt = az > 1.0e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
  if (zeta < 0.0) tt = -tt;
  const double c = rsqrt(1.0 + tt * tt), sn = c * tt;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int i = gl + e * G;
    const T vv = sc_mulc(v[e], ph);  // y * conj(phase)
    const T na = sc_sub(sc_scale(u[e], c), sc_scale(vv, sn));
    const T nb = sc_add(sc_scale(u[e], sn), sc_scale(vv, c));
    if (i < p) {
      xa[i] = na;
      xb[i] = nb;
    }
  }
  return g2 > JAC_QUAD * JAC_QUAD * al * bt ? 2 : 1;
}

// jobs[j] runs on workgroups j * B .. j * B + B - 1.  work: 3 + 3 ints of
// sweep flags (rotations; rotations above JAC_QUAD), zero on entry, then
// njobs * B doubles of partial norms at byte 32.
template <typename T>
__global__ __launch_bounds__(WS_NT) void svd_wide_kernel(const SVDJobDev* __restrict__ jobs, int B,
                                                         const T* __restrict__ store,
                                                         const T* __restrict__ alpha, double eps,
                                                         int* __restrict__ flags,
                                                         double* __restrict__ parts) {
  namespace cg = cooperative_groups;
  constexpr int NB = WideCfg<T>::NB;
  constexpr int G = WS_NT / NB;
  constexpr int EPL = (WS_PMAX + G - 1) / G;
  const cg::grid_group grid = cg::this_grid();
  const int job = blockIdx.x / B, w = blockIdx.x % B;
  const SVDJobDev Jb = jobs[job];
  const int p = Jb.p, k = Jb.k, tid = threadIdx.x;
  const int grp = tid / G, gl = tid % G;
  extern __shared__ unsigned char smem_raw[];
  T* L = (T*)smem_raw;  // 2 NB columns of p entries
  const int ldl = p;
  __shared__ int sRotW;
  __shared__ double sPart[WS_NT / 64];
  __shared__ int sR;
  T* M = (T*)Jb.W;  // W = R2^H, p x k, ld p (rotated in place)
  QRNodeDev N;
  N.store = Jb.store;
  N.ab = Jb.ab;
  auto Rat = [&](int i, int j) -> T {
    return Jb.from_node ? node_R<T>(store, alpha, N, i, j) : ((const T*)Jb.R)[(int64_t)j * p + i];
  };
  // ---- the partial Frobenius norm of W (columns w, w + B, ...)
  double f2 = 0.0;
  for (int j = w; j < k; j += B)
    for (int i = tid; i < p; i += WS_NT) f2 += sc_abs2(M[(int64_t)j * p + i]);
  f2 = wave_sum(f2);
  if ((tid & 63) == 0) sPart[tid >> 6] = f2;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < WS_NT / 64; ++q) s += sPart[q];
    parts[blockIdx.x] = s;
    sRotW = 0;
  }
  grid.sync();
  // the same sum in every workgroup of the job (fixed order: deterministic)
  f2 = 0.0;
  for (int q = 0; q < B; ++q) f2 += parts[job * B + q];
  const double negl = 1.0e-32 * (double)(p > 1 ? p : 1) * f2;
  const double tol = 4.0e-16 * (p > 4 ? (double)p : 4.0);
  const double tol2 = tol * tol;
  const int nblk = 2 * B, R1 = nblk - 1;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (blockIdx.x == 0 && tid == 0) {
      flags[(sweep + 1) % 3] = 0;
      flags[3 + (sweep + 1) % 3] = 0;
    }
    for (int t = 0; t < R1; ++t) {
      // the round-robin pairing of the blocks (block nblk - 1 stays put)
      int ba, bb;
      if (w == 0) {
        ba = t;
        bb = nblk - 1;
      } else {
        ba = (t + w) % R1;
        bb = (t - w + R1) % R1;
      }
      // local column c < NB: block ba, else block bb; columns past k load
      // as zero and never rotate (their norm is not above negl)
      for (int e = tid; e < 2 * NB * p; e += WS_NT) {
        const int c = e / p, i = e % p;
        const int gc = (c < NB ? ba * NB + c : bb * NB + c - NB);
        L[(int64_t)c * ldl + i] = gc < k ? M[(int64_t)gc * p + i] : sc_zero<T>();
      }
      __syncthreads();
      int rot = 0;
      if (t == 0) {
        // every pair of the 2 NB local columns (circle method)
        constexpr int K = 2 * NB;
        for (int u = 0; u < K - 1; ++u) {
          int a, b;
          if (grp == 0) {
            a = 0;
            b = 1 + (u % (K - 1));
          } else {
            a = 1 + (u + grp) % (K - 1);
            b = 1 + (u - grp + (K - 1)) % (K - 1);
          }
          rot = max(rot, wide_pair<T, G, EPL>(L, ldl, p, a, b, gl, tol2, negl));
          __syncthreads();
        }
      } else {
        // the pairs across the two blocks
        for (int u = 0; u < NB; ++u) {
          rot = max(rot, wide_pair<T, G, EPL>(L, ldl, p, grp, NB + (grp + u) % NB, gl, tol2, negl));
          __syncthreads();
        }
      }
      if (rot && gl == 0) atomicMax(&sRotW, rot);
      for (int e = tid; e < 2 * NB * p; e += WS_NT) {
        const int c = e / p, i = e % p;
        const int gc = (c < NB ? ba * NB + c : bb * NB + c - NB);
        if (gc < k) M[(int64_t)gc * p + i] = L[(int64_t)c * ldl + i];
      }
      __syncthreads();
      if (tid == 0 && sRotW) {
        atomicAdd(&flags[sweep % 3], 1);
        if (sRotW > 1) atomicAdd(&flags[3 + sweep % 3], 1);
        sRotW = 0;
      }
      grid.sync();
    }
    const int any = __atomic_load_n(&flags[sweep % 3], __ATOMIC_RELAXED);
    const int big = __atomic_load_n(&flags[3 + sweep % 3], __ATOMIC_RELAXED);
    if (any == 0 || big == 0) break;
  }
  // ---- singular values (column norms) sorted descending, the eps-rank:
  // workgroup 0 of the job
  __shared__ double sN[WS_PMAX];
  __shared__ int sPerm[WS_PMAX];
  if (w == 0) {
    double* sNrm = (double*)smem_raw;  // k norms (the LDS block is free now)
    for (int j = grp; j < k; j += NB) {
      const T* x = M + (int64_t)j * p;
      double s2 = 0.0;
      for (int i = gl; i < p; i += G) s2 += sc_abs2(x[i]);
      s2 = group_sum<G>(s2);
      if (gl == 0) sNrm[j] = (s2 == s2 && s2 <= 1.0e300) ? sqrt(s2) : 0.0;
    }
    __syncthreads();
    for (int j = tid; j < k; j += WS_NT) {
      const double sj = sNrm[j];
      int pos = 0;
      for (int i = 0; i < k; ++i) {
        const double si = sNrm[i];
        if (si > sj || (si == sj && i < j)) ++pos;
      }
      sPerm[pos] = j;
      sN[pos] = sj;
    }
    __syncthreads();
    if (tid == 0) {
      const double s1 = k > 0 ? sN[0] : 0.0;
      int r = 0;
      if (s1 > 0.0)
        while (r < k && sN[r] >= eps * s1) ++r;
      Jb.rank[0] = r;
      Jb.rank[1] = sweep + 1;
    }
    for (int j = tid; j < k; j += WS_NT) {
      Jb.S[j] = sN[j];
      Jb.perm[j] = sPerm[j];
    }
  }
  grid.sync();
  // ---- X = P U: X(cperm[i], pos) = W(i, perm[pos]) / S(pos);
  // Y_r = R^H X_r / S_r; the output columns are shared out over the job's
  // workgroups
  if (tid == 0) sR = Jb.rank[0];
  for (int j = tid; j < k; j += WS_NT) {
    sN[j] = Jb.S[j];
    sPerm[j] = Jb.perm[j];
  }
  __syncthreads();
  const int r = sR;
  const int* cperm = Jb.cperm;
  T* Xr = (T*)Jb.Xr;
  for (int pos = w; pos < k; pos += B) {
    const double sv = sN[pos];
    const T* x = M + (int64_t)sPerm[pos] * p;
    for (int i = tid; i < p; i += WS_NT)
      Xr[(int64_t)pos * p + cperm[i]] = sv > 0.0 ? sc_scale(x[i], 1.0 / sv) : sc_zero<T>();
  }
  grid.sync();
  T* Yr = (T*)Jb.Yr;
  for (int pos = w; pos < r; pos += B) {
    const double sv = sN[pos];
    const T* x = Xr + (int64_t)pos * p;
    for (int i = grp; i < k; i += NB) {
      const int tmax = Jb.from_node ? (i < p - 1 ? i : p - 1) : p - 1;
      T acc = sc_zero<T>();
      for (int tt = gl; tt <= tmax; tt += G) sc_cfma(acc, Rat(tt, i), x[tt]);
      acc = group_sum_sc<G, T>(acc);
      if (gl == 0) Yr[(int64_t)pos * k + i] = sc_scale(acc, 1.0 / sv);
    }
  }
}

// ------------------------------------------------------------ block GEMM ---
constexpr int BG_NT = 256;
constexpr int BG_CT = 16;

template <typename T>
__global__ __launch_bounds__(BG_NT) void block_gemm_kernel(const BlockGemmDev* __restrict__ jobs,
                                                           int /*ymax*/) {
  const BlockGemmDev Jb = jobs[blockIdx.y];
  const int row = blockIdx.x * BG_NT + threadIdx.x;
  const int nrows = Jb.n1 + Jb.n2;
  extern __shared__ unsigned char smem_raw[];
  T* sY = (T*)smem_raw;  // (r1 + r2) x BG_CT
  const int rin = Jb.r1 + Jb.r2;
  if ((int)(blockIdx.x * BG_NT) >= nrows) return;
  const bool first = row < Jb.n1;
  const T* Ab = first ? (const T*)Jb.A1 : (const T*)Jb.A2;
  const int64_t lda = first ? Jb.lda1 : Jb.lda2;
  const int rowb = first ? row : row - Jb.n1;
  const int t0 = first ? 0 : Jb.r1;
  const int tn = first ? Jb.r1 : Jb.r2;
  const T* Yg = (const T*)Jb.Y;
  T* Cg = (T*)Jb.C;
  for (int c0 = 0; c0 < Jb.r; c0 += BG_CT) {
    __syncthreads();
    for (int e = threadIdx.x; e < rin * BG_CT; e += BG_NT) {
      const int t = e % rin, cc = e / rin;
      sY[t * BG_CT + cc] = (c0 + cc < Jb.r) ? Yg[(int64_t)(c0 + cc) * Jb.ldy + t] : sc_zero<T>();
    }
    __syncthreads();
    if (row < nrows) {
      T acc[BG_CT];
#pragma unroll
      for (int cc = 0; cc < BG_CT; ++cc) acc[cc] = sc_zero<T>();
      for (int t = 0; t < tn; ++t) {
        const T a = Ab[(int64_t)t * lda + rowb];
#pragma unroll
        for (int cc = 0; cc < BG_CT; ++cc) sc_fma(acc[cc], a, sY[(t0 + t) * BG_CT + cc]);
      }
#pragma unroll
      for (int cc = 0; cc < BG_CT; ++cc)
        if (c0 + cc < Jb.r) Cg[(int64_t)(c0 + cc) * Jb.ldc + row] = acc[cc];
    }
  }
}


}  // namespace

namespace hbk {

int tsqr_mc(int, int) { return MC_ALL; }

int tsqr_kmax_for(int scalar, int k) {
  if (k <= 16) return 16;
  if (k <= 32) return 32;
  if (k <= 64) return 64;
  if (scalar == 0 && k <= 128) return 128;
  return -1;
}

template <typename T, int KMAX, int NQ, int SEG>
static int fac(const QRNodeDev* nodes, int n, const QRNodeDev* below, void* store, void* alpha,
               double* beta, hipStream_t st) {
  hipLaunchKernelGGL((tsqr_factor_kernel<T, KMAX, NQ, SEG>), dim3(n), dim3(KMAX * NQ), 0, st,
                     nodes, below, (T*)store, (T*)alpha, beta);
  return (int)hipGetLastError();
}

template <typename T, int KMAX, int NQ, int SEG>
static int app(const QRApplyDev* jobs, int n, const void* store, const double* beta,
               hipStream_t st) {
  hipLaunchKernelGGL((tsqr_apply_kernel<T, KMAX, NQ, SEG>), dim3(n), dim3(KMAX * NQ), 0, st,
                     jobs, (const T*)store, beta);
  return (int)hipGetLastError();
}

template <typename T, int KMAX, int NQ, int SEG>
static int apph(const QRApplyHDev* jobs, int n, const void* store, const double* beta,
                hipStream_t st) {
  hipLaunchKernelGGL((tsqr_applyh_kernel<T, KMAX, NQ, SEG>), dim3(n), dim3(KMAX * NQ), 0, st,
                     jobs, (const T*)store, beta);
  return (int)hipGetLastError();
}

// Lane layouts of the TSQR kernels of one width: layout 0 gives a node
// KMAX * NQ lanes with SEG rows each, layout 1 twice the lanes with half the
// rows (16 columns have a single layout).  Which one is faster depends on
// the width and on how many nodes a launch holds (one node at the top of a
// tree, hundreds at the bottom); the choice per (scalar, width, batch size)
// is a table that tsqr_autotune fills by timing both, and that starts at
// layout 1.  Both layouts compute the same reflectors up to the order of
// their partial sums.
static int g_tsqr_layout[2][4][2] = {{{1, 1}, {1, 1}, {1, 1}, {1, 1}},
                                      {{1, 1}, {1, 1}, {1, 1}, {1, 1}}};

static int kidx(int kmax) { return kmax == 16 ? 0 : kmax == 32 ? 1 : kmax == 64 ? 2 : 3; }
static int nbucket(int n) { return n < 64 ? 0 : 1; }

#define HB_TSQR_DISPATCH(FN, ...)                                                     \
  do {                                                                                \
    const int lay = g_tsqr_layout[scalar ? 1 : 0][kidx(kmax)][nbucket(n)];            \
    if (scalar == 0) {                                                                \
      if (kmax == 16) return FN<double, 16, 32, 8>(__VA_ARGS__);                      \
      if (kmax == 32) return lay ? FN<double, 32, 32, 8>(__VA_ARGS__)                 \
                                 : FN<double, 32, 16, 16>(__VA_ARGS__);               \
      if (kmax == 64) return lay ? FN<double, 64, 16, 16>(__VA_ARGS__)                \
                                 : FN<double, 64, 8, 32>(__VA_ARGS__);                \
      if (kmax == 128) return lay ? FN<double, 128, 8, 32>(__VA_ARGS__)               \
                                  : FN<double, 128, 4, 64>(__VA_ARGS__);              \
    } else {                                                                          \
      if (kmax == 16) return FN<hb_cplx, 16, 32, 8>(__VA_ARGS__);                     \
      if (kmax == 32) return lay ? FN<hb_cplx, 32, 32, 8>(__VA_ARGS__)                \
                                 : FN<hb_cplx, 32, 16, 16>(__VA_ARGS__);              \
      if (kmax == 64) return lay ? FN<hb_cplx, 64, 16, 16>(__VA_ARGS__)               \
                                 : FN<hb_cplx, 64, 8, 32>(__VA_ARGS__);               \
    }                                                                                 \
  } while (0)

int tsqr_factor_launch(int scalar, int kmax, const QRNodeDev* nodes, int n,
                       const QRNodeDev* below, void* store, void* alpha, double* beta,
                       hipStream_t st) {
  if (n == 0) return 0;
  HB_TSQR_DISPATCH(fac, nodes, n, below, store, alpha, beta, st);
  return -1;
}

int tsqr_apply_launch(int scalar, int kmax, const QRApplyDev* jobs, int n, const void* store,
                      const double* beta, hipStream_t st) {
  if (n == 0) return 0;
  HB_TSQR_DISPATCH(app, jobs, n, store, beta, st);
  return -1;
}

int tsqr_applyh_launch(int scalar, int kmax, const QRApplyHDev* jobs, int n, const void* store,
                       const double* beta, hipStream_t st) {
  if (n == 0) return 0;
  HB_TSQR_DISPATCH(apph, jobs, n, store, beta, st);
  return -1;
}
#undef HB_TSQR_DISPATCH

__global__ void tune_fill_kernel(double* x, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // a fixed pseudo-random fill (SplitMix64 of the index), values in [-1, 1)
  uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Times both lane layouts of the factor and apply kernels on synthetic
// level-0 batches (1 node: the top of a tree; 256 nodes: its bottom) of
// every width and scalar type, and keeps the faster in g_tsqr_layout.
// Writes the table to `table` (2 x 4 x 2 ints, may be null) and the
// measured times in microseconds to `us` (2 x 4 x 2 x 2, may be null).
int tsqr_autotune(hipStream_t st, int* table, double* us) {
  const int MC = MC_ALL;
  const int batches[2] = {1, 256};
  const int kmaxs[4] = {16, 32, 64, 128};
  const size_t maxk = 128, maxn = 256;
  double *B = nullptr, *store = nullptr, *alpha = nullptr, *beta = nullptr, *Z = nullptr;
  QRNodeDev* dn = nullptr;
  QRApplyDev* dj = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int err = 0;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess && err == 0) err = (int)e;
    return err == 0;
  };
  const size_t belems = maxn * MC * maxk * 2;  // complex counts twice
  if (!ok(hipMalloc(&B, belems * 8)) || !ok(hipMalloc(&store, belems * 8)) ||
      !ok(hipMalloc(&alpha, maxn * maxk * 16)) || !ok(hipMalloc(&beta, maxn * maxk * 8)) ||
      !ok(hipMalloc(&Z, belems * 8)) || !ok(hipMalloc(&dn, maxn * sizeof(QRNodeDev))) ||
      !ok(hipMalloc(&dj, maxn * sizeof(QRApplyDev))) || !ok(hipEventCreate(&e0)) ||
      !ok(hipEventCreate(&e1))) {
  } else {
    hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)((belems + 255) / 256)), dim3(256), 0, st,
                       B, (int64_t)belems, 12345ull);
    ok(hipGetLastError());
    for (int sc = 0; sc < 2 && err == 0; ++sc)
      for (int ki = 0; ki < 4 && err == 0; ++ki) {
        const int k = kmaxs[ki];
        if (sc == 1 && k == 128) continue;
        for (int bi = 0; bi < 2 && err == 0; ++bi) {
          const int n = batches[bi];
          const size_t sb = sc ? 16 : 8;
          std::vector<QRNodeDev> nodes(n);
          std::vector<QRApplyDev> jobs(n);
          for (int a = 0; a < n; ++a) {
            QRNodeDev nd{};
            nd.rows = MC;
            nd.k = k;
            nd.steps = k < MC ? k : MC;
            nd.level0 = 1;
            nd.P1 = (const char*)B + (size_t)a * MC * k * sb;
            nd.P2 = nd.P1;
            nd.ld1 = nd.ld2 = MC;
            nd.n1 = k;
            nd.store = (int64_t)a * MC * k;
            nd.ab = a * k;
            nodes[a] = nd;
            QRApplyDev J{};
            J.rows = MC;
            J.steps = nd.steps;
            J.r = k;
            J.store = nd.store;
            J.ab = nd.ab;
            J.Zin = (const char*)B + (size_t)a * MC * k * sb;
            J.ldin = MC;
            J.Zout = (char*)Z + (size_t)a * MC * k * sb;
            J.ldout = MC;
            jobs[a] = J;
          }
          if (!ok(hipMemcpyAsync(dn, nodes.data(), n * sizeof(QRNodeDev), hipMemcpyHostToDevice,
                                 st)) ||
              !ok(hipMemcpyAsync(dj, jobs.data(), n * sizeof(QRApplyDev), hipMemcpyHostToDevice,
                                 st)))
            break;
          double best = 0.0;
          int pick = 1;
          for (int lay = 0; lay < 2 && err == 0; ++lay) {
            g_tsqr_layout[sc][ki][bi] = lay;
            // warm-up, then three timed factor + apply pairs
            int le = tsqr_factor_launch(sc, k, dn, n, nullptr, store, alpha, beta, st);
            if (le == 0) le = tsqr_apply_launch(sc, k, dj, n, store, beta, st);
            if (le != 0) {
              err = le;
              break;
            }
            ok(hipEventRecord(e0, st));
            for (int rep = 0; rep < 3 && le == 0; ++rep) {
              le = tsqr_factor_launch(sc, k, dn, n, nullptr, store, alpha, beta, st);
              if (le == 0) le = tsqr_apply_launch(sc, k, dj, n, store, beta, st);
            }
            if (le != 0) {
              err = le;
              break;
            }
            ok(hipEventRecord(e1, st));
            ok(hipEventSynchronize(e1));
            float ms = 0.0f;
            ok(hipEventElapsedTime(&ms, e0, e1));
            const double t = ms * 1e3 / 3.0;
            if (us) us[((sc * 4 + ki) * 2 + bi) * 2 + lay] = t;
            if (lay == 0 || t < best) {
              best = t;
              pick = lay;
            }
          }
          g_tsqr_layout[sc][ki][bi] = pick;
        }
      }
  }
  if (table)
    for (int i = 0; i < 16; ++i) table[i] = (&g_tsqr_layout[0][0][0])[i];
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  for (void* q : {(void*)B, (void*)store, (void*)alpha, (void*)beta, (void*)Z, (void*)dn, (void*)dj})
    if (q) (void)hipFree(q);
  return err;
}

int svd_launch(int scalar, const SVDJobDev* jobs, int n, int kmax_batch, int pmax_batch,
               const void* store, const void* alpha, double eps, hipStream_t st,
               int force_storage, bool precond_only) {
  if (n == 0) return 0;
  if (kmax_batch > 512 || pmax_batch > 512) return -1;
  const size_t sb = scalar == 0 ? 8 : 16;
  const size_t lds_cap = 158 * 1024;
  const size_t aux = svd_aux_bytes(pmax_batch, kmax_batch);
  const size_t full = svd_mat_bytes(pmax_batch, kmax_batch, sb) + aux;
  const bool in_lds = full <= lds_cap && force_storage != 1;
  const size_t sh = in_lds ? full : aux;
  auto go = [&](auto kern, auto tag) {
    using TT = decltype(tag);
    if (sh > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL(kern, dim3(n), dim3(SVD_NT), sh, st, jobs, (const TT*)store, (const TT*)alpha,
                       eps, precond_only ? 1 : 0);
  };
  if (scalar == 0) {
    if (in_lds) go(svd_kernel<double, true>, 0.0);
    else go(svd_kernel<double, false>, 0.0);
  } else {
    if (in_lds) go(svd_kernel<hb_cplx, true>, hb_cplx{});
    else go(svd_kernel<hb_cplx, false>, hb_cplx{});
  }
  return (int)hipGetLastError();
}

// Workgroups per matrix of the multi-workgroup SVD for a width k (0 when the
// shape does not suit it: p < k or p > WS_PMAX, or a single block pair).
int svd_wide_blocks(int scalar, int p, int k) {
  const int nb = scalar == 0 ? WideCfg<double>::NB : WideCfg<hb_cplx>::NB;
  if (p < k || p > WS_PMAX || k <= 2 * nb) return 0;
  return (k + 2 * nb - 1) / (2 * nb);
}

// Cooperative launch of svd_wide_kernel over njobs * B workgroups.  work
// holds 3 ints and njobs * B doubles (svd_wide_work_bytes).  Returns -2 when
// the grid cannot be co-resident (svd_wide_fits tells beforehand), a HIP
// error code otherwise, 0 on success.
size_t svd_wide_work_bytes(int njobs, int B) { return 32 + (size_t)njobs * B * 8; }

static const void* wide_kernel(int scalar) {
  return scalar == 0 ? (const void*)svd_wide_kernel<double> : (const void*)svd_wide_kernel<hb_cplx>;
}
static size_t wide_lds(int scalar, int pmax) {
  const int nb = scalar == 0 ? WideCfg<double>::NB : WideCfg<hb_cplx>::NB;
  return (size_t)2 * nb * pmax * (scalar == 0 ? 8 : 16);
}

bool svd_wide_fits(int scalar, int njobs, int B, int pmax) {
  const void* kern = wide_kernel(scalar);
  const size_t sh = wide_lds(scalar, pmax);
  if (sh > 64 * 1024)
    (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WS_NT, sh) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (int64_t)njobs * B <= (int64_t)cus * per_cu;
}

int svd_wide_launch(int scalar, const SVDJobDev* jobs, int njobs, int B, int pmax,
                    const void* store, const void* alpha, double eps, void* work, hipStream_t st) {
  if (njobs == 0) return 0;
  if (!svd_wide_fits(scalar, njobs, B, pmax)) return -2;
  const void* kern = wide_kernel(scalar);
  const size_t sh = wide_lds(scalar, pmax);
  int e = zero_fill_launch(work, 32, st);
  if (e != 0) return e;
  int* flags = (int*)work;
  double* parts = (double*)((char*)work + 32);
  void* args[] = {(void*)&jobs, (void*)&B, (void*)&store, (void*)&alpha, (void*)&eps,
                  (void*)&flags, (void*)&parts};
  return (int)hipLaunchCooperativeKernel(kern, dim3(njobs * B), dim3(WS_NT), args, sh, st);
}

int block_gemm_launch(int scalar, const BlockGemmDev* jobs, int n, int max_rows, int max_rin,
                      hipStream_t st) {
  if (n == 0 || max_rows == 0) return 0;
  dim3 grid((max_rows + BG_NT - 1) / BG_NT, n);
  const size_t sh = (size_t)max_rin * BG_CT * (scalar == 0 ? 8 : 16);
  if (sh > 160 * 1024) return -1;
  if (scalar == 0)
    hipLaunchKernelGGL((block_gemm_kernel<double>), grid, dim3(BG_NT), sh, st, jobs, max_rin);
  else
    hipLaunchKernelGGL((block_gemm_kernel<hb_cplx>), grid, dim3(BG_NT), sh, st, jobs, max_rin);
  return (int)hipGetLastError();
}

int concat_launch(int scalar, const ConcatDev* jobs, int n, int64_t max_m, int, hipStream_t st) {
  if (n == 0 || max_m == 0) return 0;
  dim3 g((unsigned)((max_m + 255) / 256), n);
  if (scalar == 0)
    hipLaunchKernelGGL((concat_kernel<double>), g, dim3(256), 0, st, jobs);
  else
    hipLaunchKernelGGL((concat_kernel<hb_cplx>), g, dim3(256), 0, st, jobs);
  return (int)hipGetLastError();
}


int rcopy_launch(int scalar, const RCopyDev* jobs, int n, const void* store, const void* alpha,
                 hipStream_t st) {
  if (n == 0) return 0;
  if (scalar == 0)
    hipLaunchKernelGGL((rcopy_kernel<double>), dim3(n), dim3(256), 0, st, jobs,
                       (const double*)store, (const double*)alpha);
  else
    hipLaunchKernelGGL((rcopy_kernel<hb_cplx>), dim3(n), dim3(256), 0, st, jobs,
                       (const hb_cplx*)store, (const hb_cplx*)alpha);
  return (int)hipGetLastError();
}

int rrh_launch(int scalar, const RRhDev* jobs, int n, int64_t max_entries, hipStream_t st) {
  if (n == 0 || max_entries == 0) return 0;
  if (n > 65535) return -1;
  const dim3 g((unsigned)((max_entries + 255) / 256), (unsigned)n);
  if (scalar == 0)
    hipLaunchKernelGGL((rrh_explicit_kernel<double>), g, dim3(256), 0, st, jobs);
  else
    hipLaunchKernelGGL((rrh_explicit_kernel<hb_cplx>), g, dim3(256), 0, st, jobs);
  return (int)hipGetLastError();
}

int rcompact_launch(int scalar, const RCompactDev* jobs, int n, hipStream_t st) {
  if (n == 0) return 0;
  if (scalar == 0)
    hipLaunchKernelGGL((rcompact_kernel<double>), dim3(n), dim3(256), 0, st, jobs);
  else
    hipLaunchKernelGGL((rcompact_kernel<hb_cplx>), dim3(n), dim3(256), 0, st, jobs);
  return (int)hipGetLastError();
}

int zero_fill_launch(void* ptr, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 8;
  if (n == 0) return 0;
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (uint64_t*)ptr, n);
  return (int)hipGetLastError();
}


int copy_list_launch(const CopyDev* jobs, int n, hipStream_t st) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(copy_list_kernel, dim3(n), dim3(64), 0, st, jobs);
  return (int)hipGetLastError();
}

}  // namespace hbk
