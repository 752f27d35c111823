// Blocked adaptive cross approximation of one leaf per workgroup
// (Algorithm 2 of the paper, with its LRID, LRnorm and LRnormUp functions).
//
// Layout and work split (512 threads = 8 wave64s per leaf):
//  * the factors live in HBM: U (m0 x cap) and Vh = V^H (n0 x cap), both
//    column-major, so a wave reading one column touches consecutive rows;
//  * the residual column block C_k = A(:, J_k) - U V(:, J_k) is computed with
//    one thread per row (RPT rows per thread), V(:, J_k) staged through LDS in
//    tiles; it is written once to HBM scratch (U_k and W_k gather from it) and
//    kept in registers as the QRCP panel that picks I_k (eq. (6));
//  * the residual row block R_k = A(I_k, :) - U(I_k, :) V is computed with one
//    thread per column and never leaves registers: it feeds V_k (eq. (9))
//    and the QRCP panel that picks J_{k+1} (eq. (7));
//  * QRCP(W_k, eps) (eq. (8)) runs in one wave, one column per lane;
//  * the norm estimates (eqs. (11)-(13)) use the Gram blocks
//    [U, U_k]^H U_k and [Vh, Vh_k]^H Vh_k, accumulated from LDS-staged row
//    chunks with 4x2 register blocking and a deterministic cross-wave sum.
//
// Pivot choice follows the reading of QR(., d) stated at qrcp_select: exact
// trailing norms after each Householder step, largest first, ties to the
// lowest index; the strong rank-revealing selection refines it with swaps.
//
// This header holds the device code and the launch template; hb_baca.hip
// instantiates the kernels with greedy QRCP, hb_baca_strong.hip those with
// the strong selection (two translation units, compiled in parallel).
#pragma once

#include "hb_common.h"
#include "hb_entries.h"
#include "hb_internal.h"
#include "hb_merge.h"

namespace {

constexpr int NT = 512;
// Trailing norms below this fraction of a panel's largest column norm are
// rounding left by the earlier reflectors and count as zero in the pivot
// choice (ties go to the lowest index), so that the picks do not depend on
// the order of rounding.
constexpr double QRCP_NOISE = 1e-12;
constexpr int NW = NT / HB_WAVE;
constexpr int LCH = 8;  // HBM loads issued together before their first use

template <typename T, int DMAX>
struct GramCfg {
  static constexpr int CB = DMAX / 2;       // column blocks of 2
  static constexpr int TB = HB_WAVE / CB;   // row blocks of 4
  static constexpr int GT = 4 * TB;         // t-tile width
  // rows per staged chunk: the staging buffers hold at most 2048 + 1024
  // elements, and every chunk costs two barriers and one HBM round trip
  static constexpr int GCH = (2048 / GT < 1024 / DMAX) ? 2048 / GT : 1024 / DMAX;
  // row strides of the staged chunks, one element longer than a row: the
  // transposing stores of consecutive lanes (consecutive rows) then fall in
  // different LDS banks instead of all in one
  static constexpr int XLD = GT + 1;
  static constexpr int KLD = DMAX + 1;
};

// G[tt * DMAX + c] = sum_i conj(X(i, t0 + tt)) * X(i, k0 + c), tt < tw, c < dk.
// X is column-major with leading dimension ld and `nrows` rows.  The result
// lands in sG (GT x DMAX).  All threads of the block must call it.
template <typename T, int DMAX>
__device__ __forceinline__ void gram_tile(const T* __restrict__ X, int64_t ld, int nrows, int t0, int tw, int k0,
                          int dk, T* sXs, T* sKs, typename acc_type<T>::type* sG) {
  using C = GramCfg<T, DMAX>;
  using TA = typename acc_type<T>::type;
  constexpr int NX = (C::GCH * C::GT + NT - 1) / NT;   // staged elements per thread
  constexpr int NK = (C::GCH * DMAX + NT - 1) / NT;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int tb = lane % C::TB, cb = lane / C::TB;
  TA acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = sc_zero<TA>();
#pragma unroll 1
  for (int i0 = 0; i0 < nrows; i0 += C::GCH) {
    // all loads of the chunk are issued before any is used; indexes are
    // clamped into the matrix and out-of-range values replaced by zero
    T vx[NX], vk[NK];
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int e = tid + u * NT, ii = e % C::GCH, tt = e / C::GCH, i = i0 + ii;
      const int ic = i < nrows ? i : nrows - 1, tc = tt < tw ? tt : tw - 1;
      const T v = X[(int64_t)(t0 + tc) * ld + ic];
      vx[u] = (i < nrows && tt < tw) ? v : sc_zero<T>();
    }
#pragma unroll
    for (int u = 0; u < NK; ++u) {
      const int e = tid + u * NT, ii = e % C::GCH, c = e / C::GCH, i = i0 + ii;
      const int ic = i < nrows ? i : nrows - 1, cc = c < dk ? c : dk - 1;
      const T v = X[(int64_t)(k0 + cc) * ld + ic];
      vk[u] = (i < nrows && c < dk) ? v : sc_zero<T>();
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int e = tid + u * NT;
      if (e < C::GCH * C::GT) sXs[(e % C::GCH) * C::XLD + e / C::GCH] = vx[u];
    }
#pragma unroll
    for (int u = 0; u < NK; ++u) {
      const int e = tid + u * NT;
      if (e < C::GCH * DMAX) sKs[(e % C::GCH) * C::KLD + e / C::GCH] = vk[u];
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < C::GCH / NW; ++q) {
      const int ii = wid * (C::GCH / NW) + q;
      T xa[4], kb[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = sXs[ii * C::XLD + 4 * tb + a];
#pragma unroll
      for (int b = 0; b < 2; ++b) kb[b] = sKs[ii * C::KLD + 2 * cb + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) sc_cfma(acc[a][b], sc_to_acc(xa[a]), sc_to_acc(kb[b]));
    }
  }
  // deterministic cross-wave sum: wave 0 writes, waves 1..7 add in order
  for (int w = 0; w < NW; ++w) {
    __syncthreads();
    if (wid == w) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int idx = (4 * tb + a) * DMAX + 2 * cb + b;
          sG[idx] = (w == 0) ? acc[a][b] : sc_add(sG[idx], acc[a][b]);
        }
    }
  }
  __syncthreads();
}

// Upper Cholesky factor in place (G = T^H T, T stored over G's upper part)
// by one wave: the diagonal of row j from a wave sum, its off-diagonal
// entries one per lane.  Returns false on a pivot <= 0 (same in every lane).
template <typename T, int DMAX>
__device__ __forceinline__ bool chol_wave(T* G, int n, int lane) {
  for (int j = 0; j < n; ++j) {
    double part = 0.0;
    for (int k = lane; k < j; k += HB_WAVE) part += sc_abs2(G[k * DMAX + j]);
    part = wave_sum(part);
    const double sj = sc_re(G[j * DMAX + j]) - part;
    if (!(sj > 0.0)) return false;
    const double d = sqrt(sj);
    const double id = 1.0 / d;
    for (int c = j + 1 + lane; c < n; c += HB_WAVE) {
      T v = G[j * DMAX + c];
      for (int k = 0; k < j; ++k) v = sc_sub(v, sc_cmul(G[k * DMAX + j], G[k * DMAX + c]));
      G[j * DMAX + c] = sc_scale(v, id);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane == 0) G[j * DMAX + j] = sc_real<T>(d);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  return true;
}

// Greedy QRCP pivot selection over a register-resident panel (Algorithm 2,
// lines selecting I_k and J_{k+1}).  Each thread owns RPT candidates (index
// tid + s * NT) with panel vectors x[s][0..nrow).  `excl[idx] != 0` removes a
// candidate.  Writes the nsel chosen indices to out[].  Destroys x.  Returns
// (to every thread) how many leading picks had a trailing norm above the
// rounding level: the panel's numerical rank as the selection saw it.
// One barrier per step: every wave publishes its best candidate's vector
// with its (norm, index); after the barrier all threads take the overall
// winner from LDS.  Buffers alternate between steps.
template <typename T, int DMAX, int RPT>
__device__ __forceinline__ int qrcp_select(T (&x)[RPT][DMAX], int ncand_total, const unsigned char* excl,
                            int nrow, int nsel, int* out, T (*sPivW)[NW][DMAX], double (*redv)[NW],
                            int (*redi)[NW]) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  bool picked[RPT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) picked[s] = false;
  // the largest squared norm at the first step: later trailing norms below
  // QRCP_NOISE of it are rounding only and count as zero (ties to the
  // lowest index)
  double zero2 = 0.0;
  int nz = 0;
  bool noise = false;
#pragma unroll 1
  for (int st = 0; st < nsel; ++st) {
    const int bb = st & 1;
    double bv = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int i = tid + s * NT;
      if (i < ncand_total && excl[i] == 0 && !picked[s]) {
        double nv = 0.0;
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          if (c >= st && c < nrow) nv += sc_abs2(x[s][c]);
        // a NaN norm (non-finite data) must still leave a valid winner
        if (!(nv == nv)) nv = 0.0;
        if (nv < zero2) nv = 0.0;
        if (nv > bv || (nv == bv && i < bi)) {
          bv = nv;
          bi = i;
        }
      }
    }
    wave_argmax(bv, bi);
    if (lane == 0) {
      redv[bb][wid] = bv;
      redi[bb][wid] = bi;
    }
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      if (tid + s * NT == bi) {
#pragma unroll
        for (int c = 0; c < DMAX; ++c) sPivW[bb][wid][c] = x[s][c];
      }
    }
    __syncthreads();
    int ww = 0;
    bv = redv[bb][0];
    bi = redi[bb][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const double ov = redv[bb][w];
      const int oi = redi[bb][w];
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
        ww = w;
      }
    }
    if (st == 0) zero2 = QRCP_NOISE * QRCP_NOISE * bv;
    if (bv > 0.0 && !noise) ++nz;
    else noise = true;
#pragma unroll
    for (int s = 0; s < RPT; ++s)
      if (tid + s * NT == bi) picked[s] = true;
    if (tid == 0) out[st] = bi;
    const T* piv = sPivW[bb][ww];
    // Householder reflector of the pivot's trailing part, applied to the rest
    double sig2 = 0.0;
#pragma unroll
    for (int c = 0; c < DMAX; ++c)
      if (c >= st && c < nrow) sig2 += sc_abs2(piv[c]);
    const double sigma = sqrt(sig2);
    if (sigma > 0.0 && st + 1 < nsel) {
      const T x0 = piv[st];
      const double a0 = sqrt(sc_abs2(x0));
      const T alpha = sc_scale(sc_phase(x0), -sigma);
      const double beta = 1.0 / (sigma * (sigma + a0));
      const T v0 = sc_sub(x0, alpha);
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int i = tid + s * NT;
        if (i < ncand_total && excl[i] == 0 && !picked[s]) {
          T w = sc_zero<T>();
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nrow) sc_cfma(w, c == st ? v0 : piv[c], x[s][c]);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nrow) sc_axpy_neg(x[s][c], beta, c == st ? v0 : piv[c], w);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }
  // the chosen indices are read after the call
  __syncthreads();
  return nz;
}

// Workgroup argmax of (val, idx): larger value wins, equal values go to the
// lower index.  Every thread receives the winner.  Uses rv / ri (NW entries
// of LDS each) between two barriers, so consecutive calls may reuse them.
__device__ __forceinline__ void block_argmax(double& val, int& idx, double* rv, int* ri) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  wave_argmax(val, idx);
  if (lane == 0) {
    rv[wid] = val;
    ri[wid] = idx;
  }
  __syncthreads();
  val = rv[0];
  idx = ri[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    const double ov = rv[w];
    const int oi = ri[w];
    if (ov > val || (ov == val && oi < idx)) {
      val = ov;
      idx = oi;
    }
  }
  __syncthreads();
}

// Strong rank-revealing refinement of a QRCP selection (the alternative to
// greedy QRCP named beside eqs. (6)-(7); the swaps of Gu and Eisenstat's
// strong RRQR).  The panel is M(c, idx) = G[c * ld + idx], c < nrow (its
// conjugate gives the same coefficient magnitudes); candidates are
// idx < ncand with excl[idx] == 0.  sel[0..k) are QRCP's picks above the
// rounding level, sel[k..nsel) the rounding-level ones.  Each round
//   1. wave 0 factors M(:, sel[0..k)) = Q R by Householder reflections
//      (reflectors in sRefl / sBeta, R in sTm, 1 / diag(R) in sTinv);
//   2. every thread solves R w = Q^H M(:, j) for its candidates j outside
//      sel[0..k) and keeps the largest |w(i)| (ties: lowest j, then lowest i);
//   3. a workgroup argmax; if the winner exceeds f, j replaces sel[i].
// With the panel of numerical rank k the trailing block of the pivoted QR
// counts as zero, so |w(i)| is exactly the factor by which the swap grows
// the volume of the chosen columns.  At most SWAP_CAP * k swaps.  When a
// swap was made the picks past k are re-taken as the lowest free indices
// (the tie rule of rounding-level norms).  Returns the number of swaps, the
// same in every thread.  sRefl, sBeta, sTm, sTinv and sPcol are free at both
// call sites (the cross block's factorisation is not live there).
constexpr int SWAP_CAP = 4;

template <typename T, int DMAX, int RPT>
__device__ __forceinline__ int strong_refine(const T* __restrict__ G, int64_t ld, int nrow, int ncand,
                                             const unsigned char* excl, int* sel, int nsel, int k,
                                             double f, T* sRefl, double* sBeta, T* sTm, T* sTinv,
                                             T* sPcol, double* rv, int* ri) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int swaps = 0;
  if (k <= 0) return 0;
#pragma unroll 1
  while (swaps < SWAP_CAP * k) {
    // ---- 1. Householder QR of the k chosen columns (wave 0, lane i holds column i)
    if (wid == 0) {
      T w[DMAX];
      {
        const int idx = sel[lane < k ? lane : 0];
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          const T v = G[(int64_t)(c < nrow ? c : 0) * ld + idx];
          w[c] = (lane < k && c < nrow) ? v : sc_zero<T>();
        }
      }
#pragma unroll 1
      for (int st = 0; st < k; ++st) {
        if (lane == st) {
#pragma unroll
          for (int c = 0; c < DMAX; ++c) sPcol[c] = w[c];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        T pc[DMAX];
#pragma unroll
        for (int c = 0; c < DMAX; ++c) pc[c] = sPcol[c];
        double sig2 = 0.0;
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          if (c >= st && c < nrow) sig2 += sc_abs2(pc[c]);
        const double sigma = sqrt(sig2);
        const T x0 = sPcol[st];
        T alpha = sc_zero<T>();
        double beta = 0.0;
        if (sigma > 0.0) {
          alpha = sc_scale(sc_phase(x0), -sigma);
          beta = 1.0 / (sigma * (sigma + sqrt(sc_abs2(x0))));
        }
        const T v0 = sc_sub(x0, alpha);
        T ww = sc_zero<T>();
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          if (c >= st && c < nrow) sc_cfma(ww, c == st ? v0 : pc[c], w[c]);
        const bool upd = lane > st && lane < k && beta != 0.0;
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          if (upd && c >= st && c < nrow) sc_axpy_neg(w[c], beta, c == st ? v0 : pc[c], ww);
          if (lane == 0 && c >= st && c < nrow) sRefl[st * DMAX + c] = (c == st) ? v0 : pc[c];
        }
        if (lane == st) {
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c < st) sTm[c * DMAX + st] = w[c];
          sTm[st * DMAX + st] = alpha;
          sTinv[st] = sigma > 0.0 ? sc_div(sc_real<T>(1.0), alpha) : sc_zero<T>();
        }
        if (lane == 0) sBeta[st] = beta;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    __syncthreads();
    // ---- 2. coefficients of every other candidate in the chosen basis
    double bv = -1.0;
    int bi = 0x7fffffff;
#pragma unroll 1
    for (int s = 0; s < RPT; ++s) {
      const int j = tid + s * NT;
      bool cand = j < ncand && excl[j] == 0;
      for (int c = 0; c < k; ++c) cand = cand && sel[c] != j;
      if (cand) {
        T z[DMAX];
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          const T v = G[(int64_t)(c < nrow ? c : 0) * ld + j];
          z[c] = c < nrow ? v : sc_zero<T>();
        }
#pragma unroll 1
        for (int st = 0; st < k; ++st) {
          T ww = sc_zero<T>();
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nrow) sc_cfma(ww, sRefl[st * DMAX + c], z[c]);
          const double beta = sBeta[st];
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nrow) sc_axpy_neg(z[c], beta, sRefl[st * DMAX + c], ww);
        }
#pragma unroll 1
        for (int cc = k - 1; cc >= 0; --cc) {
          T sum = sc_zero<T>();
#pragma unroll
          for (int e = 0; e < DMAX; ++e) {
            if (e == cc) sum = sc_add(sum, z[e]);
            if (e > cc && e < k) sum = sc_sub(sum, sc_mul(sTm[cc * DMAX + e], z[e]));
          }
          sum = sc_mul(sum, sTinv[cc]);
#pragma unroll
          for (int e = 0; e < DMAX; ++e)
            if (e == cc) z[e] = sum;
        }
#pragma unroll
        for (int e = 0; e < DMAX; ++e) {
          if (e < k) {
            double a = sqrt(sc_abs2(z[e]));
            if (!(a == a)) a = 0.0;  // non-finite data must not swap
            const int ci = j * DMAX + e;
            if (a > bv || (a == bv && ci < bi)) {
              bv = a;
              bi = ci;
            }
          }
        }
      }
    }
    // ---- 3. the largest coefficient decides the swap
    block_argmax(bv, bi, rv, ri);
    if (!(bv > f)) break;
    if (tid == 0) sel[bi % DMAX] = bi / DMAX;
    ++swaps;
    __syncthreads();
  }
  if (swaps > 0 && k < nsel) {
    // the rounding-level picks: the lowest indices not chosen
#pragma unroll 1
    for (int t = k; t < nsel; ++t) {
      double bv = -1.0;
      int bi = 0x7fffffff;
#pragma unroll 1
      for (int s = 0; s < RPT; ++s) {
        const int j = tid + s * NT;
        bool cand = j < ncand && excl[j] == 0;
        for (int c = 0; c < t; ++c) cand = cand && sel[c] != j;
        if (cand && j < bi) {
          bv = 0.0;
          bi = j;
        }
      }
      block_argmax(bv, bi, rv, ri);
      if (tid == 0) sel[t] = bi;
      __syncthreads();
    }
  }
  return swaps;
}

// True when the first n entries of the LDS index list lie in [0, lim).  Every
// thread reads the same entries after a barrier, so the answer is uniform
// over the workgroup and a loop may be left on it.
__device__ __forceinline__ bool pivots_in_range(const int* idx, int n, int lim) {
  bool ok = true;
  for (int c = 0; c < n; ++c) ok = ok && idx[c] >= 0 && idx[c] < lim;
  return ok;
}

// BACA of leaf `li` by the whole workgroup.
template <typename T, int DMAX, int RPT, bool STRONG>
__device__ __forceinline__ void baca_leaf(const BacaArgs& A, const int li) {
  using C = GramCfg<T, DMAX>;
  using TA = typename acc_type<T>::type;  // FP32 data accumulate in FP64
  constexpr int TILE = 32;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const BacaLeafDev L = A.leaves[li];
  const int m0 = L.m0, n0 = L.n0, cap = L.cap;
  const int rmax = min(m0, n0);
  T* __restrict__ U = (T*)A.U + L.u_off;
  T* __restrict__ Vh = (T*)A.V + L.v_off;
  const double eps = A.eps;
  const int dim = A.E.dim;

  __shared__ int sJ[DMAX], sI[DMAX], sJbar[DMAX];
  __shared__ int sDK, sNJ;
  __shared__ unsigned char used_r[NT * RPT], used_c[NT * RPT];
  __shared__ double redv[2][NW];
  __shared__ int redi[2][NW];
  __shared__ double redd[NW];
  __shared__ T sPivW[2][NW][DMAX];
  __shared__ T sPcol[DMAX];
  __shared__ T sRefl[DMAX * DMAX];
  __shared__ double sBeta[DMAX];
  __shared__ T sTm[DMAX * DMAX];
  __shared__ T sTinv[DMAX];
  __shared__ double sTabs[DMAX];
  __shared__ double sPts[DMAX * HB_MAXDIM];
  __shared__ T sTile[DMAX * TILE];
  __shared__ T sXs[C::GCH * C::XLD];
  __shared__ T sKs[C::GCH * C::KLD];
  __shared__ TA sG[C::GT * DMAX];
  __shared__ TA sGU[C::GT * DMAX];
  __shared__ TA sGUd[DMAX * DMAX];
  __shared__ TA sGVd[DMAX * DMAX];
  __shared__ double sScal[3];
  __shared__ int sOk[2];

  for (int i = tid; i < NT * RPT; i += NT) {
    used_r[i] = 0;
    used_c[i] = 0;
  }
  if (tid < DMAX) sJ[tid] = (tid < L.nj1) ? A.j1[L.j1_off + tid] : 0;
  if (tid == 0) sNJ = L.nj1;
  __syncthreads();

  double mu2 = 0.0;
  int r = 0, iter = 0, status = 0, swaps = 0;

  while (true) {
    // The residual blocks' bases are taken anew in every iteration: the
    // empty asm hides that they do not change, so the compiler does not keep
    // the per-column addresses (2 RPT DMAX 64-bit values) live across
    // iterations, where they spilled to scratch.
    uint64_t cbase = (uint64_t)((T*)A.C + L.c_off), rbase = (uint64_t)((T*)A.R + L.r_off);
    asm volatile("" : "+v"(cbase), "+v"(rbase));
    T* __restrict__ Cg = (T*)cbase;
    T* __restrict__ Rg = (T*)rbase;
    const int nJ = sNJ;
    if (r + min(nJ, m0 - r) > cap) {
      status = 1;
      break;
    }
    // Every pivot index is checked before it addresses memory: a winner
    // outside the candidate range (possible only with non-finite data) ends
    // the leaf with status 2 instead of reading past the point arrays.
    if (!pivots_in_range(sJ, nJ, n0)) {
      status = 2;
      break;
    }
    // ------------------------------------------------ C_k = A(:,J) - U V(:,J)
    if (tid < nJ * dim) {
      const int c = tid / dim, q = tid % dim;
      sPts[c * HB_MAXDIM + q] = A.E.Y[(int64_t)q * A.E.ldy + L.col0 + sJ[c]];
    }
    __syncthreads();
    // entries A(:, J_k) straight to the scratch block
#pragma unroll 1
    for (int s = 0; s < RPT; ++s) {
      const int i = tid + s * NT;
      if (i < m0) {
        double xi[HB_MAXDIM];
#pragma unroll
        for (int q = 0; q < HB_MAXDIM; ++q)
          xi[q] = q < dim ? A.E.X[(int64_t)q * A.E.ldx + L.row0 + i] : 0.0;
#pragma unroll 1
        for (int c = 0; c < nJ; ++c)
          Cg[(int64_t)c * m0 + i] =
              eval_entry<T>(A.E, L.row0 + i, L.col0 + sJ[c], xi, &sPts[c * HB_MAXDIM]);
      }
    }
    TA xa[RPT][DMAX];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
#pragma unroll
      for (int c = 0; c < DMAX; ++c) xa[s][c] = sc_zero<TA>();
    for (int t0 = 0; t0 < r; t0 += TILE) {
      const int tw = min(TILE, r - t0);
      __syncthreads();
      for (int e = tid; e < nJ * TILE; e += NT) {
        const int c = e / TILE, tt = e % TILE;
        sTile[c * TILE + tt] =
            tt < tw ? sc_conj(Vh[(int64_t)(t0 + tt) * n0 + sJ[c]]) : sc_zero<T>();
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int i = tid + s * NT;
        const int ic = i < m0 ? i : m0 - 1;
        // TILE factor columns per pass, loaded LCH at a time before use;
        // entries past tw have zero weights in sTile
#pragma unroll 1
        for (int tb0 = 0; tb0 < tw; tb0 += LCH) {
          T uu[LCH];
#pragma unroll
          for (int u = 0; u < LCH; ++u) uu[u] = U[(int64_t)(t0 + min(tb0 + u, tw - 1)) * m0 + ic];
#pragma unroll
          for (int u = 0; u < LCH; ++u) {
#pragma unroll
            for (int c = 0; c < DMAX; ++c)
              if (c < nJ) sc_fma(xa[s][c], sc_to_acc(uu[u]), sc_to_acc(sTile[c * TILE + tb0 + u]));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
    // C_k = A(:, J_k) - U V(:, J_k); the panel is its conjugate transpose
    T x[RPT][DMAX];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int i = tid + s * NT;
      const int ic = i < m0 ? i : m0 - 1;
#pragma unroll
      for (int c0 = 0; c0 < DMAX; c0 += LCH) {
        T cv[LCH];
#pragma unroll
        for (int u = 0; u < LCH; ++u) cv[u] = Cg[(int64_t)min(c0 + u, nJ - 1) * m0 + ic];
#pragma unroll
        for (int u = 0; u < LCH; ++u) {
          const int c = c0 + u;
          const T v = sc_from_acc<T>(sc_sub(sc_to_acc(cv[u]), xa[s][c]));
          if (i < m0 && c < nJ) Cg[(int64_t)c * m0 + i] = v;
          x[s][c] = (i < m0 && c < nJ) ? sc_conj(v) : sc_zero<T>();
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // ------------------------------------------------ I_k = QR(C^H, d) (eq. (6))
    const int nI = min(nJ, m0 - r);
    {
      const int kI = qrcp_select<T, DMAX, RPT>(x, m0, used_r, nJ, nI, sI, sPivW, redv, redi);
      // the strong selection works on the residual block C_k itself (whose
      // conjugate is the panel)
      if constexpr (STRONG)
        swaps += strong_refine<T, DMAX, RPT>(Cg, m0, nJ, m0, used_r, sI, nI, kI, A.select_f, sRefl,
                                             sBeta, sTm, sTinv, sPcol, redv[0], redi[0]);
    }
    // (the selection ends with a barrier, so sI is visible)
    if (!pivots_in_range(sI, nI, m0)) {
      status = 2;
      break;
    }

    // ------------------------------------------------ R_k = A(I,:) - U(I,:) V
    if (tid < nI * dim) {
      const int c = tid / dim, q = tid % dim;
      sPts[c * HB_MAXDIM + q] = A.E.X[(int64_t)q * A.E.ldx + L.row0 + sI[c]];
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < RPT; ++s) {
      const int j = tid + s * NT;
      if (j < n0) {
        double yj[HB_MAXDIM];
#pragma unroll
        for (int q = 0; q < HB_MAXDIM; ++q)
          yj[q] = q < dim ? A.E.Y[(int64_t)q * A.E.ldy + L.col0 + j] : 0.0;
#pragma unroll 1
        for (int c = 0; c < nI; ++c)
          Rg[(int64_t)c * n0 + j] =
              eval_entry<T>(A.E, L.row0 + sI[c], L.col0 + j, &sPts[c * HB_MAXDIM], yj);
      }
    }
    {
      TA y[RPT][DMAX];
#pragma unroll
      for (int s = 0; s < RPT; ++s)
#pragma unroll
        for (int c = 0; c < DMAX; ++c) y[s][c] = sc_zero<TA>();
      for (int t0 = 0; t0 < r; t0 += TILE) {
        const int tw = min(TILE, r - t0);
        __syncthreads();
        for (int e = tid; e < nI * TILE; e += NT) {
          const int c = e / TILE, tt = e % TILE;
          sTile[c * TILE + tt] = tt < tw ? U[(int64_t)(t0 + tt) * m0 + sI[c]] : sc_zero<T>();
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int j = tid + s * NT;
          const int jc = j < n0 ? j : n0 - 1;
#pragma unroll 1
          for (int tb0 = 0; tb0 < tw; tb0 += LCH) {
            T vv[LCH];
#pragma unroll
            for (int u = 0; u < LCH; ++u)
              vv[u] = sc_conj(Vh[(int64_t)(t0 + min(tb0 + u, tw - 1)) * n0 + jc]);
#pragma unroll
            for (int u = 0; u < LCH; ++u) {
#pragma unroll
              for (int c = 0; c < DMAX; ++c)
                if (c < nI) sc_fma(y[s][c], sc_to_acc(sTile[c * TILE + tb0 + u]), sc_to_acc(vv[u]));
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      }
      // R_k = A(I_k, :) - U(I_k, :) V, kept transposed in the scratch block
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int j = tid + s * NT;
        const int jc = j < n0 ? j : n0 - 1;
#pragma unroll
        for (int c0 = 0; c0 < DMAX; c0 += LCH) {
          T rv[LCH];
#pragma unroll
          for (int u = 0; u < LCH; ++u) rv[u] = Rg[(int64_t)min(c0 + u, nI - 1) * n0 + jc];
#pragma unroll
          for (int u = 0; u < LCH; ++u) {
            const int c = c0 + u;
            if (j < n0 && c < nI)
              Rg[(int64_t)c * n0 + j] = sc_from_acc<T>(sc_sub(sc_to_acc(rv[u]), y[s][c]));
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // ------------------------------------------------ W_k and QR(W_k, eps) (eq. (8))
    if (wid == 0) {
      T w[DMAX];
      bool rem = lane < nJ;
      {
        const int lc = lane < nJ ? lane : nJ - 1;
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          const T v = Cg[(int64_t)lc * m0 + sI[c < nI ? c : nI - 1]];
          w[c] = (lane < nJ && c < nI) ? v : sc_zero<T>();
        }
      }
      const int q = min(nI, nJ);
      double zero2 = 0.0;  // rounding-level trailing norms count as zero
#pragma unroll 1
      for (int st = 0; st < q; ++st) {
        double bv = -1.0;
        if (rem) {
          bv = 0.0;
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nI) bv += sc_abs2(w[c]);
          if (!(bv == bv)) bv = 0.0;
          if (bv < zero2) bv = 0.0;
        }
        int bi = rem ? lane : 0x7fffffff;
        wave_argmax(bv, bi);
        if (st == 0) zero2 = QRCP_NOISE * QRCP_NOISE * bv;
        const int p = bi;
        // the pivot column goes through LDS to every lane of the wave
        if (lane == p) {
#pragma unroll
          for (int c = 0; c < DMAX; ++c) sPcol[c] = w[c];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // the pivot column is read from LDS where it is used (every lane
        // reads the same address): a register copy of it spilled
        double sig2 = 0.0;
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          if (c >= st && c < nI) sig2 += sc_abs2(sPcol[c]);
        const double sigma = sqrt(sig2);
        const T x0 = sPcol[st];
        T alpha = sc_zero<T>();
        double beta = 0.0;
        if (sigma > 0.0) {
          alpha = sc_scale(sc_phase(x0), -sigma);
          beta = 1.0 / (sigma * (sigma + sqrt(sc_abs2(x0))));
        }
        const T v0 = sc_sub(x0, alpha);
        {
          T ww = sc_zero<T>();
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nI) sc_cfma(ww, c == st ? v0 : sPcol[c], w[c]);
          const bool upd = rem && lane != p && beta != 0.0;
#pragma unroll
          for (int c = 0; c < DMAX; ++c) {
            if (upd && c >= st && c < nI) sc_axpy_neg(w[c], beta, c == st ? v0 : sPcol[c], ww);
            if (lane == 0 && c >= st && c < nI) sRefl[st * DMAX + c] = (c == st) ? v0 : sPcol[c];
          }
        }
        if (lane == p) {
#pragma unroll
          for (int c = 0; c < DMAX; ++c) {
            if (c == st) w[c] = alpha;
            if (c > st) w[c] = sc_zero<T>();
          }
          rem = false;
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c <= st) sTm[c * DMAX + st] = w[c];
          sTinv[st] = sigma > 0.0 ? sc_div(sc_real<T>(1.0), alpha) : sc_zero<T>();
        }
        if (lane == 0) {
          sBeta[st] = beta;
          sTabs[st] = sigma;
          sJbar[st] = p;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
      if (lane == 0) {
        int dk = 0;
        if (q > 0 && sTabs[0] > 0.0)
          while (dk < q && sTabs[dk] >= eps * sTabs[0]) ++dk;
        sDK = dk;
      }
    }
    __syncthreads();
    const int dk = sDK;
    if (!pivots_in_range(sJbar, dk, nJ)) {
      status = 2;
      break;
    }
    if (A.fz && A.fz_stride >= 3 + 3 * DMAX) {
      // the iteration's pivots in full, for a replay with frozen pivots
      int32_t* rec = A.fz + (int64_t)(L.it_off + iter) * A.fz_stride;
      if (tid == 0) {
        rec[0] = nI;
        rec[1] = nJ;
        rec[2] = dk;
      }
      if (tid < nI) rec[3 + tid] = sI[tid];
      if (tid < nJ) rec[3 + DMAX + tid] = sJ[tid];
      if (tid < dk) rec[3 + 2 * DMAX + tid] = sJbar[tid];
    }
    if (dk == 0) {
      if (tid == 0) {
        A.it_dk[L.it_off + iter] = 0;
        A.it_nu[L.it_off + iter] = 0.0;
        A.it_mu[L.it_off + iter] = sqrt(mu2);
      }
      ++iter;
      break;
    }
    // ------------------------------------------------ V_k = T11^-1 Q1^H R_k (eq. (9))
#pragma unroll 1
    for (int s = 0; s < RPT; ++s) {
      const int j = tid + s * NT;
      if (j < n0) {
        T z[DMAX];
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          const T v = Rg[(int64_t)min(c, nI - 1) * n0 + j];
          z[c] = c < nI ? v : sc_zero<T>();
        }
#pragma unroll 1
        for (int st = 0; st < dk; ++st) {
          T ww = sc_zero<T>();
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nI) sc_cfma(ww, sRefl[st * DMAX + c], z[c]);
          const double beta = sBeta[st];
#pragma unroll
          for (int c = 0; c < DMAX; ++c)
            if (c >= st && c < nI) sc_axpy_neg(z[c], beta, sRefl[st * DMAX + c], ww);
        }
        // back substitution: the row loop runs at run time, the register
        // array is addressed with compile-time indexes only
#pragma unroll 1
        for (int cc = dk - 1; cc >= 0; --cc) {
          T sum = sc_zero<T>();
#pragma unroll
          for (int e = 0; e < DMAX; ++e) {
            if (e == cc) sum = sc_add(sum, z[e]);
            if (e > cc && e < dk) sum = sc_sub(sum, sc_mul(sTm[cc * DMAX + e], z[e]));
          }
          sum = sc_mul(sum, sTinv[cc]);
#pragma unroll
          for (int e = 0; e < DMAX; ++e)
            if (e == cc) z[e] = sum;
        }
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          if (c < dk) Vh[(int64_t)(r + c) * n0 + j] = sc_conj(z[c]);
      }
    }
    // ------------------------------------------------ U_k = C_k(:, Jbar)
#pragma unroll 1
    for (int s = 0; s < RPT; ++s) {
      const int i = tid + s * NT;
      if (i < m0) {
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          if (c < dk) U[(int64_t)(r + c) * m0 + i] = Cg[(int64_t)sJbar[c] * m0 + i];
      }
    }
    // ------------------------------------------------ pivots (eq. (10)) and exclusions
    if (tid < dk) {
      A.tape_rows[L.tape_off + r + tid] = sI[tid];
      A.tape_cols[L.tape_off + r + tid] = sJ[sJbar[tid]];
    }
    if (tid < nJ) used_c[sJ[tid]] = 2;  // the whole current J leaves the next candidates
    __syncthreads();
    if (tid < dk) {
      used_c[sJ[sJbar[tid]]] = 1;
      used_r[sI[tid]] = 1;
    }
    // ------------------------------------------------ LRnorm / LRnormUp (eqs. (11)-(13))
    double cross = 0.0;
    const int ntot = r + dk;
    for (int t0 = 0; t0 < ntot; t0 += C::GT) {
      const int tw = min(C::GT, ntot - t0);
      gram_tile<T, DMAX>(U, m0, m0, t0, tw, r, dk, sXs, sKs, sGU);
      gram_tile<T, DMAX>(Vh, n0, n0, t0, tw, r, dk, sXs, sKs, sG);
      double part = 0.0;
      for (int e = tid; e < C::GT * DMAX; e += NT) {
        const int tt = e / DMAX, c = e % DMAX, t = t0 + tt;
        if (tt < tw && c < dk) {
          if (t < r) {
            part += sc_re(sc_mulc(sGU[e], sG[e]));
          } else {
            sGUd[(t - r) * DMAX + c] = sGU[e];
            sGVd[(t - r) * DMAX + c] = sG[e];
          }
        }
      }
      cross += block_sum<NT>(part, redd);
    }
    // sGUd / sGVd hold U_k^H U_k and Vh_k^H Vh_k (dk x dk, Hermitian): the
    // breakdown fallback tr(G_U G_V) first, then both Cholesky factors at once
    // (waves 0 and 1), then ||T1 T2^H||_F (eqs. (11)-(12)) and mu (eq. (13))
    if (wid == 0) {
      double fb = 0.0;
      for (int e = lane; e < dk * dk; e += HB_WAVE) {
        const int a = e / dk, b = e % dk;
        fb += sc_re(sc_mulc(sGUd[a * DMAX + b], sGVd[a * DMAX + b]));
      }
      fb = wave_sum(fb);
      if (lane == 0) sScal[2] = fb;
    }
    __syncthreads();
    if (wid < 2) {
      const bool ok = chol_wave<TA, DMAX>(wid == 0 ? sGUd : sGVd, dk, lane);
      if (lane == 0) sOk[wid] = ok ? 1 : 0;
    }
    __syncthreads();
    if (wid == 0) {
      double nu2;
      if (sOk[0] && sOk[1]) {
        double part = 0.0;
        for (int e = lane; e < dk * dk; e += HB_WAVE) {
          const int a = e / dk, b = e % dk;
          TA sv = sc_zero<TA>();
          const int k0 = a > b ? a : b;
          for (int kk = k0; kk < dk; ++kk) sc_fma(sv, sGUd[a * DMAX + kk], sc_conj(sGVd[b * DMAX + kk]));
          part += sc_abs2(sv);
        }
        nu2 = wave_sum(part);
      } else {
        nu2 = sScal[2] > 0.0 ? sScal[2] : 0.0;
      }
      if (lane == 0) {
        sScal[0] = sqrt(nu2);
        const double m2 = mu2 + nu2 + 2.0 * cross;
        sScal[1] = m2 > 0.0 ? m2 : 0.0;
      }
    }
    __syncthreads();
    const double nu = sScal[0];
    mu2 = sScal[1];
    if (tid == 0) {
      A.it_dk[L.it_off + iter] = dk;
      A.it_nu[L.it_off + iter] = nu;
      A.it_mu[L.it_off + iter] = sqrt(mu2);
    }
    ++iter;
    r += dk;
    // ------------------------------------------------ stopping test
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int j = tid + s * NT;
      if (j < n0 && used_c[j] == 0) ++cnt;
    }
    const int npc = (int)(block_sum<NT>((double)cnt, redd) + 0.5);
    const bool stop = (nu < eps * sqrt(mu2)) || npc == 0 || r >= rmax;
    if (stop) break;
    // ------------------------------------------------ J_{k+1} = QR(R_k, d) (eq. (7))
    const int nsel = min(nI, npc);
    {
      T y[RPT][DMAX];
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int j = tid + s * NT;
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
          y[s][c] = (j < n0 && c < nI) ? Rg[(int64_t)c * n0 + j] : sc_zero<T>();
      }
      const int kJ = qrcp_select<T, DMAX, RPT>(y, n0, used_c, nI, nsel, sJ, sPivW, redv, redi);
      if constexpr (STRONG)
        swaps += strong_refine<T, DMAX, RPT>(Rg, n0, nI, n0, used_c, sJ, nsel, kJ, A.select_f, sRefl,
                                             sBeta, sTm, sTinv, sPcol, redv[0], redi[0]);
    }
    for (int i = tid; i < NT * RPT; i += NT)
      if (used_c[i] == 2) used_c[i] = 0;
    if (tid == 0) sNJ = nsel;
    __syncthreads();
  }
  if (tid == 0) {
    BacaOutDev o;
    o.rank = r;
    o.iters = iter;
    o.status = status;
    o.swaps = swaps;
    o.mu = sqrt(mu2);
    A.out[li] = o;
  }
}

// One persistent launch over all leaves: each workgroup takes the next leaf
// from an atomic counter (the leaves are ordered largest first) until none
// is left, so every wave reaches the exit once the counter passes nleaves.
template <typename T, int DMAX, int RPT, bool STRONG>
__global__ __launch_bounds__(NT) void baca_leaf_kernel(BacaArgs A) {
  __shared__ int sNext;
  for (;;) {
    if (threadIdx.x == 0) sNext = atomicAdd(A.queue, 1);
    __syncthreads();
    const int li = sNext;
    if (li >= A.nleaves) break;
    baca_leaf<T, DMAX, RPT, STRONG>(A, li);
    // every thread has read sNext and left the leaf's LDS before the next take
    __syncthreads();
  }
}

}  // namespace

namespace hbk {

// Workgroups of the persistent launch: as many as fit on the device at once
// (occupancy per CU times the CU count), at most one per leaf.
template <typename T, int DMAX, int RPT, bool STRONG>
inline int launch_one(const BacaArgs& a, hipStream_t st) {
  static int resident = 0;  // per instantiation, computed on first use
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, baca_leaf_kernel<T, DMAX, RPT, STRONG>,
                                                     NT, 0) !=
            hipSuccess)
      return (int)hipGetLastError();
    resident = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const int grid = a.nleaves < resident ? a.nleaves : resident;
  int e = zero_fill_launch(a.queue, sizeof(int32_t) * 2, st);
  if (e != 0) return e;
  hipLaunchKernelGGL((baca_leaf_kernel<T, DMAX, RPT, STRONG>), dim3(grid), dim3(NT), 0, st, a);
  return (int)hipGetLastError();
}

// Every (scalar, DMAX, RPT) instantiation of the leaf kernel:
// scalar 0 FP64, 1 complex FP64, 2 FP32.
#define HB_BACA_INSTANCES(X)                                       \
  X(0, double, 8, 1) X(0, double, 8, 2) X(0, double, 8, 4)         \
  X(0, double, 16, 1) X(0, double, 16, 2) X(0, double, 16, 4)      \
  X(0, double, 32, 1) X(0, double, 32, 2)                          \
  X(1, hb_cplx, 8, 1) X(1, hb_cplx, 8, 2) X(1, hb_cplx, 8, 4)      \
  X(1, hb_cplx, 16, 1) X(1, hb_cplx, 16, 2)                        \
  X(1, hb_cplx, 32, 1)                                             \
  X(2, float, 8, 1) X(2, float, 8, 2) X(2, float, 8, 4)            \
  X(2, float, 16, 1) X(2, float, 16, 2) X(2, float, 16, 4)         \
  X(2, float, 32, 1) X(2, float, 32, 2) X(2, float, 32, 4)

}  // namespace hbk
