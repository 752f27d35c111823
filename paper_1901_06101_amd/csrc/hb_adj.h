// Frozen-pivot adjoint of the compressed operator: one-workgroup tasks.
//
// With the pivots of every BACA iteration (the row block I_k, the column
// block J_k, the pivot order of QR(W_k, eps) and d_k) and every truncation
// rank fixed to those of a forward run, the compressed operator
// A~ = U diag(s) V^T is a smooth function of the sampled entries A(:, J_k)
// and A(I_k, :) of every leaf, hence of the Gaussian width h and of the
// point coordinates.  The tasks below replay that fixed pipeline
// (Algorithm 2 with eqs. (8)-(9), the SVD re-compression, the merges of
// Algorithm 3 with eqs. (14)-(15)) and run it in reverse, from the
// cotangent of y = A~ w down to the cotangents of the sampled entries and
// on to dL/dh and dL/d(points) through the closed-form derivatives of the
// Gaussian entry.
//
// Reverse rules used (real arithmetic):
// * V_k = T^-1 Q1^T R_k is the least-squares solution W_p^+ R_k with
//   W_p = Q1 T (full column rank), so with Zb = T^-T Vb_k:
//   Rb_k = Q1 Zb,  Wb_p = -Q1 Zb V_k^T + (R_k - Q1 Q1^T R_k) (T^-1 Zb)^T.
// * A truncated SVD P ~ Ub diag(s) Vb^T kept at rank rho, with cotangents
//   Ubb = [Ub_o, 0], Vbb = [Vb_o, 0] of the kept factors (Townsend,
//   "Differentiating the singular value decomposition", 2016):
//   Pb = Ub G Vb^T + (I - Ub Ub^T) Ubb s^-1 Vb^T + Ub s^-1 Vbb^T (I - Vb Vb^T),
//   G = diag(sb) + (F o (J - J^T)) diag(s) + diag(s) (F o (K - K^T)),
//   J = Ub^T Ubb, K = Vb^T Vbb, F_ij = 1 / (s_j^2 - s_i^2).  Only the kept
//   singular values are inverted.  For the re-compression P = U Vt^T the
//   third term vanishes in Pb Vt and the second in Pb^T U; for a merge,
//   P = [P1 diag(S1), P2 diag(S2)] keeps both (one is zero up to rounding
//   when P has at least as many rows as columns, the other when it has
//   fewer).
//
// Every task runs on one workgroup; a tall merge is split into several
// row-chunk tasks with small single-workgroup steps between them (see
// "merges split over rows").  `W` supplies the lane id `tid`, the
// lane count `nt`, a reduction array `red` of 3 nt + ADJ_RED_EXTRA doubles
// and `sync()`, a barrier that every lane reaches.  Loops stride by nt over
// disjoint outputs and a phase that reads another lane's output follows a
// sync(), so the result does not depend on the lane count beyond the order
// of rounding in sums.
#pragma once

#include <math.h>
#include <stdint.h>

// hipcc compiles these tasks for the GPU (hb_adjoint.hip).  The tests also
// compile them for the host, one thread or one fiber per lane, to check
// them against the oracle; the library itself has no host path.
#if defined(__HIPCC__)
#define HBA_FN __device__ inline
#else
#define HBA_FN inline
#endif

#define HBA_DMAX 32   // largest block size d of a replayed leaf
#define HBA_MAXDIM 8  // largest point dimension

// wg_svd shares each Jacobi pair over several lanes from this many columns
// on (the host checks also build with 2, to run that path at small sizes)
#ifndef ADJ_JACOBI_SPLIT_K
#define ADJ_JACOBI_SPLIT_K 64
#endif

// `red` holds three doubles per lane (the pair sums of wg_svd) and
// ADJ_RED_EXTRA more (the partial sums of wg_sum, at red[3 nt ..], which
// nothing else touches)
constexpr int ADJ_RED_EXTRA = 16;

enum AdjTaskKind {
  ADJ_LEAF_FWD = 0,
  ADJ_REC_FWD = 1,
  ADJ_MERGE_FWD = 2,
  ADJ_ROOT = 3,
  ADJ_MERGE_BWD = 4,
  ADJ_REC_BWD = 5,
  ADJ_LEAF_BWD = 6,
  ADJ_RED_ROWS = 7,
  ADJ_RED_COLS = 8,
  ADJ_RED_H = 9,
  // merges tall enough to be split over row chunks (one task per chunk or
  // per merge, in this order within a merge step)
  ADJ_MCH_FWD1 = 10,  // chunk: its rows of B and their thin QR
  ADJ_MCH_FWD2 = 11,  // merge: QR of the stacked chunk R's, SVD
  ADJ_MCH_FWD3 = 12,  // chunk: its rows of Ub and of the new O side
  ADJ_MCH_BWD1 = 13,  // chunk: partial sums over its rows, O-side cotangents
  ADJ_MCH_BWD2 = 14,  // merge: the small matrices of the reverse rule
  ADJ_MCH_BWD3 = 15,  // chunk: its rows of the P-side cotangents
  ADJ_MCH_BWD4 = 16,  // merge: the children's sigma cotangents
};

// One leaf (offsets are in doubles from the arena base D; ws_* are offsets
// from the phase workspace).
struct AdjLeaf {
  int64_t row0, col0;  // first row / column of the leaf in the problem
  int32_t m0, n0;
  int32_t iters;       // replayed iterations (all with d_k > 0)
  int32_t rb;          // BACA rank, sum of d_k
  int32_t rho;         // rank after the SVD re-compression
  int32_t fz_off;      // index of the first iteration record
  int64_t U, Vt;       // BACA factors, m0 x rb and n0 x rb
  int64_t it, it_sz;   // iteration k: C (m0 x dmax), R (dmax x n0), Q1, T (dmax x dmax)
  int64_t Ub, Vb, S;   // re-compression: m0 x rb, n0 x rb, rb
  int64_t gU, gVt;     // cotangents of U and Vt
  int64_t gx, gy, gh;  // partial gradients: m0 x dim, n0 x dim (ld m0, n0), 1
  int64_t ws_lf, ws_rf, ws_rb, ws_lb;
};

// A compressed block U diag(S) Vt^T and the cotangents of its factors.
struct AdjBlock {
  int64_t m, n;
  int32_t r, pad;
  int64_t U, ldU, Vt, ldVt, S;
  int64_t gU, gVt, gS;  // m x r (ld m), n x r (ld n), r
};

// A merge of blocks b1 and b2 (horizontal: side by side, the P side is U;
// vertical: stacked, the P side is Vt).
struct AdjMerge {
  int32_t b1, b2, out, horiz;
  int32_t k, rho;      // k = r1 + r2 columns, rank kept
  int32_t p, G;        // p = min(rows, k) singular values; G row chunks (1: one task)
  int64_t rows;        // rows of the P side
  int64_t n1, n2;      // rows of the O sides
  int64_t Ub, Y, S;    // rows x p, k x p, p
  int64_t ws_f, ws_b;  // G == 1
  // G > 1: B and then each chunk's Q (rows x k), the chunks' R stacked and
  // then their Q' (G k x k), Q' X (G k x k, each chunk forms its k rows),
  // the SVD's left factor X (k x k), per-chunk partial sums
  // (G x (2 k rho + k)), and the reverse rule's J (k x rho), G Y^T (k x k)
  // and E2 (k x rho)
  int64_t Bq, Rs, QX, Xs, part, Jm, H, E2;
  int64_t ws_f2, ws_b2;
};

// One row chunk of a split merge: P-side rows [p0, p1), O-side rows [o0, o1).
struct AdjChunk {
  int32_t merge, c;
  int64_t p0, p1, o0, o1;
  int64_t ws_f1, ws_b3;
};

struct AdjArgs {
  double* D;            // arena
  double* ws;           // phase workspace
  const int32_t* fz;    // iteration records: nI, nJ, d_k, I_k, J_k, pivot order
  const AdjLeaf* leaves;
  const AdjBlock* blocks;
  const AdjMerge* merges;
  const AdjChunk* chunks;
  const int32_t* tasks;  // merge or chunk ids of the merge-step launches
  const double* X;      // points, structure of arrays: X[q * ldx + i]
  const double* Y;
  int64_t ldx, ldy;
  int32_t dim, dmax, fz_stride, root;
  int32_t nb, nleaves;
  double h, nic;        // Gaussian width and -1 / (c h^2)
  const double* w;      // n
  const double* ybar;   // m
  double* gw;           // n (may be null)
  double* gh;           // 1 (may be null)
  double* gX;           // m x dim, points-major (may be null)
  double* gY;           // n x dim (may be null)
};

// --------------------------------------------------------------- helpers ---
template <class W>
HBA_FN double wg_sum(W& w, double v) {
  // two barriers: ADJ_RED_EXTRA lanes each add a strided share of the nt
  // values into the partial-sum slots red[3 nt ..], then every lane adds
  // those.  Only the partial-sum slots are read after the second barrier,
  // and no other code writes them (the next call does so past its first
  // barrier), so red[0 .. 3 nt) is free again on return.
  constexpr int P = ADJ_RED_EXTRA;
  const int np = w.nt < P ? w.nt : P;
  double* part = w.red + 3 * w.nt;
  w.red[w.tid] = v;
  w.sync();
  if (w.tid < np) {
    double s = 0.0;
    for (int i = w.tid; i < w.nt; i += np) s += w.red[i];
    part[w.tid] = s;
  }
  w.sync();
  double r = 0.0;
  for (int c = 0; c < np; ++c) r += part[c];
  return r;
}

// C (m x n) = alpha op(A) op(B) + beta C, column-major, op = transpose when
// tA / tB is set; C must not overlap A or B.
template <class W>
HBA_FN void wg_gemm(W& w, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                    int64_t lda, int tA, const double* B, int64_t ldb, int tB, double beta,
                    double* C, int64_t ldc) {
  for (int64_t e = w.tid; e < m * n; e += w.nt) {
    const int64_t i = e % m, j = e / m;
    double s = 0.0;
    for (int64_t l = 0; l < k; ++l) {
      const double x = tA ? A[l + i * lda] : A[i + l * lda];
      const double y = tB ? B[j + l * ldb] : B[l + j * ldb];
      s += x * y;
    }
    C[i + j * ldc] = alpha * s + (beta == 0.0 ? 0.0 : beta * C[i + j * ldc]);
  }
  w.sync();
}

// The rows where column j can be nonzero: all m rows, or, for a stack of
// upper-triangular blk x blk blocks (m a multiple of blk), rows
// c blk + i with i <= j.  Index t < n maps to row (*this)(t).
struct QrRows {
  int64_t n, per, blk;
  HBA_FN QrRows(int64_t m, int64_t b, int j)
      : n(m), per(b > 0 && j + 1 < b ? j + 1 : 0), blk(b) {
    if (per) n = (m / b) * per;
  }
  HBA_FN int64_t operator()(int64_t t) const { return per ? (t / per) * blk + t % per : t; }
};

// Thin QR of A (m x k, m >= k) by classical Gram-Schmidt with at least one
// full re-orthogonalisation, and more (up to four passes) while a pass still
// removes more than half of the column's norm, as happens for a column
// nearly in the span of the earlier ones (Kahan and Parlett's criterion):
// Q (m x k) with orthonormal columns, R (k x k) upper triangular with a
// non-negative diagonal, A = Q R to working precision.  Q may be A itself
// (same ld).  h: k doubles of scratch.  blk > 0 declares A a stack of
// upper-triangular blk x blk blocks (blk = k): column j and every
// combination of the earlier columns vanish on block rows below j, so the
// loops skip those rows (the same result up to the order of the sums).
template <class W>
HBA_FN void wg_qr(W& w, int64_t m, int k, const double* A, int64_t lda, double* Q, int64_t ldq,
                  double* R, int64_t ldr, double* h, int blk = 0) {
  for (int j = 0; j < k; ++j) {
    if (A != Q)
      for (int64_t i = w.tid; i < m; i += w.nt) Q[i + j * ldq] = A[i + j * lda];
    for (int e = w.tid; e < k; e += w.nt) R[e + j * ldr] = 0.0;
    w.sync();
    const QrRows rows(m, blk, j);
    // nq: the norm of column j as it stands (for j > 0 the passes form it)
    double nq = 0.0;
    if (j == 0) {
      double part0 = 0.0;
      for (int64_t t = w.tid; t < rows.n; t += w.nt) {
        const int64_t l = rows(t);
        part0 += Q[l + j * ldq] * Q[l + j * ldq];
      }
      nq = sqrt(wg_sum(w, part0));
    }
    for (int pass = 0; j > 0 && pass < 4; ++pass) {
      // the dot products with the j earlier columns; pass 1 (which always
      // follows pass 0) adds column j with itself, the norm pass 0 left,
      // as h[j].  g adjacent lanes share each of the nd products (rows
      // interleaved, so neighbouring lanes read neighbouring rows) when
      // nd <= nt / 2; their partial sums meet in red
      const int nd = pass == 1 ? j + 1 : j;
      const int g = w.nt / nd >= 2 ? w.nt / nd : 1;
      if (g == 1) {
        for (int i = w.tid; i < nd; i += w.nt) {
          double s = 0.0;
          for (int64_t t = 0; t < rows.n; ++t) {
            const int64_t l = rows(t);
            s += Q[l + i * ldq] * Q[l + j * ldq];
          }
          h[i] = s;
        }
      } else {
        if (w.tid < nd * g) {
          const int i = w.tid / g, c = w.tid % g;
          double s = 0.0;
          for (int64_t t = c; t < rows.n; t += g) {
            const int64_t l = rows(t);
            s += Q[l + i * ldq] * Q[l + j * ldq];
          }
          w.red[w.tid] = s;
        }
        w.sync();
        for (int i = w.tid; i < nd; i += w.nt) {
          double s = 0.0;
          for (int c = 0; c < g; ++c) s += w.red[i * g + c];
          h[i] = s;
        }
      }
      w.sync();
      if (pass == 1) nq = sqrt(h[j]);
      for (int64_t t = w.tid; t < rows.n; t += w.nt) {
        const int64_t l = rows(t);
        double s = Q[l + j * ldq];
        for (int i = 0; i < j; ++i) s -= Q[l + i * ldq] * h[i];
        Q[l + j * ldq] = s;
      }
      for (int i = w.tid; i < j; i += w.nt) R[i + j * ldr] += h[i];
      w.sync();
      if (pass == 0) continue;
      double pn = 0.0;
      for (int64_t t = w.tid; t < rows.n; t += w.nt) {
        const int64_t l = rows(t);
        pn += Q[l + j * ldq] * Q[l + j * ldq];
      }
      const double nnow = sqrt(wg_sum(w, pn));
      const bool again = nnow < 0.5 * nq;
      nq = nnow;
      if (!again) break;
    }
    const double nrm = nq;
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t t = w.tid; t < rows.n; t += w.nt) Q[rows(t) + j * ldq] *= inv;
    if (w.tid == 0) R[j + j * ldr] = nrm;
    w.sync();
  }
}

// SVD of the k x k matrix A = X diag(s) Y^T by one-sided Jacobi (Hestenes)
// with round-robin pairs: on return A holds X (unit columns, zero for a zero
// singular value), Y the orthogonal right factor, s the singular values in
// descending order.  Aw, Yw: k x k scratch; st: k doubles of scratch.
template <class W>
HBA_FN void wg_svd(W& w, int k, double* A, int64_t lda, double* Yo, int64_t ldy, double* s,
                   double* Aw, double* Yw, double* st) {
  if (k == 0) return;
  for (int e = w.tid; e < k * k; e += w.nt) {
    const int i = e % k, j = e / k;
    Aw[e] = A[i + (int64_t)j * lda];
    Yw[e] = i == j ? 1.0 : 0.0;
  }
  w.sync();
  const int kk = k + (k & 1);
  const int npair = kk / 2;
  // g lanes per pair (rows interleaved) when the pairs leave lanes idle and
  // the columns are long enough for the split to outweigh the extra barrier
  // per round; their partial sums meet in red[0 .. 3 npair g)
  const int g = k >= ADJ_JACOBI_SPLIT_K && npair <= w.nt ? w.nt / npair : 1;
  const double tol = 4e-16 * (double)(k > 4 ? k : 4);
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rot = 0;
    for (int rd = 0; rd < kk - 1; ++rd) {
      if (g > 1) {
        if (w.tid < npair * g) {
          const int t = w.tid / g, c0 = w.tid % g;
          const int pa = t, pb = kk - 1 - t;
          const int p = pa == 0 ? 0 : 1 + (pa - 1 + rd) % (kk - 1);
          const int q = pb == 0 ? 0 : 1 + (pb - 1 + rd) % (kk - 1);
          double al = 0.0, be = 0.0, ga = 0.0;
          if (p < k && q < k)
            for (int i = c0; i < k; i += g) {
              const double x = Aw[i + p * k], y = Aw[i + q * k];
              al += x * x;
              be += y * y;
              ga += x * y;
            }
          w.red[3 * w.tid] = al;
          w.red[3 * w.tid + 1] = be;
          w.red[3 * w.tid + 2] = ga;
        }
        w.sync();
        if (w.tid < npair * g) {
          const int t = w.tid / g, c0 = w.tid % g;
          const int pa = t, pb = kk - 1 - t;
          const int p = pa == 0 ? 0 : 1 + (pa - 1 + rd) % (kk - 1);
          const int q = pb == 0 ? 0 : 1 + (pb - 1 + rd) % (kk - 1);
          // every lane of the pair adds the partials in the same order, so
          // all of them take the same rotation
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int c = 0; c < g; ++c) {
            al += w.red[3 * (t * g + c)];
            be += w.red[3 * (t * g + c) + 1];
            ga += w.red[3 * (t * g + c) + 2];
          }
          if (p < k && q < k && al > 0.0 && be > 0.0 &&
              fabs(ga) > tol * sqrt(al) * sqrt(be)) {
            const double ze = (be - al) / (2.0 * ga);
            const double tn = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + hypot(1.0, ze));
            const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
            for (int i = c0; i < k; i += g) {
              const double x = Aw[i + p * k], y = Aw[i + q * k];
              Aw[i + p * k] = cs * x - sn * y;
              Aw[i + q * k] = sn * x + cs * y;
              const double u = Yw[i + p * k], v = Yw[i + q * k];
              Yw[i + p * k] = cs * u - sn * v;
              Yw[i + q * k] = sn * u + cs * v;
            }
            if (c0 == 0) ++rot;
          }
        }
        w.sync();
        continue;
      }
      for (int t = w.tid; t < npair; t += w.nt) {
        const int pa = t, pb = kk - 1 - t;
        const int p = pa == 0 ? 0 : 1 + (pa - 1 + rd) % (kk - 1);
        const int q = pb == 0 ? 0 : 1 + (pb - 1 + rd) % (kk - 1);
        if (p >= k || q >= k) continue;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = 0; i < k; ++i) {
          const double x = Aw[i + p * k], y = Aw[i + q * k];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        if (!(al > 0.0 && be > 0.0) || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        const double ze = (be - al) / (2.0 * ga);
        const double tn = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + hypot(1.0, ze));
        const double c = 1.0 / sqrt(1.0 + tn * tn), sn = c * tn;
        for (int i = 0; i < k; ++i) {
          const double x = Aw[i + p * k], y = Aw[i + q * k];
          Aw[i + p * k] = c * x - sn * y;
          Aw[i + q * k] = sn * x + c * y;
          const double u = Yw[i + p * k], v = Yw[i + q * k];
          Yw[i + p * k] = c * u - sn * v;
          Yw[i + q * k] = sn * u + c * v;
        }
        ++rot;
      }
      w.sync();
    }
    if (wg_sum(w, (double)rot) == 0.0) break;
  }
  for (int j = w.tid; j < k; j += w.nt) {
    double nn = 0.0;
    for (int i = 0; i < k; ++i) nn += Aw[i + j * k] * Aw[i + j * k];
    st[j] = sqrt(nn);
  }
  w.sync();
  // descending order, ties by index; each column goes to its own slot
  for (int j = w.tid; j < k; j += w.nt) {
    const double sj = st[j];
    int pos = 0;
    for (int i = 0; i < k; ++i)
      if (st[i] > sj || (st[i] == sj && i < j)) ++pos;
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    s[pos] = sj;
    for (int i = 0; i < k; ++i) {
      A[i + (int64_t)pos * lda] = Aw[i + j * k] * inv;
      Yo[i + (int64_t)pos * ldy] = Yw[i + j * k];
    }
  }
  w.sync();
}

// G of the truncated-SVD reverse rule (k x k, ld k).  J and K hold their
// first rho columns (ld k); the others are zero.
template <class W>
HBA_FN void adj_svd_g(W& w, int k, int rho, const double* s, const double* sb, const double* J,
                      const double* K, double* G) {
  for (int e = w.tid; e < k * k; e += w.nt) {
    const int i = e % k, j = e / k;
    double v = 0.0;
    if (i == j) {
      if (i < rho) v = sb[i];
    } else if (i < rho || j < rho) {
      const double jij = j < rho ? J[i + j * k] : 0.0, jji = i < rho ? J[j + i * k] : 0.0;
      const double kij = j < rho ? K[i + j * k] : 0.0, kji = i < rho ? K[j + i * k] : 0.0;
      const double f = 1.0 / (s[j] * s[j] - s[i] * s[i]);
      v = f * ((jij - jji) * s[j] + s[i] * (kij - kji));
    }
    G[e] = v;
  }
  w.sync();
}

// Gaussian entry of problem row gi and column gj.
HBA_FN double adj_entry(const AdjArgs& a, int64_t gi, int64_t gj) {
  double r2 = 0.0;
  for (int q = 0; q < a.dim; ++q) {
    const double d = a.X[q * a.ldx + gi] - a.Y[q * a.ldy + gj];
    r2 += d * d;
  }
  return exp(a.nic * r2);
}

// Contribution of the entry cotangent ab of (gi, gj): g[q] += ab dA/dx_q
// (dA/dy_q is its negative); returns ab dA/dh.
HBA_FN double adj_entry_grad(const AdjArgs& a, int64_t gi, int64_t gj, double ab, double* g) {
  double d[HBA_MAXDIM];
  double r2 = 0.0;
  for (int q = 0; q < a.dim; ++q) {
    d[q] = a.X[q * a.ldx + gi] - a.Y[q * a.ldy + gj];
    r2 += d[q] * d[q];
  }
  const double f = ab * exp(a.nic * r2);
  for (int q = 0; q < a.dim; ++q) g[q] += f * 2.0 * a.nic * d[q];
  return f * r2 * (-2.0 * a.nic / a.h);
}

// ---------------------------------------------------------- forward tasks ---
// Leaf BACA with frozen pivots (Algorithm 2, eqs. (8)-(9)); keeps C_k, R_k,
// Q1 and T of every iteration.
template <class W>
HBA_FN void adj_leaf_fwd(W& w, const AdjArgs& a, int li) {
  const AdjLeaf& L = a.leaves[li];
  double* D = a.D;
  const int m0 = L.m0, n0 = L.n0, dm = a.dmax;
  double* U = D + L.U;
  double* Vt = D + L.Vt;
  double* hs = a.ws + L.ws_lf;
  int r0 = 0;
  for (int k = 0; k < L.iters; ++k) {
    const int32_t* rec = a.fz + (int64_t)(L.fz_off + k) * a.fz_stride;
    const int nI = rec[0], nJ = rec[1], dk = rec[2];
    const int32_t* I = rec + 3;
    const int32_t* J = rec + 3 + dm;
    const int32_t* Jb = rec + 3 + 2 * dm;
    double* C = D + L.it + k * L.it_sz;
    double* R = C + (int64_t)m0 * dm;
    double* Q1 = R + (int64_t)dm * n0;
    double* T = Q1 + dm * dm;
    // C_k = A(:, J_k) - U V(:, J_k)
    for (int64_t e = w.tid; e < (int64_t)m0 * nJ; e += w.nt) {
      const int i = (int)(e % m0), b = (int)(e / m0);
      double s = adj_entry(a, L.row0 + i, L.col0 + J[b]);
      for (int t = 0; t < r0; ++t) s -= U[i + (int64_t)t * m0] * Vt[J[b] + (int64_t)t * n0];
      C[i + (int64_t)b * m0] = s;
    }
    // R_k = A(I_k, :) - U(I_k, :) V
    for (int64_t e = w.tid; e < (int64_t)nI * n0; e += w.nt) {
      const int c = (int)(e % nI);
      const int64_t j = e / nI;
      double s = adj_entry(a, L.row0 + I[c], L.col0 + j);
      for (int t = 0; t < r0; ++t) s -= U[I[c] + (int64_t)t * m0] * Vt[j + (int64_t)t * n0];
      R[c + j * dm] = s;
    }
    w.sync();
    // the pivoted columns of W_k = C_k(I_k, :) and their thin QR
    for (int e = w.tid; e < nI * dk; e += w.nt) {
      const int c = e % nI, q = e / nI;
      Q1[c + q * dm] = C[I[c] + (int64_t)Jb[q] * m0];
    }
    w.sync();
    wg_qr(w, nI, dk, Q1, dm, Q1, dm, T, dm, hs);
    // U_k = C_k(:, Jbar), V_k = T^-1 Q1^T R_k
    for (int64_t e = w.tid; e < (int64_t)m0 * dk; e += w.nt) {
      const int i = (int)(e % m0), q = (int)(e / m0);
      U[i + (int64_t)(r0 + q) * m0] = C[i + (int64_t)Jb[q] * m0];
    }
    for (int64_t j = w.tid; j < n0; j += w.nt) {
      double z[HBA_DMAX];
      for (int q = 0; q < dk; ++q) {
        double s = 0.0;
        for (int c = 0; c < nI; ++c) s += Q1[c + q * dm] * R[c + j * dm];
        z[q] = s;
      }
      for (int q = dk - 1; q >= 0; --q) {
        double s = z[q];
        for (int p = q + 1; p < dk; ++p) s -= T[q + p * dm] * z[p];
        z[q] = s / T[q + q * dm];
      }
      for (int q = 0; q < dk; ++q) Vt[j + (int64_t)(r0 + q) * n0] = z[q];
    }
    w.sync();
    r0 += dk;
  }
}

// SVD re-compression of U Vt^T: U = QU TU, Vt = QV TV, TU TV^T = X diag(s) Y^T,
// Ub = QU X, Vb = QV Y; the leaf's block keeps the first rho columns.
template <class W>
HBA_FN void adj_rec_fwd(W& w, const AdjArgs& a, int li) {
  const AdjLeaf& L = a.leaves[li];
  const int m0 = L.m0, n0 = L.n0, r = L.rb;
  if (r == 0) return;
  double* D = a.D;
  double* QU = a.ws + L.ws_rf;
  double* QV = QU + (int64_t)m0 * r;
  double* TU = QV + (int64_t)n0 * r;
  double* TV = TU + r * r;
  double* M = TV + r * r;
  double* Yo = M + r * r;
  double* Aw = Yo + r * r;
  double* Yw = Aw + r * r;
  double* hs = Yw + r * r;
  wg_qr(w, m0, r, D + L.U, m0, QU, m0, TU, r, hs);
  wg_qr(w, n0, r, D + L.Vt, n0, QV, n0, TV, r, hs);
  wg_gemm(w, r, r, r, 1.0, TU, r, 0, TV, r, 1, 0.0, M, r);
  wg_svd(w, r, M, r, Yo, r, D + L.S, Aw, Yw, hs);
  wg_gemm(w, m0, r, r, 1.0, QU, m0, 0, M, r, 0, 0.0, D + L.Ub, m0);
  wg_gemm(w, n0, r, r, 1.0, QV, n0, 0, Yo, r, 0, 0.0, D + L.Vb, n0);
}

struct AdjSides {
  const double *P1, *P2, *O1, *O2, *S1, *S2;
  int64_t ldP1, ldP2, ldO1, ldO2;
};

HBA_FN AdjSides adj_sides(const AdjArgs& a, const AdjMerge& M) {
  const AdjBlock& b1 = a.blocks[M.b1];
  const AdjBlock& b2 = a.blocks[M.b2];
  AdjSides s;
  s.P1 = a.D + (M.horiz ? b1.U : b1.Vt);
  s.ldP1 = M.horiz ? b1.ldU : b1.ldVt;
  s.P2 = a.D + (M.horiz ? b2.U : b2.Vt);
  s.ldP2 = M.horiz ? b2.ldU : b2.ldVt;
  s.O1 = a.D + (M.horiz ? b1.Vt : b1.U);
  s.ldO1 = M.horiz ? b1.ldVt : b1.ldU;
  s.O2 = a.D + (M.horiz ? b2.Vt : b2.U);
  s.ldO2 = M.horiz ? b2.ldVt : b2.ldU;
  s.S1 = a.D + b1.S;
  s.S2 = a.D + b2.S;
  return s;
}

// Merge (Algorithm 3, eqs. (14)-(15)): the thin SVD B = Ub diag(s) Y^T of
// B = [P1 diag(S1), P2 diag(S2)] (rows x k, p = min(rows, k) singular
// values), through B = Q R, R = X diag(s) Y^T, Ub = Q X when rows >= k, and
// through B^T = Q R, R^T = X diag(s) Z^T, Ub = X, Y = Q Z otherwise; the new
// block is P = Ub(:, :rho), s(:rho), O = blockdiag(O1, O2) Y(:, :rho).
template <class W>
HBA_FN void adj_merge_fwd(W& w, const AdjArgs& a, int mi) {
  const AdjMerge& M = a.merges[mi];
  const int k = M.k, rho = M.rho, p = M.p;
  if (k == 0) return;
  const int r1 = a.blocks[M.b1].r, r2 = a.blocks[M.b2].r;
  const int64_t rows = M.rows, n1 = M.n1, n2 = M.n2;
  const AdjSides sd = adj_sides(a, M);
  const AdjBlock& out = a.blocks[M.out];
  double* D = a.D;
  double* B = a.ws + M.ws_f;  // rows x k (or its transpose)
  double* R = B + rows * k;   // p x p
  double* X = R + p * p;
  double* Aw = X + p * p;
  double* Yw = Aw + p * p;
  double* Z = Yw + p * p;
  double* hs = Z + p * p;     // rows + k
  const bool tall = rows >= k;
  for (int64_t e = w.tid; e < rows * k; e += w.nt) {
    const int64_t l = e % rows;
    const int c = (int)(e / rows);
    const double v =
        c < r1 ? sd.P1[l + c * sd.ldP1] * sd.S1[c] : sd.P2[l + (c - r1) * sd.ldP2] * sd.S2[c - r1];
    if (tall)
      B[e] = v;
    else
      B[c + l * k] = v;
  }
  w.sync();
  if (tall) {
    wg_qr(w, rows, k, B, rows, B, rows, R, k, hs);
    wg_svd(w, k, R, k, D + M.Y, k, D + M.S, Aw, Yw, hs);
    wg_gemm(w, rows, k, k, 1.0, B, rows, 0, R, k, 0, 0.0, D + M.Ub, rows);
  } else {
    wg_qr(w, k, (int)rows, B, k, B, k, R, p, hs);
    for (int e = w.tid; e < p * p; e += w.nt) X[e] = R[(e / p) + (e % p) * p];
    w.sync();
    wg_svd(w, p, X, p, Z, p, D + M.S, Aw, Yw, hs);
    for (int64_t e = w.tid; e < rows * p; e += w.nt) D[M.Ub + e] = X[e];
    wg_gemm(w, k, p, p, 1.0, B, k, 0, Z, p, 0, 0.0, D + M.Y, k);
  }
  double* On = D + (M.horiz ? out.Vt : out.U);
  wg_gemm(w, n1, rho, r1, 1.0, sd.O1, sd.ldO1, 0, D + M.Y, k, 0, 0.0, On, n1 + n2);
  wg_gemm(w, n2, rho, r2, 1.0, sd.O2, sd.ldO2, 0, D + M.Y + r1, k, 0, 0.0, On + n1, n1 + n2);
}

// ---------------------------------------------------------- reverse tasks ---
// y = U diag(S) Vt^T w: cotangents of the root factors from ybar, and
// wbar = Vt diag(S) U^T ybar.
template <class W>
HBA_FN void adj_root(W& w, const AdjArgs& a) {
  const AdjBlock& B = a.blocks[a.root];
  const int r = B.r;
  const int64_t m = B.m, n = B.n;
  double* D = a.D;
  const double* U = D + B.U;
  const double* Vt = D + B.Vt;
  const double* S = D + B.S;
  double* g = a.ws;      // Vt^T w
  double* u = a.ws + r;  // U^T ybar
  for (int j = w.tid; j < r; j += w.nt) {
    double sg = 0.0, su = 0.0;
    for (int64_t l = 0; l < n; ++l) sg += Vt[l + j * B.ldVt] * a.w[l];
    for (int64_t l = 0; l < m; ++l) su += U[l + j * B.ldU] * a.ybar[l];
    g[j] = sg;
    u[j] = su;
  }
  w.sync();
  for (int64_t e = w.tid; e < m * r; e += w.nt) {
    const int64_t l = e % m;
    const int j = (int)(e / m);
    D[B.gU + e] = a.ybar[l] * S[j] * g[j];
  }
  for (int64_t e = w.tid; e < n * r; e += w.nt) {
    const int64_t l = e % n;
    const int j = (int)(e / n);
    D[B.gVt + e] = a.w[l] * S[j] * u[j];
  }
  for (int j = w.tid; j < r; j += w.nt) D[B.gS + j] = u[j] * g[j];
  if (a.gw)
    for (int64_t l = w.tid; l < n; l += w.nt) {
      double s = 0.0;
      for (int j = 0; j < r; ++j) s += Vt[l + j * B.ldVt] * S[j] * u[j];
      a.gw[l] = s;
    }
  w.sync();
}

// Reverse of a merge: cotangents of the children's factors.  B = Ub
// diag(s) Y^T is a thin SVD with p = min(rows, k) columns: both projector
// terms of the truncated-SVD rule are kept (one of them vanishes, up to
// rounding, when Ub or Y is square).
template <class W>
HBA_FN void adj_merge_bwd(W& w, const AdjArgs& a, int mi) {
  const AdjMerge& M = a.merges[mi];
  const int k = M.k, rho = M.rho, p = M.p;
  if (k == 0) return;
  const AdjBlock& b1 = a.blocks[M.b1];
  const AdjBlock& b2 = a.blocks[M.b2];
  const AdjBlock& out = a.blocks[M.out];
  const int r1 = b1.r, r2 = b2.r;
  const int64_t rows = M.rows, n1 = M.n1, n2 = M.n2;
  const AdjSides sd = adj_sides(a, M);
  double* D = a.D;
  const double* gPo = D + (M.horiz ? out.gU : out.gVt);  // rows x rho
  const double* gOo = D + (M.horiz ? out.gVt : out.gU);  // (n1 + n2) x rho
  const double* gSo = D + out.gS;
  double* gP1 = D + (M.horiz ? b1.gU : b1.gVt);  // rows x r1
  double* gP2 = D + (M.horiz ? b2.gU : b2.gVt);
  double* gO1 = D + (M.horiz ? b1.gVt : b1.gU);  // n1 x r1
  double* gO2 = D + (M.horiz ? b2.gVt : b2.gU);
  const double* Ub = D + M.Ub;  // rows x p
  const double* Y = D + M.Y;    // k x p
  const double* s = D + M.S;
  double* Yb = a.ws + M.ws_b;   // k x rho
  double* Jm = Yb + k * rho;    // p x rho
  double* Km = Jm + p * rho;    // p x rho
  double* G = Km + p * rho;     // p x p
  double* H = G + p * p;        // p x k
  double* E2 = H + p * k;       // k x rho
  double* E = E2 + k * rho;     // rows x rho
  double* Bb = E + rows * rho;  // rows x k
  const int64_t ldo = n1 + n2;
  // O = blockdiag(O1, O2) Y(:, :rho)
  wg_gemm(w, r1, rho, n1, 1.0, sd.O1, sd.ldO1, 1, gOo, ldo, 0, 0.0, Yb, k);
  wg_gemm(w, r2, rho, n2, 1.0, sd.O2, sd.ldO2, 1, gOo + n1, ldo, 0, 0.0, Yb + r1, k);
  wg_gemm(w, n1, r1, rho, 1.0, gOo, ldo, 0, Y, k, 1, 0.0, gO1, n1);
  wg_gemm(w, n2, r2, rho, 1.0, gOo + n1, ldo, 0, Y + r1, k, 1, 0.0, gO2, n2);
  // B = Ub diag(s) Y^T truncated at rho
  wg_gemm(w, p, rho, rows, 1.0, Ub, rows, 1, gPo, rows, 0, 0.0, Jm, p);
  wg_gemm(w, p, rho, k, 1.0, Y, k, 1, Yb, k, 0, 0.0, Km, p);
  adj_svd_g(w, p, rho, s, gSo, Jm, Km, G);
  wg_gemm(w, p, k, p, 1.0, G, p, 0, Y, k, 1, 0.0, H, p);
  for (int64_t e = w.tid; e < rows * rho; e += w.nt) {
    const int64_t l = e % rows;
    const int j = (int)(e / rows);
    double v = gPo[e];
    for (int i = 0; i < p; ++i) v -= Ub[l + i * rows] * Jm[i + j * p];
    E[e] = v / s[j];
  }
  for (int e = w.tid; e < k * rho; e += w.nt) {
    const int c = e % k, j = e / k;
    double v = Yb[e];
    for (int i = 0; i < p; ++i) v -= Y[c + i * k] * Km[i + j * p];
    E2[e] = v / s[j];
  }
  w.sync();
  wg_gemm(w, rows, k, p, 1.0, Ub, rows, 0, H, p, 0, 0.0, Bb, rows);
  wg_gemm(w, rows, k, rho, 1.0, E, rows, 0, Y, k, 1, 1.0, Bb, rows);
  wg_gemm(w, rows, k, rho, 1.0, Ub, rows, 0, E2, k, 1, 1.0, Bb, rows);
  // B = [P1 diag(S1), P2 diag(S2)]
  for (int64_t e = w.tid; e < rows * k; e += w.nt) {
    const int64_t l = e % rows;
    const int c = (int)(e / rows);
    if (c < r1)
      gP1[l + c * rows] = Bb[e] * sd.S1[c];
    else
      gP2[l + (c - r1) * rows] = Bb[e] * sd.S2[c - r1];
  }
  for (int c = w.tid; c < k; c += w.nt) {
    double v = 0.0;
    if (c < r1) {
      for (int64_t l = 0; l < rows; ++l) v += Bb[l + c * rows] * sd.P1[l + c * sd.ldP1];
      D[b1.gS + c] = v;
    } else {
      for (int64_t l = 0; l < rows; ++l) v += Bb[l + c * rows] * sd.P2[l + (c - r1) * sd.ldP2];
      D[b2.gS + c - r1] = v;
    }
  }
  w.sync();
}

// Reverse of the re-compression: cotangents of the BACA factors U and Vt.
template <class W>
HBA_FN void adj_rec_bwd(W& w, const AdjArgs& a, int li) {
  const AdjLeaf& L = a.leaves[li];
  const AdjBlock& B = a.blocks[li];
  const int m0 = L.m0, n0 = L.n0, r = L.rb, rho = L.rho;
  if (r == 0) return;
  double* D = a.D;
  const double* Ub = D + L.Ub;
  const double* Vb = D + L.Vb;
  const double* s = D + L.S;
  const double* gUo = D + B.gU;  // m0 x rho
  const double* gVo = D + B.gVt; // n0 x rho
  double* Jm = a.ws + L.ws_rb;   // r x rho
  double* Km = Jm + r * rho;
  double* G = Km + r * rho;
  double* Wu = G + r * r;
  double* Wv = Wu + r * r;
  double* H1 = Wv + r * r;
  double* H2 = H1 + r * r;
  double* E1 = H2 + r * r;                 // m0 x rho
  double* E2 = E1 + (int64_t)m0 * rho;     // n0 x rho
  wg_gemm(w, r, rho, m0, 1.0, Ub, m0, 1, gUo, m0, 0, 0.0, Jm, r);
  wg_gemm(w, r, rho, n0, 1.0, Vb, n0, 1, gVo, n0, 0, 0.0, Km, r);
  adj_svd_g(w, r, rho, s, D + B.gS, Jm, Km, G);
  wg_gemm(w, r, r, m0, 1.0, Ub, m0, 1, D + L.U, m0, 0, 0.0, Wu, r);
  wg_gemm(w, r, r, n0, 1.0, Vb, n0, 1, D + L.Vt, n0, 0, 0.0, Wv, r);
  wg_gemm(w, r, r, r, 1.0, G, r, 0, Wv, r, 0, 0.0, H1, r);
  wg_gemm(w, r, r, r, 1.0, G, r, 1, Wu, r, 0, 0.0, H2, r);
  for (int64_t e = w.tid; e < (int64_t)m0 * rho; e += w.nt) {
    const int64_t l = e % m0;
    const int j = (int)(e / m0);
    double v = gUo[e];
    for (int i = 0; i < r; ++i) v -= Ub[l + i * (int64_t)m0] * Jm[i + j * r];
    E1[e] = v / s[j];
  }
  for (int64_t e = w.tid; e < (int64_t)n0 * rho; e += w.nt) {
    const int64_t l = e % n0;
    const int j = (int)(e / n0);
    double v = gVo[e];
    for (int i = 0; i < r; ++i) v -= Vb[l + i * (int64_t)n0] * Km[i + j * r];
    E2[e] = v / s[j];
  }
  w.sync();
  wg_gemm(w, m0, r, r, 1.0, Ub, m0, 0, H1, r, 0, 0.0, D + L.gU, m0);
  wg_gemm(w, m0, r, rho, 1.0, E1, m0, 0, Wv, r, 0, 1.0, D + L.gU, m0);
  wg_gemm(w, n0, r, r, 1.0, Vb, n0, 0, H2, r, 0, 0.0, D + L.gVt, n0);
  wg_gemm(w, n0, r, rho, 1.0, E2, n0, 0, Wu, r, 0, 1.0, D + L.gVt, n0);
}

// Reverse of the leaf BACA, last iteration first: entry cotangents of
// C_k and R_k go to the partial point and width gradients; the rest flows
// to the factor columns of earlier iterations.
template <class W>
HBA_FN void adj_leaf_bwd(W& w, const AdjArgs& a, int li) {
  const AdjLeaf& L = a.leaves[li];
  const int m0 = L.m0, n0 = L.n0, dm = a.dmax, dim = a.dim;
  double* D = a.D;
  const double* U = D + L.U;
  const double* Vt = D + L.Vt;
  double* gU = D + L.gU;
  double* gVt = D + L.gVt;
  double* gx = D + L.gx;
  double* gy = D + L.gy;
  double* Zb = a.ws + L.ws_lb;       // dm x n0
  double* Y2 = Zb + (int64_t)dm * n0;  // dm x n0
  double* E = Y2 + (int64_t)dm * n0;   // dm x n0
  double* Rb = E + (int64_t)dm * n0;   // dm x n0
  double* Cb = Rb + (int64_t)dm * n0;  // m0 x dm
  double* S1 = Cb + (int64_t)m0 * dm;  // dm x dm
  double* S2 = S1 + dm * dm;
  double* Wb = S2 + dm * dm;
  for (int64_t e = w.tid; e < (int64_t)m0 * dim; e += w.nt) gx[e] = 0.0;
  for (int64_t e = w.tid; e < (int64_t)n0 * dim; e += w.nt) gy[e] = 0.0;
  w.sync();
  double ghl = 0.0;
  int r0 = L.rb;
  for (int k = L.iters - 1; k >= 0; --k) {
    const int32_t* rec = a.fz + (int64_t)(L.fz_off + k) * a.fz_stride;
    const int nI = rec[0], nJ = rec[1], dk = rec[2];
    const int32_t* I = rec + 3;
    const int32_t* J = rec + 3 + dm;
    const int32_t* Jb = rec + 3 + 2 * dm;
    r0 -= dk;
    const double* C = D + L.it + k * L.it_sz;
    const double* R = C + (int64_t)m0 * dm;
    const double* Q1 = R + (int64_t)dm * n0;
    const double* T = Q1 + dm * dm;
    (void)C;
    // per column j of the row block: Zb = T^-T Vb_k, Y2 = T^-1 Zb,
    // E = R_k - Q1 Q1^T R_k, Rb_k = Q1 Zb
    for (int64_t j = w.tid; j < n0; j += w.nt) {
      double zb[HBA_DMAX], z[HBA_DMAX];
      for (int q = 0; q < dk; ++q) {
        double s = gVt[j + (int64_t)(r0 + q) * n0];
        for (int p = 0; p < q; ++p) s -= T[p + q * dm] * zb[p];
        zb[q] = s / T[q + q * dm];
      }
      for (int q = dk - 1; q >= 0; --q) {
        double s = zb[q];
        for (int p = q + 1; p < dk; ++p) s -= T[q + p * dm] * z[p];
        z[q] = s / T[q + q * dm];
      }
      for (int q = 0; q < dk; ++q) {
        Zb[q + j * dm] = zb[q];
        Y2[q + j * dm] = z[q];
      }
      for (int q = 0; q < dk; ++q) {
        double s = 0.0;
        for (int c = 0; c < nI; ++c) s += Q1[c + q * dm] * R[c + j * dm];
        z[q] = s;
      }
      for (int c = 0; c < nI; ++c) {
        double e = R[c + j * dm], rb = 0.0;
        for (int q = 0; q < dk; ++q) {
          e -= Q1[c + q * dm] * z[q];
          rb += Q1[c + q * dm] * zb[q];
        }
        E[c + j * dm] = e;
        Rb[c + j * dm] = rb;
      }
    }
    w.sync();
    // S1 = Zb V_k^T (dk x dk), S2 = E Y2^T (nI x dk)
    for (int e = w.tid; e < dk * dk; e += w.nt) {
      const int q = e % dk, p = e / dk;
      double s = 0.0;
      for (int64_t j = 0; j < n0; ++j) s += Zb[q + j * dm] * Vt[j + (int64_t)(r0 + p) * n0];
      S1[q + p * dm] = s;
    }
    for (int e = w.tid; e < nI * dk; e += w.nt) {
      const int c = e % nI, p = e / nI;
      double s = 0.0;
      for (int64_t j = 0; j < n0; ++j) s += E[c + j * dm] * Y2[p + j * dm];
      S2[c + p * dm] = s;
    }
    w.sync();
    // cotangent of the pivoted W_k: -Q1 S1 + S2
    for (int e = w.tid; e < nI * dk; e += w.nt) {
      const int c = e % nI, p = e / nI;
      double s = S2[c + p * dm];
      for (int q = 0; q < dk; ++q) s -= Q1[c + q * dm] * S1[q + p * dm];
      Wb[c + p * dm] = s;
    }
    w.sync();
    // cotangent of C_k: U_k = C_k(:, Jbar) and W_k = C_k(I_k, Jbar)
    for (int64_t e = w.tid; e < (int64_t)m0 * nJ; e += w.nt) {
      const int i = (int)(e % m0), b = (int)(e / m0);
      double v = 0.0;
      for (int q = 0; q < dk; ++q)
        if (Jb[q] == b) {
          v += gU[i + (int64_t)(r0 + q) * m0];
          for (int c = 0; c < nI; ++c)
            if (I[c] == i) v += Wb[c + q * dm];
        }
      Cb[i + (int64_t)b * m0] = v;
    }
    w.sync();
    // entry cotangents: A(:, J_k) carries Cb, A(I_k, :) carries Rb
    for (int64_t i = w.tid; i < m0; i += w.nt) {
      double g[HBA_MAXDIM];
      for (int q = 0; q < dim; ++q) g[q] = 0.0;
      for (int b = 0; b < nJ; ++b) {
        const double cb = Cb[i + (int64_t)b * m0];
        if (cb != 0.0) ghl += adj_entry_grad(a, L.row0 + i, L.col0 + J[b], cb, g);
      }
      for (int q = 0; q < dim; ++q) gx[i + (int64_t)q * m0] += g[q];
    }
    w.sync();
    for (int b = w.tid; b < nJ; b += w.nt) {
      double g[HBA_MAXDIM];
      for (int q = 0; q < dim; ++q) g[q] = 0.0;
      for (int64_t i = 0; i < m0; ++i) {
        const double cb = Cb[i + (int64_t)b * m0];
        if (cb != 0.0) (void)adj_entry_grad(a, L.row0 + i, L.col0 + J[b], cb, g);
      }
      for (int q = 0; q < dim; ++q) gy[J[b] + (int64_t)q * n0] -= g[q];
    }
    w.sync();
    for (int64_t j = w.tid; j < n0; j += w.nt) {
      double g[HBA_MAXDIM];
      for (int q = 0; q < dim; ++q) g[q] = 0.0;
      for (int c = 0; c < nI; ++c) {
        const double rb = Rb[c + j * dm];
        if (rb != 0.0) ghl += adj_entry_grad(a, L.row0 + I[c], L.col0 + j, rb, g);
      }
      for (int q = 0; q < dim; ++q) gy[j + (int64_t)q * n0] -= g[q];
    }
    w.sync();
    for (int c = w.tid; c < nI; c += w.nt) {
      double g[HBA_MAXDIM];
      for (int q = 0; q < dim; ++q) g[q] = 0.0;
      for (int64_t j = 0; j < n0; ++j) {
        const double rb = Rb[c + j * dm];
        if (rb != 0.0) (void)adj_entry_grad(a, L.row0 + I[c], L.col0 + j, rb, g);
      }
      for (int q = 0; q < dim; ++q) gx[I[c] + (int64_t)q * m0] += g[q];
    }
    w.sync();
    // C_k = A(:, J_k) - U V(:, J_k) and R_k = A(I_k, :) - U(I_k, :) V
    // reach the factor columns t < r0
    for (int64_t e = w.tid; e < (int64_t)m0 * r0; e += w.nt) {
      const int i = (int)(e % m0), t = (int)(e / m0);
      double s = 0.0;
      for (int b = 0; b < nJ; ++b) s += Cb[i + (int64_t)b * m0] * Vt[J[b] + (int64_t)t * n0];
      gU[e] -= s;
    }
    w.sync();
    for (int e = w.tid; e < nI * r0; e += w.nt) {
      const int c = e % nI, t = e / nI;
      double s = 0.0;
      for (int64_t j = 0; j < n0; ++j) s += Rb[c + j * dm] * Vt[j + (int64_t)t * n0];
      gU[I[c] + (int64_t)t * m0] -= s;
    }
    w.sync();
    for (int e = w.tid; e < nJ * r0; e += w.nt) {
      const int b = e % nJ, t = e / nJ;
      double s = 0.0;
      for (int64_t i = 0; i < m0; ++i) s += U[i + (int64_t)t * m0] * Cb[i + (int64_t)b * m0];
      gVt[J[b] + (int64_t)t * n0] -= s;
    }
    w.sync();
    for (int64_t e = w.tid; e < (int64_t)n0 * r0; e += w.nt) {
      const int64_t j = e % n0;
      const int t = (int)(e / n0);
      double s = 0.0;
      for (int c = 0; c < nI; ++c) s += U[I[c] + (int64_t)t * m0] * Rb[c + j * dm];
      gVt[e] -= s;
    }
    w.sync();
  }
  const double tot = wg_sum(w, ghl);
  if (w.tid == 0) D[L.gh] = tot;
}

// ------------------------------------------------- merges split over rows ---
// A tall merge (rows >= G max(k, chunk size)) runs as G row chunks: each
// chunk takes the thin QR of its rows of B, B_c = Q_c R_c; the stacked
// R_c = Q' R give B = blockdiag(Q_c) Q' R (a two-level tall-skinny QR);
// R = X diag(s) Y^T, so Ub = blockdiag(Q_c) (Q' X).  The reverse rule is the
// one of adj_merge_bwd, its sums over rows split into per-chunk partials.

template <class W>
HBA_FN void adj_mch_fwd1(W& w, const AdjArgs& a, int ci) {
  const AdjChunk& Ch = a.chunks[ci];
  const AdjMerge& M = a.merges[Ch.merge];
  const int k = M.k;
  const int r1 = a.blocks[M.b1].r;
  const int64_t rows = M.rows, len = Ch.p1 - Ch.p0;
  const AdjSides sd = adj_sides(a, M);
  double* B = a.D + M.Bq + Ch.p0;  // ld rows
  for (int64_t e = w.tid; e < len * k; e += w.nt) {
    const int64_t l = Ch.p0 + e % len;
    const int c = (int)(e / len);
    B[(l - Ch.p0) + c * rows] = c < r1 ? sd.P1[l + c * sd.ldP1] * sd.S1[c]
                                       : sd.P2[l + (c - r1) * sd.ldP2] * sd.S2[c - r1];
  }
  w.sync();
  wg_qr(w, len, k, B, rows, B, rows, a.D + M.Rs + (int64_t)Ch.c * k, (int64_t)M.G * k,
        a.ws + Ch.ws_f1);
}

template <class W>
HBA_FN void adj_mch_fwd2(W& w, const AdjArgs& a, int mi) {
  const AdjMerge& M = a.merges[mi];
  const int k = M.k;
  const int64_t gk = (int64_t)M.G * k;
  double* D = a.D;
  double* Aw = a.ws + M.ws_f2;  // k x k
  double* Yw = Aw + k * k;
  double* hs = Yw + k * k;      // gk + k
  // the stacked R's (upper-triangular k x k blocks) = Q' R; R goes to Xs,
  // where the SVD R = X diag(s) Y^T leaves X
  wg_qr(w, gk, k, D + M.Rs, gk, D + M.Rs, gk, D + M.Xs, k, hs, k);
  wg_svd(w, k, D + M.Xs, k, D + M.Y, k, D + M.S, Aw, Yw, hs);
}

template <class W>
HBA_FN void adj_mch_fwd3(W& w, const AdjArgs& a, int ci) {
  const AdjChunk& Ch = a.chunks[ci];
  const AdjMerge& M = a.merges[Ch.merge];
  const int k = M.k, rho = M.rho;
  const int r1 = a.blocks[M.b1].r, r2 = a.blocks[M.b2].r;
  const int64_t rows = M.rows, n1 = M.n1, n2 = M.n2, len = Ch.p1 - Ch.p0;
  const int64_t gk = (int64_t)M.G * k;
  const AdjSides sd = adj_sides(a, M);
  double* D = a.D;
  // this chunk's k rows of Q' X, then its rows of Ub = Q_c (Q' X)_c
  double* QXc = D + M.QX + (int64_t)Ch.c * k;
  wg_gemm(w, k, k, k, 1.0, D + M.Rs + (int64_t)Ch.c * k, gk, 0, D + M.Xs, k, 0, 0.0, QXc, gk);
  wg_gemm(w, len, k, k, 1.0, D + M.Bq + Ch.p0, rows, 0, QXc, gk, 0, 0.0, D + M.Ub + Ch.p0, rows);
  const AdjBlock& out = a.blocks[M.out];
  double* On = D + (M.horiz ? out.Vt : out.U);
  const int64_t a0 = Ch.o0, a1 = Ch.o1 < n1 ? Ch.o1 : n1;
  const int64_t b0 = Ch.o0 > n1 ? Ch.o0 : n1, b1 = Ch.o1;
  if (a1 > a0)
    wg_gemm(w, a1 - a0, rho, r1, 1.0, sd.O1 + a0, sd.ldO1, 0, D + M.Y, k, 0, 0.0, On + a0,
            n1 + n2);
  if (b1 > b0)
    wg_gemm(w, b1 - b0, rho, r2, 1.0, sd.O2 + (b0 - n1), sd.ldO2, 0, D + M.Y + r1, k, 0, 0.0,
            On + b0, n1 + n2);
}

template <class W>
HBA_FN void adj_mch_bwd1(W& w, const AdjArgs& a, int ci) {
  const AdjChunk& Ch = a.chunks[ci];
  const AdjMerge& M = a.merges[Ch.merge];
  const int k = M.k, rho = M.rho;
  const AdjBlock& b1 = a.blocks[M.b1];
  const AdjBlock& b2 = a.blocks[M.b2];
  const AdjBlock& out = a.blocks[M.out];
  const int r1 = b1.r, r2 = b2.r;
  const int64_t rows = M.rows, n1 = M.n1, n2 = M.n2, len = Ch.p1 - Ch.p0;
  const AdjSides sd = adj_sides(a, M);
  double* D = a.D;
  const double* gPo = D + (M.horiz ? out.gU : out.gVt);
  const double* gOo = D + (M.horiz ? out.gVt : out.gU);
  double* gO1 = D + (M.horiz ? b1.gVt : b1.gU);
  double* gO2 = D + (M.horiz ? b2.gVt : b2.gU);
  const double* Y = D + M.Y;
  const int64_t ldo = n1 + n2;
  double* Ybp = D + M.part + (int64_t)Ch.c * (2 * k * rho + k);  // k x rho
  double* Jmp = Ybp + k * rho;                                    // k x rho
  const int64_t a0 = Ch.o0, a1 = Ch.o1 < n1 ? Ch.o1 : n1;
  const int64_t o0 = Ch.o0 > n1 ? Ch.o0 : n1, o1 = Ch.o1;
  // partial blockdiag(O1, O2)^T gOo over this chunk's O rows
  for (int e = w.tid; e < k * rho; e += w.nt) {
    const int c = e % k, j = e / k;
    double s = 0.0;
    if (c < r1) {
      for (int64_t l = a0; l < a1; ++l) s += sd.O1[l + c * sd.ldO1] * gOo[l + j * ldo];
    } else {
      for (int64_t l = o0; l < o1; ++l)
        s += sd.O2[(l - n1) + (c - r1) * sd.ldO2] * gOo[l + j * ldo];
    }
    Ybp[e] = s;
  }
  // this chunk's rows of the children's O-side cotangents
  if (a1 > a0)
    wg_gemm(w, a1 - a0, r1, rho, 1.0, gOo + a0, ldo, 0, Y, k, 1, 0.0, gO1 + a0, n1);
  if (o1 > o0)
    wg_gemm(w, o1 - o0, r2, rho, 1.0, gOo + o0, ldo, 0, Y + r1, k, 1, 0.0, gO2 + (o0 - n1), n2);
  // partial Ub^T gPo over this chunk's P rows
  wg_gemm(w, k, rho, len, 1.0, D + M.Ub + Ch.p0, rows, 1, gPo + Ch.p0, rows, 0, 0.0, Jmp, k);
}

template <class W>
HBA_FN void adj_mch_bwd2(W& w, const AdjArgs& a, int mi) {
  const AdjMerge& M = a.merges[mi];
  const int k = M.k, rho = M.rho;
  const AdjBlock& out = a.blocks[M.out];
  double* D = a.D;
  const double* Y = D + M.Y;
  const double* s = D + M.S;
  double* Jm = D + M.Jm;
  double* Yb = a.ws + M.ws_b2;  // k x rho
  double* Km = Yb + k * rho;    // k x rho
  double* G = Km + k * rho;     // k x k
  const int64_t stride = 2 * (int64_t)k * rho + k;
  for (int e = w.tid; e < k * rho; e += w.nt) {
    double sy = 0.0, sj = 0.0;
    for (int c = 0; c < M.G; ++c) {
      sy += D[M.part + c * stride + e];
      sj += D[M.part + c * stride + k * rho + e];
    }
    Yb[e] = sy;
    Jm[e] = sj;
  }
  w.sync();
  wg_gemm(w, k, rho, k, 1.0, Y, k, 1, Yb, k, 0, 0.0, Km, k);
  adj_svd_g(w, k, rho, s, D + out.gS, Jm, Km, G);
  wg_gemm(w, k, k, k, 1.0, G, k, 0, Y, k, 1, 0.0, D + M.H, k);
  for (int e = w.tid; e < k * rho; e += w.nt) {
    const int c = e % k, j = e / k;
    double v = Yb[e];
    for (int i = 0; i < k; ++i) v -= Y[c + i * k] * Km[i + j * k];
    D[M.E2 + e] = v / s[j];
  }
  w.sync();
}

template <class W>
HBA_FN void adj_mch_bwd3(W& w, const AdjArgs& a, int ci) {
  const AdjChunk& Ch = a.chunks[ci];
  const AdjMerge& M = a.merges[Ch.merge];
  const int k = M.k, rho = M.rho;
  const AdjBlock& b1 = a.blocks[M.b1];
  const AdjBlock& b2 = a.blocks[M.b2];
  const AdjBlock& out = a.blocks[M.out];
  const int r1 = b1.r;
  const int64_t rows = M.rows, len = Ch.p1 - Ch.p0;
  const AdjSides sd = adj_sides(a, M);
  double* D = a.D;
  const double* gPo = D + (M.horiz ? out.gU : out.gVt) + Ch.p0;  // ld rows
  double* gP1 = D + (M.horiz ? b1.gU : b1.gVt);
  double* gP2 = D + (M.horiz ? b2.gU : b2.gVt);
  const double* Ub = D + M.Ub + Ch.p0;  // ld rows
  const double* Jm = D + M.Jm;
  const double* Y = D + M.Y;
  const double* s = D + M.S;
  double* gSp = D + M.part + (int64_t)Ch.c * (2 * k * rho + k) + 2 * k * rho;  // k
  double* E = a.ws + Ch.ws_b3;  // len x rho
  double* Bb = E + len * rho;   // len x k
  for (int64_t e = w.tid; e < len * rho; e += w.nt) {
    const int64_t l = e % len;
    const int j = (int)(e / len);
    double v = gPo[l + j * rows];
    for (int i = 0; i < k; ++i) v -= Ub[l + i * rows] * Jm[i + j * k];
    E[e] = v / s[j];
  }
  w.sync();
  wg_gemm(w, len, k, k, 1.0, Ub, rows, 0, D + M.H, k, 0, 0.0, Bb, len);
  wg_gemm(w, len, k, rho, 1.0, E, len, 0, Y, k, 1, 1.0, Bb, len);
  wg_gemm(w, len, k, rho, 1.0, Ub, rows, 0, D + M.E2, k, 1, 1.0, Bb, len);
  for (int64_t e = w.tid; e < len * k; e += w.nt) {
    const int64_t l = Ch.p0 + e % len;
    const int c = (int)(e / len);
    if (c < r1)
      gP1[l + c * rows] = Bb[e] * sd.S1[c];
    else
      gP2[l + (c - r1) * rows] = Bb[e] * sd.S2[c - r1];
  }
  for (int c = w.tid; c < k; c += w.nt) {
    double v = 0.0;
    if (c < r1) {
      for (int64_t l = 0; l < len; ++l) v += Bb[l + c * len] * sd.P1[Ch.p0 + l + c * sd.ldP1];
    } else {
      for (int64_t l = 0; l < len; ++l)
        v += Bb[l + c * len] * sd.P2[Ch.p0 + l + (c - r1) * sd.ldP2];
    }
    gSp[c] = v;
  }
  w.sync();
}

template <class W>
HBA_FN void adj_mch_bwd4(W& w, const AdjArgs& a, int mi) {
  const AdjMerge& M = a.merges[mi];
  const int k = M.k, rho = M.rho;
  const AdjBlock& b1 = a.blocks[M.b1];
  const AdjBlock& b2 = a.blocks[M.b2];
  const int64_t stride = 2 * (int64_t)k * rho + k;
  for (int c = w.tid; c < k; c += w.nt) {
    double v = 0.0;
    for (int g = 0; g < M.G; ++g) v += a.D[M.part + g * stride + 2 * k * rho + c];
    if (c < b1.r)
      a.D[b1.gS + c] = v;
    else
      a.D[b2.gS + c - b1.r] = v;
  }
  w.sync();
}

// Gradient rows of row cluster t: the sum over its leaves (t, v).
template <class W>
HBA_FN void adj_red_rows(W& w, const AdjArgs& a, int t) {
  const AdjLeaf& L0 = a.leaves[(int64_t)t * a.nb];
  const int m0 = L0.m0, dim = a.dim;
  for (int64_t e = w.tid; e < (int64_t)m0 * dim; e += w.nt) {
    const int64_t i = e % m0;
    const int q = (int)(e / m0);
    double s = 0.0;
    for (int v = 0; v < a.nb; ++v) s += a.D[a.leaves[(int64_t)t * a.nb + v].gx + e];
    a.gX[(L0.row0 + i) * dim + q] = s;
  }
}

template <class W>
HBA_FN void adj_red_cols(W& w, const AdjArgs& a, int v) {
  const AdjLeaf& L0 = a.leaves[v];
  const int n0 = L0.n0, dim = a.dim;
  for (int64_t e = w.tid; e < (int64_t)n0 * dim; e += w.nt) {
    const int64_t j = e % n0;
    const int q = (int)(e / n0);
    double s = 0.0;
    for (int t = 0; t < a.nb; ++t) s += a.D[a.leaves[(int64_t)t * a.nb + v].gy + e];
    a.gY[(L0.col0 + j) * dim + q] = s;
  }
}

template <class W>
HBA_FN void adj_red_h(W& w, const AdjArgs& a) {
  double s = 0.0;
  for (int i = w.tid; i < a.nleaves; i += w.nt) s += a.D[a.leaves[i].gh];
  s = wg_sum(w, s);
  if (w.tid == 0) a.gh[0] = s;
}

template <class W>
HBA_FN void adj_run_task(W& w, const AdjArgs& a, int kind, int g) {
  switch (kind) {
    case ADJ_LEAF_FWD: adj_leaf_fwd(w, a, g); break;
    case ADJ_REC_FWD: adj_rec_fwd(w, a, g); break;
    case ADJ_MERGE_FWD: adj_merge_fwd(w, a, a.tasks[g]); break;
    case ADJ_ROOT: adj_root(w, a); break;
    case ADJ_MERGE_BWD: adj_merge_bwd(w, a, a.tasks[g]); break;
    case ADJ_MCH_FWD1: adj_mch_fwd1(w, a, a.tasks[g]); break;
    case ADJ_MCH_FWD2: adj_mch_fwd2(w, a, a.tasks[g]); break;
    case ADJ_MCH_FWD3: adj_mch_fwd3(w, a, a.tasks[g]); break;
    case ADJ_MCH_BWD1: adj_mch_bwd1(w, a, a.tasks[g]); break;
    case ADJ_MCH_BWD2: adj_mch_bwd2(w, a, a.tasks[g]); break;
    case ADJ_MCH_BWD3: adj_mch_bwd3(w, a, a.tasks[g]); break;
    case ADJ_MCH_BWD4: adj_mch_bwd4(w, a, a.tasks[g]); break;
    case ADJ_REC_BWD: adj_rec_bwd(w, a, g); break;
    case ADJ_LEAF_BWD: adj_leaf_bwd(w, a, g); break;
    case ADJ_RED_ROWS: adj_red_rows(w, a, g); break;
    case ADJ_RED_COLS: adj_red_cols(w, a, g); break;
    case ADJ_RED_H: adj_red_h(w, a); break;
    default: break;
  }
}
