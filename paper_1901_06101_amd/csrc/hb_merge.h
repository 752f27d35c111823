// Kernels behind the SVD re-compression of BACA leaves and the hierarchical
// merges (Algorithm 3; eqs. (14)-(15)).  Every step computes a truncated SVD
// of a tall block B = [P1 diag(S1), P2 diag(S2)] (or a plain tall factor) as
// Householder QR of B, then the SVD of the small triangular factor.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// A node of a tall-skinny QR (TSQR) tree.  Level-0 nodes hold up to MC rows
// of B; a higher node stacks the R factors of up to MC / k children.
struct QRNodeDev {
  int32_t rows;    // stacked input rows (<= MC)
  int32_t k;       // columns of B
  int32_t steps;   // Householder steps = min(rows, k) = rows of this node's R
  int32_t level0;  // 1: rows come from B, 0: rows come from child R factors
  // level 0: B(row0 + i, j) = j < n1 ? P1(row0+i, j) * S1[j] : P2(row0+i, j-n1) * S2[j-n1]
  const void* P1;
  const void* P2;
  const double* S1;  // may be null (scale 1)
  const double* S2;
  int64_t ld1, ld2, row0;
  int32_t n1, n2;
  // level > 0
  int32_t child0, nchild;
  // this node's storage: MC x k tile (column-major, ld MC) holding R above the
  // diagonal and the reflectors on and below it; alpha = diag(R); beta
  int64_t store;  // element offset into the tile arena
  int32_t ab;     // offset into the alpha / beta arrays (k entries)
  int32_t pad;
};

// Applying the tree's Q to Z = [Zin; Ztr] (Ztr = 0 when null): one node per
// entry.  Zin holds the node's first `steps` rows, Ztr its remaining rows.
struct QRApplyDev {
  int32_t rows, steps, r;  // node rows, reflector count, columns of Z
  int32_t pad;
  int64_t store;
  int32_t ab;
  int32_t pad2;
  const void* Zin;  // steps x r (column-major, ld ldin)
  void* Zout;       // rows x r (column-major, ld ldout)
  int64_t ldin, ldout;
  const void* Ztr;  // (rows - steps) x r, ld ldtr, or null
  int64_t ldtr;
};

// Applying the tree's Q^H bottom-up: the node's rows x r input is reflected;
// its first `steps` rows go up (to the parent's stacked input, or to the
// coupling block R_12 at the top), the others to the trailing block.
struct QRApplyHDev {
  int32_t rows, steps, r;
  int32_t pad;
  int64_t store;
  int32_t ab;
  int32_t pad2;
  const void* Zin;  // rows x r, ld ldin
  void* Zup;        // steps x r, ld ldup
  void* Ztr;        // (rows - steps) x r, ld ldtr
  int64_t ldin, ldup, ldtr;
};

// B = [P1 diag(S1), P2 diag(S2)] materialised (column-major, ld ldb).
struct ConcatDev {
  const void* P1;
  const void* P2;
  const double* S1;
  const double* S2;
  int64_t m;
  int32_t n1, n2;
  void* B;
};

// One small SVD: R (p x k) read from a TSQR top node or given explicitly.
struct SVDJobDev {
  int32_t p, k;       // R is p x k
  int32_t from_node;  // 1: R from a TSQR node (store/ab), 0: explicit R
  int32_t pad;
  int64_t store;
  int32_t ab;
  int32_t pad2;
  const void* R;   // explicit R, column-major ld p
  void* A;         // HBM workspace, p x k elements (R^H and its QR when they
                   // do not fit in LDS)
  void* W;         // HBM workspace, p x k elements (R2^H)
  double* S;       // k singular values (sorted descending on return)
  int32_t* perm;   // k: sorted position -> column
  int32_t* rank;   // out: [0] eps-rank r, [1] Jacobi sweeps used
  void* Xr;        // p x k output: left singular vectors, sorted (ld p)
  void* Yr;        // k x k output: first r columns = right singular vectors
                   // R^H X_r diag(1/S_r) (ld k)
  int32_t* cperm;  // p ints: the row permutation of the preconditioner, kept
                   // for the multi-workgroup Jacobi (may be null otherwise)
};

// Batched device-to-device copies (one workgroup per entry).
struct CopyDev {
  const void* src;
  void* dst;
  int64_t bytes;  // multiple of 8
};

// C(row, c) = sum_t A_b(row, t) * Y(t0_b + t, c) for the two diagonal blocks
// of blockdiag(A1, A2) * Y (the "other side" of a merge).
struct BlockGemmDev {
  const void* A1;
  const void* A2;
  int64_t lda1, lda2;
  int32_t n1, n2;  // rows of A1, A2
  int32_t r1, r2;  // columns of A1, A2 (rows of the two Y blocks)
  const void* Y;   // (r1 + r2) x r, column-major ld ldy
  int64_t ldy;
  int32_t r;
  int32_t pad;
  void* C;  // (n1 + n2) x r, column-major ld ldc
  int64_t ldc;
};

// Copy of a TSQR top node's R (p x k) into a column-major block (ld ld).
struct RCopyDev {
  int64_t store;
  int32_t ab;
  int32_t p, k;
  int32_t pad;
  void* dst;
  int64_t ld;
};

// dst (P x k, ld P) = rows 0..P-1 of src (ld ld_src).
struct RCompactDev {
  const void* src;
  int64_t ld_src;
  void* dst;
  int32_t P, k;
};

// M (pa x pb, column-major, ld pa) = A B^H for A (pa x k, ld pa) and
// B (pb x k, ld pb), both upper trapezoidal: A(i, t) = 0 for t < i.
struct RRhDev {
  const void* A;
  const void* B;
  void* M;
  int32_t pa, pb, k;
  int32_t pad;
};

namespace hbk {
// scalar: 0 double, 1 complex double
int copy_list_launch(const CopyDev* jobs_dev, int njobs, hipStream_t st);
int rcopy_launch(int scalar, const RCopyDev* jobs_dev, int njobs, const void* store,
                 const void* alpha, hipStream_t st);
int rcompact_launch(int scalar, const RCompactDev* jobs_dev, int njobs, hipStream_t st);
int zero_fill_launch(void* ptr, size_t bytes, hipStream_t st);
int tsqr_factor_launch(int scalar, int kmax, const QRNodeDev* nodes_dev, int nnodes,
                       const QRNodeDev* level_below_dev, void* store, void* alpha,
                       double* beta, hipStream_t st);
int tsqr_apply_launch(int scalar, int kmax, const QRApplyDev* jobs_dev, int njobs,
                      const void* store, const double* beta, hipStream_t st);
int svd_launch(int scalar, const SVDJobDev* jobs_dev, int njobs, int kmax_batch, int pmax_batch,
               const void* store, const void* alpha, double eps, hipStream_t st,
               int force_storage = 0, bool precond_only = false);
int block_gemm_launch(int scalar, const BlockGemmDev* jobs_dev, int njobs, int max_rows,
                      int max_r, hipStream_t st);
int tsqr_applyh_launch(int scalar, int kmax, const QRApplyHDev* jobs_dev, int njobs,
                       const void* store, const double* beta, hipStream_t st);
int concat_launch(int scalar, const ConcatDev* jobs_dev, int njobs, int64_t max_m, int max_k,
                  hipStream_t st);
int rrh_launch(int scalar, const RRhDev* jobs_dev, int njobs, int64_t max_entries, hipStream_t st);
// Multi-workgroup Jacobi SVD (cooperative launch) of jobs with p >= k, after
// svd_launch(..., precond_only = true) has left each job's preconditioned
// W = R2^H in its W workspace and the row permutation in cperm: workgroups
// per matrix (0: not suited), whether the grid can be co-resident,
// workspace bytes, and the launch (-2: not co-resident).
int svd_wide_blocks(int scalar, int p, int k);
bool svd_wide_fits(int scalar, int njobs, int B, int pmax);
size_t svd_wide_work_bytes(int njobs, int B);
int svd_wide_launch(int scalar, const SVDJobDev* jobs_dev, int njobs, int B, int pmax,
                    const void* store, const void* alpha, double eps, void* work, hipStream_t st);
int tsqr_mc(int scalar, int kmax);
int tsqr_autotune(hipStream_t st, int* table, double* us);
int tsqr_kmax_for(int scalar, int k);
}  // namespace hbk
