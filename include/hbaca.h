/*
 * hbaca.h -- C ABI of the MI355X (gfx950) H-BACA library.
 *
 * H-BACA computes a truncated SVD  A ~ U diag(sigma) V^H  of an m x n matrix
 * whose entries are evaluated on demand in O(1) each (the paper's problem
 * statement, Abstract and Algorithm 3).  The matrix is split by two L-level
 * binary cluster trees into 4^L leaf blocks; every leaf is compressed by
 * blocked adaptive cross approximation (BACA, Algorithm 2) followed by an SVD
 * re-compression (Section "Blocked Adaptive Cross Approximation"), and the
 * leaf factors are merged level by level by truncated SVDs (Algorithm 3,
 * eqs. (14)-(15)).
 *
 * Conventions used by every call:
 *  - All array arguments are DEVICE pointers (HIP), except where a comment
 *    says "host".  Matrices are column-major; point sets are row-major
 *    (point i occupies dim consecutive doubles).
 *  - Rows and columns are assumed already ordered so that contiguous index
 *    ranges are geometric clusters (the paper applies the method to a
 *    KD-permuted matrix); the library never reorders.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  The
 *    compress calls synchronise that stream before returning, because the
 *    output ranks size the results.
 *  - The caller owns every input.  Results are owned by the library until
 *    hb_result_free().  On error *out is set to NULL and nothing leaks.
 *  - No exception or HIP error crosses the ABI: HIP failures map to
 *    HB_EDEVICE; hb_status_string() gives a text for every status.
 *  - Calls on distinct results and streams may run concurrently.
 */
#ifndef HBACA_H
#define HBACA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HB_OK = 0,
  HB_EINVAL = -1,       /* invalid argument (null pointer, size, tolerance...) */
  HB_ENOMEM = -2,       /* device allocation failed */
  HB_EDEVICE = -3,      /* a HIP call or kernel launch failed */
  HB_ERANKCAP = -4,     /* a leaf needed more than params->rank_cap columns */
  HB_ENONFINITE = -5,   /* NaN or Inf in a scalar parameter */
  HB_EUNSUPPORTED = -6  /* size outside what the kernels are built for */
} hb_status;

/* Entry functions A(i, j) for row point x_i and column point y_j. */
typedef enum {
  HB_K_GAUSS = 1,          /* exp(-|x - y|^2 / (gauss_c h^2)), real; the
                              paper's Gaussian kernel has gauss_c = 2 */
  HB_K_LAPLACE = 2,        /* 1 / |x - y|, real */
  HB_K_HELMHOLTZ3D = 3,    /* exp(i k |x - y|) / (4 pi |x - y|), complex */
  HB_K_LOWRANK_SPIKES = 4, /* (G1 G2)(i, j) + spike(i, j), real: the paper's
                              product-of-random kernel plus sparse entries */
  HB_K_EFIE2D = 5,         /* H_0^(2)(k |x - y|), the Hankel function of the
                              second kind and order 0, complex: the paper's
                              EFIE2D kernel (Section "Numerical Results") */
  HB_K_POLYNOMIAL = 6      /* (x^T y + h)^2, real: the paper's polynomial
                              kernel; dim up to HB_POLY_MAXDIM */
} hb_entry_fn;

#define HB_POLY_MAXDIM 256

typedef enum {
  HB_PREC_FP64 = 0,  /* every step in FP64 (complex: FP64 pairs) */
  HB_PREC_MIXED = 1  /* real kernels only: the leaf BACA evaluates entries and
                        forms residual blocks and factors in FP32, accumulating
                        products and Gram blocks in FP64; the norm estimates
                        nu, mu (eqs. (11)-(13)), the leaf SVD re-compression
                        and every merge stay FP64.  Complex kernels return
                        HB_EUNSUPPORTED. */
} hb_precision;

/*
 * Selection of the skeleton rows I_k and columns J_{k+1} in the leaf BACA
 * (Algorithm 2, eqs. (6)-(7)).  The paper uses greedy QRCP and names strong
 * rank-revealing QR as an alternative (Section "Blocked Adaptive Cross
 * Approximation").
 *   HB_SEL_QRCP    greedy QRCP (trailing norms below 1e-12 of the panel's
 *                  largest count as zero; ties to the lowest index)
 *   HB_SEL_STRONG  greedy QRCP, then the swaps of Gu and Eisenstat's strong
 *                  rank-revealing QR: with k the picks above the rounding
 *                  level and W = R11^-1 R12 the coefficients of every other
 *                  candidate in the basis of the k chosen panel columns,
 *                  while max |W(i, j)| > select_f the candidate j replaces
 *                  chosen column i in place (ties: lowest j, then lowest i),
 *                  at most 4 k swaps; the picks past k are then the lowest
 *                  free indices.  Each swap multiplies the volume of the
 *                  chosen columns by |W(i, j)| > select_f.
 */
typedef enum { HB_SEL_QRCP = 0, HB_SEL_STRONG = 1 } hb_selector;

typedef struct {
  int32_t dim;        /* point dimension (1..8; 1..HB_POLY_MAXDIM for
                         POLYNOMIAL); ignored by LOWRANK_SPIKES */
  double h;           /* Gaussian width h > 0; POLYNOMIAL: the shift h */
  double gauss_c;     /* Gaussian normalisation c > 0 */
  double wavenumber;  /* Helmholtz and EFIE2D k > 0 */
  /* LOWRANK_SPIKES only (device arrays): G1 is m x lr_rank row-major, G2 is
     lr_rank x n row-major; spike_lin holds n_spikes sorted linear indices
     i * n + j with values spike_val. */
  int32_t lr_rank;
  const double* lr_G1;
  const double* lr_G2;
  int32_t n_spikes;
  const int64_t* spike_lin;
  const double* spike_val;
  /* Seed of the random first column block J_1 of every leaf (Algorithm 2,
     first line).  Leaf b = t * 2^L + v (row cluster t, column cluster v)
     draws min(d, n0) distinct leaf-local columns by a partial Fisher-Yates
     shuffle driven by SplitMix64 started at seed + b * 0x632BE59BD9B4E019.
     In the batched call block p uses seed + p. */
  uint64_t seed;
  int32_t precision;   /* hb_precision */
  int32_t rank_cap;    /* max BACA rank per leaf; 0 = min(m0, n0) */
  int32_t record_tape; /* 0: nothing; 1: keep per-leaf pivots, d_k, nu, mu for
                          hb_result_leaf_tape; 2: also the frozen structure
                          (every I_k, J_k and pivot order of QR(W_k, eps), and
                          every truncation rank) that hbaca_vjp replays */
  int32_t stop_after;  /* diagnostics: 0 full H-BACA; 1 stop after the leaf
                          BACA (blocks = leaves, A_leaf ~ U Vh^H, sigma = 1);
                          2 stop after the leaf SVD re-compression;
                          2 + s stop after merge step s (odd s: horizontal,
                          even s: vertical); blocks in row-major grid order */
  int32_t diag_panel;  /* diagnostics: 0 default; > 0 merges wider than this
                          many columns use the column-panel QR with panels of
                          this width (1..128 real, 1..64 complex) */
  int32_t diag_svd_storage; /* diagnostics: 0 default (small batches of
                          wide matrices on several workgroups each, otherwise
                          one workgroup per matrix with its matrices in LDS
                          when they fit); 1 one workgroup, matrices in HBM;
                          2 one workgroup, in LDS when they fit; 3 several
                          workgroups wherever the shape allows (p >= k,
                          p <= 512), else as 2 */
  int32_t selector;    /* hb_selector; 0 (greedy QRCP) for a zeroed struct */
  double select_f;     /* HB_SEL_STRONG: swap threshold, finite and > 1
                          (HB_EINVAL otherwise); ignored by HB_SEL_QRCP */
} hb_params;

typedef struct hb_result hb_result; /* opaque */

typedef struct {
  int32_t n_blocks;          /* output blocks (problems, or leaves if stop_after > 0) */
  int32_t n_leaves;
  int32_t levels_max;        /* max L over the problems */
  int32_t leaf_rank_baca_max;
  int32_t leaf_rank_max;     /* after re-compression */
  int32_t iters_max;
  int64_t iters_total;
  int32_t step_rank_max[64]; /* max rank after merge step s (s = 0: leaves;
                                odd: horizontal, even > 0: vertical) */
  int32_t n_steps;
  double ms_setup, ms_baca, ms_recompress, ms_merge, ms_total;  /* device time */
  double entries_evaluated;  /* matrix entries computed by the leaf BACA */
  double resid_bytes;        /* algorithmic HBM bytes of the BACA residual
                                passes: U and V streamed once per iteration */
  double resid_flops;        /* 2 phi d r (m0 + n0) summed over iterations */
  int32_t svd_sweeps_max;    /* most Jacobi sweeps taken by one small SVD */
  int32_t pad;
  /* algorithmic flops (real arithmetic; complex counts 4 per product) of
     the re-compression and of the merges: thin QR of an m x k factor
     2 phi m k^2, applying its Q to k x r singular vectors 2 phi m k r, the
     block product of the other side 2 phi r (r1 n1 + r2 n2); the small SVDs
     are not counted */
  double recompress_flops;
  double merge_flops;
  double resid_cr_bytes;     /* algorithmic bytes of the residual blocks C_k
                                (m0 x d) and R_k (d x n0) written once per
                                iteration: s d (m0 + n0) */
  double ms_svd;             /* device time of the small-SVD launches */
  double ms_qr;              /* device time of the TSQR factor and apply
                                launches (re-compression and merges) */
  double ms_gemm;            /* device time of the other-side block products */
  double svd_flops;          /* algorithmic flops of the small SVDs: QRCP of
                                R^H 4 phi p k q, and 4 phi p q (q - 1) per
                                Jacobi sweep, q = min(p, k) */
  int32_t svd_launches, qr_launches;
  int64_t select_swaps;      /* swaps made by HB_SEL_STRONG over all leaves */
} hb_stats;

/*
 * H-BACA of one m x n matrix (Algorithm 3).
 *   entry_fn_id  hb_entry_fn
 *   params       kernel parameters and options (host struct, required)
 *   points_row   m x dim row points (device); NULL for LOWRANK_SPIKES
 *   points_col   n x dim column points (device); NULL for LOWRANK_SPIKES
 *   tol          relative tolerance eps of every truncation, 0 < tol < 1
 *   d            BACA block size (1..32)
 *   leaf         target leaf size; L = smallest level count with
 *                leaf * 2^L >= max(m, n), lowered until 2^L <= min(m, n)
 * Leaves larger than 2048 in either dimension return HB_EUNSUPPORTED.
 */
hb_status hbaca_compress(int entry_fn_id, const hb_params* params, const double* points_row,
                         const double* points_col, int64_t m, int64_t n, double tol, int32_t d,
                         int32_t leaf, void* stream, hb_result** out);

/*
 * Independent H-BACA of nblocks matrices in one pass: all their leaves run in
 * one leaf-kernel launch and every merge step of all blocks is one batch.
 * Block p has rows points_row[row_off[p] .. row_off[p] + row_cnt[p]) and
 * columns points_col[col_off[p] ...]; the offset/count arrays are HOST
 * arrays of nblocks entries.  LOWRANK_SPIKES is not accepted here.
 */
hb_status hbaca_compress_batched(int entry_fn_id, const hb_params* params, int64_t nblocks,
                                 const double* points_row, const int64_t* row_off,
                                 const int64_t* row_cnt, const double* points_col,
                                 const int64_t* col_off, const int64_t* col_cnt, double tol,
                                 int32_t d, int32_t leaf, void* stream, hb_result** out);

/* Number of output blocks, and rank / rows / columns of one of them
   (-1 on a bad handle or index). */
int64_t hb_result_nblocks(const hb_result* res);
int64_t hb_result_rank(const hb_result* res, int64_t block);
int64_t hb_result_rows(const hb_result* res, int64_t block);
int64_t hb_result_cols(const hb_result* res, int64_t block);
/* 1 if the factors are complex (interleaved FP64 pairs), 0 if real FP64. */
int32_t hb_result_is_complex(const hb_result* res);

/*
 * Copy block `block`: U (rows x r), sigma (r) and Vh (cols x r), all
 * column-major DEVICE buffers of the result's scalar type (sigma is real
 * FP64), such that A_block ~ U diag(sigma) Vh^H.  Any pointer may be NULL.
 * Asynchronous on `stream`.
 */
hb_status hb_result_copy(const hb_result* res, int64_t block, void* U, double* sigma, void* Vh,
                         void* stream);

/*
 * The compressed operator of block `block` applied to a DEVICE vector:
 *   adjoint = 0:  out (rows)  = U diag(sigma) Vh^H in  (in: cols entries)
 *   adjoint = 1:  out (cols)  = Vh diag(sigma) U^H in  (in: rows entries)
 * Vectors hold the result's scalar type (FP64, or interleaved FP64 pairs for
 * a complex result).  This is y = U (V^T w) of the differentiation workload
 * and its adjoint, the gradient of <y, ybar> with respect to w.  Asynchronous
 * on `stream`; `in` and `out` must not overlap.  Ranks above 4096 (8192 real)
 * return HB_EUNSUPPORTED.
 */
hb_status hbaca_apply(const hb_result* res, int64_t block, const void* in, void* out,
                      int32_t adjoint, void* stream);

/*
 * hbaca_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and the same kernels, with the r per-column products held
 * in a library-owned static device buffer of 64 KiB per GPU instead of an
 * allocation.  The call allocates nothing.  Ranks whose products exceed
 * 64 KiB (4096 complex, 8192 real) return HB_EUNSUPPORTED.  Every call on
 * one GPU shares that buffer: calls that overlap on one GPU (concurrent
 * streams or host threads) race and must be serialised by the caller.  The
 * buffer is fully written before it is read, so no clearing is needed.
 * Arguments, layouts and errors are those of hbaca_apply; HB_EDEVICE also
 * when the buffer's device address cannot be obtained.
 */
hb_status hbaca_apply_noalloc(const hb_result* res, int64_t block, const void* in, void* out,
                              int32_t adjoint, void* stream);

/*
 * Vector-Jacobian product of y = A~(h, X, Y) w with pivots and ranks frozen.
 *
 * With every BACA iteration's row block I_k, column block J_k, pivot order
 * of QR(W_k, eps) and d_k (Algorithm 2, eqs. (6)-(9)) and every truncation
 * rank of the re-compression and of the merges (Algorithm 3, eqs.
 * (14)-(15)) held at the values of the forward run, the compressed
 * operator A~ depends smoothly on the sampled Gaussian entries
 * exp(-|x_i - y_j|^2 / (c h^2)).  This call replays that fixed pipeline in
 * FP64 on the device and runs it in reverse, returning the gradient of
 * <ybar, A~ w> with respect to w, the width h, the row points and the
 * column points.
 *
 * res:   a real Gaussian (HB_K_GAUSS) result of hbaca_compress run to the
 *        end (stop_after = 0) with params->record_tape = 2; otherwise
 *        HB_EINVAL (HB_EUNSUPPORTED for another kernel).
 * w:     DEVICE, n FP64 entries;  ybar: DEVICE, m FP64 entries.
 * grad_w: DEVICE, n FP64 (= A~^T ybar of the replayed factors);
 * grad_h: DEVICE, 1 FP64;
 * grad_points_row: DEVICE, m x dim FP64 in the layout of points_row;
 * grad_points_col: DEVICE, n x dim FP64 in the layout of points_col.
 * Any gradient pointer may be NULL to skip it.  The call allocates its own
 * device workspace (the replayed factors, the saved blocks of every
 * iteration and merge, and the cotangents: about 11.3 GB for a 50000 x
 * 50000 Gaussian with leaves of 1563 and root rank 63; HB_ENOMEM when it
 * cannot), runs on `stream` and synchronises it before returning.  The replay assumes the frozen ranks sit at a gap
 * of the singular values (distinct kept values, separated from the dropped
 * ones); where they do not, the gradient is not defined and the result is
 * not finite.
 */
hb_status hbaca_vjp(const hb_result* res, const double* w, const double* ybar, double* grad_w,
                    double* grad_h, double* grad_points_row, double* grad_points_col,
                    void* stream);

/*
 * hbaca_vjp for FP32 vectors, as the differentiation workload draws w and b:
 * w (n) and ybar (m) are widened to FP64 on the device, the frozen pipeline
 * is replayed and reversed in FP64 exactly as by hbaca_vjp, and the
 * w-gradient is rounded to FP32 into wbar (n).  hbar (1), points_row_bar
 * (m x dim) and points_col_bar (n x dim) are FP64 as in hbaca_vjp.  All
 * pointers are DEVICE; wbar, hbar and the point gradients may be NULL to
 * skip them.  Same requirements, errors and workspace as hbaca_vjp, plus
 * 8 (2n + m) bytes for the widened vectors; synchronises `stream` before
 * returning.
 */
hb_status hbaca_adjoint(const hb_result* res, const float* w, const float* ybar, float* wbar,
                        double* hbar, double* points_row_bar, double* points_col_bar,
                        void* stream);

/*
 * The frozen operator at new parameters: the pipeline recorded in `tape`
 * (same requirements as hbaca_vjp) replayed in FP64 with the same pivots
 * and ranks, at new points and a new Gaussian width, without any new
 * pivot or rank decision.  This is the map whose derivative hbaca_vjp
 * returns, so central differences of it check that gradient.
 *
 * params: only dim (must equal the tape's), h and gauss_c are read.
 * points_row, points_col: DEVICE, m x dim and n x dim FP64 (the tape's
 *        m and n), copied into the new result.
 * *out:  a new single-block result (rank = the tape's root rank) owned by
 *        the caller (hb_result_free); it carries the tape's frozen
 *        structure, so hbaca_vjp and hbaca_recompute_frozen accept it too.
 *        NULL on error.
 * Runs on `stream` and synchronises it before returning.  Errors as for
 * hbaca_vjp; HB_ENONFINITE for a non-finite h or gauss_c.
 */
hb_status hbaca_recompute_frozen(const hb_result* tape, const hb_params* params,
                                 const double* points_row, const double* points_col,
                                 void* stream, hb_result** out);

/*
 * The partition hbaca_compress uses (host only, no device work): the number
 * of levels L (the smallest L with leaf 2^L >= max(m, n), lowered until
 * 2^L <= min(m, n)) and, when the arrays are given, for every leaf
 * b = t 2^L + v of the cluster trees (a node of size s splits into
 * ceil(s/2) then floor(s/2), Algorithm 3):
 *   leaves[4b .. 4b+3] = first row, rows, first column, columns;
 *   j1[b d .. b d + d - 1] = its first column block J_1 (Algorithm 2), the
 *   first min(d, n0) leaf-local columns of a partial Fisher-Yates shuffle
 *   driven by SplitMix64 from seed + b * 0x632BE59BD9B4E019, then -1.
 * Host arrays of 4^L * 4 and 4^L * d entries; either may be NULL (both
 * NULL: only *L_out).  HB_EINVAL for m, n, leaf or d below 1.
 */
hb_status hb_partition(int64_t m, int64_t n, int32_t leaf, int32_t d, uint64_t seed,
                       int32_t* L_out, int64_t* leaves, int32_t* j1);

/*
 * Hierarchical (HODLR) matrix of the kernel matrix of one point set with
 * itself, built with H-BACA: the construction of hierarchical matrices the
 * paper names as the method's use (Introduction; Section "Numerical
 * Results" compresses one off-diagonal block of a KD-permuted kernel matrix
 * and notes that the permutation yields a hierarchical representation).
 *   points  N x dim row-major DEVICE array, already in KD order
 *   nmin    leaf size: the cluster tree of [0, N) splits a node of s points
 *           into ceil(s/2) and floor(s/2) down to the smallest depth whose
 *           nodes hold at most nmin points
 *   tol, d, leaf  as for hbaca_compress, for every off-diagonal block
 * Both off-diagonal blocks A(c1, c2) and A(c2, c1) of every internal node
 * are compressed in one hbaca_compress_batched pass (block p, numbered level
 * by level from the root, nodes left to right, A(c1, c2) first, draws its
 * first column blocks from params->seed + p); the diagonal blocks of the
 * leaves are evaluated densely.  Real kernels finite at r = 0 only: GAUSS
 * and POLYNOMIAL (others return HB_EUNSUPPORTED).  Synchronises `stream`.
 * The object is library-owned until hb_hodlr_free.
 */
typedef struct hb_hodlr hb_hodlr; /* opaque */
hb_status hb_hodlr_build(int entry_fn_id, const hb_params* params, const double* points, int64_t N,
                         int32_t nmin, double tol, int32_t d, int32_t leaf, void* stream,
                         hb_hodlr** out);
/* The H-BACA result of the off-diagonal blocks (owned by the HODLR object;
   block p in the order above; NULL when N <= nmin). */
const hb_result* hb_hodlr_blocks(const hb_hodlr* h);
int64_t hb_hodlr_nblocks(const hb_hodlr* h);
int64_t hb_hodlr_nleaves(const hb_hodlr* h);
/* level, row offset, row count, column offset, column count of block p. */
hb_status hb_hodlr_block_info(const hb_hodlr* h, int64_t block, int64_t* info5);
/* y = A_H x for DEVICE vectors of N FP64 entries (must not overlap): the
   dense leaves, then the low-rank blocks level by level (the blocks of one
   level cover disjoint rows, so the sums have a fixed order).  Asynchronous
   on `stream`. */
hb_status hb_hodlr_matvec(const hb_hodlr* h, const double* x, double* y, void* stream);
void hb_hodlr_free(hb_hodlr* h);

/*
 * Autotuner of the thin-QR (TSQR) kernels that the re-compression and the
 * merges use.  Each width (16, 32, 64, 128 columns; 128 real only) has two
 * lane layouts (a node on K x NQ lanes, or on twice as many with half the
 * rows each); this call times both, factor and apply, on synthetic batches
 * of 1 node (the top of a tree) and 256 nodes (its bottom) and keeps the
 * faster for each (scalar type, width, batch size) in a process-wide table
 * that later calls use.  Both layouts give the same reflectors up to the
 * order of their partial sums.  Call it with no other library work in
 * flight (the table is shared).  Allocates and frees its own synthetic
 * data; synchronises `stream`.
 *   table  16 int32 (may be NULL): [scalar][width 16/32/64/128][batch
 *          1 / 256] -> layout 0 or 1
 *   us     32 doubles (may be NULL): the measured microseconds per factor
 *          plus apply, [scalar][width][batch][layout]
 */
hb_status hb_autotune(void* stream, int32_t* table, double* us);

/* Statistics of the call (host struct). */
hb_status hb_result_stats(const hb_result* res, hb_stats* out);

/*
 * Leaf descriptors (host, 12 int64 per leaf, in leaf order: block-major,
 * then b = t * 2^L + v):
 *   block, t, v, row0, col0, m0, n0, rank_baca, rank_leaf, iterations,
 *   status, tape_len
 */
int64_t hb_result_nleaves(const hb_result* res);
hb_status hb_result_leaf_info(const hb_result* res, int64_t leaf, int64_t* info12);

/*
 * Pivot tape of one leaf (needs params->record_tape): rows[c] and cols[c],
 * c < rank_baca, are the leaf-local rows I_k(1:d_k) and columns J_k(Jbar) in
 * the order their cross blocks were appended; dk[k], nu[k], mu[k] for each
 * iteration k < iterations (an iteration that ends with d_k = 0 is included).
 * Host buffers sized from hb_result_leaf_info; any pointer may be NULL.
 */
hb_status hb_result_leaf_tape(const hb_result* res, int64_t leaf, int32_t* rows, int32_t* cols,
                              int32_t* dk, double* nu, double* mu);

/*
 * Frozen structure of a result compressed with record_tape = 2 (host):
 * *stride = ints per iteration record; records (host, iterations x stride
 * int32, may be NULL) receives, per iteration of the leaf, nI, nJ, d_k,
 * then I_k (DMAX slots), J_k (DMAX slots) and the pivot order of
 * QR(W_k, eps) (DMAX slots), DMAX = (stride - 3) / 3.  HB_EINVAL if the
 * result holds no frozen structure.
 */
hb_status hb_result_leaf_frozen(const hb_result* res, int64_t leaf, int32_t* stride,
                                int32_t* records);
/*
 * Every merge rank of a whole-pipeline result with a frozen structure
 * (host): for l = 1..L the horizontal merges of the level (block (ti, v)
 * of the 2^(L-l+1) x 2^(L-l) grid, ti-major), then its vertical merges
 * (block (t, v), t-major).  *count receives the number; ranks may be NULL.
 */
hb_status hb_result_merge_ranks(const hb_result* res, int32_t* ranks, int64_t* count);

/*
 * Untimed check: sum over rows i = 0, stride, 2 stride, ... of
 * |A(i,j) - (U diag(sigma) Vh^H)(i,j)|^2 and of |A(i,j)|^2, every column j,
 * with A re-evaluated on the device in FP64 (host outputs).  The problem's
 * own entry function and points are used; for a batched result `block`
 * selects the problem.
 */
hb_status hb_result_error(const hb_result* res, int64_t block, int64_t row_stride, double* err2,
                          double* ref2, void* stream);

void hb_result_free(hb_result* res);
const char* hb_status_string(hb_status status);

#ifdef __cplusplus
}
#endif

#endif /* HBACA_H */
