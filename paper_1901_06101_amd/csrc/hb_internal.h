// Internal structures shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hb_adj.h"
#include "hb_entries.h"

// One BACA leaf (Algorithm 2) as the leaf kernel sees it.
struct BacaLeafDev {
  int32_t m0, n0;      // leaf size
  int64_t row0, col0;  // global offsets of the leaf's first row / column
  int64_t u_off;       // U: m0 x cap, column-major, ld m0 (elements)
  int64_t v_off;       // Vh = V^H: n0 x cap, column-major, ld n0
  int64_t c_off;       // scratch C: m0 x DMAX, ld m0
  int64_t r_off;       // scratch R^T: n0 x DMAX, ld n0
  int32_t cap;         // factor capacity in columns
  int32_t tape_off;    // offset of cap entries in the pivot tapes
  int32_t it_off;      // offset of cap+1 entries in the per-iteration records
  int32_t j1_off;      // offset of the first column block in the j1 array
  int32_t nj1;         // its length, min(d, n0)
  int32_t pad;
};

struct BacaOutDev {
  int32_t rank;
  int32_t iters;
  int32_t status;  // 0 ok, 1 factor capacity exhausted, 2 a pivot outside its candidate range
  int32_t swaps;   // swaps made by the strong rank-revealing selection
  double mu;
};

struct BacaArgs {
  const BacaLeafDev* leaves;
  BacaOutDev* out;
  EntryDev E;
  void* U;   // factor arena (scalar type of the launch)
  void* V;   // Vh arena
  void* C;   // residual column scratch
  void* R;   // residual row scratch (transposed)
  const int32_t* j1;
  int32_t* tape_rows;  // I_k(1:d_k), concatenated in U's column order
  int32_t* tape_cols;  // J_k(Jbar), concatenated in V's row order
  int32_t* it_dk;
  double* it_nu;
  double* it_mu;
  // frozen structure (NULL: not recorded): per iteration, at
  // (it_off + k) * fz_stride: nI, nJ, d_k, then I_k (DMAX slots), J_k (DMAX
  // slots) and the pivot order of QR(W_k, eps) (DMAX slots)
  int32_t* fz;
  double eps;
  int32_t nleaves;
  int32_t fz_stride;  // 3 + 3 DMAX when fz is set
  // work queue of the persistent launch: the next leaf index to take (the
  // leaves are ordered largest first); zero before the launch
  int32_t* queue;
  // pivot selection of eqs. (6)-(7): 0 greedy QRCP, 1 QRCP then strong
  // rank-revealing swaps while a coefficient exceeds select_f
  int32_t selector;
  double select_f;
};

// host launchers (defined in the .hip files)
namespace hbk {
int baca_launch(int scalar /*0 f64, 1 c128, 2 f32*/, int dmax, int rpt, const BacaArgs& a,
                hipStream_t st);
// the same with the strong rank-revealing selection (a.selector == 1)
int baca_launch_strong(int scalar, int dmax, int rpt, const BacaArgs& a, hipStream_t st);
// one launch of the adjoint tasks of one kind (AdjTaskKind), tasks
// base .. base + count - 1
int adj_launch(int kind, int base, int count, const AdjArgs& a, hipStream_t st);
}
