// Kernels of the frozen-pivot adjoint: every task of hb_adj.h runs on one
// 256-lane workgroup; a launch covers the tasks of one phase (all leaves,
// all merges of one level, the root, the gradient reductions).
#include <hip/hip_runtime.h>

#include "hb_internal.h"

namespace {

constexpr int ADJ_NT = 256;

struct WgDev {
  int tid, nt;
  double* red;
  __device__ void sync() { __syncthreads(); }
};

template <int KIND>
__global__ __launch_bounds__(ADJ_NT) void adj_kernel(AdjArgs a, int base) {
  __shared__ double red[3 * ADJ_NT + ADJ_RED_EXTRA];
  WgDev w{(int)threadIdx.x, ADJ_NT, red};
  adj_run_task(w, a, KIND, base + (int)blockIdx.x);
}

template <int KIND>
static void launch_kind(int base, int count, const AdjArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(adj_kernel<KIND>, dim3((unsigned)count), dim3(ADJ_NT), 0, st, a, base);
}

}  // namespace

namespace hbk {

int adj_launch(int kind, int base, int count, const AdjArgs& a, hipStream_t st) {
  if (count <= 0) return 0;
  switch (kind) {
    case ADJ_LEAF_FWD: launch_kind<ADJ_LEAF_FWD>(base, count, a, st); break;
    case ADJ_REC_FWD: launch_kind<ADJ_REC_FWD>(base, count, a, st); break;
    case ADJ_MERGE_FWD: launch_kind<ADJ_MERGE_FWD>(base, count, a, st); break;
    case ADJ_ROOT: launch_kind<ADJ_ROOT>(base, count, a, st); break;
    case ADJ_MERGE_BWD: launch_kind<ADJ_MERGE_BWD>(base, count, a, st); break;
    case ADJ_REC_BWD: launch_kind<ADJ_REC_BWD>(base, count, a, st); break;
    case ADJ_LEAF_BWD: launch_kind<ADJ_LEAF_BWD>(base, count, a, st); break;
    case ADJ_RED_ROWS: launch_kind<ADJ_RED_ROWS>(base, count, a, st); break;
    case ADJ_RED_COLS: launch_kind<ADJ_RED_COLS>(base, count, a, st); break;
    case ADJ_RED_H: launch_kind<ADJ_RED_H>(base, count, a, st); break;
    case ADJ_MCH_FWD1: launch_kind<ADJ_MCH_FWD1>(base, count, a, st); break;
    case ADJ_MCH_FWD2: launch_kind<ADJ_MCH_FWD2>(base, count, a, st); break;
    case ADJ_MCH_FWD3: launch_kind<ADJ_MCH_FWD3>(base, count, a, st); break;
    case ADJ_MCH_BWD1: launch_kind<ADJ_MCH_BWD1>(base, count, a, st); break;
    case ADJ_MCH_BWD2: launch_kind<ADJ_MCH_BWD2>(base, count, a, st); break;
    case ADJ_MCH_BWD3: launch_kind<ADJ_MCH_BWD3>(base, count, a, st); break;
    case ADJ_MCH_BWD4: launch_kind<ADJ_MCH_BWD4>(base, count, a, st); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

}  // namespace hbk
