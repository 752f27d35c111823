// Leaf BACA launches with greedy QRCP pivot selection (Algorithm 2); the
// kernels are in hb_baca_impl.h.  Launches with the strong rank-revealing
// selection are instantiated in hb_baca_strong.hip.
#include "hb_baca_impl.h"

namespace hbk {

int baca_launch(int scalar, int dmax, int rpt, const BacaArgs& a, hipStream_t st) {
  if (a.nleaves == 0) return 0;
  if (a.selector == 1) return baca_launch_strong(scalar, dmax, rpt, a, st);
#define HB_CASE(S, TY, D, R) \
  if (scalar == S && dmax == D && rpt == R) return launch_one<TY, D, R, false>(a, st);
  HB_BACA_INSTANCES(HB_CASE)
#undef HB_CASE
  return -1;
}

}  // namespace hbk
