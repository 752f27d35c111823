// Leaf BACA launches with the strong rank-revealing pivot selection (greedy
// QRCP refined by Gu-Eisenstat swaps, strong_refine in hb_baca_impl.h): a
// separate instantiation of the leaf kernel, so that the default kernel
// carries none of its registers.
#include "hb_baca_impl.h"

namespace hbk {

int baca_launch_strong(int scalar, int dmax, int rpt, const BacaArgs& a, hipStream_t st) {
  if (a.nleaves == 0) return 0;
#define HB_CASE(S, TY, D, R) \
  if (scalar == S && dmax == D && rpt == R) return launch_one<TY, D, R, true>(a, st);
  HB_BACA_INSTANCES(HB_CASE)
#undef HB_CASE
  return -1;
}

}  // namespace hbk
