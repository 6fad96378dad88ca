// Sparse passes with fp32 values other than the CG product: gradient,
// objective, forward and transpose products.
#include "pass.h"

namespace admmbb {

template <bool C16>
static void launch_group(int mode, const PassArgs& a, int tb, int tc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case PASS_GRAD: launch_acc<VAL_F32, C16, PASS_GRAD>(a, tb, tc, st, e0, e1); break;
    case PASS_OBJ: launch_acc<VAL_F32, C16, PASS_OBJ>(a, tb, tc, st, e0, e1); break;
    case PASS_MATVEC: launch_acc<VAL_F32, C16, PASS_MATVEC>(a, tb, tc, st, e0, e1); break;
    default: launch_acc<VAL_F32, C16, PASS_RMATVEC>(a, tb, tc, st, e0, e1); break;
  }
}

void launch_pass_f32_io(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1) {
  if (a.mat.col16)
    launch_group<true>(mode, a, tile_begin, tile_count, st, e0, e1);
  else
    launch_group<false>(mode, a, tile_begin, tile_count, st, e0, e1);
}

}  // namespace admmbb
