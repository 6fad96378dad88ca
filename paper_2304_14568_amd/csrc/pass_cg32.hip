// The CG product pass with fp32 values.
#include "pass.h"

namespace admmbb {

template <bool C16>
static void launch_group(int mode, const PassArgs& a, int tb, int tc, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  (void)mode;
  launch_acc<VAL_F32, C16, PASS_CG>(a, tb, tc, st, e0, e1);
}

void launch_pass_cg_f32(int mode, const PassArgs& a, int tile_begin, int tile_count, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1) {
  if (a.mat.col16)
    launch_group<true>(mode, a, tile_begin, tile_count, st, e0, e1);
  else
    launch_group<false>(mode, a, tile_begin, tile_count, st, e0, e1);
}

}  // namespace admmbb
