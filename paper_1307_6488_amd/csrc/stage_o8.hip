// stage_o8.hip -- instances of the fused stage kernel for order-8
// finite differences, and their launcher.
#include "stage_kernel.hpp"

namespace chemora {

namespace {
template <bool UPWIND, int MODE>
void launch(const StageArgs& a, hipStream_t s) {
  dim3 block(TILE_X, TILE_Y, 1);
  dim3 grid(a.tiles_x * a.tiles_y * a.geo.nz, 1, 1);
  hipLaunchKernelGGL((stage_kernel<8, UPWIND, MODE>), grid, block, 0, s, a);
}

template <bool UPWIND>
void by_mode(int mode, const StageArgs& a, hipStream_t s) {
  switch (mode) {
    case MODE_RHS: launch<UPWIND, MODE_RHS>(a, s); break;
    case MODE_STAGE1: launch<UPWIND, MODE_STAGE1>(a, s); break;
    case MODE_STAGE23: launch<UPWIND, MODE_STAGE23>(a, s); break;
    default: launch<UPWIND, MODE_STAGE4>(a, s); break;
  }
}
}  // namespace

void launch_stage_o8(int mode, bool upwind, const StageArgs& a, hipStream_t s) {
  if (upwind)
    by_mode<true>(mode, a, s);
  else
    by_mode<false>(mode, a, s);
}

}  // namespace chemora
