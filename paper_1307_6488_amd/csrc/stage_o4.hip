// stage_o4.hip -- order-4 instances of the stage kernel and their launcher.
// Default: the direct-load kernel (stage_kernel.hpp).  Built with
// -DCHEMORA_O4_LDS: the LDS-staged kernel (stage_lds.hpp), whose staged axis
// reach R is 2 (centred, KO r <= 2) or 3 (upwinded or KO r = 3).
#include "stage_lds.hpp"

namespace chemora {

namespace {
template <bool UPWIND, int R, int MODE>
void launch(const StageArgs& a, hipStream_t s) {
  dim3 block(TILE_X, TILE_Y, 1);
  dim3 grid(a.tiles_x * a.tiles_y * a.geo.nz, 1, 1);
#ifdef CHEMORA_O4_LDS
  hipLaunchKernelGGL((stage_lds_kernel<4, UPWIND, R, MODE>), grid, block, 0, s, a);
#else
  hipLaunchKernelGGL((stage_kernel<4, UPWIND, MODE>), grid, block, 0, s, a);
#endif
}

template <bool UPWIND, int R>
void by_mode(int mode, const StageArgs& a, hipStream_t s) {
  switch (mode) {
    case MODE_RHS: launch<UPWIND, R, MODE_RHS>(a, s); break;
    case MODE_STAGE1: launch<UPWIND, R, MODE_STAGE1>(a, s); break;
    case MODE_STAGE23: launch<UPWIND, R, MODE_STAGE23>(a, s); break;
    default: launch<UPWIND, R, MODE_STAGE4>(a, s); break;
  }
}
}  // namespace

void launch_stage_o4(int mode, bool upwind, const StageArgs& a, hipStream_t s) {
  if (upwind)
    by_mode<true, 3>(mode, a, s);
#ifdef CHEMORA_O4_LDS
  else if (a.sc.ko_r > 2)
    by_mode<false, 3>(mode, a, s);
#endif
  else
    by_mode<false, 2>(mode, a, s);
}

}  // namespace chemora
