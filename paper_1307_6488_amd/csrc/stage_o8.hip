// stage_o8.hip -- order-8 instances of the stage kernel and their launcher.
// The staged axis reach R is 4 (centred, Kreiss-Oliger r <= 4) or 5 (upwinded, or r = 5).
#include "stage_kernel.hpp"

// Staging depth and work-groups per CU.  The staged neighbourhood of one
// grid function is 62-70 KB, so two buffers and one work-group (one wave per
// SIMD) per CU is all the LDS holds.
#ifndef CHEMORA_STAGING_DEPTH_O8
#define CHEMORA_STAGING_DEPTH_O8 2
#endif
#ifndef CHEMORA_WAVES_O8
#define CHEMORA_WAVES_O8 1
#endif

namespace chemora {

namespace {
template <bool UPWIND, int R>
void launch(const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s) {
  hipLaunchKernelGGL((stage_kernel<8, UPWIND, R, CHEMORA_STAGING_DEPTH_O8, CHEMORA_WAVES_O8>), dim3(grid), dim3(TILE_X, TILE_Y, 1), 0, s, a, bt);
}
}  // namespace

void launch_stage_o8(bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s) {
  if (upwind)
    launch<true, 5>(a, bt, grid, s);
  else if (ko_r > 4)
    launch<false, 5>(a, bt, grid, s);
  else
    launch<false, 4>(a, bt, grid, s);
}

}  // namespace chemora
