// stage_o4.hip -- order-4 instances of the stage kernel and their launcher.
// The staged axis reach R is 2 (centred, Kreiss-Oliger r <= 2) or 3 (upwinded, or r = 3).
#include "stage_kernel.hpp"

// Staging depth and work-groups per CU.  The staged neighbourhood of one
// grid function is 22-28 KB: two buffers per work-group let two work-groups
// share a CU (one wave per SIMD each, 256 registers per lane), which hides
// more latency than a deeper pipeline at one wave per SIMD (4.0 vs 4.3 ms
// per 128^3 RK4 step).
#ifndef CHEMORA_STAGING_DEPTH_O4
#define CHEMORA_STAGING_DEPTH_O4 2
#endif
#ifndef CHEMORA_WAVES_O4
#define CHEMORA_WAVES_O4 2
#endif

namespace chemora {

namespace {
template <int TX, int WPG, bool UPWIND, int R>
void launch(const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s) {
  hipLaunchKernelGGL((stage_kernel<4, UPWIND, R, CHEMORA_STAGING_DEPTH_O4, CHEMORA_WAVES_O4, TX, WPG>), dim3(grid),
                     dim3(64, WPG, 1), 0, s, a, bt);
}

template <int TX, int WPG>
void by_reach(bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s) {
  if (upwind)
    launch<TX, WPG, true, 3>(a, bt, grid, s);
  else if (ko_r > 2)
    launch<TX, WPG, false, 3>(a, bt, grid, s);
  else
    launch<TX, WPG, false, 2>(a, bt, grid, s);
}
}  // namespace

void launch_stage_o4(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid,
                     hipStream_t s) {
  switch (variant) {
    case 1: by_reach<64, 8>(upwind, ko_r, a, bt, grid, s); break;
    case 2: by_reach<32, 4>(upwind, ko_r, a, bt, grid, s); break;
    case 3: by_reach<32, 8>(upwind, ko_r, a, bt, grid, s); break;
    default: by_reach<64, 4>(upwind, ko_r, a, bt, grid, s); break;
  }
}

}  // namespace chemora
