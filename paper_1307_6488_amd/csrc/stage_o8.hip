// stage_o8.hip -- order-8 instances of the stage kernel and their launcher.
// The staged axis reach R is 4 (centred, Kreiss-Oliger r <= 4) or 5 (upwinded, or r = 5).
// Built once per part: persistent batched form (CHEMORA_PART_PERSIST) or not.
#include "stage_kernel.hpp"

#ifndef CHEMORA_PART_PERSIST
#define CHEMORA_PART_PERSIST 0
#endif

// Staging depth and waves per SIMD.  The staged neighbourhood of one grid
// function is 54-70 KB, so the LDS holds either two buffers of one
// work-group (one wave per SIMD: a wave's LDS, staging and barrier waits go
// uncovered) or one buffer of each of two work-groups (two waves per SIMD,
// each work-group waiting for its staging while the other computes; the
// axis taps are then read axis by axis to fit 256 registers).
#ifndef CHEMORA_STAGING_DEPTH_O8
#define CHEMORA_STAGING_DEPTH_O8 1
#endif
#ifndef CHEMORA_WAVES_O8
#define CHEMORA_WAVES_O8 2
#endif

namespace chemora {

namespace {
// wgs != nullptr: no launch, *wgs receives the kernel's resident
// work-groups per CU instead
template <int TX, int WPG, bool UPWIND, int R, bool KOQ = false>
void launch(const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s, int* wgs) {
  const auto k = stage_kernel<8, UPWIND, R, CHEMORA_STAGING_DEPTH_O8, CHEMORA_WAVES_O8, TX, WPG, double, 1, KOQ,
                              CHEMORA_PART_PERSIST != 0>;
  if (wgs) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs, k, 64 * WPG, 0) != hipSuccess) *wgs = 0;
    return;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(64, WPG, 1), 0, s, a, bt);
}

// the upwinded kernels reuse the tenth difference of the lopsided stencils as
// the Kreiss-Oliger sum when the dissipation radius is 5 (or 0)
template <int TX, int WPG>
void by_reach(bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s,
              int* wgs) {
  if (upwind && (ko_r == Stencil<8>::UR || ko_r == 0))
    launch<TX, WPG, true, 5, true>(a, bt, grid, s, wgs);
  else if (upwind)
    launch<TX, WPG, true, 5>(a, bt, grid, s, wgs);
  else if (ko_r > 4)
    launch<TX, WPG, false, 5>(a, bt, grid, s, wgs);
  else
    launch<TX, WPG, false, 4>(a, bt, grid, s, wgs);
}
}  // namespace

// the 8-wave shapes are not built for order 8 (variant_supported)
template <>
void launch_stage_o8_part<CHEMORA_PART_PERSIST != 0>(int variant, bool upwind, int ko_r, const StageArgs& a,
                                                     const BatchTable& bt, int grid, hipStream_t s, int* wgs) {
  if (variant == 2)
    by_reach<32, 4>(upwind, ko_r, a, bt, grid, s, wgs);
  else
    by_reach<64, 4>(upwind, ko_r, a, bt, grid, s, wgs);
}

}  // namespace chemora
