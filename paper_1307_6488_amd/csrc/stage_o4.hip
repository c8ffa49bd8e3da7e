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
// Waves per SIMD: FP64 uses CHEMORA_WAVES_O4; split precision (about 156
// registers) takes a third wave wherever three work-groups' staging
// buffers fit the LDS.
template <int TX, int WPG, int R, typename T>
constexpr int occupancy() {
  if (!std::is_same<T, float>::value) return CHEMORA_WAVES_O4;
  using L = LdsLayout<R, 2, Shape<TX, WPG>>;
  constexpr int bytes = CHEMORA_STAGING_DEPTH_O4 * L::SIZEP * 8;
  constexpr int wgs = 12 / WPG > 1 ? 12 / WPG : 1;
  return wgs * bytes <= 160 * 1024 ? 3 : 2;
}

template <int TX, int WPG, bool UPWIND, int R, typename T>
void launch(const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s) {
  hipLaunchKernelGGL(
      (stage_kernel<4, UPWIND, R, CHEMORA_STAGING_DEPTH_O4, occupancy<TX, WPG, R, T>(), TX, WPG, T>),
      dim3(grid), dim3(64, WPG, 1), 0, s, a, bt);
}

template <int TX, int WPG, typename T>
void by_reach(bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s) {
  if (upwind)
    launch<TX, WPG, true, 3, T>(a, bt, grid, s);
  else if (ko_r > 2)
    launch<TX, WPG, false, 3, T>(a, bt, grid, s);
  else
    launch<TX, WPG, false, 2, T>(a, bt, grid, s);
}

template <typename T>
void by_variant(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid,
                hipStream_t s) {
  switch (variant) {
    case 1: by_reach<64, 8, T>(upwind, ko_r, a, bt, grid, s); break;
    case 2: by_reach<32, 4, T>(upwind, ko_r, a, bt, grid, s); break;
    case 3: by_reach<32, 8, T>(upwind, ko_r, a, bt, grid, s); break;
    default: by_reach<64, 4, T>(upwind, ko_r, a, bt, grid, s); break;
  }
}
}  // namespace

void launch_stage_o4(int variant, bool split, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt,
                     int grid, hipStream_t s) {
  if (split)
    by_variant<float>(variant, upwind, ko_r, a, bt, grid, s);
  else
    by_variant<double>(variant, upwind, ko_r, a, bt, grid, s);
}

}  // namespace chemora
