// stage_o4.hip -- order-4 instances of the stage kernel and their launcher.
// The staged axis reach R is 2 (centred, Kreiss-Oliger r <= 2) or 3 (upwinded, or r = 3).
// Built once per part -- precision (CHEMORA_PART_SPLIT) and persistent batched
// form or not (CHEMORA_PART_PERSIST) -- so that the parts compile in parallel.
#include "stage_kernel.hpp"

#ifndef CHEMORA_PART_SPLIT
#define CHEMORA_PART_SPLIT 0
#endif
#ifndef CHEMORA_PART_PERSIST
#define CHEMORA_PART_PERSIST 0
#endif

// Waves per SIMD and staging depth.  FP64 runs two waves per SIMD (256
// registers per lane): more latency hiding than a deeper pipeline at one
// wave per SIMD (4.0 vs 4.3 ms per 128^3 RK4 step).  The staged
// neighbourhood of one grid function is 20-44 KB depending on the tile, and
// each variant takes the deepest pipeline (up to CHEMORA_MAX_DEPTH_O4
// buffers) whose work-groups still fit the LDS at that occupancy.
#ifndef CHEMORA_WAVES_O4
#define CHEMORA_WAVES_O4 2
#endif
#ifndef CHEMORA_MAX_DEPTH_O4
#define CHEMORA_MAX_DEPTH_O4 3
#endif

namespace chemora {

namespace {
// LDS of one work-group: nb staging buffers, plus the parked staging
// offsets where the kernel keeps them in LDS (FP64 at two waves per SIMD)
template <int TX, int WPG, int R, typename T, int TZ>
constexpr int lds_bytes(int nb, int occ) {
  using L = LdsLayout<R, 2, Shape<TX, WPG, TZ>>;
  return nb * L::SIZEP * 8 + ((occ == 2 && sizeof(T) == 8) ? L::CPW * 64 * WPG * 4 : 0);
}
template <int WPG>
constexpr int wgs_per_cu(int occ) {
  return occ * 4 / WPG > 1 ? occ * 4 / WPG : 1;
}

// Waves per SIMD: FP64 uses CHEMORA_WAVES_O4; split precision (about 160
// registers) takes a third wave wherever three work-groups fit the LDS with
// two buffers each.
#ifndef CHEMORA_SPLIT_MAX_WAVES
#define CHEMORA_SPLIT_MAX_WAVES 3
#endif
template <int TX, int WPG, int R, typename T, int TZ>
constexpr int occupancy() {
  if (!std::is_same<T, float>::value) return CHEMORA_WAVES_O4;
  return CHEMORA_SPLIT_MAX_WAVES >= 3 && wgs_per_cu<WPG>(3) * lds_bytes<TX, WPG, R, T, TZ>(2, 3) <= 160 * 1024 ? 3
                                                                                                           : 2;
}

template <int TX, int WPG, int R, typename T, int TZ>
constexpr int depth() {
  constexpr int occ = occupancy<TX, WPG, R, T, TZ>();
  int nb = 2;
  while (nb < CHEMORA_MAX_DEPTH_O4 &&
         wgs_per_cu<WPG>(occ) * lds_bytes<TX, WPG, R, T, TZ>(nb + 1, occ) <= 160 * 1024)
    ++nb;
  return nb;
}

// wgs != nullptr: no launch, *wgs receives the kernel's resident
// work-groups per CU instead
template <int TX, int WPG, int TZ, bool UPWIND, int R, typename T, bool KOQ = false>
void launch(const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s, int* wgs) {
  const auto k = stage_kernel<4, UPWIND, R, depth<TX, WPG, R, T, TZ>(), occupancy<TX, WPG, R, T, TZ>(), TX, WPG, T,
                              TZ, KOQ, CHEMORA_PART_PERSIST != 0>;
  if (wgs) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs, k, 64 * WPG, 0) != hipSuccess) *wgs = 0;
    return;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(64, WPG, 1), 0, s, a, bt);
}

// Upwinded FP64 kernels reuse the sixth difference of the lopsided stencils
// as the Kreiss-Oliger sum when the dissipation radius is 3 (or 0: zero scale)
template <int TX, int WPG, typename T, int TZ = 1>
void by_reach(bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid, hipStream_t s,
              int* wgs) {
  constexpr bool FP64 = !std::is_same<T, float>::value;
  if (upwind && FP64 && (ko_r == Stencil<4>::UR || ko_r == 0))
    launch<TX, WPG, TZ, true, 3, T, FP64>(a, bt, grid, s, wgs);
  else if (upwind)
    launch<TX, WPG, TZ, true, 3, T>(a, bt, grid, s, wgs);
  else if (ko_r > 2)
    launch<TX, WPG, TZ, false, 3, T>(a, bt, grid, s, wgs);
  else
    launch<TX, WPG, TZ, false, 2, T>(a, bt, grid, s, wgs);
}

template <typename T>
void by_variant(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid,
                hipStream_t s, int* wgs) {
  switch (variant) {
    case 1: by_reach<64, 8, T>(upwind, ko_r, a, bt, grid, s, wgs); break;
    case 2: by_reach<32, 4, T>(upwind, ko_r, a, bt, grid, s, wgs); break;
    case 3: by_reach<32, 8, T>(upwind, ko_r, a, bt, grid, s, wgs); break;
    case 4: by_reach<32, 8, T, 2>(upwind, ko_r, a, bt, grid, s, wgs); break;
    case 5: by_reach<32, 8, T, 4>(upwind, ko_r, a, bt, grid, s, wgs); break;
    default: by_reach<64, 4, T>(upwind, ko_r, a, bt, grid, s, wgs); break;
  }
}
}  // namespace

template <>
void launch_stage_o4_part<CHEMORA_PART_SPLIT != 0, CHEMORA_PART_PERSIST != 0>(int variant, bool upwind, int ko_r,
                                                                              const StageArgs& a,
                                                                              const BatchTable& bt, int grid,
                                                                              hipStream_t s, int* wgs) {
  by_variant<std::conditional_t<CHEMORA_PART_SPLIT != 0, float, double>>(variant, upwind, ko_r, a, bt, grid, s, wgs);
}

}  // namespace chemora
