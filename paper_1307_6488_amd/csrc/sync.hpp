// sync.hpp -- ghost exchange between the patches of a plan, 2:1 prolongation
// into refined patches' ghosts and restriction to coarser patches (the
// framework services around the evolution kernel: section "Cactus-Carpet
// Computational Infrastructure" -- ghost-zone synchronisation, refinement,
// multi-block -- named as the next step in section "Conclusion").
//
// Patches sit on vertex-centred refinement levels, h_L = h_0 / 2^L (h_0 the
// coarsest spacing); every origin lies on its level's lattice through the
// first coarsest patch's origin, so each stored point has a global integer
// index per level and a level-L point with an even index along an axis
// coincides with a level-(L-1) point.  A ghost point of a level-L patch
// takes, in this order of preference,
//   - the value of the lowest-numbered other level-L patch whose interior
//     holds the point (a copy), else
//   - on a refined level, the order-p tensor Lagrange interpolation (p = the
//     finite-difference order; per axis the coincident coarse point or the p
//     coarse points around a midpoint) from the lowest-numbered level-(L-1)
//     patch whose stored box (interior and ghosts) holds every tap, else
//   - (coarsest level only) nothing: an outer-boundary point keeping the
//     patch's own boundary treatment.
// Levels are refilled coarsest first, so interpolation reads coarse ghosts
// that are complete.  Restriction: a coarse interior point that coincides
// with a finer level's interior point takes its value (lowest-numbered fine
// patch), finest level first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "chemora.h"

namespace chemora {

// One refilled point: all 24 grid functions of patch dst at element offset
// dst_off (GF 0) from patch src at src_off -- the point itself (mid == 0) or
// the lowest-corner tap of the interpolation stencil, with bit a of mid set
// where the point is a midpoint along axis a.
struct SyncItem {
  int dst, src;
  int mid, pad;
  int64_t dst_off, src_off;
};

// Per-patch geometry the sync kernels need (element strides).
struct SyncGeo {
  int64_t sy, sz, sf;
};

struct SyncMaps {
  int nlevels = 0;
  std::vector<SyncItem> fill;        // ghost refills, level by level
  std::vector<int> fill_start;       // nlevels + 1 offsets into fill
  std::vector<int> fill_copies;      // per level: its first fill_copies[L] items are copies (mid == 0)
  std::vector<SyncItem> restr;       // restriction, finest level pair first
  std::vector<int> restr_start;      // pair L -> L-1 for L = max .. 1: nlevels offsets into restr (the last = end)
  std::vector<int> level;            // per patch
};

// Builds the maps of patches[0 .. np); returns CHEMORA_OK, or CHEMORA_EINVAL
// with a message in *err (spacings not a power-of-two hierarchy, an origin
// off its lattice, a refined patch's ghost point that no source covers).
// Host only, no HIP call.
int build_sync_maps(const chemora_params* P, const chemora_patch* patches, int np, SyncMaps* out, std::string* err);

// Launches the refill of one level's items (or one restriction pair's), the
// first ncopy of which are copies: bufs[p] is patch p's state of the stage
// being refilled.
void launch_sync(int order, const SyncItem* items, int n, int ncopy, double* const* bufs, const SyncGeo* geo,
                 hipStream_t s);

}  // namespace chemora
