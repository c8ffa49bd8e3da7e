// stage_kernel.hpp -- the fused RK-stage kernel for gfx950: stencils, BSSN
// algebra, upwinded advection, Kreiss-Oliger dissipation and the RK4 stage
// combination in one pass over the grid, instantiated per finite-difference
// order in stage_o4.hip / stage_o8.hip.
//
// Equations (section "Scientific Motivation": the BSSN form of the Einstein
// equations; section "Binary Black Hole Simulations": the McLachlan kernels),
// in the chi form with 1+log / harmonic / frozen slicing and the advective
// Gamma-driver shift (eta damping, 3/4 coupling):
//   d0 chi   = 2/3 chi (alpha K - div beta)
//   d0 gt_ij = -2 alpha At_ij + gt_ik d_j b^k + gt_jk d_i b^k - 2/3 gt_ij div beta
//   d0 K     = -D^2 alpha + alpha (At_ij At^ij + K^2/3)
//   d0 At_ij = chi [-D_i D_j alpha + alpha R_ij]^TF + alpha (K At_ij - 2 At_ik At^k_j)
//              + At_ik d_j b^k + At_jk d_i b^k - 2/3 At_ij div beta
//   d0 Gt^i  = gt^jk d_j d_k b^i + 1/3 gt^ij d_j d_k b^k - Gd^j d_j b^i
//              + 2/3 Gd^i div beta - 2 At^ij d_j alpha
//              + 2 alpha (Gt^i_jk At^jk - 3/(2chi) At^ij d_j chi - 2/3 gt^ij d_j K)
//   d0 alpha = -2 alpha K (1+log) | -alpha^2 K (harmonic) ;  d0 beta^i = 3/4 B^i
//   d0 B^i   = d0 Gt^i - eta B^i
// with d0 = d_t - beta^k d_k, Gd^i = gt^jk Gt^i_jk from the metric, and
//   R_ij  = -1/2 gt^lm d_l d_m gt_ij + gt_k(i d_j) Gt^k + Gd^k Gt_(ij)k
//           + gt^lm (2 Gt^k_l(i Gt_j)km + Gt^k_im Gt_klj)
//           + [D~_i D~_j chi + gt_ij D~^2 chi] / (2 chi)
//           - [d_i chi d_j chi + 3 gt_ij |d chi|^2] / (4 chi^2).
// Each variable's right-hand side is (algebra + advection) + dissipation.
//
// Work decomposition.  A work-group owns a TX x TY tile of one z-plane (TX =
// 32 or 64 columns, one wave per 64 / TX rows), one work-item per point.  The
// paper's kernels spill because every derivative is formed before the
// algebra (section "Fat Kernel Detection"); here the right-hand side is
// evaluated grid function by grid function in dependency order
//     beta(3) gt(6) chi alpha Gt(3) K At(6) B(3)
// and every stencil result is consumed at once: second derivatives are
// contracted straight into the Ricci, D_i D_j alpha and Gt-source
// accumulators, and each variable's right-hand side goes through the RK
// epilogue (loads of u_n / the accumulator, stores) as soon as its inputs are
// complete.
//
// Staging.  Each grid function's stencil neighbourhood is copied into LDS by
// direct global->LDS loads (buffer_load_dwordx4 ... lds: lane l moves two
// doubles to LDS bytes [16 l, 16 l + 16) of the instruction's 1 KiB chunk), no
// registers involved, through NB buffers: the chunks of the next NB - 1 grid
// functions are in flight while the work-items evaluate the current one's
// stencils from LDS with compile-time offsets.  Every lane's global offset
// for each of its wave's chunks is computed once per tile, so issuing a grid
// function costs one instruction per chunk.  One barrier per grid function.
//
// LDS layout per staged grid function (one-plane tiles):
//   plane dz = 0            rows y in [-R,  TY-1+R]   (x and y stencils, xy mixed)
//   planes 1 <= |dz| <= RM  rows y in [-RM, TY-1+RM]  (xz / yz mixed, z stencils)
//   planes RM < |dz| <= R   rows y in [0, TY-1]       (z stencils only)
// with R the axis reach (upwind, Kreiss-Oliger) and RM = ORDER/2 the mixed
// reach; planes are ordered dz = 0, +1, -1, +2, -2, ...; rows span columns
// [-R, TX-1+R] (pitch P = TX + 2R).
#pragma once

#include <cstddef>
#include <type_traits>
#include <utility>

#include "fd_ops.hpp"
#include "stage_common.hpp"

namespace chemora {

// Tile shape: TX (32 or 64) columns, WPG waves per work-group, TZ planes; a
// wave covers 64 / TX rows of TX points of one plane, WPG / TZ waves cover a
// plane, so a tile is TX x TY x TZ with TY = (WPG / TZ) * 64 / TX.
template <int TX_, int WPG_, int TZ_ = 1>
struct Shape {
  static constexpr int TX = TX_, WPG = WPG_, TZ = TZ_;
  static constexpr int RPW = 64 / TX;          // rows per wave
  static constexpr int WPP = WPG / TZ;         // waves per plane
  static constexpr int TY = WPP * RPW;
  static constexpr int NT = 64 * WPG;          // work-items per work-group
  static_assert(TX == 32 || TX == 64, "tile width");
  static_assert(TZ >= 1 && WPG % TZ == 0, "tile depth");
};

template <int R, int RM, class SH, int TZ = SH::TZ>
struct LdsLayout;

// Every layout maps a tap (dx, dy, dz) of a work-item to its anchor plus
// off(dx, dy, dz), a compile-time constant; decode() is the inverse over the
// buffer, and stage_point() the clamped point a staging lane loads.

// One plane per tile: the neighbourhood is cut to what the stencils reach
// (see the file header).  Plane kinds by |dz|: 0 (dz = 0), 1 (|dz| <= RM)
// and 2 (RM < |dz| <= R), with y halos R, RM, 0; every row has pitch
// P = TX + 2R.
template <int R, int RM, class SH>
struct LdsLayout<R, RM, SH, 1> {
  static constexpr int TX = SH::TX, TY = SH::TY;
  static constexpr int P = TX + 2 * R;
  __host__ __device__ static constexpr int kind(int dz) {
    const int a = dz < 0 ? -dz : dz;
    return a == 0 ? 0 : (a <= RM ? 1 : 2);
  }
  __host__ __device__ static constexpr int yh(int k) { return k == 0 ? R : (k == 1 ? RM : 0); }
  __host__ __device__ static constexpr int psize(int k) { return P * (TY + 2 * yh(k)); }
  static constexpr int SIZE = psize(0) + 2 * RM * psize(1) + 2 * (R - RM) * psize(2);
  static constexpr int CHUNK = 128;                          // doubles per LDS-DMA instruction
  static constexpr int NCHUNK = (SIZE + CHUNK - 1) / CHUNK;
  static constexpr int SIZEP = NCHUNK * CHUNK;               // buffer size incl. padding
  static constexpr int CPW = (NCHUNK + SH::WPG - 1) / SH::WPG;  // chunks per wave (at most)
  static constexpr int CMIN = NCHUNK / SH::WPG;                 // chunks per wave (at least)
  static_assert(P % 2 == 0, "a lane's pair of doubles must not straddle rows");

  // anchor of the work-item at tile point (xr, yr) (of the one plane)
  __host__ __device__ static constexpr int anchor(int xr, int yr, int) { return yr * P + xr; }
  // first element of plane dz (planes ordered dz = 0, +1, -1, +2, -2, ...)
  __host__ __device__ static constexpr int plane(int dz) {
    const int a = dz < 0 ? -dz : dz;
    if (a == 0) return 0;
    if (a <= RM) return psize(0) + ((dz > 0 ? 2 * a - 1 : 2 * a) - 1) * psize(1);
    return psize(0) + 2 * RM * psize(1) + ((dz > 0 ? 2 * (a - RM) - 1 : 2 * (a - RM)) - 1) * psize(2);
  }
  // offset (doubles) of tap (dx, dy, dz) from the work-item's anchor
  __host__ __device__ static constexpr int off(int dx, int dy, int dz) {
    return plane(dz) + (dy + yh(kind(dz))) * P + (dx + R);
  }
  // inverse of off(): the tile-relative point (x, y, dz) stored at LDS double
  // idx; the padding past SIZE maps to the anchor (0, 0, 0)
  __host__ __device__ static constexpr void decode(int idx, int& x, int& y, int& dz) {
    if (idx >= SIZE) {
      x = 0; y = 0; dz = 0;
      return;
    }
    int k = 0, q = 0, r = idx;   // plane kind, plane index within the kind, offset in the plane
    if (r < psize(0)) {
      dz = 0;
    } else if ((r -= psize(0)) < 2 * RM * psize(1)) {
      k = 1;
      q = r / psize(1);
      r -= q * psize(1);
      dz = (q & 1) ? -(q / 2 + 1) : q / 2 + 1;
    } else {
      r -= 2 * RM * psize(1);
      k = 2;
      q = r / psize(2);
      r -= q * psize(2);
      dz = (q & 1) ? -(RM + q / 2 + 1) : RM + q / 2 + 1;
    }
    const int row = r / P;
    y = row - yh(k);
    x = r - row * P - R;
  }
  // the point a staging lane loads for LDS double idx of a tile at (i0, j0,
  // k0), clamped into the staged reach of a patch of nx x ny x nz interior
  // points: a row / column / plane of a ragged tile past it re-reads one
  // inside (never used by a valid work-item).  Pairs start on even column
  // offsets from -R; one whose first column is the last one inside is
  // possible for odd nx only, and its second element then lies at most one
  // column past the ghost zone (row padding, which the host guarantees for
  // odd nx).
  __host__ __device__ static constexpr void stage_point(int idx, int i0, int j0, int k0, int nx, int ny, int nz,
                                                        int& x, int& y, int& dz) {
    decode(idx, x, y, dz);
    const int xmax = nx - 1 + R - i0, ymax = ny - 1 + R - j0, zmax = nz - 1 + R - k0;
    y = y < ymax ? y : ymax;
    dz = dz < zmax ? dz : zmax;
    if (x > xmax) x = xmax - 1;
  }
};

// TZ planes per tile: the TZ + 2R planes dz = -R .. TZ-1+R are stored whole
// (rows -R .. TY-1+R, columns -R .. TX-1+R) and in order, so that a tap of a
// work-item on tile plane tz is at a compile-time offset from its anchor
// tz * PLANE + y * P + x whatever tz is -- the z halo is shared by the TZ
// planes instead of staged once per plane.
template <int R, int RM, class SH, int TZ>
struct LdsLayout {
  static constexpr int TX = SH::TX, TY = SH::TY;
  static constexpr int P = TX + 2 * R;
  static constexpr int ROWS = TY + 2 * R;
  static constexpr int PLANE = ROWS * P;
  static constexpr int NPL = TZ + 2 * R;
  static constexpr int SIZE = NPL * PLANE;
  static constexpr int CHUNK = 128;
  static constexpr int NCHUNK = (SIZE + CHUNK - 1) / CHUNK;
  static constexpr int SIZEP = NCHUNK * CHUNK;
  static constexpr int CPW = (NCHUNK + SH::WPG - 1) / SH::WPG;
  static constexpr int CMIN = NCHUNK / SH::WPG;
  static_assert(P % 2 == 0, "a lane's pair of doubles must not straddle rows");
  __host__ __device__ static constexpr int anchor(int xr, int yr, int tz) { return tz * PLANE + yr * P + xr; }
  // offset of tap (dx, dy, dz) from the anchor of a work-item on plane 0
  __host__ __device__ static constexpr int off(int dx, int dy, int dz) {
    return (dz + R) * PLANE + (dy + R) * P + (dx + R);
  }
  // tile-relative point (x, y, dz) stored at LDS double idx (the padding
  // past SIZE maps to (0, 0, 0))
  __host__ __device__ static constexpr void decode(int idx, int& x, int& y, int& dz) {
    if (idx >= SIZE) {
      x = 0; y = 0; dz = 0;
      return;
    }
    const int q = idx / PLANE, r = idx - q * PLANE;
    const int row = r / P;
    dz = q - R;
    y = row - R;
    x = r - row * P - R;
  }
  // as for one plane
  __host__ __device__ static constexpr void stage_point(int idx, int i0, int j0, int k0, int nx, int ny, int nz,
                                                        int& x, int& y, int& dz) {
    decode(idx, x, y, dz);
    const int xmax = nx - 1 + R - i0, ymax = ny - 1 + R - j0, zmax = nz - 1 + R - k0;
    y = y < ymax ? y : ymax;
    dz = dz < zmax ? dz : zmax;
    if (x > xmax) x = xmax - 1;
  }
};

// Cross layout (one-plane tiles): what the axis stencils of a grid function
// without mixed derivatives read.  Plane dz = 0 as in the full layout (rows
// [-R, TY-1+R], pitch P), padded to whole chunks (the padding is staged with
// the full layout's points, never read), then the 2R planes dz = +1, -1, +2,
// -2, ... holding only the tile's own TX x TY points (pitch TX).  x and y
// taps sit at the full layout's offsets from the full anchor; z taps at
// zoff(dz) from the column anchor Z0 + yr TX + xr.
template <int R, int RM, class SH>
struct CrossLayout {
  using F = LdsLayout<R, RM, SH, 1>;
  static constexpr int TX = SH::TX, TY = SH::TY;
  static constexpr int CHUNK = F::CHUNK;
  static constexpr int NCHUNK0 = (F::psize(0) + CHUNK - 1) / CHUNK;   // chunks of plane 0
  static constexpr int Z0 = NCHUNK0 * CHUNK;
  static constexpr int CPP = TX * TY / CHUNK;                          // chunks per column plane
  static constexpr int SIZE = Z0 + 2 * R * TX * TY;
  static constexpr int NCHUNK = SIZE / CHUNK;
  static_assert(TX * TY % CHUNK == 0 && SH::WPG % CPP == 0, "a wave's column chunks share one place in their plane");
  static_assert(SIZE <= F::SIZEP, "the cross layout fits the full layout's buffer");
  __host__ __device__ static constexpr int zplane(int dz) { return dz > 0 ? 2 * (dz - 1) : 2 * (-dz) - 1; }
  __host__ __device__ static constexpr int col_anchor(int xr, int yr) { return Z0 + yr * TX + xr; }
  __host__ __device__ static constexpr int zoff(int dz) { return zplane(dz) * TX * TY; }
  // the tile-relative point stored at LDS double idx
  __host__ __device__ static constexpr void decode(int idx, int& x, int& y, int& dz) {
    if (idx < Z0) {
      F::decode(idx, x, y, dz);
      return;
    }
    const int r = idx - Z0, j = r / (TX * TY), e = r - j * TX * TY;
    dz = (j & 1) ? -(j / 2 + 1) : j / 2 + 1;
    y = e / TX;
    x = e - y * TX;
  }
  // the point a staging lane loads for LDS double idx, clamped as in the
  // full layout
  __host__ __device__ static constexpr void stage_point(int idx, int i0, int j0, int k0, int nx, int ny, int nz,
                                                        int& x, int& y, int& dz) {
    if (idx < Z0) {
      F::stage_point(idx, i0, j0, k0, nx, ny, nz, x, y, dz);
      return;
    }
    decode(idx, x, y, dz);
    const int xmax = nx - 1 + R - i0, ymax = ny - 1 + R - j0, zmax = nz - 1 + R - k0;
    y = y < ymax ? y : ymax;
    dz = dz < zmax ? dz : zmax;
    // column pairs start at even x, so a pair starting at xmax would leave
    // the row; no valid work-item reads a column element past nx - 1 - i0
    if (x >= xmax) x = xmax - 1;
  }
};

// Cross layout at order 4 (any tile depth): what the axis stencils of a
// grid function without mixed derivatives read.  The TZ tile planes whole
// (rows [-R, TY-1+R], pitch P: the x and y taps, at the full layout's
// in-plane offsets), padded to whole chunks, then the TZ + 2R planes dz =
// -R .. TZ-1+R holding only the tile's TX x TY points (pitch TX: the z taps,
// at zoff(dz) from the column anchor of the work-item's plane).  The tile
// planes' own points are staged twice, so that every z tap sits at a
// compile-time offset whatever the wave's plane.
template <int R, class SH>
struct CrossLayoutZ {
  static constexpr int TX = SH::TX, TY = SH::TY, TZ = SH::TZ;
  static constexpr int P = TX + 2 * R, ROWS = TY + 2 * R, PLANE = P * ROWS;
  static constexpr int CHUNK = 128;
  static constexpr int NCHUNK0 = (TZ * PLANE + CHUNK - 1) / CHUNK;   // chunks of the tile planes
  static constexpr int Z0 = NCHUNK0 * CHUNK;
  static constexpr int NPL = TZ + 2 * R;
  static constexpr int CPP = TX * TY / CHUNK;                        // chunks per column plane
  static constexpr int SIZE = Z0 + NPL * TX * TY;
  static constexpr int NCHUNK = SIZE / CHUNK;
  static constexpr int CPW0 = (NCHUNK0 + SH::WPG - 1) / SH::WPG;     // tile-plane chunks per wave (at most)
  static constexpr int CMIN = NCHUNK / SH::WPG;                      // chunks per wave (at least)
  static_assert(TX * TY % CHUNK == 0 && SH::WPG % CPP == 0, "a wave's column chunks share one place in their plane");
  static_assert(P % 2 == 0, "a lane's pair of doubles must not straddle rows");
  __host__ __device__ static constexpr int anchor(int xr, int yr, int tz) { return tz * PLANE + yr * P + xr; }
  __host__ __device__ static constexpr int off(int dx, int dy) { return (dy + R) * P + (dx + R); }
  __host__ __device__ static constexpr int col_anchor(int xr, int yr, int tz) {
    return Z0 + (tz + R) * TX * TY + yr * TX + xr;
  }
  __host__ __device__ static constexpr int zoff(int dz) { return dz * TX * TY; }
  // the tile-relative point stored at LDS double idx (padding: (0, 0, 0))
  __host__ __device__ static constexpr void decode(int idx, int& x, int& y, int& dz) {
    if (idx < Z0) {
      if (idx >= TZ * PLANE) {
        x = 0; y = 0; dz = 0;
        return;
      }
      const int q = idx / PLANE, r = idx - q * PLANE, row = r / P;
      dz = q;
      y = row - R;
      x = r - row * P - R;
      return;
    }
    const int r = idx - Z0, j = r / (TX * TY), e = r - j * TX * TY;
    dz = j - R;
    y = e / TX;
    x = e - y * TX;
  }
  // the point a staging lane loads for LDS double idx, clamped as in the
  // full layouts (tile-plane pairs start at odd columns -R + 2m, column
  // pairs at even ones)
  __host__ __device__ static constexpr void stage_point(int idx, int i0, int j0, int k0, int nx, int ny, int nz,
                                                        int& x, int& y, int& dz) {
    decode(idx, x, y, dz);
    const int xmax = nx - 1 + R - i0, ymax = ny - 1 + R - j0, zmax = nz - 1 + R - k0;
    y = y < ymax ? y : ymax;
    dz = dz < zmax ? dz : zmax;
    if (idx < Z0) {
      if (x > xmax) x = xmax - 1;
    } else {
      if (x >= xmax) x = xmax - 1;
    }
  }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// the double v of lane src mod 64 of the wave (every lane active)
__device__ __forceinline__ double lane_read(double v, int src) {
  const int a = (src & 63) << 2;
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(a, (int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(a, (int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// a staged grid function's advection and dissipation terms; its right-hand
// side is (algebra + advection) + dissipation, or algebra + (advection and
// dissipation summed together) where MERGED
template <typename TC, bool MERGED = false>
struct AdvDiss {
  TC adv, diss;
  __device__ __forceinline__ TC rhs(TC alg) const {
    if constexpr (MERGED)
      return alg + adv;
    else
      return (alg + adv) + diss;
  }
};

// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding: vmcnt bits 3:0 and 15:14,
// expcnt 6:4 left at its maximum, lgkmcnt 11:8)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// Work-group barrier for LDS hand-over.  __syncthreads() adds work-group
// scope release / acquire fences, which on gfx9 wait for every outstanding
// vector-memory operation -- the staging loads of later phases included.
// The LDS data a barrier hands over is already complete (wait_staged waits
// for this wave's staging loads and, lgkmcnt(0), its LDS accesses), so only
// the compiler must be kept from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wait until this wave's staging loads of the next phase have landed in LDS
// while the loads of the m phases issued after it (C chunks each at least)
// may stay in flight.  Vector-memory loads complete in issue order, so at
// most m*C outstanding operations imply the older loads are done; stores and
// extra loads issued in between only make the wait longer.  m is
// wave-uniform; NB - 2 is the most phases in flight behind the next one.
template <int NB, int C>
__device__ __forceinline__ void wait_staged(int m) {
  if (NB >= 5 && m >= 3) wait_vm<3 * C>();
  else if (NB >= 4 && m >= 2) wait_vm<2 * C>();
  else if (NB >= 3 && m >= 1) wait_vm<C>();
  else wait_vm<0>();
}

// One tile t of a patch, staged through the NB LDS buffers bufs[]
// (LdsLayout::SIZEP doubles each): grid function p of the sequence goes to
// bufs[p % NB], issued NB - 1 phases before it is used.  Tiles are numbered
// x fastest, then z, then y, so that the work-groups in flight on one XCD
// cover a block that is deep in z and share their z halos in its L2.  Every
// work-item of the work-group must call it (it synchronises); it ends with a
// barrier, so the buffers may be reused right after.
template <int ORDER, bool UPWIND, int R, int NB, bool BOUND, bool OFFS_LDS, bool PARK, class SH, typename T,
          bool KOQ, bool AXIS_GROUPS, bool CROSSZ>
__device__ __forceinline__ void stage_tile(const StageArgs& a, int t, double* const (&bufs)[NB], unsigned* offs,
                                           double* park) {
  // T: the arithmetic type of stencil combinations and algebra -- double, or
  // float for split precision (FP64 differences rounded to FP32, FP32
  // algebra, FP64 state, RK combination and near-puncture chi terms)
  constexpr bool SPLIT = std::is_same<T, float>::value;
  static_assert(!SPLIT || ORDER == 4, "split precision is built for order 4");
  using St = Stencil<ORDER>;
  constexpr int RM = ORDER / 2;
  using L = LdsLayout<R, RM, SH>;
  const Geo G = a.geo;
  const int nzb = (G.nz + SH::TZ - 1) / SH::TZ;   // tile planes
  const int txi = t % a.tiles_x;
  const int kb = (t / a.tiles_x) % nzb;
  const int tyi = t / (a.tiles_x * nzb);
  // threadIdx.y is the wave index: uniform across the wave, so keep it (and
  // everything the staging derives from it) in scalar registers
  const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tz = wave / SH::WPP;                                        // the wave's tile plane
  const int xr = lane % SH::TX, yr = (wave % SH::WPP) * SH::RPW + lane / SH::TX;   // tile-relative point
  const int i0 = txi * SH::TX, j0 = tyi * SH::TY, k0 = kb * SH::TZ;
  const int k = k0 + tz;
  const bool valid = (i0 + xr < G.nx) && (j0 + yr < G.ny) && (k < G.nz);
  // pointwise accesses of work-items outside the interior use a clamped point
  const int ic = min(i0 + xr, G.nx - 1), jc = min(j0 + yr, G.ny - 1), kc = min(k, G.nz - 1);

  // byte offsets are unsigned 32-bit (the host limits a state to 4 GiB)
  const unsigned sy = (unsigned)G.sy, sz = (unsigned)G.sz, sf = (unsigned)G.sf, gg = (unsigned)G.g;
  const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, G.sf);
  const unsigned vpt = (jc * sy + ic + gg) * 8u + XB * 8u;       // the point (pointwise accesses)
  const unsigned spt = ((kc + gg) * sz + gg * sy) * 8u;         // its z plane / ghost offset
  auto val = [&](int f) __attribute__((always_inline)) { return bload(rin, vpt, spt + f * sf * 8u); };

  // ---- staging offsets of this tile.  Lane l of wave w moves LDS doubles
  // [c*128 + 2l, c*128 + 2l + 1] of chunks c = w, w+WPG, ...  Points outside
  // the patch's stored box (rows / columns of a ragged tile past the ghost
  // zone) are clamped into it by the layout's stage_point(): their LDS
  // values are never read by a valid work-item.  A pair whose first column
  // is the last one of the box (odd nx only) reads one element of row
  // padding, which the host guarantees (sy >= nx + 2g + 1 for odd nx), so no
  // access leaves its row.  voff is biased by (R sz + R sy + R) so that it
  // stays non-negative.
  const unsigned bias = (unsigned)R * (sz + sy + 1u);
  unsigned voff[L::CPW];
  // opaque copies: the decode depends only on lane and wave, and hoisted out
  // of a batched kernel's tile loop it would hold 3 registers per chunk for
  // the whole kernel; recomputed per tile it is a few dozen instructions
  int lane_t = lane, wave_t = wave;
  asm volatile("" : "+v"(lane_t));
  asm volatile("" : "+s"(wave_t));
#pragma unroll
  for (int q = 0; q < L::CPW; ++q) {
    int x, y, dz;
    L::stage_point((wave_t + SH::WPG * q) * L::CHUNK + 2 * lane_t, i0, j0, k0, G.nx, G.ny, G.nz, x, y, dz);
    voff[q] = (unsigned)(dz * (int)sz + y * (int)sy + x + (int)bias) * 8u;
    // OFFS_LDS: park the offsets in LDS (each lane reads back only its own
    // slots, so no barrier is involved) and free their registers
    if (OFFS_LDS) offs[q * SH::NT + wave * 64 + lane] = voff[q];
  }
  // CROSSZ (order 4, FP64 with parked offsets): the 13 grid functions
  // without mixed derivatives stage CrossLayoutZ; its tile-plane chunks have
  // offsets of their own, parked after the full layout's
  using LZ = CrossLayoutZ<R, SH>;
  if constexpr (CROSSZ) {
#pragma unroll
    for (int q = 0; q < LZ::CPW0; ++q) {
      int x, y, dz;
      LZ::stage_point((wave_t + SH::WPG * q) * LZ::CHUNK + 2 * lane_t, i0, j0, k0, G.nx, G.ny, G.nz, x, y, dz);
      offs[(L::CPW + q) * SH::NT + wave * 64 + lane] = (unsigned)(dz * (int)sz + y * (int)sy + x + (int)bias) * 8u;
    }
  }
  const unsigned tile_base = ((k0 + gg) * sz + (j0 + gg) * sy + i0 + gg + XB) * 8u - bias * 8u;
  // whether chunk wave + WPG q exists: with q a compile-time constant the
  // wave-uniform test remains only for the last q, so that the loads before
  // it are unconditional and their offsets are read from LDS together
  // rather than with one wait per load
  auto chunk_exists = [&](int q) __attribute__((always_inline)) {
    return SH::WPG * (q + 1) <= L::NCHUNK ? true : wave + SH::WPG * q < L::NCHUNK;
  };
  auto issue = [&](int f, double* dst) __attribute__((always_inline)) {
    const unsigned so = tile_base + f * sf * 8u;
#pragma unroll
    for (int q = 0; q < L::CPW; ++q) {
      const int c = wave + SH::WPG * q;
      if (!chunk_exists(q)) break;   // wave-uniform
      const unsigned vo = OFFS_LDS ? offs[q * SH::NT + wave * 64 + lane] : voff[q];
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr_t)(dst + c * L::CHUNK), 16, vo, so, 0, 0);
    }
  };
  // CROSS (order 8, one buffer): the 13 grid functions without mixed
  // derivatives (phases 11-23: Gt, K, At, B) stage only the cross of
  // CrossLayout, less than half the full neighbourhood.  Its plane-0 chunks
  // are the full layout's; a column chunk holds CHUNK points of one plane
  // z = k + dz, and all of a wave's column chunks sit at the same place in
  // their planes, so one per-lane offset serves them, the plane entering
  // through the scalar offset.
  constexpr bool CROSS = AXIS_GROUPS && NB == 1 && ORDER == 8 && SH::TZ == 1;
  using LC = std::conditional_t<CROSS, CrossLayout<R, RM, SH>, L>;
  using XKIND = std::integral_constant<int, CROSSZ ? 2 : (CROSS ? 1 : 0)>;
  auto issue_cross = [&](int f, double* dst) __attribute__((always_inline)) {
    if constexpr (CROSS) {
      const unsigned so = tile_base + f * sf * 8u;
#pragma unroll
      for (int q = 0; q < L::CPW; ++q) {
        const int c = wave + SH::WPG * q;
        if (c >= LC::NCHUNK0) break;   // wave-uniform
        const unsigned vo = OFFS_LDS ? offs[q * SH::NT + wave * 64 + lane] : voff[q];
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr_t)(dst + c * L::CHUNK), 16, vo, so, 0, 0);
      }
      const int pos = ((wave - LC::NCHUNK0) % LC::CPP + LC::CPP) % LC::CPP;
      const int e = pos * LC::CHUNK + 2 * lane;
      int y = e / SH::TX, x = e - y * SH::TX;
      const int xmax = G.nx - 1 + R - i0, ymax = G.ny - 1 + R - j0, zmax = G.nz - 1 + R - k0;
      y = y < ymax ? y : ymax;
      if (x >= xmax) x = xmax - 1;
      // the plane offset (dz + R) sz >= 0 goes to the scalar part, the rest
      // of the full layout's bias to the lane's part
      const unsigned vo = (unsigned)(y * (int)sy + x + R * ((int)sy + 1)) * 8u;
#pragma unroll
      for (int q = 0; q < (LC::NCHUNK + SH::WPG - 1) / SH::WPG; ++q) {
        const int c = wave + SH::WPG * q;
        if (c < LC::NCHUNK0) continue;
        if (c >= LC::NCHUNK) break;   // wave-uniform
        const int j = (c - LC::NCHUNK0) / LC::CPP;
        int dz = (j & 1) ? -(j / 2 + 1) : j / 2 + 1;
        dz = dz < zmax ? dz : zmax;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr_t)(dst + c * L::CHUNK), 16, vo,
                                                 so + (unsigned)(dz + R) * sz * 8u, 0, 0);
      }
    }
  };

  // CROSSZ staging of grid function f into dst: the tile-plane chunks with
  // their parked offsets, then the column chunks, whose per-lane part is the
  // same in every plane (the plane enters through the scalar offset, as
  // (dz + R) sz >= 0).  Wave-uniform tests remain only where a range of
  // chunks ends inside a round of the waves.
  auto issue_crossz = [&](int f, double* dst) __attribute__((always_inline)) {
    if constexpr (CROSSZ) {
      const unsigned so = tile_base + f * sf * 8u;
      auto in_range = [&](int q, int lo, int hi) __attribute__((always_inline)) {
        const int c = wave + SH::WPG * q;
        const bool above = SH::WPG * q >= lo ? true : (SH::WPG * (q + 1) <= lo ? false : c >= lo);
        const bool below = SH::WPG * (q + 1) <= hi ? true : (SH::WPG * q >= hi ? false : c < hi);
        return above && below;
      };
#pragma unroll
      for (int q = 0; q < LZ::CPW0; ++q) {
        if (!in_range(q, 0, LZ::NCHUNK0)) continue;
        const int c = wave + SH::WPG * q;
        const unsigned vo = offs[(L::CPW + q) * SH::NT + wave * 64 + lane];
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr_t)(dst + c * LZ::CHUNK), 16, vo, so, 0, 0);
      }
      const int pos = ((wave - LZ::NCHUNK0) % LZ::CPP + LZ::CPP) % LZ::CPP;
      const int e = pos * LZ::CHUNK + 2 * lane;
      int y = e / SH::TX, x = e - y * SH::TX;
      const int xmax = G.nx - 1 + R - i0, ymax = G.ny - 1 + R - j0, zmax = G.nz - 1 + R - k0;
      y = y < ymax ? y : ymax;
      if (x >= xmax) x = xmax - 1;
      const unsigned vo = (unsigned)(y * (int)sy + x + R * ((int)sy + 1)) * 8u;
#pragma unroll
      for (int q = 0; q < (LZ::NCHUNK + SH::WPG - 1) / SH::WPG; ++q) {
        if (!in_range(q, LZ::NCHUNK0, LZ::NCHUNK)) continue;
        const int c = wave + SH::WPG * q;
        int dz = (c - LZ::NCHUNK0) / LZ::CPP - R;
        dz = dz < zmax ? dz : zmax;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr_t)(dst + c * LZ::CHUNK), 16, vo,
                                                 so + (unsigned)(dz + R) * sz * 8u, 0, 0);
      }
    }
  };

  // Stencil taps of the current phase's buffer.  Each phase addresses it from
  // an opaque copy of the anchor: LDS reads are merged in pairs (8-bit
  // offsets, +-2 KB), so a buffer needs a base register per 2 KB it spans,
  // and shared across phases those bases would stay live through the whole
  // kernel.  Every stencil group also takes a fresh copy, so a tap used by
  // several groups is read again from LDS instead of being held in a
  // register across the phase.
  struct Taps {
    const double* cur;
    int anc;
    __device__ __forceinline__ double operator()(int dx, int dy, int dz) const {
      return cur[anc + L::off(dx, dy, dz)];
    }
    __device__ __forceinline__ Taps fresh() const {
      Taps t = *this;
      if (BOUND) asm volatile("" : "+v"(t.anc));
      return t;
    }
  };
  // BOUND: each stencil's result is materialised and followed by a
  // scheduling barrier, so its taps die there.  Otherwise the combining
  // arithmetic sinks below later stencils' reads, and with order-8 stencils
  // the 64 taps of a mixed derivative (or more) are live at once and spill.
  // It costs instruction-level parallelism, so order 4 uses it only where
  // two waves share a SIMD (half the registers each).
  auto bound = [&](auto& v) __attribute__((always_inline)) {
    if (BOUND) {
      keep(v);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto make_ops = [&](const double* cur) __attribute__((always_inline)) {
    int anc = L::anchor(xr, yr, tz);
    asm volatile("" : "+v"(anc));
    return Taps{cur, anc};
  };
  // the taps of a CROSSZ buffer: its tile planes hold the x and y taps at
  // the full layout's in-plane offsets, from the work-item's plane
  auto cross_ops = [&](const double* cur) __attribute__((always_inline)) {
    if constexpr (!CROSSZ) {
      return make_ops(cur);
    } else {
      int anc = LZ::anchor(xr, yr, tz) - (L::off(0, 0, 0) - LZ::off(0, 0));
      asm volatile("" : "+v"(anc));
      return Taps{cur, anc};
    }
  };
  // Taps along the three axes through the point serve a phase's first and
  // pure second derivatives, advection and dissipation.  A phase reads all
  // 1 + 6R of them from LDS in one group into registers, so a work-item
  // waits for LDS a few times per phase instead of once per stencil.  At
  // order 4 each mixed derivative also reads its 16 taps in one group; at
  // order 8 (64 taps, more than the registers to spare) a mixed derivative
  // reads the inner stencils at +-oa together, 16 taps per group (measured
  // against 8, 32 and all 64 per group).
  constexpr bool MIXED_GROUP = ORDER == 4;
  // Order 8: the mixed derivatives whose outer direction is x (xy, xz) take
  // their inner stencils from the neighbouring lanes (16 taps and 16 lane
  // reads each instead of 64 taps)
#ifndef CHEMORA_MIXED_SHUFFLE
#define CHEMORA_MIXED_SHUFFLE 1
#endif
  constexpr bool XSHUF = CHEMORA_MIXED_SHUFFLE && ORDER == 8 && SH::TZ == 1 && AXIS_GROUPS;
  struct Axes {
    Taps t;                  // the mixed derivatives read from LDS
    double c;
    double v[3][2 * R];      // offsets -R..-1, 1..R along each axis
    __device__ __forceinline__ double operator()(int ax, int o) const {
      return o == 0 ? c : v[ax][o < 0 ? o + R : o + R - 1];
    }
  };
  // the axis taps of a phase's buffer, read in one group
  auto phase_src = [&](const Taps& t0) __attribute__((always_inline)) {
    const Taps tap = t0.fresh();
    Axes r;
    r.t = t0;
    r.c = tap(0, 0, 0);
#pragma unroll
    for (int o = 1; o <= R; ++o) {
      r.v[0][R - o] = tap(-o, 0, 0);
      r.v[0][R + o - 1] = tap(o, 0, 0);
      r.v[1][R - o] = tap(0, -o, 0);
      r.v[1][R + o - 1] = tap(0, o, 0);
      r.v[2][R - o] = tap(0, 0, -o);
      r.v[2][R + o - 1] = tap(0, 0, o);
    }
    keep(r.c);
    keep(r.v);
    return r;
  };
  // the same from a CROSSZ buffer (z taps from the column planes)
  auto phase_src_cross = [&](const Taps& t0) __attribute__((always_inline)) {
    const Taps tap = t0.fresh();
    int az = LZ::col_anchor(xr, yr, tz);
    asm volatile("" : "+v"(az));
    Axes r;
    r.t = t0;
    r.c = tap(0, 0, 0);
#pragma unroll
    for (int o = 1; o <= R; ++o) {
      r.v[0][R - o] = tap(-o, 0, 0);
      r.v[0][R + o - 1] = tap(o, 0, 0);
      r.v[1][R - o] = tap(0, -o, 0);
      r.v[1][R + o - 1] = tap(0, o, 0);
      r.v[2][R - o] = t0.cur[az + LZ::zoff(-o)];
      r.v[2][R + o - 1] = t0.cur[az + LZ::zoff(o)];
    }
    keep(r.c);
    keep(r.v);
    return r;
  };
  // The stencils below take a precision tag: double() gives the FP64 forms,
  // float() the split forms (FP64 differences rounded to FP32, FP32 weights).
  const double bet_d[3] = {val(gBETA), val(gBETA + 1), val(gBETA + 2)};
  // FP64 upwinding as UA beta A + UQ |beta| Q per axis (fd_ops.hpp), with
  // velocity factors (UA / (DU h)) beta and (UQ / (DU h)) |beta| formed in
  // each phase (two multiplies per axis; held through the kernel they would
  // take six registers more than beta)
  const double cA = St::UA * a.sc.up, cQ = St::UQ * a.sc.up;
  // The stencils along the three axes read the phase's register-held axis
  // taps.  FENCE_AXES 0: the first and pure second derivatives of the three
  // axes (and, below, the advection and dissipation of the three axes) form
  // one scheduling region each, so that their independent dependency chains
  // interleave -- a dependent FP64 operation waits several issue slots for
  // its operand -- and one fence follows the group.  1: a fence after every
  // stencil.
#ifndef CHEMORA_FENCE_AXES
#define CHEMORA_FENCE_AXES 0
#endif
  constexpr bool FENCE_AXES = CHEMORA_FENCE_AXES != 0;
  auto abound = [&](auto& v) __attribute__((always_inline)) {
    if (FENCE_AXES) bound(v);
  };
  auto gbound = [&](auto& v) __attribute__((always_inline)) {
    if (!FENCE_AXES) bound(v);
  };
  auto D1 = [&](auto tag, const auto& src, int ax) __attribute__((always_inline)) {
    using TC = decltype(tag);
    auto along = [&](int o) __attribute__((always_inline)) { return src(ax, o); };
    TC v;
    if constexpr (std::is_same<TC, float>::value)
      v = St::first_f(along) * float(a.sc.d1);
    else
      v = St::first(along) * a.sc.d1;
    abound(v);
    return v;
  };
  // pure second derivative along ax
  auto D2d = [&](auto tag, const auto& src, int ax) __attribute__((always_inline)) {
    using TC = decltype(tag);
    auto along = [&](int o) __attribute__((always_inline)) { return src(ax, o); };
    TC v;
    if constexpr (std::is_same<TC, float>::value)
      v = St::second_f(along) * float(a.sc.d2);
    else
      v = St::second(along) * a.sc.d2;
    abound(v);
    return v;
  };
  // the first (and pure second) derivatives along the three axes
  auto D1all = [&](auto tag, const auto& src, auto (&d)[3]) __attribute__((always_inline)) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) d[ax] = D1(tag, src, ax);
    gbound(d);
  };
  auto D12all = [&](auto tag, const auto& src, auto (&d)[3], auto (&d2)[3]) __attribute__((always_inline)) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) d[ax] = D1(tag, src, ax);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) d2[ax] = D2d(tag, src, ax);
    gbound(d);
    gbound(d2);
  };
  // mixed second derivative of slot (ai != bj): outer D1 along ai of inner
  // D1's along bj (the inner ones FP64 in both precisions)
  auto D2m = [&](auto tag, const auto& src, int slot) __attribute__((always_inline)) {
    using TC = decltype(tag);
    constexpr bool F32 = std::is_same<TC, float>::value;
    constexpr int M = St::R;
    const Taps tap = src.t.fresh();
    const int ai = SI(slot), bj = SJ(slot);
    auto at2 = [&](int oa, int ob) __attribute__((always_inline)) {
      int d[3] = {0, 0, 0};
      d[ai] = oa;
      d[bj] = ob;
      return tap(d[0], d[1], d[2]);
    };
    auto idx = [](int o) { return o < 0 ? o + M : o + M - 1; };
    TC v;
    if (XSHUF && ai == 0) {
      // outer direction x: the inner stencil at column x + oa is the one the
      // work-item oa columns away evaluates at its own column -- the same
      // taps and arithmetic, so the same bits -- read across lanes.  The
      // lane rotation (lane + oa) mod 64 carries rows past the tile's x
      // edges to the first / last M lanes of a row, which hold the halo
      // columns' inner stencils (hal) for the row that reads them there:
      // with two rows per wave the other row, with one row its own.
      auto inner = [&](const Taps& tt) __attribute__((always_inline)) {
        return St::first([&](int ob) __attribute__((always_inline)) {
          int d[3] = {0, 0, 0};
          d[bj] = ob;
          return tt(d[0], d[1], d[2]);
        });
      };
      // the first M lanes of a row hold columns TX.., the last M columns -M..
      const bool first = xr < M, last = xr >= SH::TX - M;
      Taps th = tap.fresh();
      th.anc += (first ? SH::TX : (last ? -SH::TX : 0)) +
                (SH::RPW == 2 && (first || last) ? (lane < 32 ? L::P : -L::P) : 0);
      // the lane's own inner stencil is the unscaled first derivative
      // along bj that the phase's axis stencils kept (src.fu)
      double own = src.fu[bj];
      double hal = inner(th);
      bound(own);
      bound(hal);
      // each lane offers hal where the lanes oa away read a halo column
      // through it, else own
      auto outer = [&](int oa) __attribute__((always_inline)) {
        const bool offer_hal = oa > 0 ? xr < oa : xr >= SH::TX + oa;
        return lane_read(offer_hal ? hal : own, lane + oa);
      };
      if constexpr (F32)
        v = St::first_f(outer) * float(a.sc.d11);
      else
        v = St::first(outer) * a.sc.d11;
    } else if constexpr (MIXED_GROUP) {
      // the 4M^2 taps in one group
      double m[2 * M][2 * M];
#pragma unroll
      for (int oa = -M; oa <= M; ++oa)
#pragma unroll
        for (int ob = -M; ob <= M; ++ob)
          if (oa != 0 && ob != 0) m[idx(oa)][idx(ob)] = at2(oa, ob);
      keep(m);
      auto outer = [&](int oa) __attribute__((always_inline)) {
        return St::first([&](int ob) { return m[idx(oa)][idx(ob)]; });
      };
      if constexpr (F32)
        v = St::first_f(outer) * float(a.sc.d11);
      else
        v = St::first(outer) * a.sc.d11;
    } else {
      // the inner derivatives at +oa and -oa (4M taps) in one group; the
      // barrier after each pair bounds the live taps to two inner stencils
      double inner[2 * M];
#pragma unroll
      for (int k = 1; k <= M; ++k) {
        const Taps ti = tap.fresh();
        auto in_at = [&](int oa) __attribute__((always_inline)) {
          return St::first([&](int ob) {
            int d[3] = {0, 0, 0};
            d[ai] = oa;
            d[bj] = ob;
            return ti(d[0], d[1], d[2]);
          });
        };
        double ip = in_at(k);
        // with axis-by-axis taps (two waves per SIMD at order 8) one inner
        // stencil per group
        if constexpr (AXIS_GROUPS) bound(ip);
        double im = in_at(-k);
        if constexpr (!AXIS_GROUPS) bound(ip);
        bound(im);
        inner[idx(k)] = ip;
        inner[idx(-k)] = im;
      }
      auto outer = [&](int oa) __attribute__((always_inline)) { return inner[idx(oa)]; };
      if constexpr (F32)
        v = St::first_f(outer) * float(a.sc.d11);
      else
        v = St::first(outer) * a.sc.d11;
    }
    bound(v);
    return v;
  };
  // Order 4: the three mixed derivatives of a phase (slots xy, xz, yz) with
  // their tap reads pipelined -- the taps of the next one are read from LDS
  // before the current one is combined, so that their latency overlaps that
  // arithmetic.  Each value is computed exactly as D2m computes it.
  struct Mix16 {
    double m[4][4];
  };
  auto mixed_taps = [&](const auto& src, int slot) __attribute__((always_inline)) {
    constexpr int M = 2;
    const Taps tap = src.t.fresh();
    const int ai = SI(slot), bj = SJ(slot);
    Mix16 r;
#pragma unroll
    for (int oa = -M; oa <= M; ++oa)
#pragma unroll
      for (int ob = -M; ob <= M; ++ob)
        if (oa != 0 && ob != 0) {
          int d[3] = {0, 0, 0};
          d[ai] = oa;
          d[bj] = ob;
          r.m[oa < 0 ? oa + M : oa + M - 1][ob < 0 ? ob + M : ob + M - 1] = tap(d[0], d[1], d[2]);
        }
    return r;
  };
  auto mixed_from = [&](auto tag, Mix16& r) __attribute__((always_inline)) {
    using TC = decltype(tag);
    keep(r.m);
    auto outer = [&](int oa) __attribute__((always_inline)) {
      const int i = oa < 0 ? oa + 2 : oa + 1;
      return St::first([&](int ob) { return r.m[i][ob < 0 ? ob + 2 : ob + 1]; });
    };
    TC v;
    if constexpr (std::is_same<TC, float>::value)
      v = St::first_f(outer) * float(a.sc.d11);
    else
      v = St::first(outer) * a.sc.d11;
    bound(v);
    return v;
  };
  // mx[1], mx[2], mx[4] (the off-diagonal slots) of the staged GF
  auto mixed3 = [&](auto tag, const auto& src, auto (&mx)[6]) __attribute__((always_inline)) {
    static_assert(ORDER == 4, "pipelined mixed derivatives are built for order 4");
    Mix16 A = mixed_taps(src, 1);
    Mix16 B = mixed_taps(src, 2);
    __builtin_amdgcn_sched_barrier(0);
    mx[1] = mixed_from(tag, A);
    Mix16 C = mixed_taps(src, 4);
    __builtin_amdgcn_sched_barrier(0);
    mx[2] = mixed_from(tag, B);
    mx[4] = mixed_from(tag, C);
  };
#ifndef CHEMORA_PIPE_MIXED
#define CHEMORA_PIPE_MIXED 1
#endif
  constexpr bool PIPE = MIXED_GROUP && CHEMORA_PIPE_MIXED && !AXIS_GROUPS;

  // Advection and dissipation of the staged GF, one axis at a time: its
  // right-hand side is (algebra + advection) + dissipation.  ad_step adds
  // axis ax (ax = 0, 1, 2 in turn) to the running sums st[0] (advection)
  // and st[1] (dissipation).
  auto ad_step = [&](auto tag, auto&& along, int ax, auto (&st)[2]) __attribute__((always_inline)) {
    using TC = decltype(tag);
    constexpr bool F32 = std::is_same<TC, float>::value;
    if constexpr (UPWIND && !F32 && KOQ) {
      // the dissipation is Q times its scale (its radius is Q's, or 0), so
      // per axis beta * lopsided + dissipation = cA beta A + (cQ |beta| + ko) Q:
      // one sum of both terms (st[0]), Q summed exactly as Kreiss-Oliger sums
      const double Qs = ko_sum<St::UR>(along, St::USYM);
      const double As = St::upwind_anti(along);
      const double kq = __builtin_fma(cQ, __builtin_fabs(bet_d[ax]), a.sc.ko);
      st[0] = __builtin_fma(cA * bet_d[ax], As, ax == 0 ? kq * Qs : __builtin_fma(kq, Qs, st[0]));
      abound(st[0]);
    } else {
      const TC b = TC(bet_d[ax]);
      TC qd;
      if constexpr (UPWIND && !F32) {
        // the antisymmetric part and the symmetric difference Q of the
        // lopsided stencils, Q summed exactly as Kreiss-Oliger sums
        const double Qs = ko_sum<St::UR>(along, St::USYM);
        const double As = St::upwind_anti(along);
        st[0] = __builtin_fma(cA * bet_d[ax], As, __builtin_fma(cQ * __builtin_fabs(bet_d[ax]), Qs, st[0]));
        qd = ko_axis<R>(along, a.sc.kow, a.sc.ko);
      } else {
        TC d;
        if constexpr (UPWIND) {
          // both lopsided stencils from the same taps, then select by the sign of beta
          const float dp = St::lopsided_f(along, 1);
          const float dm = -St::lopsided_f([&](int o) { return along(-o); }, 1);
          d = (bet_d[ax] >= 0.0 ? dp : dm) * float(a.sc.up);
        } else {
          if constexpr (F32)
            d = St::first_f(along) * float(a.sc.d1);
          else
            d = St::first(along) * a.sc.d1;
        }
        st[0] += b * d;
        // radius 0 has zero weights and scale: the term is an exact zero
        if constexpr (F32)
          qd = ko_axis_f<R>(along, a.sc.kow, float(a.sc.ko));
        else
          qd = ko_axis<R>(along, a.sc.kow, a.sc.ko);
      }
      st[1] = (ax == 0) ? qd : st[1] + qd;
      bound(st[0]);
      bound(st[1]);
    }
  };
  auto ad_result = [&](auto tag, auto (&st)[2]) __attribute__((always_inline)) {
    using TC = decltype(tag);
    if constexpr (UPWIND && !std::is_same<TC, float>::value && KOQ) {
      gbound(st[0]);
      return AdvDiss<TC, true>{st[0], TC(0.0)};
    } else {
      return AdvDiss<TC>{st[0], st[1]};
    }
  };
  auto advdiss = [&](auto tag, const auto& src) __attribute__((always_inline)) {
    using TC = decltype(tag);
    TC st[2] = {TC(0.0), TC(0.0)};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) ad_step(tag, [&](int o) __attribute__((always_inline)) { return src(ax, o); }, ax, st);
    return ad_result(tag, st);
  };
  // A phase's stencils along the axes through the point: the first
  // derivatives into d1 and the pure second derivatives into d2 (either may
  // be nullptr: not wanted), and the advection and dissipation terms.
  // AXIS_GROUPS 0: the 1 + 6R axis taps are read in one group (phase_src);
  // 1: axis by axis, each axis' 1 + 2R taps read in one group and all of that
  // axis' stencils formed from them before the next axis is read (fewer
  // live registers, the same arithmetic in the same order).  The result's
  // t is the phase's LDS view for the mixed derivatives.
  // cross: the buffer holds the CrossLayout (CROSS phases): z taps at the
  // column anchor
  auto stencils = [&](auto tag, const Taps& t0, auto d1, auto d2, auto cross) __attribute__((always_inline)) {
    // cross: 0 the full layout, 1 CrossLayout (order 8), 2 CrossLayoutZ (order 4)
    constexpr int XK = int(decltype(cross)::value);
    constexpr bool XC = XK == 1, XZ = XK == 2;
    // dependent on the call, so that only cross calls name CrossLayout's members
    using LX = std::conditional_t<XC, LC, CrossLayout<R, RM, Shape<32, 4, 1>>>;
    using TC = decltype(tag);
    constexpr bool W1 = !std::is_same<decltype(d1), std::nullptr_t>::value;
    constexpr bool W2 = !std::is_same<decltype(d2), std::nullptr_t>::value;
    struct Out {
      struct {
        Taps t;
        double fu[3];   // XSHUF: the unscaled first derivatives (with d1)
      } src;
      decltype(advdiss(tag, std::declval<Axes>())) ad;
    } out;
    out.src.t = t0;
    if constexpr (!AXIS_GROUPS) {
      static_assert(!XC, "the cross layout is read axis by axis");
      const auto src = [&]() __attribute__((always_inline)) {
        if constexpr (XZ)
          return phase_src_cross(t0);
        else
          return phase_src(t0);
      }();
      if constexpr (W1 && W2)
        D12all(tag, src, *d1, *d2);
      else if constexpr (W1)
        D1all(tag, src, *d1);
      out.ad = advdiss(tag, src);
    } else {
      static_assert(!XZ, "CrossLayoutZ is read in one group");
      TC st[2] = {TC(0.0), TC(0.0)};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const Taps tap = t0.fresh();
        double c = tap(0, 0, 0), v[2 * R];
        if constexpr (XC) {
          if (ax == 2) {
            int az = LX::col_anchor(xr, yr);
            asm volatile("" : "+v"(az));
#pragma unroll
            for (int o = 1; o <= R; ++o) {
              v[R - o] = t0.cur[az + LX::zoff(-o)];
              v[R + o - 1] = t0.cur[az + LX::zoff(o)];
            }
          }
        }
        if (!XC || ax != 2) {
#pragma unroll
          for (int o = 1; o <= R; ++o) {
            int d[3] = {0, 0, 0};
            d[ax] = -o;
            v[R - o] = tap(d[0], d[1], d[2]);
            d[ax] = o;
            v[R + o - 1] = tap(d[0], d[1], d[2]);
          }
        }
        keep(c);
        keep(v);
        auto along = [&](int o) __attribute__((always_inline)) { return o == 0 ? c : v[o < 0 ? o + R : o + R - 1]; };
        struct One {
          decltype(along)& f;
          __device__ __forceinline__ double operator()(int, int o) const { return f(o); }
        } one{along};
        if constexpr (W1 && XSHUF) {
          // D1 as D1() forms it, its unscaled stencil kept for the mixed
          // derivatives with outer direction x
          out.src.fu[ax] = St::first(along);
          (*d1)[ax] = out.src.fu[ax] * a.sc.d1;
          abound((*d1)[ax]);
        } else if constexpr (W1) {
          (*d1)[ax] = D1(tag, one, ax);
        }
        if constexpr (W2) (*d2)[ax] = D2d(tag, one, ax);
        ad_step(tag, along, ax, st);
        if constexpr (W1) bound((*d1)[ax]);
        if constexpr (W2) bound((*d2)[ax]);
      }
      out.ad = ad_result(tag, st);
    }
    return out;
  };
  // RK epilogue.  Its operands (u_n / accumulator values at the point) are
  // loaded by epi_load() before the phase issues its staging loads: loads
  // complete in issue order, so a load issued after them would make its use
  // wait for every staging load in flight.
  const int mode = a.mode;
  struct Epi {
    double y, u;
  };
  const __amdgpu_buffer_rsrc_t ryin = state_rsrc(a.yin, G.sf), run = state_rsrc(a.un, G.sf);
  auto epi_load = [&](int f) __attribute__((always_inline)) {
    const unsigned so = spt + f * sf * 8u;
    return Epi{bload(ryin, vpt, so), bload(run, vpt, so)};
  };
  // the right-hand side k arrives in T and is combined in FP64; every mode
  // but HAM stores out = fma(cs, k, fma(cyo, Y, cu U)), RK4 stages 1-3 also
  // the accumulator
  const bool store_out = mode != MODE_HAM;
  const bool store_y = mode == MODE_STAGE1 || mode == MODE_STAGE23;
  auto emit = [&](int f, auto kt, const Epi& e) __attribute__((always_inline)) {
    if (!(valid && store_out)) return;
    const double kf = double(kt);
    const unsigned so = spt + f * sf * 8u;
    if (store_y) bstore(state_rsrc(a.y, G.sf), vpt, so, e.y + a.cy * kf);
    bstore(state_rsrc(a.out, G.sf), vpt, so, __builtin_fma(a.cs, kf, __builtin_fma(a.cyo, e.y, a.cu * e.u)));
  };

  // staging sequence: 24 phases (B only with the Gamma-driver shift)
  const Gauge& gauge = a.gauge;
  const bool driver = gauge.shift == 0;
  auto seq_gf = [&](int p) __attribute__((always_inline)) -> int {
    if (p < 3) return gBETA + p;
    if (p < 9) return gGT + (p - 3);
    if (p == 9) return gCHI;
    if (p == 10) return gALPHA;
    if (p < 14) return gXT + (p - 11);
    if (p == 14) return gK;
    if (p < 21) return gAT + (p - 15);
    return gB + (p - 21);
  };
  const int nphase = driver ? 24 : 21;
  // phase p computes from bufs[p % NB] after issuing phase p + NB - 1 into the
  // buffer phase p - 1 used; at its end the next phase's buffer must be
  // complete in every wave (own loads waited for, then the barrier)
  // The scheduling barrier keeps the phase's pointwise loads (issued just
  // before) ahead of its staging loads in the instruction stream.
  // One buffer (NB = 1): phase p issues its own grid function, waits for it
  // and meets the barrier before computing, and meets another at its end so
  // that no wave overwrites the buffer while another still reads it; the
  // other work-groups on the CU compute in the meantime.
  // With CROSS the cross phases 11.. are double-buffered inside the one
  // buffer (two cross neighbourhoods fit it): phase p >= 11 reads half p & 1,
  // and the grid function of phase p + 1 is issued into the other half at the
  // start of phase p, once every wave has left phase p - 1.
  static_assert(!CROSS || 2 * LC::SIZE <= L::SIZEP, "two cross neighbourhoods fit one buffer");
  auto cross_half = [&](int p) __attribute__((always_inline)) { return bufs[0] + (p & 1) * LC::SIZE; };
  auto buf_of = [&](int p) __attribute__((always_inline)) {
    return (CROSS && p >= 11) ? cross_half(p) : bufs[p % NB];
  };
  auto begin = [&](int p) __attribute__((always_inline)) {
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (NB == 1) {
      if (CROSS && p >= 11) {
        if (p == 11) {   // the first cross phase: nothing staged ahead yet
          issue_cross(seq_gf(p), cross_half(p));
          wait_vm<0>();
          lds_barrier();
        }
        if (p + 1 < nphase) issue_cross(seq_gf(p + 1), cross_half(p + 1));
      } else {
        issue(seq_gf(p), bufs[0]);
        wait_vm<0>();
        lds_barrier();
      }
    } else {
      if (p + NB - 1 < nphase) {
        if (CROSSZ && p + NB - 1 >= 11)
          issue_crossz(seq_gf(p + NB - 1), bufs[(p + NB - 1) % NB]);
        else
          issue(seq_gf(p + NB - 1), bufs[(p + NB - 1) % NB]);
      }
    }
  };
  auto sync = [&](int p) __attribute__((always_inline)) {
    if constexpr (NB == 1) {
      // a cross phase waits for the next phase's staging (and its own stores)
      if (CROSS && p >= 11) wait_vm<0>();
      if (p >= 0) lds_barrier();
    } else {
      // the phases issued after the next one hold at least C chunks per
      // wave each: fewer where CROSSZ phases are among them
      const int m = min(p + NB - 1, nphase - 1) - (p + 1);
      if (CROSSZ && p + NB - 1 >= 11)
        wait_staged<NB, (LZ::CMIN < L::CMIN ? LZ::CMIN : L::CMIN)>(m);
      else
        wait_staged<NB, L::CMIN>(m);
      lds_barrier();
    }
  };

  const double alpha_d = val(gALPHA), chi_d = val(gCHI), K_d = val(gK);
  const T alpha = T(alpha_d), chi = T(chi_d), K = T(K_d);
  // split precision: a point with chi < chi_split (near a puncture, where
  // the 1/chi terms are large) takes the chi phase in FP64
  const bool near = SPLIT && chi_d < a.chi_split;
  T g[6], gu[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) g[s] = T(val(gGT + s));
  {
    const T c00 = g[3] * g[5] - g[4] * g[4];
    const T c01 = g[2] * g[4] - g[1] * g[5];
    const T c02 = g[1] * g[4] - g[2] * g[3];
    const T c11 = g[0] * g[5] - g[2] * g[2];
    const T c12 = g[1] * g[2] - g[0] * g[4];
    const T c22 = g[0] * g[3] - g[1] * g[1];
    const T idet = T(1.0) / (g[0] * c00 + g[1] * c01 + g[2] * c02);
    gu[0] = c00 * idet; gu[1] = c01 * idet; gu[2] = c02 * idet;
    gu[3] = c11 * idet; gu[4] = c12 * idet; gu[5] = c22 * idet;
  }
  // traceless extrinsic curvature, raised (point values only)

  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int p = 0; p < NB - 1; ++p)
    if (p < nphase) issue(seq_gf(p), bufs[p]);
  sync(-1);

  // ---- shift (phases 0-2)
  T db[3][3];
  T xts[3] = {T(0.0), T(0.0), T(0.0)};
  T ddiv[3] = {T(0.0), T(0.0), T(0.0)};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Epi e = epi_load(gBETA + c);
    const T Bc = T(val(gB + c));
    begin(c);
    // the axis stencils first, so that register-held axis taps die before
    // the mixed derivatives read theirs
    T d2p[3];
    const auto ps = stencils(T(), make_ops(bufs[c % NB]), &db[c], &d2p, std::false_type());
    const auto& src = ps.src;
    const auto& ad = ps.ad;
    T mx[6];
    if constexpr (PIPE) mixed3(T(), src, mx);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int qi = SI(q), qj = SJ(q);
      const T dd = qi == qj ? d2p[qi] : (PIPE ? mx[q] : D2m(T(), src, q));
      xts[c] += T(W(q)) * gu[q] * dd;
      if (qj == c) ddiv[qi] += dd;
      if (qi == c && qi != qj) ddiv[qj] += dd;
    }
    emit(gBETA + c, driver ? ad.rhs(T(0.75) * Bc) : T(0.0), e);
    keep(db[c]);
    keep(xts);
    keep(ddiv);
    sync(c);
  }
  const T divb = db[0][0] + db[1][1] + db[2][2];
  // PARK: the Gt-source accumulators are not needed again before the K
  // phase; parked in LDS (each lane its own slots, no barrier) they do not
  // hold six registers through the metric phases, where pressure peaks
  auto park_slot = [&](int q) __attribute__((always_inline)) {
    int lin = wave * 64 + lane;
    asm volatile("" : "+v"(lin));
    return park + q * SH::NT + lin;
  };
  if constexpr (PARK) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      *park_slot(c) = double(xts[c]);
      *park_slot(3 + c) = double(ddiv[c]);
    }
  }

  // ---- conformal metric (phases 3-8)
  T Ric[6];
  T Gu[3][6];
  T Gd[3];
  {
    T dg[6][3];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int p = 3 + s;
      const Epi e = epi_load(gGT + s);
      const T As = T(val(gAT + s));
      begin(p);
      T d2p[3];
      const auto ps = stencils(T(), make_ops(bufs[p % NB]), &dg[s], &d2p, std::false_type());
      const auto& src = ps.src;
      const auto& ad = ps.ad;
      T r = T(0.0);
      T mx[6];
      if constexpr (PIPE) mixed3(T(), src, mx);
#pragma unroll
      for (int q = 0; q < 6; ++q)
        r += T(W(q)) * gu[q] * (SI(q) == SJ(q) ? d2p[SI(q)] : (PIPE ? mx[q] : D2m(T(), src, q)));
      Ric[s] = -T(0.5) * r;
      const int i = SI(s), jj = SJ(s);
      T lie = T(0.0);
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) lie += g[S(i, kk)] * db[kk][jj] + g[S(jj, kk)] * db[kk][i];
      emit(gGT + s, ad.rhs(-T(2.0) * alpha * As + lie - (T(2.0) / T(3.0)) * g[s] * divb), e);
      keep(Ric[s]);
      keep(dg[s]);
      sync(p);
    }
    T Gl[3][6];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), jj = SJ(s);
        Gl[kk][s] = T(0.5) * (dg[S(kk, i)][jj] + dg[S(kk, jj)][i] - dg[s][kk]);
      }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int s = 0; s < 6; ++s)
        Gu[kk][s] = gu[S(kk, 0)] * Gl[0][s] + gu[S(kk, 1)] * Gl[1][s] + gu[S(kk, 2)] * Gl[2][s];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      T acc = T(0.0);
#pragma unroll
      for (int s = 0; s < 6; ++s) acc += T(W(s)) * gu[s] * Gu[kk][s];
      Gd[kk] = acc;
    }
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), jj = SJ(s);
      T r = Ric[s];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) r += T(0.5) * Gd[kk] * (Gl[i][S(jj, kk)] + Gl[jj][S(i, kk)]);
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const T gmi = gu[S(0, m)] * Gu[kk][S(0, i)] + gu[S(1, m)] * Gu[kk][S(1, i)] +
                             gu[S(2, m)] * Gu[kk][S(2, i)];
          const T gmj = gu[S(0, m)] * Gu[kk][S(0, jj)] + gu[S(1, m)] * Gu[kk][S(1, jj)] +
                             gu[S(2, m)] * Gu[kk][S(2, jj)];
          r += gmi * (Gl[jj][S(kk, m)] + Gl[kk][S(m, jj)]) + gmj * Gl[i][S(kk, m)];
        }
      Ric[s] = r;
    }
  }
  keep(Gu);
  keep(Gd);
  keep(Ric);

  // ---- chi (phase 9), in precision TC: FP64, or FP32 in split waves away
  // from the punctures; dchi is kept in FP64 for the later 1/chi terms
  double dchi[3];
  const double ichi = 1.0 / chi_d;
  {
    const Epi e = epi_load(gCHI);
    begin(9);
    const auto tap = make_ops(bufs[9 % NB]);
    // the chi phase in precision TC, returned rather than applied: its Ricci
    // contributions, d chi (FP64) and the right-hand side of chi
    struct ChiPart {
      T ric[6];
      double dchi[3];
      T k;
    };
    auto chi_phase = [&](auto tag) __attribute__((always_inline)) {
      using TC = decltype(tag);
      ChiPart out;
      TC dc[3];
      TC d2p[3];
      const auto ps = stencils(tag, tap, &dc, &d2p, std::false_type());
      const auto& src = ps.src;
      const auto& ad = ps.ad;
      TC cdd[6], mx[6];
      if constexpr (PIPE) mixed3(tag, src, mx);
#pragma unroll
      for (int s = 0; s < 6; ++s)
        cdd[s] = (SI(s) == SJ(s) ? d2p[SI(s)] : (PIPE ? mx[s] : D2m(tag, src, s))) -
                 (TC(Gu[0][s]) * dc[0] + TC(Gu[1][s]) * dc[1] + TC(Gu[2][s]) * dc[2]);
      TC trc = TC(0.0), dchi2 = TC(0.0);
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        trc += TC(W(s)) * TC(gu[s]) * cdd[s];
        dchi2 += TC(W(s)) * TC(gu[s]) * dc[SI(s)] * dc[SJ(s)];
      }
      const TC ic = TC(ichi);
#pragma unroll
      for (int s = 0; s < 6; ++s)
        out.ric[s] = T(TC(0.5) * ic * (cdd[s] + TC(g[s]) * trc) -
                       TC(0.25) * ic * ic * (dc[SI(s)] * dc[SJ(s)] + TC(3.0) * TC(g[s]) * dchi2));
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) out.dchi[ax] = double(dc[ax]);
      out.k = T(ad.rhs(TC(2.0 / 3.0) * TC(chi_d) * (TC(alpha_d) * TC(K_d) - TC(divb))));
      return out;
    };
    // apply a chi-phase result to the points that take it
    auto apply = [&](const ChiPart& c, bool take) __attribute__((always_inline)) {
#pragma unroll
      for (int s = 0; s < 6; ++s) Ric[s] += take ? c.ric[s] : T(0.0);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) dchi[ax] = take ? c.dchi[ax] : dchi[ax];
      if (take) emit(gCHI, c.k, e);
    };
    if constexpr (!SPLIT) {
      apply(chi_phase(double()), true);
    } else {
      // waves entirely on one side of chi_split evaluate one precision; a
      // wave that straddles it evaluates both, each applied to its own
      // points, so a point's arithmetic does not depend on which points
      // share its wave (tile variants agree bitwise)
      const uint64_t in_near = __builtin_amdgcn_ballot_w64(valid && near);
      const uint64_t in_far = __builtin_amdgcn_ballot_w64(valid && !near);
      if (!in_far) {
        apply(chi_phase(double()), true);
      } else if (!in_near) {
        apply(chi_phase(float()), true);
      } else {
        apply(chi_phase(double()), near);
        apply(chi_phase(float()), !near);
      }
    }
    keep(Ric);
    keep(dchi);
    sync(9);
  }

  // ---- lapse (phase 10)
  T da[3];
  T DDa[6];
  {
    const Epi e = epi_load(gALPHA);
    begin(10);
    T d2p[3];
    const auto ps = stencils(T(), make_ops(bufs[10 % NB]), &da, &d2p, std::false_type());
    const auto& src = ps.src;
    const auto& ad = ps.ad;
    T mx[6];
    if constexpr (PIPE) mixed3(T(), src, mx);
    // the 1/chi correction is evaluated in FP64 in both precisions
    double gudchi_da = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
      gudchi_da += (double(gu[S(kk, 0)]) * dchi[0] + double(gu[S(kk, 1)]) * dchi[1] +
                    double(gu[S(kk, 2)]) * dchi[2]) * double(da[kk]);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), jj = SJ(s);
      const double corr = 0.5 * ichi * (double(g[s]) * gudchi_da - dchi[jj] * double(da[i]) - dchi[i] * double(da[jj]));
      DDa[s] = (SI(s) == SJ(s) ? d2p[SI(s)] : (PIPE ? mx[s] : D2m(T(), src, s))) - (Gu[0][s] * da[0] + Gu[1][s] * da[1] + Gu[2][s] * da[2]) -
               T(corr);
    }
    keep(da);
    keep(DDa);
    if (gauge.lapse == 2)
      emit(gALPHA, T(0.0), e);
    else
      emit(gALPHA, ad.rhs(gauge.lapse == 0 ? -T(2.0) * alpha * K : -alpha * alpha * K), e);
    sync(10);
  }

  // At_ij and At^ij (point values), loaded and formed here rather than at
  // the start so that they are not live through the metric, chi and lapse
  // phases, where register pressure peaks (each metric phase loads the one
  // component it needs; these loads hit in L2)
  T A[6], Au[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) A[s] = T(val(gAT + s));
  {
    T Am[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
        Am[i][jj] = gu[S(i, 0)] * A[S(0, jj)] + gu[S(i, 1)] * A[S(1, jj)] + gu[S(i, 2)] * A[S(2, jj)];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), jj = SJ(s);
      Au[s] = Am[i][0] * gu[S(0, jj)] + Am[i][1] * gu[S(1, jj)] + Am[i][2] * gu[S(2, jj)];
    }
  }
  // Gt^c_jk At^jk, the only later use of the Christoffel symbols besides chi/alpha
  T ga[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T acc = T(0.0);
#pragma unroll
    for (int q = 0; q < 6; ++q) acc += T(W(q)) * Gu[c][q] * Au[q];
    ga[c] = acc;
  }
  keep(ga);

  // ---- evolved Gt (phases 11-13)
  T xt_ad[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int p = 11 + c;
    begin(p);
    T dx[3];
    const auto ps = stencils(T(), cross_ops(buf_of(p)), &dx, nullptr, XKIND());
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T d = dx[ax];
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), jj = SJ(s);
        if (jj == ax) Ric[s] += T(0.5) * g[S(c, i)] * d;
        if (i == ax) Ric[s] += T(0.5) * g[S(c, jj)] * d;
      }
    }
    xt_ad[c] = ps.ad.rhs(T(0.0));
    keep(xt_ad[c]);
    keep(Ric);
    sync(p);
  }

  // ---- K (phase 14)
  T AA = T(0.0);
  {
    T Am[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
        Am[i][jj] = gu[S(i, 0)] * A[S(0, jj)] + gu[S(i, 1)] * A[S(1, jj)] + gu[S(i, 2)] * A[S(2, jj)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) AA += Am[i][jj] * Am[jj][i];
  }
  T trDDa = T(0.0), trRic = T(0.0);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    trDDa += T(W(s)) * gu[s] * DDa[s];
    trRic += T(W(s)) * gu[s] * Ric[s];
  }
  // the Hamiltonian constraint H = chi gt^ij R_ij + 2/3 K^2 - At_ij At^ij
  // (diagnostic mode; every phase still runs, so the staging drains normally)
  if (mode == MODE_HAM && valid)
    bstore(state_rsrc(a.out, G.sf), vpt, spt, double(chi * trRic + (T(2.0) / T(3.0)) * K * K - AA));
  T xsrc[3];
  {
    const Epi e = epi_load(gK);
    const Epi ex[3] = {epi_load(gXT), epi_load(gXT + 1), epi_load(gXT + 2)};
    begin(14);
    T dK[3];
    const auto ps = stencils(T(), cross_ops(buf_of(14)), &dK, nullptr, XKIND());
    emit(gK, ps.ad.rhs(-chi * trDDa + alpha * (AA + K * K * (T(1.0) / T(3.0)))), e);
    if constexpr (PARK) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xts[c] = T(*park_slot(c));
        ddiv[c] = T(*park_slot(3 + c));
      }
    }
    // Gt source, complete now
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T r = xts[c];
      r += (T(1.0) / T(3.0)) * (gu[S(c, 0)] * ddiv[0] + gu[S(c, 1)] * ddiv[1] + gu[S(c, 2)] * ddiv[2]);
      r += (T(2.0) / T(3.0)) * Gd[c] * divb - (Gd[0] * db[c][0] + Gd[1] * db[c][1] + Gd[2] * db[c][2]);
      r -= T(2.0) * (Au[S(c, 0)] * da[0] + Au[S(c, 1)] * da[1] + Au[S(c, 2)] * da[2]);
      const double adchi = double(Au[S(c, 0)]) * dchi[0] + double(Au[S(c, 1)]) * dchi[1] + double(Au[S(c, 2)]) * dchi[2];
      const T gdK = gu[S(c, 0)] * dK[0] + gu[S(c, 1)] * dK[1] + gu[S(c, 2)] * dK[2];
      r += T(2.0) * alpha * (ga[c] - T(1.5 * ichi * adchi) - (T(2.0) / T(3.0)) * gdK);
      xsrc[c] = r;
      emit(gXT + c, xt_ad[c] + r, ex[c]);
    }
    keep(xsrc);
    sync(14);
  }

  // ---- At (phases 15-20)
  const T trX = alpha * trRic - trDDa;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int p = 15 + s;
    const Epi e = epi_load(gAT + s);
    begin(p);
    const auto ps = stencils(T(), cross_ops(buf_of(p)), nullptr, nullptr, XKIND());
    const int i = SI(s), jj = SJ(s);
    T la = T(0.0), aa = T(0.0);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      la += A[S(i, kk)] * db[kk][jj] + A[S(jj, kk)] * db[kk][i];
      // At_ik At^k_j = At_ik gt^kl At_lj
      const T amkj = gu[S(kk, 0)] * A[S(0, jj)] + gu[S(kk, 1)] * A[S(1, jj)] + gu[S(kk, 2)] * A[S(2, jj)];
      aa += A[S(i, kk)] * amkj;
    }
    const T X = alpha * Ric[s] - DDa[s];
    emit(gAT + s, ps.ad.rhs(chi * (X - (T(1.0) / T(3.0)) * g[s] * trX) + alpha * (K * A[s] - T(2.0) * aa) + la -
                            (T(2.0) / T(3.0)) * A[s] * divb), e);
    sync(p);
  }

  // ---- Gamma-driver B (phases 21-23)
  if (driver) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int p = 21 + c;
      const Epi e = epi_load(gB + c);
      const T Bc = T(val(gB + c));
      begin(p);
      const auto ps = stencils(T(), cross_ops(buf_of(p)), nullptr, nullptr, XKIND());
      emit(gB + c, ps.ad.rhs(xsrc[c] - gauge.eta * Bc), e);
      sync(p);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) emit(gB + c, T(0.0), epi_load(gB + c));
  }
}

// The stage kernel.  Single-patch form (bt.ntiles == 0): the tiles of patch
// a1, one per work-group, hardware block ids remapped so that each XCD gets
// a contiguous range of tiles (neighbours share its L2).  Batched form: the
// concatenated tiles of all patches of a plan, each work-group finding its
// patch by binary search -- one tile per work-group in the same XCD order
// (bt.queue null), or persistent: a grid sized to the resident work-groups,
// each pulling tiles from its XCD's queue (the same contiguous eighth of
// the tile list) until all queues are empty.
// OCC waves share a SIMD (OCC * 4 / WPG work-groups per CU): their NB
// staging buffers must fit the 160 KB LDS together, and the registers per
// lane drop to 512 / OCC.
// PERSIST: the persistent batched form (bt.queue set); the other forms are
// separate instances without its loop, whose loop-carried state would cost
// them scalar registers.
template <int ORDER, bool UPWIND, int R, int NB, int OCC, int TX, int WPG, typename T, int TZ = 1, bool KOQ = false,
          bool PERSIST = false>
__global__ __launch_bounds__(64 * WPG) __attribute__((amdgpu_waves_per_eu(OCC)))
void stage_kernel(StageArgs a1, BatchTable bt) {
  using SH = Shape<TX, WPG, TZ>;
  using L = LdsLayout<R, ORDER / 2, SH>;
  static_assert(NB >= 1 && NB <= 5, "staging depth");
  constexpr bool BOUND = ORDER >= 8 || OCC >= 2;
  // order 8 at two waves per SIMD and split precision at three read their
  // axis taps axis by axis (256 and 168 registers per lane)
#ifndef CHEMORA_SPLIT_AXIS_GROUPS
#define CHEMORA_SPLIT_AXIS_GROUPS 1
#endif
#ifndef CHEMORA_O4_AXIS_GROUPS
#define CHEMORA_O4_AXIS_GROUPS 0
#endif
  constexpr bool AXIS_GROUPS = (ORDER >= 8 && OCC >= 2) ||
                               (CHEMORA_SPLIT_AXIS_GROUPS && std::is_same<T, float>::value && OCC >= 3) ||
                               (CHEMORA_O4_AXIS_GROUPS && ORDER == 4);
  constexpr int WG_PER_CU = (OCC * 4) / WPG > 1 ? (OCC * 4) / WPG : 1;
  constexpr int LDS_STAGE = NB * L::SIZEP * 8, LDS_OFFS = L::CPW * SH::NT * 4;
  // FP64 with two waves per SIMD keeps the per-lane staging offsets in LDS
  // where they fit (its 256 registers are otherwise exhausted); FP32 algebra
  // needs ~156
  constexpr bool OFFS_LDS = OCC == 2 && sizeof(T) == 8 && WG_PER_CU * (LDS_STAGE + LDS_OFFS) <= 160 * 1024;
  constexpr int LDS_BASE = LDS_STAGE + (OFFS_LDS ? LDS_OFFS : 0);
  static_assert(WG_PER_CU * LDS_BASE <= 160 * 1024, "LDS");
  // two waves per SIMD park six accumulators in LDS where they fit (beside
  // the persistent form's tile slot)
  constexpr bool PARK = OFFS_LDS && WG_PER_CU * (LDS_BASE + 6 * SH::NT * 8 + (PERSIST ? 16 : 0)) <= 160 * 1024;
  // order 4, FP64 with parked offsets and a staging pipeline: the 13 grid
  // functions without mixed derivatives stage CrossLayoutZ, whose tile-plane
  // chunk offsets are parked too, where that still fits
#ifndef CHEMORA_CROSS_O4
#define CHEMORA_CROSS_O4 1
#endif
  constexpr int LDS_OFFS_Z = CrossLayoutZ<R, SH>::CPW0 * SH::NT * 4;
  constexpr bool CROSSZ = CHEMORA_CROSS_O4 && ORDER == 4 && OFFS_LDS && PARK && NB >= 2 &&
                          !AXIS_GROUPS &&
                          WG_PER_CU * (LDS_BASE + LDS_OFFS_Z + 6 * SH::NT * 8 + (PERSIST ? 16 : 0)) <= 160 * 1024;
  // separate arrays, so the compiler can tell the buffers' staging loads apart
  __shared__ double b0[L::SIZEP];
  __shared__ double b1[NB > 1 ? L::SIZEP : 1];
  __shared__ double b2[NB > 2 ? L::SIZEP : 1];
  __shared__ double b3[NB > 3 ? L::SIZEP : 1];
  __shared__ double b4[NB > 4 ? L::SIZEP : 1];
  __shared__ unsigned offs[OFFS_LDS ? (L::CPW + (CROSSZ ? CrossLayoutZ<R, SH>::CPW0 : 0)) * SH::NT : 1];
  __shared__ double park[PARK ? 6 * SH::NT : 1];
  double* const all[5] = {b0, b1, b2, b3, b4};
  double* bufs[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) bufs[i] = all[i];
  if constexpr (!PERSIST) {
    int t = xcd_tile(blockIdx.x, gridDim.x);
    StageArgs a = a1;
    if (bt.ntiles > 0) {
      const int p = batch_patch(bt, t);
      a = uniform_args(bt.args + p);
      t -= uniform(table_load(bt.tile_start, p));
    }
    stage_tile<ORDER, UPWIND, R, NB, BOUND, OFFS_LDS, PARK, SH, T, KOQ, AXIS_GROUPS, CROSSZ>(a, t, bufs, offs, park);
  } else {
    // One work-item fetches each tile and hands it over through LDS.  Every
    // work-item reads the slot before stage_tile's first barrier, and the
    // fetch after it comes after stage_tile's last barrier, so one slot
    // suffices.
    const bool leader = threadIdx.x == 0 && threadIdx.y == 0;
    const int x = xcd_id();
    __shared__ int next;
    for (;;) {
      if (leader) next = pull_tile(bt, x);
      __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the LDS write is done
      lds_barrier();
      const int t = uniform(next);
      if (t < 0) break;
      const int p = batch_patch(bt, t);
      const StageArgs a = uniform_args(bt.args + p);
      stage_tile<ORDER, UPWIND, R, NB, BOUND, OFFS_LDS, PARK, SH, T, KOQ, AXIS_GROUPS, CROSSZ>(a, t - uniform(table_load(bt.tile_start, p)), bufs,
                                                                          offs, park);
    }
    // the last work-group to finish leaves the counters zeroed for the next
    // launch: every other work-group has made its last pull by then
    if (leader && atomicAdd(bt.queue + NXCD, 1) == (int)gridDim.x - 1) {
#pragma unroll
      for (int q = 0; q <= NXCD; ++q) atomicExch(bt.queue + q, 0);
    }
  }
}

}  // namespace chemora
