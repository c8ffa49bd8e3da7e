// stage_kernel.hpp -- the fused RK-stage kernel (stencils + BSSN algebra +
// advection + dissipation + RK4 stage combination), one work-item per
// interior point.  Instantiated per finite-difference order in
// stage_o4.hip / stage_o8.hip.
//
// The paper's McLachlan kernels spill badly ("fat kernels", section "Fat
// Kernel Detection") because every derivative is formed before the
// algebra.  Here the right-hand side is evaluated grid function by grid
// function in dependency order
//     beta -> gt -> chi -> Gt -> alpha -> K -> At -> (Gt, B)
// so each stencil result is consumed as soon as it is formed: second
// derivatives are contracted at once into the Ricci, D_i D_j alpha and
// Gt-source accumulators, and each variable's right-hand side is finished
// and passed through the RK epilogue (loads of u_n / the accumulator,
// stores) as soon as its inputs are complete.  Only the first derivatives of
// beta, chi, alpha, K and the Christoffel symbols stay live.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bssn_algebra.hpp"
#include "fd_ops.hpp"

namespace chemora {

// Geometry of a launch (all offsets in elements).
struct Geo {
  int nx, ny, nz, g;
  int64_t sy, sz, sf;
};

struct Scales {
  double d1;    // 1 / (D1 h)
  double d2;    // 1 / (D2 h^2)
  double d11;   // 1 / (D1 h)^2
  double up;    // 1 / (DU h)
  double ko;    // 2^(-2r) * (eps / h)
  int ko_r;
};

enum Mode : int { MODE_RHS = 0, MODE_STAGE1 = 1, MODE_STAGE23 = 2, MODE_STAGE4 = 4 };

struct StageArgs {
  const double* __restrict__ in;   // stencil input of this stage
  const double* __restrict__ un;   // u_n (stages 1-3)
  double* __restrict__ y;          // RK accumulator
  double* __restrict__ out;        // rhs (MODE_RHS), next stage input, or u (stage 4)
  Geo geo;
  Scales sc;
  Gauge gauge;
  double cy;                       // weight of k in the accumulator update
  double cs;                       // weight of k in the next stage input
  int tiles_x, tiles_y;            // tile grid (64 x 4 points per tile)
};

// Keeps the scheduler from hoisting the next phase's loads above this point
// (which would make every stencil value live at once and spill).
#ifndef CHEMORA_NO_PHASE
#define CHEMORA_PHASE() __builtin_amdgcn_sched_barrier(0)
#else
#define CHEMORA_PHASE()
#endif

// Materialises a value in registers at this point.  Without it the compiler
// sinks the arithmetic of an accumulator to its last use near the end of the
// kernel while the stencil loads feeding it stay early (stores intervene),
// which keeps every loaded tap live across the kernel.
__device__ inline void keep(double& x) { asm volatile("" : "+v"(x)); }
template <int N>
__device__ inline void keep(double (&x)[N]) {
#pragma unroll
  for (int n = 0; n < N; ++n) keep(x[n]);
}
template <int N, int M>
__device__ inline void keep(double (&x)[N][M]) {
#pragma unroll
  for (int n = 0; n < N; ++n) keep(x[n]);
}

#ifndef CHEMORA_WAVES_PER_EU
#define CHEMORA_WAVES_PER_EU 2
#endif

constexpr int TILE_X = 64;
constexpr int TILE_Y = 4;
constexpr int NXCD = 8;

// Raw buffer access (gfx9 descriptor word 3 = 0x00020000).  Each state
// buffer (24 GFs) is one buffer resource whose base sits XB elements before
// the array, and an access is
//   base + voffset (per lane: the point) + soffset (uniform: GF, y/z offsets)
//        + imm ((XB + dx) * 8, a compile-time immediate),
// so the ~1000 stencil taps of a point share a single address register and
// every y/z/GF offset is scalar arithmetic.  Offsets are 32-bit: the host
// rejects patches whose 24-GF state exceeds 4 GiB.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int XB = 8;

__device__ inline __amdgpu_buffer_rsrc_t state_rsrc(const double* base, int64_t sf) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(base - XB), (short)0, (int)((24 * sf + XB) * 8), 0x00020000);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)voff, (int)soff, 0);
}

// Work-groups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the hardware block id so that each XCD receives a contiguous
// range of tiles (neighbours share halos in that XCD's L2).
__device__ inline int xcd_tile(int bid, int nblocks) {
  const int full = (nblocks / NXCD) * NXCD;
  if (bid >= full) return bid;
  return (bid % NXCD) * (nblocks / NXCD) + bid / NXCD;
}

template <int ORDER, bool UPWIND, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CHEMORA_WAVES_PER_EU))) void stage_kernel(StageArgs a) {
  using St = Stencil<ORDER>;
  const Geo G = a.geo;
  const int nblocks = a.tiles_x * a.tiles_y * G.nz;
  const int t = xcd_tile(blockIdx.x, nblocks);
  const int tx = t % a.tiles_x;
  const int ty = (t / a.tiles_x) % a.tiles_y;
  const int k = t / (a.tiles_x * a.tiles_y);
  const int i = tx * TILE_X + threadIdx.x;
  const int j = ty * TILE_Y + threadIdx.y;
  if (i >= G.nx || j >= G.ny) return;
  // byte offsets: lane part (the point, x and y), uniform part (GF, z plane,
  // y/z stencil offsets), immediate (x stencil offset)
  const unsigned sy = (unsigned)G.sy, sz = (unsigned)G.sz, sf = (unsigned)G.sf, gg = (unsigned)G.g;
  const unsigned vb = (j * sy + i + gg) * 8u;
  const unsigned zb = k * sz;
  const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, G.sf);
  auto soff = [&](int f, int dy, int dz) { return (f * sf + zb + (gg + dz) * sz + (gg + dy) * sy) * 8u; };
  auto tap = [&](int f, int dx, int dy, int dz) { return bload(rin, vb + (XB + dx) * 8, soff(f, dy, dz)); };
  auto along = [&](int f, int ax, int o) {
    return ax == 0 ? tap(f, o, 0, 0) : (ax == 1 ? tap(f, 0, o, 0) : tap(f, 0, 0, o));
  };
  auto val = [&](int f) { return tap(f, 0, 0, 0); };
  auto D1 = [&](int f, int ax) {
    return St::first([&](int o) { return along(f, ax, o); }) * a.sc.d1;
  };
  auto D2 = [&](int f, int slot) {
    const int ai = SI(slot), bj = SJ(slot);
    if (ai == bj) return St::second([&](int o) { return along(f, ai, o); }) * a.sc.d2;
    const double v = St::first([&](int oa) {
      return St::first([&](int ob) {
        int d[3] = {0, 0, 0};
        d[ai] = oa;
        d[bj] = ob;
        return tap(f, d[0], d[1], d[2]);
      });
    });
    return v * a.sc.d11;
  };
  const double bet[3] = {val(gBETA), val(gBETA + 1), val(gBETA + 2)};
  // advection + dissipation of GF f; rhs = (algebra + adv) + diss
  auto finish = [&](int f, double alg) {
    double adv = 0.0, diss = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      double d;
      if (UPWIND) {
        const int sg = bet[ax] >= 0.0 ? 1 : -1;
        d = (double)sg * St::lopsided([&](int o) { return along(f, ax, o); }, sg) * a.sc.up;
      } else {
        d = St::first([&](int o) { return along(f, ax, o); }) * a.sc.d1;
      }
      adv += bet[ax] * d;
      if (a.sc.ko_r > 0) {
        const double qd = ko_axis([&](int o) { return along(f, ax, o); }, a.sc.ko_r, a.sc.ko);
        diss = (ax == 0) ? qd : diss + qd;
      }
    }
    return (alg + adv) + diss;
  };
  // RK epilogue of GF f with right-hand side kf (pointwise buffers)
  const unsigned vo = vb + XB * 8u;
  auto emit = [&](int f, double kf) {
    const unsigned so = soff(f, 0, 0);
    if (MODE == MODE_RHS) {
      bstore(state_rsrc(a.out, G.sf), vo, so, kf);
    } else if (MODE == MODE_STAGE1) {
      const double u0 = val(f);
      bstore(state_rsrc(a.y, G.sf), vo, so, u0 + a.cy * kf);
      bstore(state_rsrc(a.out, G.sf), vo, so, u0 + a.cs * kf);
    } else if (MODE == MODE_STAGE23) {
      const double y0 = bload(state_rsrc(a.y, G.sf), vo, so);
      const double u0 = bload(state_rsrc(a.un, G.sf), vo, so);
      bstore(state_rsrc(a.y, G.sf), vo, so, y0 + a.cy * kf);
      bstore(state_rsrc(a.out, G.sf), vo, so, u0 + a.cs * kf);
    } else {
      const double y0 = bload(state_rsrc(a.y, G.sf), vo, so);
      bstore(state_rsrc(a.out, G.sf), vo, so, y0 + a.cy * kf);
    }
  };
  const Gauge& gauge = a.gauge;
  const double alpha = val(gALPHA), chi = val(gCHI), K = val(gK);

  // conformal metric and its inverse (point values only)
  double g[6], gu[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) g[s] = val(gGT + s);
  {
    const double c00 = g[3] * g[5] - g[4] * g[4];
    const double c01 = g[2] * g[4] - g[1] * g[5];
    const double c02 = g[1] * g[4] - g[2] * g[3];
    const double c11 = g[0] * g[5] - g[2] * g[2];
    const double c12 = g[1] * g[2] - g[0] * g[4];
    const double c22 = g[0] * g[3] - g[1] * g[1];
    const double idet = 1.0 / (g[0] * c00 + g[1] * c01 + g[2] * c02);
    gu[0] = c00 * idet; gu[1] = c01 * idet; gu[2] = c02 * idet;
    gu[3] = c11 * idet; gu[4] = c12 * idet; gu[5] = c22 * idet;
  }

  CHEMORA_PHASE();
  // ---- shift: d beta kept; d d beta contracted into the Gt source
  double db[3][3];          // db[i][k] = d_k beta^i
  double xts[3] = {0.0, 0.0, 0.0};
  double ddiv[3] = {0.0, 0.0, 0.0};   // d_j d_k beta^k
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CHEMORA_PHASE();
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) db[c][ax] = D1(gBETA + c, ax);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double dd = D2(gBETA + c, q);
      xts[c] += W(q) * gu[q] * dd;
      const int qi = SI(q), qj = SJ(q);
      if (qj == c) ddiv[qi] += dd;
      if (qi == c && qi != qj) ddiv[qj] += dd;
    }
  }
  keep(db);
  keep(xts);
  keep(ddiv);
  CHEMORA_PHASE();
  const double divb = db[0][0] + db[1][1] + db[2][2];
  if (gauge.shift == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) emit(gBETA + c, finish(gBETA + c, 0.75 * val(gB + c)));
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) emit(gBETA + c, 0.0);
  }

  CHEMORA_PHASE();
  // ---- conformal metric: Christoffels, the d d gt part of the Ricci tensor
  double Ric[6];
  double Gl[3][6];          // Gt_{k,ij}
  {
    double dg[6][3];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      CHEMORA_PHASE();
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) dg[s][ax] = D1(gGT + s, ax);
      double r = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) r += W(q) * gu[q] * D2(gGT + s, q);
      Ric[s] = -0.5 * r;
      keep(Ric[s]);
      keep(dg[s]);
      const int i = SI(s), jj = SJ(s);
      double lie = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) lie += g[S(i, kk)] * db[kk][jj] + g[S(jj, kk)] * db[kk][i];
      const double At_s = val(gAT + s);
      emit(gGT + s, finish(gGT + s, -2.0 * alpha * At_s + lie - (2.0 / 3.0) * g[s] * divb));
    }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), jj = SJ(s);
        Gl[kk][s] = 0.5 * (dg[S(kk, i)][jj] + dg[S(kk, jj)][i] - dg[s][kk]);
      }
  }
  CHEMORA_PHASE();
  double Gu[3][6];          // Gt^k_ij
#pragma unroll
  for (int kk = 0; kk < 3; ++kk)
#pragma unroll
    for (int s = 0; s < 6; ++s)
      Gu[kk][s] = gu[S(kk, 0)] * Gl[0][s] + gu[S(kk, 1)] * Gl[1][s] + gu[S(kk, 2)] * Gl[2][s];
  double Gd[3];
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) acc += W(s) * gu[s] * Gu[kk][s];
    Gd[kk] = acc;
  }
  keep(Gl);
  keep(Gu);
  keep(Gd);
  // quadratic Christoffel terms of the Ricci tensor
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), jj = SJ(s);
    double r = Ric[s];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) r += 0.5 * Gd[kk] * (Gl[i][S(jj, kk)] + Gl[jj][S(i, kk)]);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        // gt^lm Gt^k_li and gt^lm Gt^k_lj
        const double gmi = gu[S(0, m)] * Gu[kk][S(0, i)] + gu[S(1, m)] * Gu[kk][S(1, i)] +
                           gu[S(2, m)] * Gu[kk][S(2, i)];
        const double gmj = gu[S(0, m)] * Gu[kk][S(0, jj)] + gu[S(1, m)] * Gu[kk][S(1, jj)] +
                           gu[S(2, m)] * Gu[kk][S(2, jj)];
        r += gmi * (Gl[jj][S(kk, m)] + Gl[kk][S(m, jj)]) + gmj * Gl[i][S(kk, m)];
      }
    Ric[s] = r;
  }
  keep(Ric);

  CHEMORA_PHASE();
  // ---- chi
  double dchi[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) dchi[ax] = D1(gCHI, ax);
  const double ichi = 1.0 / chi;
  {
    double cdd[6];
#pragma unroll
    for (int s = 0; s < 6; ++s)
      cdd[s] = D2(gCHI, s) - (Gu[0][s] * dchi[0] + Gu[1][s] * dchi[1] + Gu[2][s] * dchi[2]);
    double trc = 0.0, dchi2 = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      trc += W(s) * gu[s] * cdd[s];
      dchi2 += W(s) * gu[s] * dchi[SI(s)] * dchi[SJ(s)];
    }
#pragma unroll
    for (int s = 0; s < 6; ++s)
      Ric[s] += 0.5 * ichi * (cdd[s] + g[s] * trc) -
                0.25 * ichi * ichi * (dchi[SI(s)] * dchi[SJ(s)] + 3.0 * g[s] * dchi2);
  }
  keep(Ric);
  keep(dchi);
  emit(gCHI, finish(gCHI, (2.0 / 3.0) * chi * (alpha * K - divb)));

  CHEMORA_PHASE();
  // ---- evolved Gt: d Gt into the Ricci tensor; advection/dissipation kept
  double xt_ad[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CHEMORA_PHASE();
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double d = D1(gXT + c, ax);
      // +1/2 (gt_ci d_j Gt^c + gt_cj d_i Gt^c) for every (i, j) with ax in {i, j}
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), jj = SJ(s);
        if (jj == ax) Ric[s] += 0.5 * g[S(c, i)] * d;
        if (i == ax) Ric[s] += 0.5 * g[S(c, jj)] * d;
      }
    }
    xt_ad[c] = finish(gXT + c, 0.0);
    keep(xt_ad[c]);
    keep(Ric);
  }

  CHEMORA_PHASE();
  // ---- lapse: D_i D_j alpha
  double da[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) da[ax] = D1(gALPHA, ax);
  double DDa[6];
  {
    double gudchi_da = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
      gudchi_da += (gu[S(kk, 0)] * dchi[0] + gu[S(kk, 1)] * dchi[1] + gu[S(kk, 2)] * dchi[2]) * da[kk];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), jj = SJ(s);
      DDa[s] = D2(gALPHA, s) - (Gu[0][s] * da[0] + Gu[1][s] * da[1] + Gu[2][s] * da[2]) -
               0.5 * ichi * (g[s] * gudchi_da - dchi[jj] * da[i] - dchi[i] * da[jj]);
    }
  }
  keep(da);
  keep(DDa);
  if (gauge.lapse == 2) {
    emit(gALPHA, 0.0);
  } else {
    const double ra = gauge.lapse == 0 ? -2.0 * alpha * K : -alpha * alpha * K;
    emit(gALPHA, finish(gALPHA, ra));
  }

  CHEMORA_PHASE();
  // ---- traceless extrinsic curvature: mixed / raised forms
  double A[6], Am[3][3], Au[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) A[s] = val(gAT + s);
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
  double AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) AA += Am[i][jj] * Am[jj][i];

  CHEMORA_PHASE();
  // ---- K
  double trDDa = 0.0, trRic = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    trDDa += W(s) * gu[s] * DDa[s];
    trRic += W(s) * gu[s] * Ric[s];
  }
  double dK[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) dK[ax] = D1(gK, ax);
  keep(dK);
  emit(gK, finish(gK, -chi * trDDa + alpha * (AA + K * K * (1.0 / 3.0))));

  CHEMORA_PHASE();
  // ---- At
  const double trX = alpha * trRic - trDDa;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    CHEMORA_PHASE();
    const int i = SI(s), jj = SJ(s);
    double la = 0.0, aa = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      la += A[S(i, kk)] * db[kk][jj] + A[S(jj, kk)] * db[kk][i];
      aa += A[S(i, kk)] * Am[kk][jj];
    }
    const double X = alpha * Ric[s] - DDa[s];
    emit(gAT + s, finish(gAT + s, chi * (X - (1.0 / 3.0) * g[s] * trX) + alpha * (K * A[s] - 2.0 * aa) + la -
                                      (2.0 / 3.0) * A[s] * divb));
  }

  CHEMORA_PHASE();
  // ---- Gt and the Gamma-driver B
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    CHEMORA_PHASE();
    double r = xts[c];
    r += (1.0 / 3.0) * (gu[S(c, 0)] * ddiv[0] + gu[S(c, 1)] * ddiv[1] + gu[S(c, 2)] * ddiv[2]);
    r += (2.0 / 3.0) * Gd[c] * divb - (Gd[0] * db[c][0] + Gd[1] * db[c][1] + Gd[2] * db[c][2]);
    r -= 2.0 * (Au[S(c, 0)] * da[0] + Au[S(c, 1)] * da[1] + Au[S(c, 2)] * da[2]);
    double ga = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) ga += W(q) * Gu[c][q] * Au[q];
    const double adchi = Au[S(c, 0)] * dchi[0] + Au[S(c, 1)] * dchi[1] + Au[S(c, 2)] * dchi[2];
    const double gdK = gu[S(c, 0)] * dK[0] + gu[S(c, 1)] * dK[1] + gu[S(c, 2)] * dK[2];
    r += 2.0 * alpha * (ga - 1.5 * ichi * adchi - (2.0 / 3.0) * gdK);
    // r is the Gt source without advection and dissipation
    emit(gXT + c, xt_ad[c] + r);
    if (gauge.shift == 0)
      emit(gB + c, finish(gB + c, r - gauge.eta * val(gB + c)));
    else
      emit(gB + c, 0.0);
  }
}

// host-side launchers, one per order (defined in stage_o4.hip / stage_o8.hip)
void launch_stage_o4(int mode, bool upwind, const StageArgs& a, hipStream_t s);
void launch_stage_o8(int mode, bool upwind, const StageArgs& a, hipStream_t s);

}  // namespace chemora
