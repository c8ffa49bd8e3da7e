// stage_kernel.hpp -- the fused RK-stage kernel (stencils + BSSN algebra +
// advection + dissipation + RK4 stage combination), one work-item per
// interior point.  Instantiated per finite-difference order in
// stage_o4.hip / stage_o8.hip.
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
};

template <int ORDER, bool UPWIND, int MODE>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs a) {
  using St = Stencil<ORDER>;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const Geo& G = a.geo;
  if (i >= G.nx || j >= G.ny) return;
  const int64_t idx = (int64_t)(k + G.g) * G.sz + (int64_t)(j + G.g) * G.sy + (i + G.g);
  const int64_t st[3] = {1, G.sy, G.sz};

  PointIn p;
#pragma unroll
  for (int f = 0; f < 24; ++f) p.u[f] = a.in[f * G.sf + idx];

  auto D1 = [&](int f, int ax) {
    const double* q = a.in + f * G.sf + idx;
    const int64_t s = st[ax];
    return St::first([&](int o) { return q[o * s]; }) * a.sc.d1;
  };
  auto D2 = [&](int f, int slot) {
    const double* q = a.in + f * G.sf + idx;
    const int ai = SI(slot), bj = SJ(slot);
    if (ai == bj) {
      const int64_t s = st[ai];
      return St::second([&](int o) { return q[o * s]; }) * a.sc.d2;
    }
    const int64_t sa = st[ai], sb = st[bj];
    const double v = St::first([&](int oa) {
      const double* r = q + oa * sa;
      return St::first([&](int ob) { return r[ob * sb]; });
    });
    return v * a.sc.d11;
  };

#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    p.dchi[ax] = D1(gCHI, ax);
    p.dK[ax] = D1(gK, ax);
    p.dalpha[ax] = D1(gALPHA, ax);
#pragma unroll
    for (int s = 0; s < 6; ++s) p.dgt[s][ax] = D1(gGT + s, ax);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p.dXt[c][ax] = D1(gXT + c, ax);
      p.dbeta[c][ax] = D1(gBETA + c, ax);
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    p.ddchi[q] = D2(gCHI, q);
    p.ddalpha[q] = D2(gALPHA, q);
#pragma unroll
    for (int s = 0; s < 6; ++s) p.ddgt[s][q] = D2(gGT + s, q);
#pragma unroll
    for (int c = 0; c < 3; ++c) p.ddbeta[c][q] = D2(gBETA + c, q);
  }

  double rhs[24];
  bssn_algebra(p, a.gauge, rhs);

  // advection and dissipation, GF by GF: rhs = (algebra + advection) + dissipation
  const double bet[3] = {p.u[gBETA], p.u[gBETA + 1], p.u[gBETA + 2]};
#pragma unroll 1
  for (int f = 0; f < 24; ++f) {
    if (!evolves(f, a.gauge)) continue;
    const double* q = a.in + f * G.sf + idx;
    double adv = 0.0, diss = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int64_t s = st[ax];
      double d;
      if (UPWIND) {
        const int sg = bet[ax] >= 0.0 ? 1 : -1;
        d = (double)sg * St::lopsided([&](int o) { return q[o * s]; }, sg) * a.sc.up;
      } else {
        d = St::first([&](int o) { return q[o * s]; }) * a.sc.d1;
      }
      adv += bet[ax] * d;
      if (a.sc.ko_r > 0) {
        const double qd = ko_axis([&](int o) { return q[o * s]; }, a.sc.ko_r, a.sc.ko);
        diss = (ax == 0) ? qd : diss + qd;
      }
    }
    rhs[f] = (rhs[f] + adv) + diss;
  }

#pragma unroll
  for (int f = 0; f < 24; ++f) {
    const int64_t o = f * G.sf + idx;
    const double kf = rhs[f];
    if (MODE == MODE_RHS) {
      a.out[o] = kf;
    } else if (MODE == MODE_STAGE1) {
      const double u0 = p.u[f];
      a.y[o] = u0 + a.cy * kf;
      a.out[o] = u0 + a.cs * kf;
    } else if (MODE == MODE_STAGE23) {
      a.y[o] = a.y[o] + a.cy * kf;
      a.out[o] = a.un[o] + a.cs * kf;
    } else {
      a.out[o] = a.y[o] + a.cy * kf;
    }
  }
}

// host-side launchers, one per order (defined in stage_o4.hip / stage_o8.hip)
void launch_stage_o4(int mode, bool upwind, const StageArgs& a, hipStream_t s);
void launch_stage_o8(int mode, bool upwind, const StageArgs& a, hipStream_t s);

}  // namespace chemora
