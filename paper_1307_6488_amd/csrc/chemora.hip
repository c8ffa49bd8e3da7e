// chemora.hip -- gfx950 kernels and host ABI of the BSSN right-hand side, the
// RK4 and third-order SSP steps, batched plans, the tuner and the constraint
// kernels (see include/chemora.h for the contract).
//
// Stage kernel: one work-item per interior point.  It evaluates every
// stencil the point needs straight from the stage input (the paper's
// "RHS derivatives" step), the pointwise BSSN algebra ("RHS evaluations"),
// the upwinded advection ("RHS advection") and Kreiss-Oliger dissipation,
// and applies the RK4 stage combination in the same pass, so derivatives
// never travel through HBM (section "Binary Black Hole Simulations", timer
// table; the paper's derivative/RHS split costs bandwidth, section
// "Automated Code Generation with Kranc", "Optimization").
#include <hip/hip_runtime.h>

#include <cctype>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "chemora.h"
#include "fd_ops.hpp"
#include "host_internal.hpp"
#include "stage_common.hpp"
#include "sync.hpp"

namespace chemora {

constexpr int GHOST_THREADS = 256;

// Ghost shells, one work-group per stored row (j, k) of the full extent.
// STATIC: copy the ghosts of `src` into dst0 and dst1.  PERIODIC: fill the
// ghosts of dst0 with periodic images of its own interior.  A row inside the
// y/z ghost layers is a ghost row whole; any other row has 2g ghost points,
// g at each end.  The work-items of a row share out its (grid function,
// point) pairs, points fastest, so all 24 grid functions are in flight at
// once.
template <bool PERIODIC>
__global__ __launch_bounds__(GHOST_THREADS) void ghost_kernel(const double* __restrict__ src, double* dst0,
                                                              double* dst1, Geo G) {
  const int j = blockIdx.x, k = blockIdx.y;
  const int ex = G.nx + 2 * G.g;
  const bool ghost_row = j < G.g || j >= G.ny + G.g || k < G.g || k >= G.nz + G.g;
  const int per_f = ghost_row ? ex : 2 * G.g;
  int jj = j, kk = k;
  if (PERIODIC) {
    jj = ((j - G.g) % G.ny + G.ny) % G.ny + G.g;
    kk = ((k - G.g) % G.nz + G.nz) % G.nz + G.g;
  }
  const int64_t row = (int64_t)k * G.sz + (int64_t)j * G.sy;
  const int64_t srow = (int64_t)kk * G.sz + (int64_t)jj * G.sy;
  for (int t = threadIdx.x; t < 24 * per_f; t += GHOST_THREADS) {
    const int f = t / per_f, c = t - f * per_f;
    const int i = ghost_row ? c : (c < G.g ? c : G.nx + c);
    const int64_t at = f * G.sf + row + i;
    if (PERIODIC) {
      const int ii = ((i - G.g) % G.nx + G.nx) % G.nx + G.g;
      dst0[at] = dst0[f * G.sf + srow + ii];
    } else {
      const double v = src[at];
      dst0[at] = v;
      dst1[at] = v;
    }
  }
}

// Radiative (Sommerfeld) outer boundary: at every ghost point of the stage
// input a.in, the right-hand side of the outgoing-wave condition
//   d_t u = -v (x^i / r) d_i u - v (u - u_inf) / r,   r = |x| (at least h/2),
// with d_i u the second-order centred difference where both neighbours are
// stored points and the second-order one-sided difference into the box
// otherwise; v = rb.vlapse for the lapse and 1 for the rest, u_inf the
// flat-space value, frozen gauge variables 0.  The right-hand side k goes
// through the same stage combination as at interior points:
// out = fma(cs, k, fma(cyo, Y, cu U)), and y = Y + cy k in RK4 stages 1-3.
// One work-group per stored row (j, k), as ghost_kernel.
struct Radiative {
  double origin[3];
  double h;
  double vlapse;
  int frozen_lapse, frozen_shift;
};

__device__ __forceinline__ double rad_diff(const double* p, int64_t s, int c, int e, double inv2h) {
  if (c > 0 && c < e - 1) return (p[s] - p[-s]) * inv2h;
  if (c == 0) return (4.0 * (p[s] - p[0]) - (p[2 * s] - p[0])) * inv2h;
  return -(4.0 * (p[-s] - p[0]) - (p[-2 * s] - p[0])) * inv2h;
}

__global__ __launch_bounds__(GHOST_THREADS) void radiative_kernel(StageArgs a, Radiative rb) {
  const Geo G = a.geo;
  const int j = blockIdx.x, k = blockIdx.y;
  const int ex = G.nx + 2 * G.g, ey = G.ny + 2 * G.g, ez = G.nz + 2 * G.g;
  const bool ghost_row = j < G.g || j >= G.ny + G.g || k < G.g || k >= G.nz + G.g;
  const int per_f = ghost_row ? ex : 2 * G.g;
  const double inv2h = 1.0 / (2.0 * rb.h), half_h = rb.h / 2.0;
  const double y = rb.origin[1] + (double)(j - G.g) * rb.h, z = rb.origin[2] + (double)(k - G.g) * rb.h;
  const int64_t row = (int64_t)k * G.sz + (int64_t)j * G.sy;
  const bool store_y = a.mode == MODE_STAGE1 || a.mode == MODE_STAGE23;
  for (int t = threadIdx.x; t < 24 * per_f; t += GHOST_THREADS) {
    const int f = t / per_f, c = t - f * per_f;
    const int i = ghost_row ? c : (c < G.g ? c : G.nx + c);
    const int64_t at = f * G.sf + row + i;
    const double x = rb.origin[0] + (double)(i - G.g) * rb.h;
    double r = sqrt(x * x + y * y + z * z);
    if (r < half_h) r = half_h;
    const bool frozen = (f == gALPHA && rb.frozen_lapse) || (f >= gBETA && rb.frozen_shift);
    double kf = 0.0;
    if (!frozen) {
      const double* p = a.in + at;
      const double v = f == gALPHA ? rb.vlapse : 1.0;
      const double uinf = (f == gCHI || f == gALPHA || f == gGT || f == gGT + 3 || f == gGT + 5) ? 1.0 : 0.0;
      double xd = x * rad_diff(p, 1, i, ex, inv2h);
      xd += y * rad_diff(p, G.sy, j, ey, inv2h);
      xd += z * rad_diff(p, G.sz, k, ez, inv2h);
      kf = -(v * xd) / r - v * (p[0] - uinf) / r;
    }
    const double Y = a.yin[at], U = a.un[at];
    if (store_y) a.y[at] = Y + a.cy * kf;
    a.out[at] = __builtin_fma(a.cs, kf, __builtin_fma(a.cyo, Y, a.cu * U));
  }
}

// Algebraic constraints det(gt) = 1 and gt^ij At_ij = 0 restored at every
// interior point, one work-item per point (64 x 4 work-groups, x fastest):
// gt_ij <- gt_ij / det(gt)^(1/3), then At_ij <- At_ij - gt_ij tr / 3 with
// tr = gt^kl At_kl of the rescaled metric (its inverse = adjugate / det).
// 12 loads and 12 stores per point, coalesced along x.
__global__ __launch_bounds__(256) void enforce_kernel(double* __restrict__ u, Geo G) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= G.nx || j >= G.ny) return;
  const int64_t at = (int64_t)(k + G.g) * G.sz + (int64_t)(j + G.g) * G.sy + (i + G.g);
  double m[6], A[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    m[s] = u[(gGT + s) * G.sf + at];
    A[s] = u[(gAT + s) * G.sf + at];
  }
  // symmetric slots 0..5 = xx xy xz yy yz zz
  const double det = m[0] * (m[3] * m[5] - m[4] * m[4]) - m[1] * (m[1] * m[5] - m[4] * m[2]) +
                     m[2] * (m[1] * m[4] - m[3] * m[2]);
  const double sc = cbrt(det);
#pragma unroll
  for (int s = 0; s < 6; ++s) m[s] = m[s] / sc;
  const double c00 = m[3] * m[5] - m[4] * m[4], c01 = m[2] * m[4] - m[1] * m[5], c02 = m[1] * m[4] - m[2] * m[3];
  const double c11 = m[0] * m[5] - m[2] * m[2], c12 = m[1] * m[2] - m[0] * m[4], c22 = m[0] * m[3] - m[1] * m[1];
  const double dn = m[0] * c00 + m[1] * c01 + m[2] * c02;
  const double tr = (c00 * A[0] + c11 * A[3] + c22 * A[5] + 2.0 * (c01 * A[1] + c02 * A[2] + c12 * A[4])) / dn;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    u[(gGT + s) * G.sf + at] = m[s];
    u[(gAT + s) * G.sf + at] = A[s] - m[s] * tr / 3.0;
  }
}

// Momentum constraint (a diagnostic, not part of the step), one work-item
// per interior point (64 x 4 work-groups): centred first derivatives of chi,
// gt, K and At read straight from the state (neighbours come from L2), then
//   M_i = gt^jk (d_j At_ki - Gt^l_jk At_li - Gt^l_ji At_kl)
//         - 3/(2 chi) gt^kl At_il d_k chi - 2/3 d_i K
// stored as three grid functions M[i * sf + point].
template <int ORDER>
__global__ __launch_bounds__(256) void momentum_kernel(const double* __restrict__ u, double* __restrict__ M, Geo G,
                                                       double d1s) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= G.nx || j >= G.ny) return;
  // loads as in psi4_kernel: one biased per-lane offset, the grid function
  // and tap offsets in the scalar offset
  const int at = (k + G.g) * (int)G.sz + (j + G.g) * (int)G.sy + (i + G.g);
  const int st[3] = {1, (int)G.sy, (int)G.sz};
  constexpr int R = Stencil<ORDER>::R;
  const int bias = R * ((int)G.sz + (int)G.sy + 1);
  const __amdgpu_buffer_rsrc_t rs = state_rsrc(u, G.sf);
  const unsigned vat = (unsigned)(at - bias + XB) * 8u;
  auto tap = [&](int f, int off) __attribute__((always_inline)) {
    return bload(rs, vat, (unsigned)(f * (unsigned)G.sf + (unsigned)(bias + off)) * 8u);
  };
  auto D = [&](int f, int a) {
    const int s = st[a];
    return Stencil<ORDER>::first([&](int o) { return tap(f, o * s); }) * d1s;
  };
  double g[6], A[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    g[q] = tap(gGT + q, 0);
    A[q] = tap(gAT + q, 0);
  }
  const double chi = tap(gCHI, 0);
  const double c00 = g[3] * g[5] - g[4] * g[4], c01 = g[2] * g[4] - g[1] * g[5], c02 = g[1] * g[4] - g[2] * g[3];
  const double c11 = g[0] * g[5] - g[2] * g[2], c12 = g[1] * g[2] - g[0] * g[4], c22 = g[0] * g[3] - g[1] * g[1];
  const double idet = 1.0 / (g[0] * c00 + g[1] * c01 + g[2] * c02);
  const double gu[6] = {c00 * idet, c01 * idet, c02 * idet, c11 * idet, c12 * idet, c22 * idet};
  // Gt_{m,jk} = 1/2 (d_j gt_mk + d_k gt_mj - d_m gt_jk), then raised
  double dg[3][6];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int q = 0; q < 6; ++q) dg[m][q] = D(gGT + q, m);
  double Gu[3][6];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int jj = SI(q), kk = SJ(q);
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m)
        acc += gu[S(l, m)] * 0.5 * (dg[jj][S(m, kk)] + dg[kk][S(m, jj)] - dg[m][q]);
      Gu[l][q] = acc;
    }
  double dchi[3], dK[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dchi[a] = D(gCHI, a);
    dK[a] = D(gK, a);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        double t = D(gAT + S(kk, a), jj);
#pragma unroll
        for (int l = 0; l < 3; ++l) t -= Gu[l][S(jj, kk)] * A[S(l, a)] + Gu[l][S(jj, a)] * A[S(kk, l)];
        acc += gu[S(jj, kk)] * t;
      }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int l = 0; l < 3; ++l) acc -= 1.5 / chi * gu[S(kk, l)] * A[S(a, l)] * dchi[kk];
    (M + (int64_t)a * G.sf)[at] = acc - (2.0 / 3.0) * dK[a];
  }
}

// Psi4, the Newman-Penrose Weyl scalar of outgoing radiation (a diagnostic
// beside the step: the paper's "Compute Psi4" kernel), one work-item per
// interior point (64 x 4 work-groups), stencils read straight from the state
// (neighbours come from L2).  From the 3+1 data in vacuum:
//   gamma_ij = gt_ij / chi,   K_ij = (At_ij + gt_ij K / 3) / chi,
//   E_ij = R_ij - K_ik K^k_j + K K_ij,   B_ij = sym_ij eps_i^kl D_k K_lj,
// R_ij the physical Ricci tensor of the evolution (conformal Ricci with the
// evolved Gt^i in its d Gt term, plus the chi terms), eps_ijk =
// sqrt(det gamma) [ijk].  Tetrad: Gram-Schmidt in the physical metric of
// v2 = (x, y, z), v3^a = gamma^ad eps_dbc v1^b v2^c, v1 = (-y, x, 0) (in that
// order; v1 = (0, 1, 0) on the z axis, v2 = (0, 0, 1) at the origin) gives
// e_r, e_theta, e_phi, and with mbar = (e_theta - i e_phi)/sqrt 2
//   Psi4 = (E_ij - i B_ij) mbar^i mbar^j
//        = (E_tt - E_pp)/2 - B_tp + i (-E_tp - (B_tt - B_pp)/2),
// stored as out[point] (real part) and out[sf + point] (imaginary part).
// Coordinates: origin + (index - ghost) h.
template <int ORDER>
__global__ __launch_bounds__(256) void psi4_kernel(const double* __restrict__ u, double* __restrict__ out, Geo G,
                                                   double h, double ox, double oy, double oz) {
  using St = Stencil<ORDER>;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= G.nx || j >= G.ny) return;
  // Loads through one buffer resource: the per-lane part of every address is
  // the point (one register, biased by the stencils' reach so that it stays
  // non-negative), the grid function and the tap offset are uniform (scalar
  // offset), so no load needs address arithmetic of its own.
  const int at = (k + G.g) * (int)G.sz + (j + G.g) * (int)G.sy + (i + G.g);
  const int st[3] = {1, (int)G.sy, (int)G.sz};
  const int bias = St::R * ((int)G.sz + (int)G.sy + 1);
  const __amdgpu_buffer_rsrc_t rs = state_rsrc(u, G.sf);
  const unsigned vat = (unsigned)(at - bias + XB) * 8u;
  const double d1s = 1.0 / (St::D1 * h), d2s = 1.0 / (St::D2 * h * h), d11s = d1s * d1s;
  auto tap = [&](int f, int off) __attribute__((always_inline)) {
    return bload(rs, vat, (unsigned)(f * (unsigned)G.sf + (unsigned)(bias + off)) * 8u);
  };
  auto val = [&](int f) { return tap(f, 0); };
  // every derivative is materialised and fenced off by a scheduling barrier:
  // hoisting the loads of all of them ahead (to hide latency) would keep
  // hundreds of values live and spill
  auto fence = [](double& v) __attribute__((always_inline)) {
    keep(v);
    __builtin_amdgcn_sched_barrier(0);
  };
  auto D1 = [&](int f, int a) __attribute__((always_inline)) {
    const int s = st[a];
    double v = St::first([&](int o) { return tap(f, o * s); }) * d1s;
    fence(v);
    return v;
  };
  // second derivative of slot q (xx xy xz yy yz zz); a mixed one is the
  // outer first derivative of inner ones, fenced per inner derivative
  auto D2 = [&](int f, int q) __attribute__((always_inline)) {
    const int a = SI(q), b = SJ(q);
    double v;
    if (a == b) {
      v = St::second([&](int o) { return tap(f, o * st[a]); }) * d2s;
    } else {
      double in[2 * St::R];
#pragma unroll
      for (int k = 1; k <= St::R; ++k) {
        in[St::R - k] = St::first([&](int ob) { return tap(f, -k * st[a] + ob * st[b]); });
        fence(in[St::R - k]);
        in[St::R + k - 1] = St::first([&](int ob) { return tap(f, k * st[a] + ob * st[b]); });
        fence(in[St::R + k - 1]);
      }
      v = St::first([&](int oa) { return oa < 0 ? in[St::R + oa] : in[St::R + oa - 1]; }) * d11s;
    }
    fence(v);
    return v;
  };
  double g[6], A[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    g[q] = val(gGT + q);
    A[q] = val(gAT + q);
  }
  const double chi = val(gCHI), K = val(gK);
  const double c00 = g[3] * g[5] - g[4] * g[4], c01 = g[2] * g[4] - g[1] * g[5], c02 = g[1] * g[4] - g[2] * g[3];
  const double c11 = g[0] * g[5] - g[2] * g[2], c12 = g[1] * g[2] - g[0] * g[4], c22 = g[0] * g[3] - g[1] * g[1];
  const double detg = g[0] * c00 + g[1] * c01 + g[2] * c02;
  const double idet = 1.0 / detg;
  const double gu[6] = {c00 * idet, c01 * idet, c02 * idet, c11 * idet, c12 * idet, c22 * idet};

  // conformal Christoffel symbols: Gl[k][ij] = Gt_{k,ij}, Gu[k][ij] = Gt^k_ij
  double Gl[3][6];
  {
    double dg[3][6];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int q = 0; q < 6; ++q) dg[m][q] = D1(gGT + q, m);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int a = SI(q), b = SJ(q);
        Gl[kk][q] = 0.5 * (dg[b][S(kk, a)] + dg[a][S(kk, b)] - dg[kk][q]);
      }
  }
  double Gu[3][6];
#pragma unroll
  for (int kk = 0; kk < 3; ++kk)
#pragma unroll
    for (int q = 0; q < 6; ++q) Gu[kk][q] = gu[S(kk, 0)] * Gl[0][q] + gu[S(kk, 1)] * Gl[1][q] + gu[S(kk, 2)] * Gl[2][q];
  double Gd[3];
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc += W(q) * gu[q] * Gu[kk][q];
    Gd[kk] = acc;
  }
  double dchi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) dchi[a] = D1(gCHI, a);

  // physical Ricci tensor
  double Ric[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int a = SI(q), b = SJ(q);
    double r = 0.0;
#pragma unroll
    for (int s2 = 0; s2 < 6; ++s2) r -= 0.5 * W(s2) * gu[s2] * D2(gGT + q, s2);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      r += 0.5 * (g[S(kk, a)] * D1(gXT + kk, b) + g[S(kk, b)] * D1(gXT + kk, a));
      r += 0.5 * Gd[kk] * (Gl[a][S(b, kk)] + Gl[b][S(a, kk)]);
    }
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
          r += gu[S(l, m)] * (Gu[kk][S(l, a)] * Gl[b][S(kk, m)] + Gu[kk][S(l, b)] * Gl[a][S(kk, m)] +
                              Gu[kk][S(a, m)] * Gl[kk][S(l, b)]);
    fence(r);
    Ric[q] = r;
  }
  {
    double cdd[6], trc = 0.0, dchi2 = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      cdd[q] = D2(gCHI, q) - (Gu[0][q] * dchi[0] + Gu[1][q] * dchi[1] + Gu[2][q] * dchi[2]);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      trc += W(q) * gu[q] * cdd[q];
      dchi2 += W(q) * gu[q] * dchi[SI(q)] * dchi[SJ(q)];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
      Ric[q] += (cdd[q] + g[q] * trc) / (2.0 * chi) -
                (dchi[SI(q)] * dchi[SJ(q)] + 3.0 * g[q] * dchi2) / (4.0 * chi * chi);
  }

  // physical metric, curvature, electric part
  const double ichi = 1.0 / chi;
  double gam[6], gamu[6], Kd[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    gam[q] = g[q] * ichi;
    gamu[q] = chi * gu[q];
    Kd[q] = (A[q] + g[q] * K * (1.0 / 3.0)) * ichi;
  }
  double Km[3][3];   // K^a_b
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      Km[a][b] = gamu[S(a, 0)] * Kd[S(0, b)] + gamu[S(a, 1)] * Kd[S(1, b)] + gamu[S(a, 2)] * Kd[S(2, b)];
  const double trK = Km[0][0] + Km[1][1] + Km[2][2];
  double Ew[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int a = SI(q), b = SJ(q);
    Ew[q] = Ric[q] - (Kd[S(a, 0)] * Km[0][b] + Kd[S(a, 1)] * Km[1][b] + Kd[S(a, 2)] * Km[2][b]) + trK * Kd[q];
  }

  // magnetic part: D_k K_ij with the physical Christoffel symbols
  // Gamma^m_ij = Gt^m_ij + (gt_ij gt^mn d_n chi - delta^m_i d_j chi - delta^m_j d_i chi) / (2 chi)
  double gudchi[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) gudchi[m] = gu[S(m, 0)] * dchi[0] + gu[S(m, 1)] * dchi[1] + gu[S(m, 2)] * dchi[2];
  auto Gam = [&](int m, int a, int b) {
    double c = g[S(a, b)] * gudchi[m];
    if (m == a) c -= dchi[b];
    if (m == b) c -= dchi[a];
    return Gu[m][S(a, b)] + c * (0.5 * ichi);
  };
  double dK[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) dK[a] = D1(gK, a);
  const double sq = sqrt(detg * ichi * ichi * ichi);   // sqrt(det gamma)
  double Bn[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Bn[a][b] = 0.0;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    // D_k K_lj for this k
    double DK[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int l = SI(q), jj = SJ(q);
      double d = (D1(gAT + q, kk) + D1(gGT + q, kk) * K * (1.0 / 3.0) + g[q] * dK[kk] * (1.0 / 3.0)) * ichi -
                 Kd[q] * dchi[kk] * ichi;
#pragma unroll
      for (int m = 0; m < 3; ++m) d -= Gam(m, kk, l) * Kd[S(m, jj)] + Gam(m, kk, jj) * Kd[S(l, m)];
      fence(d);
      DK[q] = d;
    }
    // eps_a^{kl} = gamma^{kc} gamma^{ld} eps_acd, eps_acd = sq [acd]
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double e = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int pm = (c == d || a == c || a == d) ? 0 : (((c - a + 3) % 3 == 1) ? 1 : -1);
            if (pm) e += double(pm) * gamu[S(kk, c)] * gamu[S(l, d)];
          }
        e *= sq;
#pragma unroll
        for (int b = 0; b < 3; ++b) Bn[a][b] += e * DK[S(l, b)];
      }
  }
  double Bw[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) Bw[q] = 0.5 * (Bn[SI(q)][SJ(q)] + Bn[SJ(q)][SI(q)]);

  // tetrad
  const double x = ox + (double)i * h, y = oy + (double)j * h, z = oz + (double)k * h;
  double v1[3] = {-y, x, 0.0}, v2[3] = {x, y, z};
  if (x == 0.0 && y == 0.0) {
    v1[0] = 0.0;
    v1[1] = 1.0;
    if (z == 0.0) v2[2] = 1.0;
  }
  auto dot = [&](const double* p, const double* q) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc += gam[S(a, b)] * p[a] * q[b];
    return acc;
  };
  double v3[3];
  {
    // eps_dbc v1^b v2^c = sq (v1 x v2)_d, then raised
    const double c0 = sq * (v1[1] * v2[2] - v1[2] * v2[1]);
    const double c1 = sq * (v1[2] * v2[0] - v1[0] * v2[2]);
    const double c2 = sq * (v1[0] * v2[1] - v1[1] * v2[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) v3[a] = gamu[S(a, 0)] * c0 + gamu[S(a, 1)] * c1 + gamu[S(a, 2)] * c2;
  }
  double er[3], et[3], ep[3];
  {
    const double n = 1.0 / sqrt(dot(v2, v2));
#pragma unroll
    for (int a = 0; a < 3; ++a) er[a] = v2[a] * n;
    const double c = dot(v3, er);
#pragma unroll
    for (int a = 0; a < 3; ++a) et[a] = v3[a] - c * er[a];
    const double nt = 1.0 / sqrt(dot(et, et));
#pragma unroll
    for (int a = 0; a < 3; ++a) et[a] *= nt;
    const double cr = dot(v1, er), ct = dot(v1, et);
#pragma unroll
    for (int a = 0; a < 3; ++a) ep[a] = v1[a] - cr * er[a] - ct * et[a];
    const double np = 1.0 / sqrt(dot(ep, ep));
#pragma unroll
    for (int a = 0; a < 3; ++a) ep[a] *= np;
  }
  auto contract = [&](const double* T, const double* p, const double* q) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc += T[S(a, b)] * p[a] * q[b];
    return acc;
  };
  const double Ett = contract(Ew, et, et), Epp = contract(Ew, ep, ep), Etp = contract(Ew, et, ep);
  const double Btt = contract(Bw, et, et), Bpp = contract(Bw, ep, ep), Btp = contract(Bw, et, ep);
  out[at] = 0.5 * (Ett - Epp) - Btp;
  (out + G.sf)[at] = -Etp - 0.5 * (Btt - Bpp);
}

__global__ __launch_bounds__(256) void finite_kernel(const double* __restrict__ u, Geo G,
                                                     unsigned long long* count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= G.nx) return;
  const int64_t idx = (int64_t)(k + G.g) * G.sz + (int64_t)(j + G.g) * G.sy + (i + G.g);
  unsigned int bad = 0;
  for (int f = 0; f < 24; ++f) bad += isfinite(u[f * G.sf + idx]) ? 0u : 1u;
  if (bad) atomicAdd(count, (unsigned long long)bad);
}

}  // namespace chemora

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int required_ghost(int order, int upwind, int ko) {
  if (order != 4 && order != 8) return -1;
  int g = order / 2;
  if (upwind) g = order / 2 + 1;
  return ko > g ? ko : g;
}

int validate(const chemora_params* P, const chemora_patch* X) {
  if (!P) return fail(CHEMORA_EINVAL, "params is NULL");
  if (!X) return fail(CHEMORA_EINVAL, "patch is NULL");
  if (P->fd_order != 4 && P->fd_order != 8)
    return fail(CHEMORA_EINVAL, "fd_order %d not in {4, 8}", P->fd_order);
  if (P->upwind != 0 && P->upwind != 1) return fail(CHEMORA_EINVAL, "upwind must be 0 or 1");
  if (P->ko_radius != 0 && P->ko_radius != 2 && P->ko_radius != 3 && P->ko_radius != 5)
    return fail(CHEMORA_EUNSUPPORTED, "ko_radius %d not in {0, 2, 3, 5}", P->ko_radius);
  const int need = required_ghost(P->fd_order, P->upwind, P->ko_radius);
  if (P->ghost < need)
    return fail(CHEMORA_EINVAL, "ghost %d < %d required by order %d, upwind %d, ko_radius %d", P->ghost,
                need, P->fd_order, P->upwind, P->ko_radius);
  if (!(P->eps_diss >= 0.0) || !std::isfinite(P->eps_diss))
    return fail(CHEMORA_EINVAL, "eps_diss must be finite and >= 0");
  if (P->lapse < 0 || P->lapse > 2) return fail(CHEMORA_EINVAL, "lapse %d unknown", P->lapse);
  if (P->shift < 0 || P->shift > 1) return fail(CHEMORA_EINVAL, "shift %d unknown", P->shift);
  if (!std::isfinite(P->eta)) return fail(CHEMORA_EINVAL, "eta must be finite");
  if (P->bc < CHEMORA_BC_STATIC || P->bc > CHEMORA_BC_RADIATIVE) return fail(CHEMORA_EINVAL, "bc %d unknown", P->bc);
  if (P->precision != CHEMORA_PREC_FP64 && P->precision != CHEMORA_PREC_SPLIT)
    return fail(CHEMORA_EUNSUPPORTED, "precision %d unknown", P->precision);
  if (P->precision == CHEMORA_PREC_SPLIT) {
    if (P->fd_order != 4) return fail(CHEMORA_EUNSUPPORTED, "split precision is built for fd_order 4 only");
    if (!(P->chi_split >= 0.0) || std::isnan(P->chi_split))
      return fail(CHEMORA_EINVAL, "chi_split must be >= 0 (+inf: FP64 chi terms everywhere)");
  }
  for (int a = 0; a < 3; ++a) {
    if (X->n[a] < 1) return fail(CHEMORA_EINVAL, "n[%d] = %d < 1", a, X->n[a]);
    if (P->bc == CHEMORA_BC_PERIODIC && X->n[a] < P->ghost)
      return fail(CHEMORA_EINVAL, "periodic boundary needs n[%d] = %d >= ghost %d", a, X->n[a], P->ghost);
  }
  if (X->reserved != 0) return fail(CHEMORA_EINVAL, "patch.reserved must be 0");
  const int64_t g2 = 2 * (int64_t)P->ghost;
  if (X->sy < X->n[0] + g2) return fail(CHEMORA_EINVAL, "sy %lld < nx + 2g", (long long)X->sy);
  if ((X->n[0] & 1) && X->sy < X->n[0] + g2 + 1)
    return fail(CHEMORA_EINVAL, "sy %lld: odd nx needs one element of row padding (sy >= nx + 2g + 1)",
                (long long)X->sy);
  if (X->sz < X->sy * (X->n[1] + g2)) return fail(CHEMORA_EINVAL, "sz %lld < sy*(ny + 2g)", (long long)X->sz);
  if (X->sf < X->sz * (X->n[2] + g2)) return fail(CHEMORA_EINVAL, "sf %lld < sz*(nz + 2g)", (long long)X->sf);
  // the most tiles any variant makes (32 columns, 4 rows)
  const int64_t tiles = (int64_t)((X->n[0] + 31) / 32) * ((X->n[1] + 3) / 4) * X->n[2];
  if (X->sz > INT32_MAX || tiles > INT32_MAX || X->n[1] + g2 > 65535 || X->n[2] + g2 > 65535)
    return fail(CHEMORA_EINVAL, "patch too large for the launch geometry");
  if (((uint64_t)CHEMORA_NGF * (uint64_t)X->sf + 8) * 8 > 0xFFFFFFFFull)
    return fail(CHEMORA_EUNSUPPORTED, "patch state of %lld bytes exceeds 4 GiB; split it into patches",
                (long long)((uint64_t)CHEMORA_NGF * X->sf * 8));
  if (P->fd_order == 4 && P->ko_radius > 3)
    return fail(CHEMORA_EUNSUPPORTED, "order 4 supports ko_radius <= 3");
  if (!(X->h > 0.0) || !std::isfinite(X->h)) return fail(CHEMORA_EINVAL, "h must be finite and > 0");
  if (P->bc == CHEMORA_BC_RADIATIVE)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(X->origin[a])) return fail(CHEMORA_EINVAL, "radiative boundary needs a finite origin");
  if (!X->u) return fail(CHEMORA_EINVAL, "patch.u is NULL");
  if (((uintptr_t)X->u) % 8) return fail(CHEMORA_EINVAL, "patch.u not 8-byte aligned");
  return CHEMORA_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

chemora::Geo make_geo(const chemora_params* P, const chemora_patch* X) {
  chemora::Geo G;
  G.nx = X->n[0]; G.ny = X->n[1]; G.nz = X->n[2]; G.g = P->ghost;
  G.sy = X->sy; G.sz = X->sz; G.sf = X->sf;
  return G;
}

chemora::Scales make_scales(const chemora_params* P, double h) {
  chemora::Scales s;
  const bool o8 = P->fd_order == 8;
  const double D1 = o8 ? 840.0 : 12.0, D2 = o8 ? 5040.0 : 12.0;
  s.d1 = 1.0 / (D1 * h);
  s.d2 = 1.0 / (D2 * h * h);
  s.d11 = s.d1 * s.d1;
  s.up = 1.0 / (D1 * h);
  s.ko_r = P->ko_radius;
  s.ko = P->ko_radius > 0 ? std::ldexp(P->eps_diss / h, -2 * P->ko_radius) : 0.0;
  // binomial weights of the 2r-th difference in symmetric differences
  static const double kw2[5] = {4.0, -1.0, 0.0, 0.0, 0.0}, kw3[5] = {15.0, -6.0, 1.0, 0.0, 0.0},
                      kw5[5] = {210.0, -120.0, 45.0, -10.0, 1.0};
  const double* kw = P->ko_radius == 2 ? kw2 : (P->ko_radius == 3 ? kw3 : (P->ko_radius == 5 ? kw5 : nullptr));
  for (int k = 0; k < 5; ++k) s.kow[k] = kw ? kw[k] : 0.0;
  return s;
}

// tile planes of tile variant v over nz planes
int tile_planes(int nz, int v) { return (nz + chemora::variant_tz(v) - 1) / chemora::variant_tz(v); }

// tile counts of tile variant v
void set_tiles(chemora::StageArgs& a, int v) {
  a.tiles_x = (a.geo.nx + chemora::VARIANTS[v].tx - 1) / chemora::VARIANTS[v].tx;
  a.tiles_y = (a.geo.ny + chemora::variant_ty(v) - 1) / chemora::variant_ty(v);
}

// single-patch form: one work-group per tile (a's tile counts are set here)
void dispatch_stage(const chemora_params* P, chemora::StageArgs& a, int v, hipStream_t s) {
  chemora::BatchTable none;
  std::memset(&none, 0, sizeof none);
  set_tiles(a, v);
  const int tiles = a.tiles_x * a.tiles_y * tile_planes(a.geo.nz, v);
  if (P->fd_order == 4)
    chemora::launch_stage_o4(v, P->precision == CHEMORA_PREC_SPLIT, false, P->upwind != 0, P->ko_radius, a, none,
                             tiles, s);
  else
    chemora::launch_stage_o8(v, false, P->upwind != 0, P->ko_radius, a, none, tiles, s);
}

// batched form over the plan's tile list: grid work-groups, one per tile
// (bt.queue null, grid = bt.ntiles) or persistent (grid from
// persistent_grid())
void dispatch_batch(const chemora_params* P, int v, const chemora::BatchTable& bt, int grid, hipStream_t s) {
  chemora::StageArgs none;
  std::memset(&none, 0, sizeof none);
  if (P->fd_order == 4)
    chemora::launch_stage_o4(v, P->precision == CHEMORA_PREC_SPLIT, bt.queue != nullptr, P->upwind != 0,
                             P->ko_radius, none, bt, grid, s);
  else
    chemora::launch_stage_o8(v, bt.queue != nullptr, P->upwind != 0, P->ko_radius, none, bt, grid, s);
}

// Work-groups of a persistent stage launch over ntiles tiles of variant v:
// as many as are resident at once on the current device (its CUs times the
// kernel's work-groups per CU, from the occupancy query), a multiple of the
// XCD count when there are that many, never more than the tiles.  0 if the
// device cannot be queried.
int persistent_grid(const chemora_params* P, int v, int ntiles) {
  chemora::StageArgs none;
  std::memset(&none, 0, sizeof none);
  chemora::BatchTable bt;
  std::memset(&bt, 0, sizeof bt);
  int wgs = 0, dev = 0, cus = 0;
  if (P->fd_order == 4)
    chemora::launch_stage_o4(v, P->precision == CHEMORA_PREC_SPLIT, true, P->upwind != 0, P->ko_radius, none, bt,
                             0, nullptr, &wgs);
  else
    chemora::launch_stage_o8(v, true, P->upwind != 0, P->ko_radius, none, bt, 0, nullptr, &wgs);
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (wgs < 1 || cus < 1) return 0;
  int64_t g = std::min<int64_t>((int64_t)wgs * cus, ntiles);
  if (g >= chemora::NXCD) g -= g % chemora::NXCD;
  return (int)g;
}

// how plans created from now on launch their stage kernels
std::atomic<int> g_plan_dispatch{CHEMORA_DISPATCH_AUTO};

// ---------------------------------------------------------------------------
// tile variants: the per-class choice and its cache
// ---------------------------------------------------------------------------
// Patches fall into classes by (GPU architecture, order, upwinding, staged
// reach, precision, x-extent bucket, y-extent bucket); each class maps to a
// tile variant, default_variant() unless tuned, set or loaded.
std::mutex g_tune_mu;
std::map<std::string, int> g_variant;            // class -> variant
std::map<std::string, std::string> g_timing;     // class -> measured times (cache file detail)

std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> known;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = known.find(dev);
  if (it != known.end()) return it->second;
  std::string arch = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  } else {
    (void)hipGetLastError();
  }
  known[dev] = arch;
  return arch;
}

int bucket(int n, const int* edges, int ne) {
  int b = 0;
  while (b < ne && n > edges[b]) ++b;
  return b;
}

std::string class_key(const chemora_params* P, const chemora_patch* X) {
  static const int xe[] = {32, 64, 96, 128};   // x extent: <=32 <=64 <=96 <=128 >128
  static const int ye[] = {16, 32, 64};        // y extent: <=16 <=32 <=64 >64
  char buf[192];
  std::snprintf(buf, sizeof buf, "%s/o%d/u%d/r%d/%s/x%d/y%d", device_arch().c_str(), P->fd_order,
                P->upwind ? 1 : 0, required_ghost(P->fd_order, P->upwind, P->ko_radius),
                P->precision == CHEMORA_PREC_SPLIT ? "split" : "fp64", bucket(X->n[0], xe, 4),
                bucket(X->n[1], ye, 3));
  return buf;
}

// Variant of a class nobody tuned or set: 32 x 8 for both orders (order 4:
// within 3 % of the fastest, 32 x 16, at 128^3 and 256^3 and without its
// ragged-tile waste on small patches; order 8: fastest at 192^3, 6.4 ms per
// stage-2 launch against 7.2 ms for 64 x 4, measured on MI355X).
int default_variant(const chemora_params*) { return 2; }

int choose_variant(const chemora_params* P, const chemora_patch* X) {
  const std::string key = class_key(P, X);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_variant.find(key);
  return (it != g_variant.end() && chemora::variant_supported(P->fd_order, it->second)) ? it->second
                                                                                      : default_variant(P);
}

std::string variant_name(int v) {
  std::string n = std::to_string(chemora::VARIANTS[v].tx) + "x" + std::to_string(chemora::variant_ty(v));
  if (chemora::variant_tz(v) > 1) n += "x" + std::to_string(chemora::variant_tz(v));
  return n;
}

// Reads a cache file (the JSON save_cache writes, in any whitespace layout):
// every object member  "<class>": { ... "variant": <v> ... }  becomes a table
// entry.  Entries already in the table (tuned or set in this process) win.
void load_cache(const char* path) {
  std::ifstream in(path);
  if (!in) return;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string text = ss.str();
  auto skip = [&](size_t i) {
    while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
    return i;
  };
  std::string key;                     // the member whose object is open
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (size_t i = 0; i < text.size(); ++i) {
    if (text[i] != '"') continue;
    const size_t end = text.find('"', i + 1);
    if (end == std::string::npos) break;
    const std::string str = text.substr(i + 1, end - i - 1);
    size_t k = skip(end + 1);
    i = end;
    if (k >= text.size() || text[k] != ':') continue;
    k = skip(k + 1);
    if (k < text.size() && text[k] == '{') {
      key = str;
    } else if (str == "variant" && !key.empty()) {
      char* stop = nullptr;
      const long v = std::strtol(text.c_str() + k, &stop, 10);
      if (stop != text.c_str() + k && v >= 0 && v < chemora::NVARIANT && !g_variant.count(key)) g_variant[key] = (int)v;
    }
  }
}

int save_cache(const char* path) {
  std::ostringstream o;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    o << "{\n  \"format\": \"chemora tile-variant cache\",\n  \"version\": 1,\n  \"entries\": {\n";
    size_t i = 0;
    for (const auto& kv : g_variant) {
      o << "    \"" << kv.first << "\": {\"variant\": " << kv.second << ", \"tile\": \"" << variant_name(kv.second)
        << "\"";
      auto t = g_timing.find(kv.first);
      if (t != g_timing.end()) o << ", \"ms\": {" << t->second << "}";
      o << "}" << (++i < g_variant.size() ? "," : "") << "\n";
    }
    o << "  }\n}\n";
  }
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out || !(out << o.str()) || !out.flush()) return fail(CHEMORA_EINVAL, "cannot write %s", tmp.c_str());
  }
  if (std::rename(tmp.c_str(), path) != 0) return fail(CHEMORA_EINVAL, "cannot rename %s to %s", tmp.c_str(), path);
  return CHEMORA_OK;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return CHEMORA_OK;
}

chemora::StageArgs base_args(const chemora_params* P, const chemora_patch* X) {
  chemora::StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.geo = make_geo(P, X);
  a.sc = make_scales(P, X->h);
  a.gauge.lapse = P->lapse;
  a.gauge.shift = P->shift;
  a.gauge.eta = P->eta;
  a.chi_split = P->precision == CHEMORA_PREC_SPLIT ? P->chi_split : 0.0;
  set_tiles(a, 0);
  return a;
}

void launch_ghosts(bool periodic, const chemora::Geo& G, const double* src, double* d0, double* d1,
                   hipStream_t s) {
  dim3 grid(G.ny + 2 * G.g, G.nz + 2 * G.g, 1);
  if (periodic)
    hipLaunchKernelGGL((chemora::ghost_kernel<true>), grid, dim3(chemora::GHOST_THREADS), 0, s, src, d0, d1, G);
  else
    hipLaunchKernelGGL((chemora::ghost_kernel<false>), grid, dim3(chemora::GHOST_THREADS), 0, s, src, d0, d1, G);
}

// the radiative boundary of a stage whose arguments are a (bc RADIATIVE only)
void launch_radiative(const chemora_params* P, const chemora_patch* X, const chemora::StageArgs& a,
                      hipStream_t s) {
  chemora::Radiative rb;
  for (int d = 0; d < 3; ++d) rb.origin[d] = X->origin[d];
  rb.h = X->h;
  rb.vlapse = P->lapse == CHEMORA_LAPSE_ONE_PLUS_LOG ? std::sqrt(2.0) : 1.0;
  rb.frozen_lapse = P->lapse == CHEMORA_LAPSE_FROZEN;
  rb.frozen_shift = P->shift == CHEMORA_SHIFT_FROZEN;
  dim3 grid(a.geo.ny + 2 * a.geo.g, a.geo.nz + 2 * a.geo.g, 1);
  hipLaunchKernelGGL(chemora::radiative_kernel, grid, dim3(chemora::GHOST_THREADS), 0, s, a, rb);
}

}  // namespace

extern "C" {

int chemora_abi_version(void) { return 103; }

const char* chemora_last_error(void) { return g_error.c_str(); }

int chemora_required_ghost(int fd_order, int upwind, int ko_radius) {
  return required_ghost(fd_order, upwind, ko_radius);
}

size_t chemora_rk4_scratch_elems(const chemora_patch* patch) {
  if (!patch || patch->sf <= 0) return 0;
  return (size_t)3 * CHEMORA_NGF * (size_t)patch->sf;
}

int chemora_bssn_rhs(const chemora_params* params, const chemora_patch* patch, double* rhs, void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!rhs) return fail(CHEMORA_EINVAL, "rhs is NULL");
  if (((uintptr_t)rhs) % 8) return fail(CHEMORA_EINVAL, "rhs not 8-byte aligned");
  const size_t bytes = (size_t)CHEMORA_NGF * patch->sf * sizeof(double);
  if (overlap(rhs, bytes, patch->u, bytes)) return fail(CHEMORA_EINVAL, "rhs overlaps patch.u");
  chemora::StageArgs a = base_args(params, patch);
  a.in = a.un = a.yin = patch->u;
  a.out = rhs;
  a.cu = 0.0;
  a.cs = 1.0;
  a.mode = chemora::MODE_RHS;
  dispatch_stage(params, a, choose_variant(params, patch), (hipStream_t)stream);
  if (params->bc == CHEMORA_BC_RADIATIVE) launch_radiative(params, patch, a, (hipStream_t)stream);
  return check_launch("bssn_rhs");
}

int chemora_hamiltonian(const chemora_params* params, const chemora_patch* patch, double* H, void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!H) return fail(CHEMORA_EINVAL, "H is NULL");
  if (((uintptr_t)H) % 8) return fail(CHEMORA_EINVAL, "H not 8-byte aligned");
  const size_t bytes = (size_t)CHEMORA_NGF * patch->sf * sizeof(double);
  if (overlap(H, patch->sf * sizeof(double), patch->u, bytes)) return fail(CHEMORA_EINVAL, "H overlaps patch.u");
  chemora::StageArgs a = base_args(params, patch);
  a.in = a.un = a.yin = patch->u;
  a.y = a.out = H;
  a.mode = chemora::MODE_HAM;
  dispatch_stage(params, a, choose_variant(params, patch), (hipStream_t)stream);
  return check_launch("hamiltonian");
}

}  // extern "C"

namespace {

// checks of a Runge-Kutta call whose scratch holds nstates states
int rk_checks(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch, int nstates) {
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CHEMORA_EINVAL, "dt must be finite and > 0");
  if (!scratch) return fail(CHEMORA_EINVAL, "scratch is NULL");
  if (((uintptr_t)scratch) % 8) return fail(CHEMORA_EINVAL, "scratch not 8-byte aligned");
  const size_t state = (size_t)CHEMORA_NGF * patch->sf;
  if (overlap(scratch, nstates * state * sizeof(double), patch->u, state * sizeof(double)))
    return fail(CHEMORA_EINVAL, "scratch overlaps patch.u");
  return CHEMORA_OK;
}

int rk4_checks(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch) {
  return rk_checks(params, patch, dt, scratch, 3);
}

// Arguments of RK4 stage `stage` (1-4).  Buffers: u = u_n (overwritten by
// stage 4), SA/SB stage inputs, Y accumulator.
//   1: Y = u + dt/6 k1(u),  SA = u + dt/2 k1      3: Y += dt/3 k3(SB), SA = u + dt k3
//   2: Y += dt/3 k2(SA),    SB = u + dt/2 k2      4: u = Y + dt/6 k4(SA)
// Returns the buffer the stage writes.
double* stage_args(chemora::StageArgs& a, int stage, double dt, double* u, double* SA, double* SB, double* Y) {
  a.y = Y;
  a.cu = 1.0;
  switch (stage) {
    case 1:
      a.in = u; a.un = u; a.yin = u; a.out = SA; a.cy = dt / 6.0; a.cs = 0.5 * dt;
      a.mode = chemora::MODE_STAGE1;
      return SA;
    case 2:
      a.in = SA; a.un = u; a.yin = Y; a.out = SB; a.cy = dt / 3.0; a.cs = 0.5 * dt;
      a.mode = chemora::MODE_STAGE23;
      return SB;
    case 3:
      a.in = SB; a.un = u; a.yin = Y; a.out = SA; a.cy = dt / 3.0; a.cs = dt;
      a.mode = chemora::MODE_STAGE23;
      return SA;
    default:
      a.in = SA; a.un = Y; a.yin = Y; a.out = u; a.cy = dt / 6.0; a.cs = dt / 6.0;
      a.mode = chemora::MODE_STAGE4;
      return u;
  }
}

// Arguments of stage `stage` (1-3) of the third-order strong-stability-
// preserving Runge-Kutta scheme of Shu and Osher.  Buffers: u = u_n
// (overwritten by stage 3, each point read and written by its own
// work-item only), SA/SB stage inputs.
//   1: SA = u + dt k(u)
//   2: SB = 3/4 u + 1/4 SA + dt/4 k(SA)
//   3: u  = 1/3 u + 2/3 SB + 2 dt/3 k(SB)
// Returns the buffer the stage writes.
double* rk3_stage_args(chemora::StageArgs& a, int stage, double dt, double* u, double* SA, double* SB) {
  a.mode = chemora::MODE_RK3;
  a.un = u;
  switch (stage) {
    case 1:
      a.in = u; a.yin = u; a.out = SA; a.cu = 1.0; a.cyo = 0.0; a.cs = dt;
      break;
    case 2:
      a.in = SA; a.yin = SA; a.out = SB; a.cu = 0.75; a.cyo = 0.25; a.cs = 0.25 * dt;
      break;
    default:
      a.in = SB; a.yin = SB; a.out = u; a.cu = 1.0 / 3.0; a.cyo = 2.0 / 3.0; a.cs = dt * (2.0 / 3.0);
      break;
  }
  a.y = a.out;   // not written in this mode
  return a.out;
}

int rk4_stage(const chemora_params* params, const chemora_patch* patch, int stage, double dt, double* scratch,
              hipStream_t s) {
  if (stage < 1 || stage > 4) return fail(CHEMORA_EINVAL, "stage %d not in 1..4", stage);
  const size_t state = (size_t)CHEMORA_NGF * patch->sf;
  double* u = patch->u;
  double* SA = scratch;
  double* SB = scratch + state;
  double* Y = scratch + 2 * state;
  const bool periodic = params->bc == CHEMORA_BC_PERIODIC;
  chemora::StageArgs a = base_args(params, patch);
  if (stage == 1 && params->bc == CHEMORA_BC_STATIC) launch_ghosts(false, a.geo, u, SA, SB, s);
  double* written = stage_args(a, stage, dt, u, SA, SB, Y);
  dispatch_stage(params, a, choose_variant(params, patch), s);
  if (periodic) launch_ghosts(true, a.geo, nullptr, written, nullptr, s);
  if (params->bc == CHEMORA_BC_RADIATIVE) launch_radiative(params, patch, a, s);
  return check_launch("rk4 stage");
}

}  // namespace

namespace chemora {
namespace host {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

void clear_error() { g_error.clear(); }

int check_step(const chemora_params* params, const chemora_patch* patch, double dt) {
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt)) return ::fail(CHEMORA_EINVAL, "dt must be finite and > 0");
  return CHEMORA_OK;
}

int rk4_step(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch, hipStream_t s) {
  int rc;
  for (int st = 1; st <= 4; ++st)
    if ((rc = rk4_stage(params, patch, st, dt, scratch, s))) return rc;
  return CHEMORA_OK;
}

}  // namespace host
}  // namespace chemora

// Scratch of chemora_rk4_step_noalloc: S_A, S_B and the accumulator Y of
// one patch, in a device array loaded with the code object (no allocation
// call).  Host code never passes the array's name to a kernel -- on the host
// it is only a stand-in for the symbol -- but the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current (each GPU holds its own copy at its own address).
static __device__ __align__(256) double noalloc_scratch_array[CHEMORA_NOALLOC_SCRATCH_ELEMS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of the current device's copy of noalloc_scratch_array
int noalloc_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "rk4_step_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(CHEMORA_EDEVICE, "rk4_step_noalloc: device %d beyond the %d supported", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch_array));
    if (e != hipSuccess || !p)
      return fail(CHEMORA_EDEVICE, "rk4_step_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return CHEMORA_OK;
}

}  // namespace

extern "C" {

int chemora_rk4_step(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch,
                     void* stream) {
  g_error.clear();
  int rc = rk4_checks(params, patch, dt, scratch);
  if (rc) return rc;
  return chemora::host::rk4_step(params, patch, dt, scratch, (hipStream_t)stream);
}

int chemora_rk4_step_noalloc(const chemora_params* params, const chemora_patch* patch, double dt, void* stream) {
  g_error.clear();
  int rc = chemora::host::check_step(params, patch, dt);
  if (rc) return rc;
  const size_t need = chemora_rk4_scratch_elems(patch);
  if (need > CHEMORA_NOALLOC_SCRATCH_ELEMS)
    return fail(CHEMORA_EINVAL, "rk4_step_noalloc: the patch needs %zu doubles of scratch, more than the %zu held "
                "per GPU (chemora_rk4_step takes a caller's scratch of any size)",
                need, (size_t)CHEMORA_NOALLOC_SCRATCH_ELEMS);
  double* scratch = nullptr;
  if ((rc = noalloc_scratch(&scratch))) return rc;
  return chemora::host::rk4_step(params, patch, dt, scratch, (hipStream_t)stream);
}

size_t chemora_rk3_scratch_elems(const chemora_patch* patch) {
  if (!patch || patch->sf <= 0) return 0;
  return (size_t)2 * CHEMORA_NGF * (size_t)patch->sf;
}

int chemora_rk3_step(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch,
                     void* stream) {
  g_error.clear();
  int rc = rk_checks(params, patch, dt, scratch, 2);
  if (rc) return rc;
  const size_t state = (size_t)CHEMORA_NGF * patch->sf;
  double* u = patch->u;
  double* SA = scratch;
  double* SB = scratch + state;
  hipStream_t s = (hipStream_t)stream;
  const bool periodic = params->bc == CHEMORA_BC_PERIODIC;
  const int v = choose_variant(params, patch);
  for (int st = 1; st <= 3; ++st) {
    chemora::StageArgs a = base_args(params, patch);
    if (st == 1 && params->bc == CHEMORA_BC_STATIC) launch_ghosts(false, a.geo, u, SA, SB, s);
    double* written = rk3_stage_args(a, st, dt, u, SA, SB);
    dispatch_stage(params, a, v, s);
    if (periodic) launch_ghosts(true, a.geo, nullptr, written, nullptr, s);
    if (params->bc == CHEMORA_BC_RADIATIVE) launch_radiative(params, patch, a, s);
    if ((rc = check_launch("rk3 stage"))) return rc;
  }
  return CHEMORA_OK;
}

int chemora_rk4_stage(const chemora_params* params, const chemora_patch* patch, int stage, double dt,
                      double* scratch, void* stream) {
  g_error.clear();
  int rc = rk4_checks(params, patch, dt, scratch);
  if (rc) return rc;
  if (stage < 1 || stage > 4) return fail(CHEMORA_EINVAL, "stage %d not in 1..4", stage);
  return rk4_stage(params, patch, stage, dt, scratch, (hipStream_t)stream);
}

int chemora_momentum_constraint(const chemora_params* params, const chemora_patch* patch, double* M,
                                void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!M) return fail(CHEMORA_EINVAL, "M is NULL");
  if (((uintptr_t)M) % 8) return fail(CHEMORA_EINVAL, "M not 8-byte aligned");
  const size_t bytes = (size_t)CHEMORA_NGF * patch->sf * sizeof(double);
  if (overlap(M, 3 * patch->sf * sizeof(double), patch->u, bytes)) return fail(CHEMORA_EINVAL, "M overlaps patch.u");
  const chemora::Geo G = make_geo(params, patch);
  const double d1s = 1.0 / ((params->fd_order == 8 ? 840.0 : 12.0) * patch->h);
  hipStream_t s = (hipStream_t)stream;
  dim3 grid((G.nx + 63) / 64, (G.ny + 3) / 4, G.nz);
  if (params->fd_order == 8)
    hipLaunchKernelGGL(chemora::momentum_kernel<8>, grid, dim3(64, 4), 0, s, patch->u, M, G, d1s);
  else
    hipLaunchKernelGGL(chemora::momentum_kernel<4>, grid, dim3(64, 4), 0, s, patch->u, M, G, d1s);
  return check_launch("momentum_constraint");
}

int chemora_psi4(const chemora_params* params, const chemora_patch* patch, double* psi4, void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!psi4) return fail(CHEMORA_EINVAL, "psi4 is NULL");
  if (((uintptr_t)psi4) % 8) return fail(CHEMORA_EINVAL, "psi4 not 8-byte aligned");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(patch->origin[a])) return fail(CHEMORA_EINVAL, "psi4 needs a finite origin");
  const size_t bytes = (size_t)CHEMORA_NGF * patch->sf * sizeof(double);
  if (overlap(psi4, 2 * patch->sf * sizeof(double), patch->u, bytes))
    return fail(CHEMORA_EINVAL, "psi4 overlaps patch.u");
  const chemora::Geo G = make_geo(params, patch);
  hipStream_t s = (hipStream_t)stream;
  dim3 grid((G.nx + 63) / 64, (G.ny + 3) / 4, G.nz);
  const double* o = patch->origin;
  if (params->fd_order == 8)
    hipLaunchKernelGGL(chemora::psi4_kernel<8>, grid, dim3(64, 4), 0, s, patch->u, psi4, G, patch->h, o[0], o[1],
                       o[2]);
  else
    hipLaunchKernelGGL(chemora::psi4_kernel<4>, grid, dim3(64, 4), 0, s, patch->u, psi4, G, patch->h, o[0], o[1],
                       o[2]);
  return check_launch("psi4");
}

int chemora_enforce_constraints(const chemora_params* params, const chemora_patch* patch, void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  const chemora::Geo G = make_geo(params, patch);
  hipStream_t s = (hipStream_t)stream;
  dim3 grid((G.nx + 63) / 64, (G.ny + 3) / 4, G.nz);
  hipLaunchKernelGGL(chemora::enforce_kernel, grid, dim3(64, 4), 0, s, patch->u, G);
  if (params->bc == CHEMORA_BC_PERIODIC) launch_ghosts(true, G, nullptr, patch->u, nullptr, s);
  return check_launch("enforce_constraints");
}

int chemora_check_finite(const chemora_params* params, const chemora_patch* patch, int64_t* bad_count,
                         void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!bad_count) return fail(CHEMORA_EINVAL, "bad_count is NULL");
  const chemora::Geo G = make_geo(params, patch);
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  if (hipMallocAsync((void**)&d, sizeof *d, s) != hipSuccess) return fail(CHEMORA_EDEVICE, "hipMallocAsync failed");
  hipError_t e = hipMemsetAsync(d, 0, sizeof *d, s);
  dim3 grid((G.nx + 255) / 256, G.ny, G.nz);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(chemora::finite_kernel, grid, dim3(256), 0, s, patch->u, G, d);
    e = hipGetLastError();
  }
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, s);
  const hipError_t ef = hipFreeAsync(d, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "check_finite: %s", hipGetErrorString(e));
  *bad_count = (int64_t)h;
  return h ? fail(CHEMORA_ENOTFINITE, "%llu non-finite interior values", h) : CHEMORA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner (tile variants)
// ---------------------------------------------------------------------------
namespace {

// Times every tile variant built for the patch's order on a stage-2 launch
// of the patch itself (reads u and S_A, writes S_B and Y of `scratch`): one
// warm-up and three timed launches each, HIP events on `s`.  Synchronous.
int time_variants(const chemora_params* P, const chemora_patch* X, double* scratch, hipStream_t s, int* best,
                  std::string* timing) {
  const size_t state = (size_t)CHEMORA_NGF * X->sf;
  chemora::StageArgs a = base_args(P, X);
  stage_args(a, 2, X->h * 0.25, X->u, scratch, scratch + state, scratch + 2 * state);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // one warm-up launch per variant, then rounds that time every variant in
  // turn (2 launches per sample) and keep each variant's fastest sample, so
  // that clock ramps and stray interference do not favour one variant
  constexpr int ROUNDS = 3, PER_SAMPLE = 2;
  float ms_v[chemora::NVARIANT];
  for (int v = 0; v < chemora::NVARIANT; ++v) ms_v[v] = -1.0f;
  for (int v = 0; v < chemora::NVARIANT && e == hipSuccess; ++v)
    if (chemora::variant_supported(P->fd_order, v)) dispatch_stage(P, a, v, s);
  for (int r = 0; r < ROUNDS && e == hipSuccess; ++r) {
    for (int v = 0; v < chemora::NVARIANT && e == hipSuccess; ++v) {
      if (!chemora::variant_supported(P->fd_order, v)) continue;
      e = hipEventRecord(e0, s);
      for (int k = 0; k < PER_SAMPLE && e == hipSuccess; ++k) dispatch_stage(P, a, v, s);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      ms /= PER_SAMPLE;
      if (ms_v[v] < 0.0f || ms < ms_v[v]) ms_v[v] = ms;
    }
  }
  float best_ms = 0.0f;
  *best = -1;
  std::ostringstream t;
  for (int v = 0; v < chemora::NVARIANT && e == hipSuccess; ++v) {
    if (ms_v[v] < 0.0f) continue;
    char buf[64];
    std::snprintf(buf, sizeof buf, "%s\"%s\": %.4f", t.tellp() > 0 ? ", " : "", variant_name(v).c_str(), ms_v[v]);
    t << buf;
    if (*best < 0 || ms_v[v] < best_ms) {
      best_ms = ms_v[v];
      *best = v;
    }
  }
  if (*best < 0) *best = 0;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "tuning: %s", hipGetErrorString(e));
  *timing = t.str();
  return CHEMORA_OK;
}

// The patch's class: its cached / set variant, else timed now (and recorded).
int tune_class(const chemora_params* P, const chemora_patch* X, double* scratch, hipStream_t s, int* variant) {
  const std::string key = class_key(P, X);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_variant.find(key);
    if (it != g_variant.end() && chemora::variant_supported(P->fd_order, it->second)) {
      *variant = it->second;
      return CHEMORA_OK;
    }
  }
  std::string timing;
  int rc = time_variants(P, X, scratch, s, variant, &timing);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_variant[key] = *variant;
  g_timing[key] = timing;
  return CHEMORA_OK;
}

}  // namespace

extern "C" {

int chemora_tune(const chemora_params* params, const chemora_patch* patch, double* scratch,
                 const char* cache_path, void* stream, int32_t* variant) {
  g_error.clear();
  int rc = rk4_checks(params, patch, 1.0, scratch);
  if (rc) return rc;
  if (cache_path) load_cache(cache_path);
  int v = 0;
  if ((rc = tune_class(params, patch, scratch, (hipStream_t)stream, &v))) return rc;
  if (cache_path && (rc = save_cache(cache_path))) return rc;
  if (variant) *variant = v;
  return CHEMORA_OK;
}

int chemora_tile_variant(const chemora_params* params, const chemora_patch* patch) {
  g_error.clear();
  int rc = validate(params, patch);
  return rc ? rc : choose_variant(params, patch);
}

int chemora_set_tile_variant(const chemora_params* params, const chemora_patch* patch, int32_t variant) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (variant < 0 || variant >= chemora::NVARIANT) return fail(CHEMORA_EINVAL, "tile variant %d unknown", variant);
  if (!chemora::variant_supported(params->fd_order, variant))
    return fail(CHEMORA_EUNSUPPORTED, "tile variant %d not built for order %d", variant, params->fd_order);
  const std::string key = class_key(params, patch);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_variant[key] = variant;
  g_timing.erase(key);
  return CHEMORA_OK;
}

int chemora_tile_variant_shape(int32_t variant, int32_t* tile_x, int32_t* tile_y) {
  g_error.clear();
  if (variant < 0 || variant >= chemora::NVARIANT) return fail(CHEMORA_EINVAL, "tile variant %d unknown", variant);
  if (tile_x) *tile_x = chemora::VARIANTS[variant].tx;
  if (tile_y) *tile_y = chemora::variant_ty(variant);
  return CHEMORA_OK;
}

int chemora_tile_variant_depth(int32_t variant) {
  g_error.clear();
  if (variant < 0 || variant >= chemora::NVARIANT) return fail(CHEMORA_EINVAL, "tile variant %d unknown", variant);
  return chemora::variant_tz(variant);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// plans (batched form)
// ---------------------------------------------------------------------------
// The plan's patches are grouped by tile variant; per RK stage every group
// is one launch over the concatenated tiles of its patches.
struct PlanGroup {
  int variant;
  int first;       // first entry of the group in the stage tables
  int count;       // patches
  int ntiles;
  int toff;        // offset of its tile-start prefix sums (count + 1 entries)
  int grid;        // work-groups per launch: ntiles, or the persistent grid
};

struct chemora_plan {
  chemora_params params;
  int npatch = 0;
  int64_t points = 0;
  std::vector<PlanGroup> groups;
  std::vector<int> variant_of;                    // per patch (caller's order)
  chemora::StageArgs* d_args = nullptr;           // 4 (RK4) or 3 (RK3) stage tables of npatch entries, group order
  int* d_tile_start = nullptr;
  int dispatch = CHEMORA_DISPATCH_PERSISTENT;
  int* d_queue = nullptr;                         // persistent: QUEUE_INTS counters per stage and group
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // synchronised plans: ghost refill / restriction maps and their buffers
  bool synced = false;
  std::vector<int> fill_start, fill_copies, restr_start;
  chemora::SyncItem* d_fill = nullptr;
  chemora::SyncItem* d_restr = nullptr;
  chemora::SyncGeo* d_geo = nullptr;
  double** d_bufs = nullptr;                      // per stage, npatch state pointers (caller's order); then u
};

namespace {

void plan_free(chemora_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->capture) {
    (void)hipStreamSynchronize(pl->capture);
    (void)hipStreamDestroy(pl->capture);
  }
  if (pl->d_args) (void)hipFree(pl->d_args);
  if (pl->d_tile_start) (void)hipFree(pl->d_tile_start);
  if (pl->d_queue) (void)hipFree(pl->d_queue);
  if (pl->d_fill) (void)hipFree(pl->d_fill);
  if (pl->d_restr) (void)hipFree(pl->d_restr);
  if (pl->d_geo) (void)hipFree(pl->d_geo);
  if (pl->d_bufs) (void)hipFree(pl->d_bufs);
  delete pl;
}

}  // namespace

namespace {

// Time of one RK4 stage-2 pass over all patches of a plan with tile variants
// var[p]: the patches grouped by variant, one batched launch per group, the
// groups one after another as in the plan's graph.  One warm-up pass, then
// the fastest of three samples of two passes (as the per-class tuner).
// Overwrites the S_B and accumulator parts of scratch.
int plan_pass_ms(const chemora_params* P, const chemora_patch* X, double* const* scratch, int npatch,
                 const std::vector<int>& var, int dispatch, hipStream_t s, float* best_ms) {
  std::vector<int> order(npatch);
  for (int p = 0; p < npatch; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return var[x] < var[y]; });
  std::vector<chemora::StageArgs> args(npatch);
  std::vector<int> starts;
  std::vector<PlanGroup> groups;
  for (int r = 0; r < npatch;) {
    PlanGroup g{var[order[r]], r, 0, 0, (int)starts.size(), 0};
    starts.push_back(0);
    int64_t tiles = 0;
    for (; r < npatch && var[order[r]] == g.variant; ++r) {
      const chemora_patch* Y = &X[order[r]];
      const size_t state = (size_t)CHEMORA_NGF * Y->sf;
      chemora::StageArgs a = base_args(P, Y);
      set_tiles(a, g.variant);
      tiles += (int64_t)a.tiles_x * a.tiles_y * tile_planes(a.geo.nz, g.variant);
      if (tiles > INT32_MAX) return fail(CHEMORA_EINVAL, "too many tiles in the plan");
      starts.push_back((int)tiles);
      double* sc = scratch[order[r]];
      stage_args(a, 2, Y->h * 0.25, Y->u, sc, sc + state, sc + 2 * state);
      args[r] = a;
      ++g.count;
    }
    g.ntiles = (int)tiles;
    g.grid = dispatch == CHEMORA_DISPATCH_PERSISTENT ? persistent_grid(P, g.variant, g.ntiles) : g.ntiles;
    if (g.grid < 1) return fail(CHEMORA_EDEVICE, "plan tuning: occupancy or device query failed");
    groups.push_back(g);
  }
  chemora::StageArgs* d_args = nullptr;
  int* d_starts = nullptr;
  int* d_queue = nullptr;   // one set of counters: the launches run one after another
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&d_args, args.size() * sizeof(chemora::StageArgs));
  if (e == hipSuccess) e = hipMalloc((void**)&d_starts, starts.size() * sizeof(int));
  if (e == hipSuccess && dispatch == CHEMORA_DISPATCH_PERSISTENT)
    e = hipMalloc((void**)&d_queue, chemora::QUEUE_INTS * sizeof(int));
  if (e == hipSuccess && d_queue) e = hipMemsetAsync(d_queue, 0, chemora::QUEUE_INTS * sizeof(int), s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_args, args.data(), args.size() * sizeof(chemora::StageArgs), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_starts, starts.data(), starts.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto pass = [&]() {
    for (const PlanGroup& g : groups) {
      chemora::BatchTable bt;
      bt.args = d_args + g.first;
      bt.tile_start = d_starts + g.toff;
      bt.queue = d_queue;
      bt.npatch = g.count;
      bt.ntiles = g.ntiles;
      dispatch_batch(P, g.variant, bt, g.grid, s);
    }
  };
  constexpr int ROUNDS = 3, PER_SAMPLE = 2;
  *best_ms = -1.0f;
  if (e == hipSuccess) {
    pass();
    e = hipGetLastError();
  }
  for (int r = 0; r < ROUNDS && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    for (int k = 0; k < PER_SAMPLE && e == hipSuccess; ++k) pass();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (*best_ms < 0.0f || ms / PER_SAMPLE < *best_ms)) *best_ms = ms / PER_SAMPLE;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d_args) (void)hipFree(d_args);
  if (d_starts) (void)hipFree(d_starts);
  if (d_queue) (void)hipFree(d_queue);
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "plan tuning: %s", hipGetErrorString(e));
  return CHEMORA_OK;
}

// A plan capturing one step of RK4 (4 stages) or of the third-order SSP
// scheme (3 stages); scratch holds 3 states per patch either way (the
// tuner times RK4 stage-2 launches in it).
// Restriction (if asked, finest level pair first) and the ghost refill of
// every level, coarsest first, of the states bufs[0 .. npatch) (device table).
void plan_restrict_and_fill(const chemora_plan* pl, double* const* bufs, bool restrict_first, hipStream_t s) {
  const int order = pl->params.fd_order;
  if (restrict_first)
    for (size_t q = 0; q + 1 < pl->restr_start.size(); ++q) {
      const int n = pl->restr_start[q + 1] - pl->restr_start[q];   // all copies
      chemora::launch_sync(order, pl->d_restr + pl->restr_start[q], n, n, bufs, pl->d_geo, s);
    }
  for (size_t L = 0; L + 1 < pl->fill_start.size(); ++L)
    chemora::launch_sync(order, pl->d_fill + pl->fill_start[L], pl->fill_start[L + 1] - pl->fill_start[L],
                         pl->fill_copies[L], bufs, pl->d_geo, s);
}

// dt_all > 0: a synchronised plan -- every patch steps with dt_all and the
// ghosts are exchanged between patches (sync.hpp); else dt = courant * h per
// patch and the patches are independent.
int plan_create(const chemora_params* params, const chemora_patch* patches, double* const* scratch, int32_t npatch,
                double courant, const char* tune_cache_path, void* stream, chemora_plan** out, bool rk3,
                double dt_all = 0.0) {
  const int nst = rk3 ? 3 : 4;
  const bool synced = dt_all > 0.0;
  int dispatch = g_plan_dispatch.load();
  // the variant timing passes below run one work-group per tile when the
  // dispatch is still to be chosen
  const int pass_dispatch = dispatch == CHEMORA_DISPATCH_AUTO ? CHEMORA_DISPATCH_PER_TILE : dispatch;
  if (!out) return fail(CHEMORA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!patches || !scratch) return fail(CHEMORA_EINVAL, "patches or scratch is NULL");
  if (npatch < 1) return fail(CHEMORA_EINVAL, "npatch %d < 1", npatch);
  if (!synced && (!(courant > 0.0) || !std::isfinite(courant)))
    return fail(CHEMORA_EINVAL, "courant must be finite and > 0");
  auto dt_of = [&](int p) { return synced ? dt_all : courant * patches[p].h; };
  int rc;
  int64_t points = 0;
  for (int p = 0; p < npatch; ++p) {
    if ((rc = rk4_checks(params, &patches[p], dt_of(p), scratch[p]))) {
      const std::string m = g_error;
      return fail(rc, "patch %d: %s", p, m.c_str());
    }
    points += (int64_t)patches[p].n[0] * patches[p].n[1] * patches[p].n[2];
  }
  // every patch state and scratch buffer is its own memory: the stage
  // launches of a plan write them concurrently
  {
    struct Range {
      uintptr_t lo, hi;
      int patch;
      const char* what;
    };
    std::vector<Range> rs;
    rs.reserve(2 * (size_t)npatch);
    for (int p = 0; p < npatch; ++p) {
      const size_t state = (size_t)CHEMORA_NGF * patches[p].sf * sizeof(double);
      rs.push_back({(uintptr_t)patches[p].u, (uintptr_t)patches[p].u + state, p, "state"});
      rs.push_back({(uintptr_t)scratch[p], (uintptr_t)scratch[p] + 3 * state, p, "scratch"});
    }
    std::sort(rs.begin(), rs.end(), [](const Range& x, const Range& y) { return x.lo < y.lo; });
    for (size_t i = 1; i < rs.size(); ++i)
      if (rs[i].lo < rs[i - 1].hi)
        return fail(CHEMORA_EINVAL, "patch %d %s overlaps patch %d %s", rs[i].patch, rs[i].what, rs[i - 1].patch,
                    rs[i - 1].what);
  }
  chemora::SyncMaps maps;
  if (synced) {
    if (params->bc == CHEMORA_BC_PERIODIC)
      return fail(CHEMORA_EUNSUPPORTED, "a synchronised plan does not combine with periodic ghosts");
    std::string why;
    if (chemora::build_sync_maps(params, patches, npatch, &maps, &why)) return fail(CHEMORA_EINVAL, "%s", why.c_str());
  }
  hipStream_t s = (hipStream_t)stream;

  // tile variant of every patch: tuned classes from the cache, the rest
  // timed now on the largest patch of the class (longer launches, less
  // noise; then the cache is rewritten)
  std::vector<int> var(npatch, 0);
  if (tune_cache_path) {
    load_cache(tune_cache_path);
    std::vector<int> by_size(npatch);
    for (int p = 0; p < npatch; ++p) by_size[p] = p;
    auto pts = [&](int p) { return (int64_t)patches[p].n[0] * patches[p].n[1] * patches[p].n[2]; };
    std::stable_sort(by_size.begin(), by_size.end(), [&](int x, int y) { return pts(x) > pts(y); });
    for (int p : by_size)
      if ((rc = tune_class(params, &patches[p], scratch[p], s, &var[p]))) return rc;
    if ((rc = save_cache(tune_cache_path))) return rc;
    // The classes were timed one patch at a time, but a plan launches each
    // variant group after the other, so a mix of variants also pays for
    // every group's tail.  FP64 plans (whose variants are bit-identical)
    // therefore also time one pass with every built variant for all
    // patches and keep whichever assignment is fastest.
    bool mixed = false;
    for (int p = 1; p < npatch; ++p) mixed |= var[p] != var[0];
    if (mixed && params->precision == CHEMORA_PREC_FP64) {
      float best = 0.0f;
      if ((rc = plan_pass_ms(params, patches, scratch, npatch, var, pass_dispatch, s, &best))) return rc;
      for (int v = 0; v < chemora::NVARIANT; ++v) {
        if (!chemora::variant_supported(params->fd_order, v)) continue;
        const std::vector<int> uni(npatch, v);
        float ms = 0.0f;
        if ((rc = plan_pass_ms(params, patches, scratch, npatch, uni, pass_dispatch, s, &ms))) return rc;
        if (ms < best) {
          best = ms;
          var = uni;
        }
      }
    }
  } else {
    for (int p = 0; p < npatch; ++p) var[p] = choose_variant(params, &patches[p]);
  }

  // AUTO: time the stage-2 pass of the final assignment both ways and keep
  // the faster (they compute the same bits)
  if (dispatch == CHEMORA_DISPATCH_AUTO) {
    float persistent_ms = 0.0f, per_tile_ms = 0.0f;
    if ((rc = plan_pass_ms(params, patches, scratch, npatch, var, CHEMORA_DISPATCH_PERSISTENT, s, &persistent_ms)))
      return rc;
    if ((rc = plan_pass_ms(params, patches, scratch, npatch, var, CHEMORA_DISPATCH_PER_TILE, s, &per_tile_ms)))
      return rc;
    dispatch = persistent_ms < per_tile_ms ? CHEMORA_DISPATCH_PERSISTENT : CHEMORA_DISPATCH_PER_TILE;
  }

  chemora_plan* pl = new (std::nothrow) chemora_plan;
  if (!pl) return fail(CHEMORA_ENOMEM, "host allocation failed");
  pl->params = *params;
  pl->npatch = npatch;
  pl->points = points;
  pl->variant_of = var;
  pl->dispatch = dispatch;

  // group order: patches sorted by variant (stable); per-stage argument
  // tables in that order and per-group tile prefix sums (host side first)
  std::vector<int> order(npatch);
  for (int p = 0; p < npatch; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return var[x] < var[y]; });
  std::vector<chemora::StageArgs> args(nst * (size_t)npatch);
  std::vector<int> starts;
  for (int r = 0; r < npatch;) {
    PlanGroup g{var[order[r]], r, 0, 0, (int)starts.size(), 0};
    starts.push_back(0);
    int64_t tiles = 0;
    for (; r < npatch && var[order[r]] == g.variant; ++r) {
      const chemora_patch* X = &patches[order[r]];
      double* sc = scratch[order[r]];
      const size_t state = (size_t)CHEMORA_NGF * X->sf;
      chemora::StageArgs a = base_args(params, X);
      set_tiles(a, g.variant);
      tiles += (int64_t)a.tiles_x * a.tiles_y * tile_planes(a.geo.nz, g.variant);
      if (tiles > INT32_MAX) {
        plan_free(pl);
        return fail(CHEMORA_EINVAL, "too many tiles in the plan");
      }
      starts.push_back((int)tiles);
      for (int st = 0; st < nst; ++st) {
        chemora::StageArgs sa = a;
        if (rk3)
          rk3_stage_args(sa, st + 1, dt_of(order[r]), X->u, sc, sc + state);
        else
          stage_args(sa, st + 1, dt_of(order[r]), X->u, sc, sc + state, sc + 2 * state);
        args[st * (size_t)npatch + r] = sa;
      }
      ++g.count;
    }
    g.ntiles = (int)tiles;
    g.grid = dispatch == CHEMORA_DISPATCH_PERSISTENT ? persistent_grid(params, g.variant, g.ntiles) : g.ntiles;
    if (g.grid < 1) {
      plan_free(pl);
      return fail(CHEMORA_EDEVICE, "plan setup: occupancy or device query failed");
    }
    pl->groups.push_back(g);
  }
  // persistent launches: one set of queue counters per stage and group,
  // zeroed here; every launch leaves its set zeroed again
  const size_t nqueue = dispatch == CHEMORA_DISPATCH_PERSISTENT ? nst * pl->groups.size() * chemora::QUEUE_INTS : 0;
  hipError_t e = hipMalloc((void**)&pl->d_args, args.size() * sizeof(chemora::StageArgs));
  if (e == hipSuccess) e = hipMalloc((void**)&pl->d_tile_start, starts.size() * sizeof(int));
  if (e == hipSuccess && nqueue) e = hipMalloc((void**)&pl->d_queue, nqueue * sizeof(int));
  if (e != hipSuccess) {
    plan_free(pl);
    (void)hipGetLastError();
    return fail(CHEMORA_ENOMEM, "device allocation of plan tables failed");
  }
  // synchronised plans: maps, per-patch strides and the state pointers of
  // every stage output (caller's patch order), then u
  std::vector<chemora::SyncGeo> geo;
  std::vector<double*> bufs;
  if (synced) {
    pl->synced = true;
    pl->fill_start = maps.fill_start;
    pl->fill_copies = maps.fill_copies;
    pl->restr_start = maps.restr_start;
    for (int p = 0; p < npatch; ++p) geo.push_back({patches[p].sy, patches[p].sz, patches[p].sf});
    bufs.assign((size_t)(nst + 1) * npatch, nullptr);
    for (int st = 0; st < nst; ++st)
      for (int r = 0; r < npatch; ++r) bufs[st * (size_t)npatch + order[r]] = args[st * (size_t)npatch + r].out;
    for (int p = 0; p < npatch; ++p) bufs[nst * (size_t)npatch + p] = patches[p].u;
    if (e == hipSuccess && !maps.fill.empty())
      e = hipMalloc((void**)&pl->d_fill, maps.fill.size() * sizeof(chemora::SyncItem));
    if (e == hipSuccess && !maps.restr.empty())
      e = hipMalloc((void**)&pl->d_restr, maps.restr.size() * sizeof(chemora::SyncItem));
    if (e == hipSuccess) e = hipMalloc((void**)&pl->d_geo, geo.size() * sizeof(chemora::SyncGeo));
    if (e == hipSuccess) e = hipMalloc((void**)&pl->d_bufs, bufs.size() * sizeof(double*));
    if (e != hipSuccess) {
      plan_free(pl);
      (void)hipGetLastError();
      return fail(CHEMORA_ENOMEM, "device allocation of the plan's synchronisation maps failed");
    }
  }
  e = hipMemcpyAsync(pl->d_args, args.data(), args.size() * sizeof(chemora::StageArgs), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pl->d_tile_start, starts.data(), starts.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nqueue) e = hipMemsetAsync(pl->d_queue, 0, nqueue * sizeof(int), s);   // before capture
  if (synced) {
    if (e == hipSuccess && !maps.fill.empty())
      e = hipMemcpyAsync(pl->d_fill, maps.fill.data(), maps.fill.size() * sizeof(chemora::SyncItem),
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !maps.restr.empty())
      e = hipMemcpyAsync(pl->d_restr, maps.restr.data(), maps.restr.size() * sizeof(chemora::SyncItem),
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pl->d_geo, geo.data(), geo.size() * sizeof(chemora::SyncGeo), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pl->d_bufs, bufs.data(), bufs.size() * sizeof(double*), hipMemcpyHostToDevice, s);
    // the state made consistent once: restriction, then the ghost refill of u
    if (e == hipSuccess) {
      plan_restrict_and_fill(pl, pl->d_bufs + nst * (size_t)npatch, true, s);
      e = hipGetLastError();
    }
  }
  // static ghosts of the stage buffers, once
  if (e == hipSuccess && params->bc == CHEMORA_BC_STATIC) {
    for (int p = 0; p < npatch && e == hipSuccess; ++p) {
      const size_t state = (size_t)CHEMORA_NGF * patches[p].sf;
      launch_ghosts(false, make_geo(params, &patches[p]), patches[p].u, scratch[p], scratch[p] + state, s);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // tables and ghosts in place before capture
  if (e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "plan setup: %s", hipGetErrorString(e));
  }

  // capture one RK4 step
  e = hipStreamCreateWithFlags(&pl->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(pl->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "graph capture start: %s", hipGetErrorString(e));
  }
  const bool periodic = params->bc == CHEMORA_BC_PERIODIC;
  for (int st = 0; st < nst; ++st) {
    for (size_t gi = 0; gi < pl->groups.size(); ++gi) {
      const PlanGroup& g = pl->groups[gi];
      chemora::BatchTable bt;
      bt.args = pl->d_args + st * (size_t)npatch + g.first;
      bt.tile_start = pl->d_tile_start + g.toff;
      bt.queue = nqueue ? pl->d_queue + (st * pl->groups.size() + gi) * chemora::QUEUE_INTS : nullptr;
      bt.npatch = g.count;
      bt.ntiles = g.ntiles;
      dispatch_batch(params, g.variant, bt, g.grid, pl->capture);
    }
    if (periodic)
      for (int r = 0; r < npatch; ++r) {
        const double* wr = args[st * (size_t)npatch + r].out;
        launch_ghosts(true, make_geo(params, &patches[order[r]]), nullptr, const_cast<double*>(wr), nullptr,
                      pl->capture);
      }
    if (params->bc == CHEMORA_BC_RADIATIVE)
      for (int r = 0; r < npatch; ++r)
        launch_radiative(params, &patches[order[r]], args[st * (size_t)npatch + r], pl->capture);
    // ghost exchange of the stage outputs; after the last stage (which
    // writes u) restriction first
    if (synced) plan_restrict_and_fill(pl, pl->d_bufs + st * (size_t)npatch, st == nst - 1, pl->capture);
  }
  hipError_t le = hipGetLastError();
  e = hipStreamEndCapture(pl->capture, &pl->graph);
  if (le != hipSuccess || e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "graph capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
  }
  e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  *out = pl;
  return CHEMORA_OK;
}

}  // namespace

extern "C" {

int chemora_plan_create(const chemora_params* params, const chemora_patch* patches, double* const* scratch,
                        int32_t npatch, double courant, const char* tune_cache_path, void* stream,
                        chemora_plan** out) {
  g_error.clear();
  return plan_create(params, patches, scratch, npatch, courant, tune_cache_path, stream, out, false);
}

int chemora_plan_create_rk3(const chemora_params* params, const chemora_patch* patches, double* const* scratch,
                            int32_t npatch, double courant, const char* tune_cache_path, void* stream,
                            chemora_plan** out) {
  g_error.clear();
  return plan_create(params, patches, scratch, npatch, courant, tune_cache_path, stream, out, true);
}

int chemora_plan_create_synced(const chemora_params* params, const chemora_patch* patches, double* const* scratch,
                               int32_t npatch, double dt, int32_t integrator, const char* tune_cache_path,
                               void* stream, chemora_plan** out) {
  g_error.clear();
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CHEMORA_EINVAL, "dt must be finite and > 0");
  if (integrator != 3 && integrator != 4) return fail(CHEMORA_EINVAL, "integrator %d not 3 or 4", integrator);
  return plan_create(params, patches, scratch, npatch, 0.0, tune_cache_path, stream, out, integrator == 3, dt);
}

int chemora_set_plan_dispatch(int32_t mode) {
  g_error.clear();
  if (mode != CHEMORA_DISPATCH_PERSISTENT && mode != CHEMORA_DISPATCH_PER_TILE && mode != CHEMORA_DISPATCH_AUTO)
    return fail(CHEMORA_EINVAL, "unknown plan dispatch mode %d", mode);
  g_plan_dispatch.store(mode);
  return CHEMORA_OK;
}

int chemora_plan_dispatch(const chemora_plan* plan) {
  g_error.clear();
  if (!plan) return fail(CHEMORA_EINVAL, "plan is NULL");
  return plan->dispatch;
}

int chemora_plan_patch_variant(const chemora_plan* plan, int32_t p) {
  g_error.clear();
  if (!plan) return fail(CHEMORA_EINVAL, "plan is NULL");
  if (p < 0 || p >= plan->npatch) return fail(CHEMORA_EINVAL, "patch %d not in the plan", p);
  return plan->variant_of[p];
}

int chemora_batch_step(chemora_plan* plan, int32_t nsteps, void* stream) {
  g_error.clear();
  if (!plan) return fail(CHEMORA_EINVAL, "plan is NULL");
  if (nsteps < 0) return fail(CHEMORA_EINVAL, "nsteps %d < 0", nsteps);
  for (int n = 0; n < nsteps; ++n) {
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "graph launch: %s", hipGetErrorString(e));
  }
  return CHEMORA_OK;
}

int64_t chemora_plan_points(const chemora_plan* plan) { return plan ? plan->points : 0; }

int chemora_plan_destroy(chemora_plan* plan) {
  g_error.clear();
  if (!plan) return CHEMORA_OK;
  const hipError_t e = hipDeviceSynchronize();
  plan_free(plan);
  return e == hipSuccess ? CHEMORA_OK : fail(CHEMORA_EDEVICE, "plan destroy: %s", hipGetErrorString(e));
}

}  // extern "C"
