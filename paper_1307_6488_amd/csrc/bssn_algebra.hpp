// bssn_algebra.hpp -- pointwise right-hand side of the moving-puncture BSSN
// system (device code for gfx950).
//
// The paper's application is the McLachlan BSSN code (section "Scientific
// Motivation": the BSSN form of the Einstein equations, thousands of terms
// per point; section "Binary Black Hole Simulations": the "RHS evaluations"
// kernel).  The equations are the chi form of BSSN (Baumgarte & Shapiro 1998,
// Alcubierre et al. 2003) with 1+log or harmonic slicing and the advective
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
// where d0 = d_t - beta^k d_k (the advection term is added by the caller),
// Gd^i = gt^jk Gt^i_jk is the contracted Christoffel symbol computed from the
// metric (used in the Ricci tensor and in the undifferentiated shift terms;
// the evolved Gt^i enters only through d_j Gt^i), and
//   R_ij = Rt_ij + R^chi_ij,
//   Rt_ij = -1/2 gt^lm d_l d_m gt_ij + gt_k(i d_j) Gt^k + Gd^k Gt_(ij)k
//           + gt^lm (2 Gt^k_l(i Gt_j)km + Gt^k_im Gt_klj),
//   R^chi_ij = [D~_i D~_j chi + gt_ij D~^2 chi] / (2 chi)
//              - [d_i chi d_j chi + 3 gt_ij |d chi|^2] / (4 chi^2).
#pragma once

#include <hip/hip_runtime.h>

namespace chemora {

// packed symmetric index: xx xy xz yy yz zz
__device__ __forceinline__ constexpr int S(int i, int j) {
  return (i == 0) ? j : (j == 0 ? i : (i == 1 ? (j == 1 ? 3 : 4) : (j == 1 ? 4 : 5)));
}
// weight of a packed slot in a full double sum over (i, j)
__device__ __forceinline__ constexpr double W(int s) { return (s == 1 || s == 2 || s == 4) ? 2.0 : 1.0; }
// row/column of packed slot
__device__ __forceinline__ constexpr int SI(int s) { return s < 3 ? 0 : (s < 5 ? 1 : 2); }
__device__ __forceinline__ constexpr int SJ(int s) { return s < 3 ? s : (s < 5 ? s - 2 : 2); }

enum : int {
  gCHI = 0, gGT = 1, gK = 7, gAT = 8, gXT = 14, gALPHA = 17, gBETA = 18, gB = 21
};

struct Gauge {
  int lapse;   // 0 1+log, 1 harmonic, 2 frozen
  int shift;   // 0 Gamma-driver, 1 frozen
  double eta;
};

// Point data: values and the derivatives the algebra needs.
struct PointIn {
  double u[24];
  double dchi[3], dgt[6][3], dK[3], dXt[3][3], dalpha[3], dbeta[3][3];
  double ddchi[6], ddgt[6][6], ddalpha[6], ddbeta[3][6];
};

// Right-hand side without advection and dissipation.  rhs[] is fully written.
__device__ inline void bssn_algebra(const PointIn& p, const Gauge& gauge, double rhs[24]) {
  const double chi = p.u[gCHI], K = p.u[gK], alpha = p.u[gALPHA];
  const double* g = &p.u[gGT];
  const double* A = &p.u[gAT];

  // inverse conformal metric (adjugate / determinant)
  double gu[6];
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

  // Christoffel symbols: Gl[k][s(ij)] = Gt_{k,ij}, Gu[k][s(ij)] = Gt^k_ij
  double Gl[3][6], Gu[3][6];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), j = SJ(s);
      Gl[k][s] = 0.5 * (p.dgt[S(k, i)][j] + p.dgt[S(k, j)][i] - p.dgt[s][k]);
    }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 6; ++s)
      Gu[k][s] = gu[S(k, 0)] * Gl[0][s] + gu[S(k, 1)] * Gl[1][s] + gu[S(k, 2)] * Gl[2][s];
  double Gd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) acc += W(s) * gu[s] * Gu[k][s];
    Gd[k] = acc;
  }
  // Gm[k][i][m] = gt^lm Gt^k_li
  double Gm[3][3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        Gm[k][i][m] = gu[S(0, m)] * Gu[k][S(0, i)] + gu[S(1, m)] * Gu[k][S(1, i)] +
                      gu[S(2, m)] * Gu[k][S(2, i)];

  const double ichi = 1.0 / chi;
  // conformal covariant second derivative of chi and its traces
  double cdd[6];
#pragma unroll
  for (int s = 0; s < 6; ++s)
    cdd[s] = p.ddchi[s] - (Gu[0][s] * p.dchi[0] + Gu[1][s] * p.dchi[1] + Gu[2][s] * p.dchi[2]);
  double trc = 0.0, dchi2 = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    trc += W(s) * gu[s] * cdd[s];
    dchi2 += W(s) * gu[s] * p.dchi[SI(s)] * p.dchi[SJ(s)];
  }

  // Ricci tensor
  double Ric[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) r += W(q) * gu[q] * p.ddgt[s][q];
    r *= -0.5;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      r += 0.5 * (g[S(k, i)] * p.dXt[k][j] + g[S(k, j)] * p.dXt[k][i]) +
           0.5 * Gd[k] * (Gl[i][S(j, k)] + Gl[j][S(i, k)]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        r += Gm[k][i][m] * (Gl[j][S(k, m)] + Gl[k][S(m, j)]) + Gm[k][j][m] * Gl[i][S(k, m)];
    r += 0.5 * ichi * (cdd[s] + g[s] * trc) -
         0.25 * ichi * ichi * (p.dchi[i] * p.dchi[j] + 3.0 * g[s] * dchi2);
    Ric[s] = r;
  }

  // D_i D_j alpha with the physical Christoffel symbols
  double gudchi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    gudchi[k] = gu[S(k, 0)] * p.dchi[0] + gu[S(k, 1)] * p.dchi[1] + gu[S(k, 2)] * p.dchi[2];
  const double gudchi_da = gudchi[0] * p.dalpha[0] + gudchi[1] * p.dalpha[1] + gudchi[2] * p.dalpha[2];
  double DDa[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    DDa[s] = p.ddalpha[s] -
             (Gu[0][s] * p.dalpha[0] + Gu[1][s] * p.dalpha[1] + Gu[2][s] * p.dalpha[2]) -
             0.5 * ichi * (g[s] * gudchi_da - p.dchi[j] * p.dalpha[i] - p.dchi[i] * p.dalpha[j]);
  }
  double trDDa = 0.0, trRic = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    trDDa += W(s) * gu[s] * DDa[s];
    trRic += W(s) * gu[s] * Ric[s];
  }

  // mixed and raised extrinsic curvature
  double Am[3][3];   // At^i_j
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Am[i][j] = gu[S(i, 0)] * A[S(0, j)] + gu[S(i, 1)] * A[S(1, j)] + gu[S(i, 2)] * A[S(2, j)];
  double Au[6];      // At^ij
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    Au[s] = Am[i][0] * gu[S(0, j)] + Am[i][1] * gu[S(1, j)] + Am[i][2] * gu[S(2, j)];
  }
  double AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AA += Am[i][j] * Am[j][i];

  const double (&db)[3][3] = p.dbeta;   // db[i][k] = d_k beta^i
  const double divb = db[0][0] + db[1][1] + db[2][2];
  const double two3 = 2.0 / 3.0;

  rhs[gCHI] = two3 * chi * (alpha * K - divb);
  rhs[gK] = -chi * trDDa + alpha * (AA + K * K * (1.0 / 3.0));

  // trace of X_ij = alpha R_ij - D_i D_j alpha with gt^ij
  const double trX = alpha * trRic - trDDa;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = SI(s), j = SJ(s);
    double lg = 0.0, la = 0.0, aa = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lg += g[S(i, k)] * db[k][j] + g[S(j, k)] * db[k][i];
      la += A[S(i, k)] * db[k][j] + A[S(j, k)] * db[k][i];
      aa += A[S(i, k)] * Am[k][j];
    }
    rhs[gGT + s] = -2.0 * alpha * A[s] + lg - two3 * g[s] * divb;
    const double X = alpha * Ric[s] - DDa[s];
    rhs[gAT + s] = chi * (X - (1.0 / 3.0) * g[s] * trX) + alpha * (K * A[s] - 2.0 * aa) + la -
                   two3 * A[s] * divb;
  }

#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) r += W(q) * gu[q] * p.ddbeta[i][q];
    double gdd = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double ddk = p.ddbeta[0][S(j, 0)] + p.ddbeta[1][S(j, 1)] + p.ddbeta[2][S(j, 2)];
      gdd += gu[S(i, j)] * ddk;
    }
    r += (1.0 / 3.0) * gdd;
    r += two3 * Gd[i] * divb - (Gd[0] * db[i][0] + Gd[1] * db[i][1] + Gd[2] * db[i][2]);
    r -= 2.0 * (Au[S(i, 0)] * p.dalpha[0] + Au[S(i, 1)] * p.dalpha[1] + Au[S(i, 2)] * p.dalpha[2]);
    double ga = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) ga += W(q) * Gu[i][q] * Au[q];
    const double adchi = Au[S(i, 0)] * p.dchi[0] + Au[S(i, 1)] * p.dchi[1] + Au[S(i, 2)] * p.dchi[2];
    const double gdK = gu[S(i, 0)] * p.dK[0] + gu[S(i, 1)] * p.dK[1] + gu[S(i, 2)] * p.dK[2];
    r += 2.0 * alpha * (ga - 1.5 * ichi * adchi - two3 * gdK);
    rhs[gXT + i] = r;
  }

  if (gauge.lapse == 0)
    rhs[gALPHA] = -2.0 * alpha * K;
  else if (gauge.lapse == 1)
    rhs[gALPHA] = -alpha * alpha * K;
  else
    rhs[gALPHA] = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (gauge.shift == 0) {
      rhs[gBETA + i] = 0.75 * p.u[gB + i];
      rhs[gB + i] = rhs[gXT + i] - gauge.eta * p.u[gB + i];
    } else {
      rhs[gBETA + i] = 0.0;
      rhs[gB + i] = 0.0;
    }
  }
}

// whether GF f evolves (a frozen gauge variable gets no advection/dissipation)
__device__ __forceinline__ bool evolves(int f, const Gauge& gauge) {
  if (f == gALPHA) return gauge.lapse != 2;
  if (f >= gBETA) return gauge.shift == 0;
  return true;
}

}  // namespace chemora
