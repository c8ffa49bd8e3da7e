// bssn_oracle.cpp -- CPU reference of the BSSN right-hand side and the RK4
// and RK3 steps.
//
// TEST INFRASTRUCTURE ONLY.  This is the plain, slow, FP64 oracle that the HIP
// library is checked against.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg load it; the library never links or calls it,
// and it shares no source, header or table with the library.
//
// What it computes (Chemora, arXiv:1307.6488): the paper's showcase is the
// McLachlan BSSN evolution code -- the Einstein equations in BSSN form with
// high-order finite differences (section "Scientific Motivation"), 8th-order
// partially upwinded stencils needing 5 ghost zones and a third-order
// Runge-Kutta time integrator (section "Binary Black Hole Simulations", timer
// table: RHS derivatives / advection / evaluations, boundary condition,
// time-integrator copy); the classic RK4 step is here too.  The paper cites
// but does not print the equations; they are taken here from the
// formulation it cites (Nakamura 1987; Shibata & Nakamura 1995;
// Baumgarte & Shapiro 1998; Alcubierre et al. 1999/2003), in the chi variant
// with 1+log slicing and the advective Gamma-driver shift used by moving-
// puncture codes, plus Kreiss-Oliger dissipation (Kreiss & Oliger 1973).
//
// Style: every operator is a direct transcription of its definition, tensor
// sums are explicit loops over 3x3 arrays, nothing is fused or reordered for
// speed.  The scalar type is a template parameter so the same code, run on a
// counting scalar, reports the exact number of floating-point operations per
// grid point (+, -, *, /; no FMA), and, run in x87 extended precision (64-bit
// significand), gives a reference of the same discrete scheme 11 bits more
// accurate than FP64, against which the rounding error of any FP64
// evaluation (this oracle's own included) can be measured.  Every rational
// constant is formed in the scalar's own precision (the FP64 values are the
// correctly rounded quotients, as before).  Build: g++ -O2 -ffp-contract=off.

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t fd_order;   // 4 or 8
  int32_t ghost;      // ghost width of the arrays
  int32_t upwind;     // 1: lopsided advection stencils, 0: centred
  int32_t ko_radius;  // Kreiss-Oliger radius r, 0 = off
  double eps_diss;    // Kreiss-Oliger strength
  int32_t lapse;      // 0 1+log, 1 harmonic, 2 frozen
  int32_t shift;      // 0 Gamma-driver, 1 frozen
  double eta;         // Gamma-driver damping
  int32_t bc;         // 0 static ghosts, 1 periodic, 2 radiative (Sommerfeld)
  int32_t nthreads;   // OpenMP threads (<= 0: runtime default)
} oracle_params;

typedef struct {
  int32_t n[3];       // interior extents
  int32_t ghost;
  int64_t sy, sz, sf; // element strides (x stride 1)
  double h;           // grid spacing
  double origin[3];   // coordinates of interior point (0, 0, 0) (radiative boundary)
} oracle_grid;

}  // extern "C"

namespace {

enum {
  CHI = 0, GT = 1, TRK = 7, AT = 8, XT = 14, ALPHA = 17, BETA = 18, BDRV = 21, NGF = 24
};
const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
// pairs (a,b) of the 6 packed second-derivative slots
const int PAIR[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};

// ---------------------------------------------------------------------------
// counting scalar
// ---------------------------------------------------------------------------
struct Counted {
  double v;
  static long long nadd, nmul, ndiv;
  Counted() : v(0.0) {}
  Counted(double x) : v(x) {}
};
long long Counted::nadd = 0, Counted::nmul = 0, Counted::ndiv = 0;
inline Counted operator+(Counted a, Counted b) { ++Counted::nadd; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++Counted::nadd; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { ++Counted::nmul; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++Counted::ndiv; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline bool nonneg(Counted a) { return a.v >= 0.0; }
inline bool nonneg(double a) { return a >= 0.0; }
inline bool nonneg(long double a) { return a >= 0.0L; }

// ---------------------------------------------------------------------------
// finite-difference weights.  Centred weights are the classical 4th/8th-order
// ones (Fornberg 1988); the lopsided (partially upwinded) ones use offsets
// -1..3 (order 4) and -3..5 (order 8) for a non-negative advecting velocity.
// Every operator is applied to differences u_{+k} - u_0 so that a constant
// field gives exactly zero.
// ---------------------------------------------------------------------------
// Rational constants and per-grid factors in the scalar's own precision.  The
// counting scalar takes FP64 constants without counting them.
template <class R>
struct Exact {
  typedef double W;   // storage type of the stencil weights
  static R ratio(int p, int q) { return R(double(p) / double(q)); }
  static R quot(double a, double b) { return R(a / b); }
  static R inv_sq(double h) { return R(1.0 / (h * h)); }
};
template <>
struct Exact<long double> {
  typedef long double W;
  static long double ratio(int p, int q) { return (long double)p / (long double)q; }
  static long double quot(double a, double b) { return (long double)a / (long double)b; }
  static long double inv_sq(double h) { return 1.0L / ((long double)h * (long double)h); }
};

template <class W>
struct WeightsT {
  int order;
  int nc;          // number of centred offsets (order/2)
  W c1[4];         // first derivative, offsets 1..nc (antisymmetric)
  W c2[4];         // second derivative, offsets 1..nc (symmetric)
  int up_lo, up_hi;
  W up[9];         // lopsided weights for offsets up_lo..up_hi (entry for 0 unused)
};
typedef WeightsT<double> Weights;

template <class W>
WeightsT<W> make_weights_t(int order) {
  auto q = [](int a, int b) { return Exact<W>::ratio(a, b); };
  WeightsT<W> w;
  std::memset(&w, 0, sizeof w);
  w.order = order;
  w.nc = order / 2;
  if (order == 4) {
    w.c1[0] = q(2, 3);  w.c1[1] = q(-1, 12);
    w.c2[0] = q(4, 3);  w.c2[1] = q(-1, 12);
    w.up_lo = -1; w.up_hi = 3;
    const int u4[5] = {-3, -10, 18, -6, 1};
    for (int i = 0; i < 5; ++i) w.up[i] = q(u4[i], 12);
  } else {
    w.c1[0] = q(4, 5);  w.c1[1] = q(-1, 5);  w.c1[2] = q(4, 105);  w.c1[3] = q(-1, 280);
    w.c2[0] = q(8, 5);  w.c2[1] = q(-1, 5);  w.c2[2] = q(8, 315);  w.c2[3] = q(-1, 560);
    w.up_lo = -3; w.up_hi = 5;
    const int un[9] = {-1, 1, -1, -9, 5, -1, 1, -1, 1};
    const int ud[9] = {168, 14, 2, 20, 4, 2, 6, 28, 280};
    for (int i = 0; i < 9; ++i) w.up[i] = q(un[i], ud[i]);
  }
  return w;
}
Weights make_weights(int order) { return make_weights_t<double>(order); }

double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Pointwise operators on one grid function.  f points at the evaluation point,
// s is the element stride along the differentiation axis.
template <class R, class T, class W>
R op_d1(const T* f, long s, const WeightsT<W>& w, R inv_h) {
  R acc = R(0.0);
  for (int k = 1; k <= w.nc; ++k) acc = acc + R(w.c1[k - 1]) * (R(f[k * s]) - R(f[-k * s]));
  return acc * inv_h;
}

template <class R, class T, class W>
R op_d2(const T* f, long s, const WeightsT<W>& w, R inv_h2) {
  R acc = R(0.0);
  const R c = R(f[0]);
  for (int k = 1; k <= w.nc; ++k)
    acc = acc + R(w.c2[k - 1]) * ((R(f[k * s]) - c) + (R(f[-k * s]) - c));
  return acc * inv_h2;
}

// mixed derivative d_a d_b: outer first derivative (stride sa) of inner first
// derivatives (stride sb), the inner differences formed at each outer offset.
template <class R, class T, class W>
R op_d11(const T* f, long sa, long sb, const WeightsT<W>& w, R inv_h) {
  R acc = R(0.0);
  for (int k = 1; k <= w.nc; ++k) {
    R dp = op_d1<R>(f + k * sa, sb, w, inv_h);
    R dm = op_d1<R>(f - k * sa, sb, w, inv_h);
    acc = acc + R(w.c1[k - 1]) * (dp - dm);
  }
  return acc * inv_h;
}

// lopsided first derivative; positive = stencil shifted toward +axis (used
// for a non-negative advecting velocity), else the mirror image.
template <class R, class T, class W>
R op_upwind(const T* f, long s, const WeightsT<W>& w, bool positive, R inv_h) {
  R acc = R(0.0);
  const R c = R(f[0]);
  for (int o = w.up_lo; o <= w.up_hi; ++o) {
    if (o == 0) continue;
    const W wt = w.up[o - w.up_lo];
    if (positive)
      acc = acc + R(wt) * (R(f[o * s]) - c);
    else
      acc = acc - R(wt) * (R(f[-o * s]) - c);
  }
  return acc * inv_h;
}

// Kreiss-Oliger dissipation along one axis with radius r:
//   Q u = (-1)^(r+1) eps / (2^(2r) h) * sum_m (-1)^m C(2r, m) u_{i + r - m},
// written on the symmetric differences u_{+k} + u_{-k} - 2 u_0.
template <class R, class T>
R op_ko(const T* f, long s, int r, R eps_over_h) {
  R acc = R(0.0);
  const R c = R(f[0]);
  const double scale = std::ldexp(1.0, -2 * r);
  for (int k = 1; k <= r; ++k) {
    double coef = binom(2 * r, r + k) * scale * (((k + 1) % 2 == 0) ? 1.0 : -1.0);
    acc = acc + R(coef) * ((R(f[k * s]) - c) + (R(f[-k * s]) - c));
  }
  return acc * eps_over_h;
}

// ---------------------------------------------------------------------------
// pointwise right-hand side.  Inputs: the 24 values, first derivatives
// d1[f][k] = d_k u_f, second derivatives d2[f][slot] (slot as in PAIR),
// advection terms adv[f] = beta^k D_k u_f and dissipation diss[f].
// ---------------------------------------------------------------------------
struct Opts {
  int lapse, shift;
  double eta;
};

template <class R>
struct Geometry {
  R gt[3][3], gtu[3][3];       // conformal metric and inverse
  R Gl[3][3][3];               // Gt_{k,ij}  (first index lowered)
  R Gu[3][3][3];               // Gt^k_{ij}
  R Xtd[3];                    // Gt^k computed from the metric
  R Ric[3][3];                 // physical Ricci tensor R_ij
};

// steps 1-5: inverse metric, Christoffels, Ricci tensor
template <class R>
void geometry(const R u[NGF], const R d1[NGF][3], const R d2[NGF][6], Geometry<R>& G) {
  const R half = R(0.5);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) G.gt[i][j] = u[GT + SYM[i][j]];

  // inverse by cofactors / determinant (no unit-determinant assumption)
  const R(&g)[3][3] = G.gt;
  R cof[3][3];
  cof[0][0] = g[1][1] * g[2][2] - g[1][2] * g[2][1];
  cof[0][1] = g[0][2] * g[2][1] - g[0][1] * g[2][2];
  cof[0][2] = g[0][1] * g[1][2] - g[0][2] * g[1][1];
  cof[1][1] = g[0][0] * g[2][2] - g[0][2] * g[2][0];
  cof[1][2] = g[0][2] * g[1][0] - g[0][0] * g[1][2];
  cof[2][2] = g[0][0] * g[1][1] - g[0][1] * g[1][0];
  // expansion along the first row; the adjugate of a symmetric matrix is symmetric
  R det = g[0][0] * cof[0][0] + g[0][1] * cof[0][1] + g[0][2] * cof[0][2];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      G.gtu[i][j] = cof[i][j] / det;
      G.gtu[j][i] = G.gtu[i][j];
    }

  // dg[m][a][b] = d_m gt_ab
  R dg[3][3][3];
  for (int m = 0; m < 3; ++m)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) dg[m][a][b] = d1[GT + SYM[a][b]][m];

  // Gt_{k,ij} = 1/2 (d_j gt_ki + d_i gt_kj - d_k gt_ij)
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) {
        G.Gl[k][i][j] = half * (dg[j][k][i] + dg[i][k][j] - dg[k][i][j]);
        G.Gl[k][j][i] = G.Gl[k][i][j];
      }
  // Gt^k_{ij} = gtu^{kl} Gt_{l,ij}
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) {
        R s = R(0.0);
        for (int l = 0; l < 3; ++l) s = s + G.gtu[k][l] * G.Gl[l][i][j];
        G.Gu[k][i][j] = s;
        G.Gu[k][j][i] = s;
      }
  // Gt^k computed: gtu^{ij} Gt^k_{ij}
  for (int k = 0; k < 3; ++k) {
    R s = R(0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) s = s + G.gtu[i][j] * G.Gu[k][i][j];
    G.Xtd[k] = s;
  }

  // conformal Ricci tensor
  R Rt[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      R s = R(0.0);
      // -1/2 gtu^{lm} d_l d_m gt_ij
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) s = s - half * G.gtu[l][m] * d2[GT + SYM[i][j]][SYM[l][m]];
      // +1/2 (gt_ki d_j Gt^k + gt_kj d_i Gt^k), Gt^k the evolved variable
      for (int k = 0; k < 3; ++k)
        s = s + half * (G.gt[k][i] * d1[XT + k][j] + G.gt[k][j] * d1[XT + k][i]);
      // +1/2 Gtd^k (Gt_{i,jk} + Gt_{j,ik})
      for (int k = 0; k < 3; ++k) s = s + half * G.Xtd[k] * (G.Gl[i][j][k] + G.Gl[j][i][k]);
      // + gtu^{lm} (Gt^k_li Gt_{j,km} + Gt^k_lj Gt_{i,km} + Gt^k_im Gt_{k,lj})
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m)
          for (int k = 0; k < 3; ++k)
            s = s + G.gtu[l][m] * (G.Gu[k][l][i] * G.Gl[j][k][m] + G.Gu[k][l][j] * G.Gl[i][k][m] +
                                   G.Gu[k][i][m] * G.Gl[k][l][j]);
      Rt[i][j] = s;
    }

  // conformal-factor part of the Ricci tensor
  const R chi = u[CHI];
  R cddchi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      R s = d2[CHI][SYM[i][j]];
      for (int k = 0; k < 3; ++k) s = s - G.Gu[k][i][j] * d1[CHI][k];
      cddchi[i][j] = s;
      cddchi[j][i] = s;
    }
  R trc = R(0.0), dchi2 = R(0.0);
  for (int l = 0; l < 3; ++l)
    for (int m = 0; m < 3; ++m) {
      trc = trc + G.gtu[l][m] * cddchi[l][m];
      dchi2 = dchi2 + G.gtu[l][m] * d1[CHI][l] * d1[CHI][m];
    }
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      R rchi = (cddchi[i][j] + G.gt[i][j] * trc) / (R(2.0) * chi) -
               (d1[CHI][i] * d1[CHI][j] + R(3.0) * G.gt[i][j] * dchi2) / (R(4.0) * chi * chi);
      G.Ric[i][j] = Rt[i][j] + rchi;
      G.Ric[j][i] = G.Ric[i][j];
    }
}

template <class R>
void rhs_point(const Opts& P, const R u[NGF], const R d1[NGF][3], const R d2[NGF][6],
               const R adv[NGF], const R diss[NGF], R rhs[NGF]) {
  Geometry<R> G;
  geometry<R>(u, d1, d2, G);
  const R third = Exact<R>::ratio(1, 3), two3 = Exact<R>::ratio(2, 3), two = R(2.0);

  const R chi = u[CHI], K = u[TRK], alpha = u[ALPHA];
  R At[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) At[i][j] = u[AT + SYM[i][j]];
  // db[i][k] = d_k beta^i
  R db[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) db[i][k] = d1[BETA + i][k];
  R divb = db[0][0] + db[1][1] + db[2][2];

  // At^i_j and At^{ij}
  R Atm[3][3], Atu[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      R s = R(0.0);
      for (int k = 0; k < 3; ++k) s = s + G.gtu[i][k] * At[k][j];
      Atm[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      R s = R(0.0);
      for (int k = 0; k < 3; ++k) s = s + Atm[i][k] * G.gtu[k][j];
      Atu[i][j] = s;
      Atu[j][i] = s;
    }
  R AA = R(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) AA = AA + Atm[i][j] * Atm[j][i];

  // physical Christoffel symbols and D_i D_j alpha
  R gtu_dchi[3];
  for (int k = 0; k < 3; ++k) {
    R s = R(0.0);
    for (int l = 0; l < 3; ++l) s = s + G.gtu[k][l] * d1[CHI][l];
    gtu_dchi[k] = s;
  }
  R DDa[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      R s = d2[ALPHA][SYM[i][j]];
      for (int k = 0; k < 3; ++k) {
        R corr = G.gt[i][j] * gtu_dchi[k];
        if (k == i) corr = corr - d1[CHI][j];
        if (k == j) corr = corr - d1[CHI][i];
        // Gamma^k_ij = Gt^k_ij + corr / (2 chi)
        R Gam = G.Gu[k][i][j] + corr / (two * chi);
        s = s - Gam * d1[ALPHA][k];
      }
      DDa[i][j] = s;
      DDa[j][i] = s;
    }
  R LapA = R(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) LapA = LapA + G.gtu[i][j] * DDa[i][j];
  LapA = chi * LapA;

  // trace-free part of -D_i D_j alpha + alpha R_ij
  R X[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      X[i][j] = alpha * G.Ric[i][j] - DDa[i][j];
      X[j][i] = X[i][j];
    }
  R trX = R(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trX = trX + G.gtu[i][j] * X[i][j];

  // chi
  rhs[CHI] = adv[CHI] + two3 * chi * (alpha * K - divb);
  // gt_ij and At_ij
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      const int s = SYM[i][j];
      R lie_g = R(0.0), lie_a = R(0.0), AtAt = R(0.0);
      for (int k = 0; k < 3; ++k) {
        lie_g = lie_g + G.gt[i][k] * db[k][j] + G.gt[j][k] * db[k][i];
        lie_a = lie_a + At[i][k] * db[k][j] + At[j][k] * db[k][i];
        AtAt = AtAt + At[i][k] * Atm[k][j];
      }
      rhs[GT + s] = adv[GT + s] - two * alpha * At[i][j] + lie_g - two3 * G.gt[i][j] * divb;
      R XTF = X[i][j] - third * G.gt[i][j] * trX;
      rhs[AT + s] = adv[AT + s] + chi * XTF + alpha * (K * At[i][j] - two * AtAt) + lie_a -
                    two3 * At[i][j] * divb;
    }
  // K
  rhs[TRK] = adv[TRK] - LapA + alpha * (AA + third * K * K);

  // Gt^i (without advection first; the Gamma-driver reuses it)
  R Xt_src[3];
  for (int i = 0; i < 3; ++i) {
    R s = R(0.0);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) s = s + G.gtu[j][k] * d2[BETA + i][SYM[j][k]];
    R ddiv = R(0.0);  // gtu^{ij} d_j d_k beta^k
    for (int j = 0; j < 3; ++j) {
      R dj_div = R(0.0);
      for (int k = 0; k < 3; ++k) dj_div = dj_div + d2[BETA + k][SYM[j][k]];
      ddiv = ddiv + G.gtu[i][j] * dj_div;
    }
    s = s + third * ddiv;
    for (int j = 0; j < 3; ++j) s = s - G.Xtd[j] * db[i][j];
    s = s + two3 * G.Xtd[i] * divb;
    R t = R(0.0);
    for (int j = 0; j < 3; ++j) s = s - two * Atu[i][j] * d1[ALPHA][j];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) t = t + G.Gu[i][j][k] * Atu[j][k];
    R tchi = R(0.0), tK = R(0.0);
    for (int j = 0; j < 3; ++j) {
      tchi = tchi + Atu[i][j] * d1[CHI][j];
      tK = tK + G.gtu[i][j] * d1[TRK][j];
    }
    t = t - R(1.5) * tchi / chi - two3 * tK;
    s = s + two * alpha * t;
    Xt_src[i] = s;
    rhs[XT + i] = adv[XT + i] + s;
  }

  // lapse
  if (P.lapse == 0)
    rhs[ALPHA] = adv[ALPHA] - two * alpha * K;
  else if (P.lapse == 1)
    rhs[ALPHA] = adv[ALPHA] - alpha * alpha * K;
  else
    rhs[ALPHA] = R(0.0);
  // shift
  for (int i = 0; i < 3; ++i) {
    if (P.shift == 0) {
      rhs[BETA + i] = adv[BETA + i] + R(0.75) * u[BDRV + i];
      rhs[BDRV + i] = adv[BDRV + i] + Xt_src[i] - R(P.eta) * u[BDRV + i];
    } else {
      rhs[BETA + i] = R(0.0);
      rhs[BDRV + i] = R(0.0);
    }
  }
  // dissipation on every evolved variable
  for (int f = 0; f < NGF; ++f) {
    if (f == ALPHA && P.lapse == 2) continue;
    if ((f >= BETA) && P.shift == 1) continue;
    rhs[f] = rhs[f] + diss[f];
  }
}

// Hamiltonian constraint H = chi gtu^{ij} R_ij + 2/3 K^2 - At^i_j At^j_i
template <class R>
R ham_point(const R u[NGF], const R d1[NGF][3], const R d2[NGF][6]) {
  Geometry<R> G;
  geometry<R>(u, d1, d2, G);
  R trR = R(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trR = trR + G.gtu[i][j] * G.Ric[i][j];
  R Atm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      R s = R(0.0);
      for (int k = 0; k < 3; ++k) s = s + G.gtu[i][k] * u[AT + SYM[k][j]];
      Atm[i][j] = s;
    }
  R AA = R(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) AA = AA + Atm[i][j] * Atm[j][i];
  return u[CHI] * trR + Exact<R>::ratio(2, 3) * u[TRK] * u[TRK] - AA;
}

// which GFs need first / second derivatives
bool needs_d1(int f) { return !((f >= AT && f < AT + 6) || f >= BDRV); }
bool needs_d2(int f) { return f == CHI || (f >= GT && f < GT + 6) || f == ALPHA || (f >= BETA && f < BETA + 3); }

// ---------------------------------------------------------------------------
// grid-point gather: every stencil the right-hand side needs at one point
// ---------------------------------------------------------------------------
// Momentum constraint, lower index, in the conformal variables:
//   M_i = gt^jk (d_j At_ki - Gt^l_jk At_li - Gt^l_ji At_kl)
//         - 3/(2 chi) gt^kl At_il d_k chi - 2/3 d_i K,
// which is D_j K^j_i - d_i K of the physical metric gt/chi and curvature
// (At + gt K/3)/chi when At is trace-free (conformal decomposition of the
// ADM momentum constraint; first derivatives only).
template <class R>
void mom_point(const R u[NGF], const R d1[NGF][3], R M[3]) {
  const R half = R(0.5), three_halves = R(3.0) / R(2.0), two_thirds = R(2.0) / R(3.0);
  R g[3][3], At[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      g[i][j] = u[GT + SYM[i][j]];
      At[i][j] = u[AT + SYM[i][j]];
    }
  R cof[3][3];
  cof[0][0] = g[1][1] * g[2][2] - g[1][2] * g[2][1];
  cof[0][1] = g[0][2] * g[2][1] - g[0][1] * g[2][2];
  cof[0][2] = g[0][1] * g[1][2] - g[0][2] * g[1][1];
  cof[1][1] = g[0][0] * g[2][2] - g[0][2] * g[2][0];
  cof[1][2] = g[0][2] * g[1][0] - g[0][0] * g[1][2];
  cof[2][2] = g[0][0] * g[1][1] - g[0][1] * g[1][0];
  const R det = g[0][0] * cof[0][0] + g[0][1] * cof[0][1] + g[0][2] * cof[0][2];
  R gu[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      gu[i][j] = cof[i][j] / det;
      gu[j][i] = gu[i][j];
    }
  // Gt^l_jk = 1/2 gt^lm (d_j gt_mk + d_k gt_mj - d_m gt_jk)
  R Gam[3][3][3];
  for (int l = 0; l < 3; ++l)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        R s = R(0.0);
        for (int m = 0; m < 3; ++m)
          s = s + gu[l][m] * (d1[GT + SYM[m][k]][j] + d1[GT + SYM[m][j]][k] - d1[GT + SYM[j][k]][m]);
        Gam[l][j][k] = half * s;
      }
  const R chi = u[CHI];
  for (int i = 0; i < 3; ++i) {
    R s = R(0.0);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        R t = d1[AT + SYM[k][i]][j];
        for (int l = 0; l < 3; ++l) t = t - Gam[l][j][k] * At[l][i] - Gam[l][j][i] * At[k][l];
        s = s + gu[j][k] * t;
      }
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) s = s - three_halves / chi * gu[k][l] * At[i][l] * d1[CHI][k];
    M[i] = s - two_thirds * d1[TRK][i];
  }
}

// ---------------------------------------------------------------------------
// Psi4, the Newman-Penrose Weyl scalar of outgoing radiation, from the 3+1
// data in vacuum (the paper's second GPU workload, section "Binary Black Hole
// Simulations with Chemora": the WeylScal4 step, timer row "Compute Psi4";
// the paper does not print it).  With the physical metric gamma_ij = gt_ij /
// chi, the extrinsic curvature K_ij = (At_ij + gt_ij K / 3) / chi (the sign of
// d_t gamma_ij = -2 alpha K_ij + ...), its Ricci tensor R_ij (the one the
// evolution uses: the conformal Ricci with the evolved Gt^i in its d Gt term,
// plus the chi terms) and covariant derivative D:
//   E_ij = R_ij - K_ik K^k_j + K K_ij                 (electric Weyl part)
//   B_ij = sym_ij eps_i^kl D_k K_lj                    (magnetic Weyl part)
// with eps_ijk = sqrt(det gamma) [ijk].  Tetrad: the coordinate vectors
//   v1 = (-y, x, 0) (phi-like; (0, 1, 0) on the z axis),
//   v2 = (x, y, z)  (radial; (0, 0, 1) at the origin),
//   v3^a = gamma^ad eps_dbc v1^b v2^c (theta-like)
// orthonormalised by Gram-Schmidt in the order v2, v3, v1 with the physical
// metric give e_r, e_theta, e_phi; l = (n + e_r)/sqrt2 is the outgoing null
// vector, mbar = (e_theta - i e_phi)/sqrt2 and
//   Psi4 = (E_ij - i B_ij) mbar^i mbar^j
//        = [ (E_tt - E_pp)/2 - B_tp ] + i [ -E_tp - (B_tt - B_pp)/2 ]
// (t = theta, p = phi components), so that an outgoing wave h(t - r) gives
// Psi4 = -d_t^2 h_+ + i d_t^2 h_x to linear order (h_+ = (h_tt - h_pp)/2,
// h_x = h_tp) and an ingoing one gives zero.  Coordinates x, y, z are the
// point's (origin + index * h).
// ---------------------------------------------------------------------------
template <class R>
struct Psi4Out {
  R re, im;
  R E[3][3], B[3][3];
  R tet[3][3];    // e_r, e_theta, e_phi (contravariant components)
};

template <class R>
void psi4_point(const R u[NGF], const R d1[NGF][3], const R d2[NGF][6], const R xyz[3], Psi4Out<R>& out) {
  Geometry<R> G;
  geometry<R>(u, d1, d2, G);
  const R chi = u[CHI], K = u[TRK], third = Exact<R>::ratio(1, 3), half = R(0.5);
  R gam[3][3], gamu[3][3], Kd[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gam[i][j] = G.gt[i][j] / chi;
      gamu[i][j] = chi * G.gtu[i][j];
      Kd[i][j] = (u[AT + SYM[i][j]] + G.gt[i][j] * K * third) / chi;
    }
  // K^i_j and its trace
  R Km[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      R s = R(0.0);
      for (int k = 0; k < 3; ++k) s = s + gamu[i][k] * Kd[k][j];
      Km[i][j] = s;
    }
  const R trK = Km[0][0] + Km[1][1] + Km[2][2];
  // electric part
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      R kk = R(0.0);
      for (int k = 0; k < 3; ++k) kk = kk + Kd[i][k] * Km[k][j];
      out.E[i][j] = G.Ric[i][j] - kk + trK * Kd[i][j];
    }
  // physical Christoffel symbols Gamma^k_ij = Gt^k_ij + (gt_ij gt^kl d_l chi
  // - delta^k_i d_j chi - delta^k_j d_i chi) / (2 chi)
  R Gam[3][3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        R gd = R(0.0);
        for (int l = 0; l < 3; ++l) gd = gd + G.gtu[k][l] * d1[CHI][l];
        R c = G.gt[i][j] * gd;
        if (k == i) c = c - d1[CHI][j];
        if (k == j) c = c - d1[CHI][i];
        Gam[k][i][j] = G.Gu[k][i][j] + c / (R(2.0) * chi);
      }
  // d_k K_ij of K_ij = (At_ij + gt_ij K / 3) / chi, then D_k K_ij
  R DK[3][3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int s = SYM[i][j];
        R dK = (d1[AT + s][k] + d1[GT + s][k] * K * third + G.gt[i][j] * d1[TRK][k] * third) / chi -
               Kd[i][j] * d1[CHI][k] / chi;
        for (int m = 0; m < 3; ++m) dK = dK - Gam[m][k][i] * Kd[m][j] - Gam[m][k][j] * Kd[i][m];
        DK[k][i][j] = dK;
      }
  // Levi-Civita tensor of the physical metric
  R detg = gam[0][0] * (gam[1][1] * gam[2][2] - gam[1][2] * gam[2][1]) -
           gam[0][1] * (gam[1][0] * gam[2][2] - gam[1][2] * gam[2][0]) +
           gam[0][2] * (gam[1][0] * gam[2][1] - gam[1][1] * gam[2][0]);
  const R sq = std::sqrt(detg);
  auto perm = [](int a, int b, int c) -> int {
    if (a == b || b == c || a == c) return 0;
    return ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) ? 1 : -1;
  };
  R eps[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) eps[a][b][c] = R(double(perm(a, b, c))) * sq;
  // magnetic part: eps_i^kl D_k K_lj, symmetrised
  R Bn[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      R s = R(0.0);
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          R e = R(0.0);   // eps_i^kl = gamma^ka gamma^lb eps_iab
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) e = e + gamu[k][a] * gamu[l][b] * eps[i][a][b];
          s = s + e * DK[k][l][j];
        }
      Bn[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out.B[i][j] = half * (Bn[i][j] + Bn[j][i]);

  // tetrad
  const R x = xyz[0], y = xyz[1], z = xyz[2];
  R v1[3] = {-y, x, R(0.0)}, v2[3] = {x, y, z};
  if (x == R(0.0) && y == R(0.0)) { v1[0] = R(0.0); v1[1] = R(1.0); }
  if (x == R(0.0) && y == R(0.0) && z == R(0.0)) v2[2] = R(1.0);
  R v3[3];
  for (int a = 0; a < 3; ++a) {
    R s = R(0.0);
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) s = s + gamu[a][d] * eps[d][b][c] * v1[b] * v2[c];
    v3[a] = s;
  }
  auto dot = [&](const R* p, const R* q) {
    R s = R(0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s = s + gam[a][b] * p[a] * q[b];
    return s;
  };
  R er[3], et[3], ep[3];
  {
    const R n = std::sqrt(dot(v2, v2));
    for (int a = 0; a < 3; ++a) er[a] = v2[a] / n;
  }
  {
    const R c = dot(v3, er);
    R w[3];
    for (int a = 0; a < 3; ++a) w[a] = v3[a] - c * er[a];
    const R n = std::sqrt(dot(w, w));
    for (int a = 0; a < 3; ++a) et[a] = w[a] / n;
  }
  {
    const R cr = dot(v1, er), ct = dot(v1, et);
    R w[3];
    for (int a = 0; a < 3; ++a) w[a] = v1[a] - cr * er[a] - ct * et[a];
    const R n = std::sqrt(dot(w, w));
    for (int a = 0; a < 3; ++a) ep[a] = w[a] / n;
  }
  for (int a = 0; a < 3; ++a) {
    out.tet[0][a] = er[a];
    out.tet[1][a] = et[a];
    out.tet[2][a] = ep[a];
  }
  auto contract = [&](R (&T)[3][3], const R* p, const R* q) {
    R s = R(0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s = s + T[a][b] * p[a] * q[b];
    return s;
  };
  const R Ett = contract(out.E, et, et), Epp = contract(out.E, ep, ep), Etp = contract(out.E, et, ep);
  const R Btt = contract(out.B, et, et), Bpp = contract(out.B, ep, ep), Btp = contract(out.B, et, ep);
  out.re = half * (Ett - Epp) - Btp;
  out.im = -Etp - half * (Btt - Bpp);
}

template <class R>
struct Point {
  R u[NGF], d1[NGF][3], d2[NGF][6], adv[NGF], diss[NGF];
};

template <class R, class T>
void gather(const oracle_params& P, const oracle_grid& g, const WeightsT<typename Exact<R>::W>& w, const T* u,
            long idx, bool want_rhs_terms, Point<R>& pt) {
  const long st[3] = {1, g.sy, g.sz};
  const R inv_h = Exact<R>::quot(1.0, g.h), inv_h2 = Exact<R>::inv_sq(g.h);
  for (int f = 0; f < NGF; ++f) {
    const T* p = u + f * g.sf + idx;
    pt.u[f] = R(p[0]);
    for (int k = 0; k < 3; ++k) pt.d1[f][k] = R(0.0);
    for (int s = 0; s < 6; ++s) pt.d2[f][s] = R(0.0);
    if (needs_d1(f) || (want_rhs_terms && !P.upwind))
      for (int k = 0; k < 3; ++k) pt.d1[f][k] = op_d1<R>(p, st[k], w, inv_h);
    if (needs_d2(f))
      for (int s = 0; s < 6; ++s) {
        const int a = PAIR[s][0], b = PAIR[s][1];
        pt.d2[f][s] = (a == b) ? op_d2<R>(p, st[a], w, inv_h2) : op_d11<R>(p, st[a], st[b], w, inv_h);
      }
  }
  if (!want_rhs_terms) return;
  const R beta[3] = {pt.u[BETA], pt.u[BETA + 1], pt.u[BETA + 2]};
  const R eps_over_h = Exact<R>::quot(P.eps_diss, g.h);
  for (int f = 0; f < NGF; ++f) {
    const T* p = u + f * g.sf + idx;
    R a = R(0.0);
    for (int k = 0; k < 3; ++k) {
      R dk = P.upwind ? op_upwind<R>(p, st[k], w, nonneg(beta[k]), inv_h) : pt.d1[f][k];
      a = a + beta[k] * dk;
    }
    pt.adv[f] = a;
    R d = R(0.0);
    if (P.ko_radius > 0)
      for (int k = 0; k < 3; ++k) d = d + op_ko<R>(p, st[k], P.ko_radius, eps_over_h);
    pt.diss[f] = d;
  }
}

int check(const oracle_params* P, const oracle_grid* g) {
  if (!P || !g) return -1;
  if (P->fd_order != 4 && P->fd_order != 8) return -1;
  if (P->bc < 0 || P->bc > 2) return -1;
  int need = P->fd_order / 2;
  if (P->upwind) need = need > P->fd_order / 2 + 1 ? need : P->fd_order / 2 + 1;
  if (P->ko_radius > need) need = P->ko_radius;
  if (g->ghost < need || g->h <= 0.0) return -1;
  for (int a = 0; a < 3; ++a)
    if (g->n[a] < 1) return -1;
  if (g->sy < g->n[0] + 2 * g->ghost || g->sz < g->sy * (g->n[1] + 2 * g->ghost) ||
      g->sf < g->sz * (g->n[2] + 2 * g->ghost))
    return -1;
  return 0;
}

void set_threads(const oracle_params* P) {
#ifdef _OPENMP
  if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
}

long at(const oracle_grid& g, int i, int j, int k) {
  return (long)(k + g.ghost) * g.sz + (long)(j + g.ghost) * g.sy + (i + g.ghost);
}

template <class T>
void rhs_grid(const oracle_params& P, const oracle_grid& g, const T* u, T* rhs) {
  const WeightsT<typename Exact<T>::W> w = make_weights_t<typename Exact<T>::W>(P.fd_order);
  const Opts o = {P.lapse, P.shift, P.eta};
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < g.n[2]; ++k) {
    Point<T> pt;
    T r[NGF];
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const long idx = at(g, i, j, k);
        gather<T>(P, g, w, u, idx, true, pt);
        rhs_point<T>(o, pt.u, pt.d1, pt.d2, pt.adv, pt.diss, r);
        for (int f = 0; f < NGF; ++f) rhs[f * g.sf + idx] = r[f];
      }
  }
}

// periodic images into every ghost point (edges and corners included)
template <class T>
void fill_periodic(const oracle_grid& g, T* u) {
  const int G = g.ghost;
#pragma omp parallel for schedule(static)
  for (int k = -G; k < g.n[2] + G; ++k)
    for (int j = -G; j < g.n[1] + G; ++j)
      for (int i = -G; i < g.n[0] + G; ++i) {
        const bool inside = i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2];
        if (inside) continue;
        const int ii = ((i % g.n[0]) + g.n[0]) % g.n[0];
        const int jj = ((j % g.n[1]) + g.n[1]) % g.n[1];
        const int kk = ((k % g.n[2]) + g.n[2]) % g.n[2];
        for (int f = 0; f < NGF; ++f) u[f * g.sf + at(g, i, j, k)] = u[f * g.sf + at(g, ii, jj, kk)];
      }
}

// ---------------------------------------------------------------------------
// Radiative (Sommerfeld) outer boundary.  With bc = 2 every ghost point is an
// evolved boundary point whose right-hand side is the outgoing-wave condition
//   d_t u = -v (x^i / r) d_i u - v (u - u_inf) / r,   r = |x| (at least h/2),
// which every u = u_inf + f(t - r/v) / r satisfies exactly.  x are the point's
// coordinates (origin + index * h), v = sqrt(2) for the lapse under 1+log
// slicing (its gauge speed in the asymptotic region) and 1 otherwise, u_inf
// the flat-space value (chi, alpha and gt_ii 1, all else 0).  d_i u is the
// second-order centred difference where both neighbours are stored points,
// else the second-order one-sided difference into the box.  Frozen gauge
// variables get zero, as in the interior.
// ---------------------------------------------------------------------------
template <class T>
T asymptotic_value(int f) {
  return (f == CHI || f == ALPHA || f == GT + 0 || f == GT + 3 || f == GT + 5) ? T(1.0) : T(0.0);
}

template <class T>
void boundary_rhs(const oracle_params& P, const oracle_grid& g, const T* u, T* rhs) {
  const int G = g.ghost;
  const long st[3] = {1, g.sy, g.sz};
  const T h = T(g.h), inv2h = Exact<T>::quot(1.0, 2.0 * g.h), half_h = h / T(2.0);
  const T root2 = std::sqrt(T(2.0));
#pragma omp parallel for schedule(static)
  for (int k = -G; k < g.n[2] + G; ++k)
    for (int j = -G; j < g.n[1] + G; ++j)
      for (int i = -G; i < g.n[0] + G; ++i) {
        const int c[3] = {i, j, k};
        const bool inside = i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2];
        if (inside) continue;
        T x[3];
        for (int a = 0; a < 3; ++a) x[a] = T(g.origin[a]) + T(double(c[a])) * h;
        T r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (r < half_h) r = half_h;
        const long idx = at(g, i, j, k);
        for (int f = 0; f < NGF; ++f) {
          const bool frozen = (f == ALPHA && P.lapse == 2) || (f >= BETA && P.shift == 1);
          if (frozen) {
            rhs[f * g.sf + idx] = T(0.0);
            continue;
          }
          const T v = (f == ALPHA && P.lapse == 0) ? root2 : T(1.0);
          const T* p = u + f * g.sf + idx;
          T xd = T(0.0);
          for (int a = 0; a < 3; ++a) {
            const long s = st[a];
            T d;
            if (c[a] > -G && c[a] < g.n[a] + G - 1)
              d = (p[s] - p[-s]) * inv2h;                                   // centred
            else if (c[a] == -G)
              d = (T(4.0) * (p[s] - p[0]) - (p[2 * s] - p[0])) * inv2h;     // forward
            else
              d = -(T(4.0) * (p[-s] - p[0]) - (p[-2 * s] - p[0])) * inv2h;  // backward
            xd = xd + x[a] * d;
          }
          rhs[f * g.sf + idx] = -(v * xd) / r - v * (p[0] - asymptotic_value<T>(f)) / r;
        }
      }
}

// the semi-discrete right-hand side: the BSSN equations at the interior
// points, and with the radiative boundary the boundary condition at the
// ghost points
template <class T>
void rhs_full(const oracle_params& P, const oracle_grid& g, const T* u, T* rhs) {
  rhs_grid<T>(P, g, u, rhs);
  if (P.bc == 2) boundary_rhs<T>(P, g, u, rhs);
}

// out = base + c * k at the points a step advances: the interior, and with
// the radiative boundary the ghost points too
template <class T>
void axpy_points(const oracle_params& P, const oracle_grid& g, const T* base, T c, const T* k, T* out) {
  const int G = P.bc == 2 ? g.ghost : 0;
#pragma omp parallel for schedule(static)
  for (int kz = -G; kz < g.n[2] + G; ++kz)
    for (int f = 0; f < NGF; ++f)
      for (int j = -G; j < g.n[1] + G; ++j)
        for (int i = -G; i < g.n[0] + G; ++i) {
          const long idx = f * g.sf + at(g, i, j, kz);
          out[idx] = base[idx] + c * k[idx];
        }
}

// nsteps classic RK4 steps, u advanced in place.  Stage inputs take their
// ghosts from u (static), from periodic images (periodic) or from their own
// boundary evolution (radiative).
// loop_seconds (may be null) receives the wall time of the step loop alone,
// without the allocation of the stage vectors.
template <class T>
void rk4(const oracle_params& P, const oracle_grid& g, double dt_in, int nsteps, T* u,
         double* loop_seconds = nullptr) {
  const size_t N = (size_t)g.sf * NGF;
  const T dt = T(dt_in), half = T(0.5), two = T(2.0), sixth = dt / T(6.0);
  std::vector<T> k1(N, T(0.0)), k2(N, T(0.0)), k3(N, T(0.0)), k4(N, T(0.0)), s(u, u + N);
  const auto t0 = std::chrono::steady_clock::now();
  const int G = P.bc == 2 ? g.ghost : 0;
  for (int step = 0; step < nsteps; ++step) {
    rhs_full<T>(P, g, u, k1.data());
    std::copy(u, u + N, s.begin());   // ghosts of the stage input
    axpy_points<T>(P, g, u, half * dt, k1.data(), s.data());
    if (P.bc == 1) fill_periodic<T>(g, s.data());
    rhs_full<T>(P, g, s.data(), k2.data());
    axpy_points<T>(P, g, u, half * dt, k2.data(), s.data());
    if (P.bc == 1) fill_periodic<T>(g, s.data());
    rhs_full<T>(P, g, s.data(), k3.data());
    axpy_points<T>(P, g, u, dt, k3.data(), s.data());
    if (P.bc == 1) fill_periodic<T>(g, s.data());
    rhs_full<T>(P, g, s.data(), k4.data());
#pragma omp parallel for schedule(static)
    for (int kz = -G; kz < g.n[2] + G; ++kz)
      for (int f = 0; f < NGF; ++f)
        for (int j = -G; j < g.n[1] + G; ++j)
          for (int i = -G; i < g.n[0] + G; ++i) {
            const long idx = f * g.sf + at(g, i, j, kz);
            u[idx] = u[idx] + sixth * (k1[idx] + two * k2[idx] + two * k3[idx] + k4[idx]);
          }
    if (P.bc == 1) fill_periodic<T>(g, u);
  }
  if (loop_seconds)
    *loop_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// nsteps third-order Runge-Kutta steps, u advanced in place: the strong
// stability preserving scheme of Shu and Osher (1988), each stage a convex
// combination of u_n and a forward-Euler step of the previous stage:
//   u1      = u_n + dt L(u_n)
//   u2      = 3/4 u_n + 1/4 (u1 + dt L(u1))
//   u_{n+1} = 1/3 u_n + 2/3 (u2 + dt L(u2))
// Stage inputs take their ghosts from u (static) or periodic images.
template <class T>
void rk3(const oracle_params& P, const oracle_grid& g, double dt_in, int nsteps, T* u) {
  const size_t N = (size_t)g.sf * NGF;
  const T dt = T(dt_in), three = T(3.0), four = T(4.0), one = T(1.0), two = T(2.0);
  const T a2 = three / four, b2 = one / four, a3 = one / three, b3 = two / three;
  std::vector<T> k(N, T(0.0)), s1(u, u + N), s2(u, u + N);
  const int G = P.bc == 2 ? g.ghost : 0;
  for (int step = 0; step < nsteps; ++step) {
    std::copy(u, u + N, s1.begin());   // ghosts of the stage inputs
    std::copy(u, u + N, s2.begin());
    rhs_full<T>(P, g, u, k.data());
    axpy_points<T>(P, g, u, dt, k.data(), s1.data());
    if (P.bc == 1) fill_periodic<T>(g, s1.data());
    rhs_full<T>(P, g, s1.data(), k.data());
#pragma omp parallel for schedule(static)
    for (int kz = -G; kz < g.n[2] + G; ++kz)
      for (int f = 0; f < NGF; ++f)
        for (int j = -G; j < g.n[1] + G; ++j)
          for (int i = -G; i < g.n[0] + G; ++i) {
            const long idx = f * g.sf + at(g, i, j, kz);
            s2[idx] = a2 * u[idx] + b2 * (s1[idx] + dt * k[idx]);
          }
    if (P.bc == 1) fill_periodic<T>(g, s2.data());
    rhs_full<T>(P, g, s2.data(), k.data());
#pragma omp parallel for schedule(static)
    for (int kz = -G; kz < g.n[2] + G; ++kz)
      for (int f = 0; f < NGF; ++f)
        for (int j = -G; j < g.n[1] + G; ++j)
          for (int i = -G; i < g.n[0] + G; ++i) {
            const long idx = f * g.sf + at(g, i, j, kz);
            u[idx] = a3 * u[idx] + b3 * (s2[idx] + dt * k[idx]);
          }
    if (P.bc == 1) fill_periodic<T>(g, u);
  }
}

// ---------------------------------------------------------------------------
// Several patches advanced together (the paper's framework owns ghost-zone
// synchronisation between grid sections, refinement and multi-block,
// section "Cactus-Carpet Computational Infrastructure"; its conclusion names
// adaptive mesh refinement and multi-block as the next step).  Reading:
//  * patches sit on refinement levels, h_L = h_0 / 2^L with h_0 the coarsest
//    spacing, vertex-centred (a level-L point with even global index along an
//    axis coincides with a level-(L-1) point); every origin lies on its
//    level's lattice through the first coarsest patch's origin;
//  * all patches take the same time step (no subcycling);
//  * after every Runge-Kutta stage the ghost points of every stage output are
//    refilled, level by level from the coarsest: a ghost point inside the
//    interior of another patch of its level takes that value (the lowest
//    such patch); otherwise on a refined level it is prolongated from the
//    first patch of the next coarser level whose stored box holds the whole
//    interpolation stencil -- per axis, the coincident coarse point, or for a
//    midpoint the order-p Lagrange interpolation of the p coarse points
//    around it (p = the finite-difference order; tensor product over the
//    axes); otherwise (coarsest level only) it is an outer-boundary point
//    and keeps the patch's own boundary treatment;
//  * at the end of every step, and once before the first, coarse interior
//    points that coincide with a finer level's interior point take its value
//    (injection, finest level first), then the ghosts are refilled.
// ---------------------------------------------------------------------------
struct HPatch {
  oracle_grid g;
  int level;
  long I0[3];   // global index of interior point (0,0,0) on its level's lattice
};

int make_hierarchy(const oracle_grid* gs, int np, std::vector<HPatch>& H) {
  if (np < 1) return -1;
  double h0 = 0.0;
  for (int p = 0; p < np; ++p) h0 = std::max(h0, gs[p].h);
  H.resize(np);
  int first = -1;
  for (int p = 0; p < np; ++p) {
    const double ratio = h0 / gs[p].h;
    const int L = (int)std::lround(std::log2(ratio));
    if (L < 0 || L > 20 || std::fabs(std::ldexp(h0, -L) - gs[p].h) > 1e-12 * gs[p].h) return -1;
    H[p].g = gs[p];
    H[p].level = L;
    if (L == 0 && first < 0) first = p;
  }
  for (int p = 0; p < np; ++p)
    for (int a = 0; a < 3; ++a) {
      const double q = (gs[p].origin[a] - gs[first].origin[a]) / gs[p].h;
      const long I = std::lround(q);
      if (std::fabs(q - (double)I) > 1e-9) return -1;
      H[p].I0[a] = I;
    }
  return 0;
}

bool in_interior(const HPatch& q, const long* I) {
  for (int a = 0; a < 3; ++a)
    if (I[a] < q.I0[a] || I[a] >= q.I0[a] + q.g.n[a]) return false;
  return true;
}

bool in_stored_box(const HPatch& q, long lo, long hi, int a) {
  return lo >= q.I0[a] - q.g.ghost && hi < q.I0[a] + q.g.n[a] + q.g.ghost;
}

// Lagrange weights of the p points at offsets -p/2+1 .. p/2 for the midpoint
// between offsets 0 and 1 (exact binary fractions: numerator and denominator
// are formed exactly, then divided once)
void midpoint_weights(int p, double* w) {
  const int m = p / 2;
  for (int k = -m + 1; k <= m; ++k) {
    double num = 1.0, den = 1.0;
    for (int j = -m + 1; j <= m; ++j) {
      if (j == k) continue;
      num *= 0.5 - j;
      den *= (double)(k - j);
    }
    w[k + m - 1] = num / den;
  }
}

// refill the ghost points of every patch (states: one state per patch)
template <class T>
int sync_ghosts(const std::vector<HPatch>& H, int order, T* const* st) {
  int maxL = 0;
  for (const HPatch& q : H) maxL = std::max(maxL, q.level);
  double wmid[8];
  midpoint_weights(order, wmid);
  const int m = order / 2;
  int bad = 0;
  for (int L = 0; L <= maxL; ++L)
    for (size_t p = 0; p < H.size(); ++p) {
      const HPatch& P = H[p];
      if (P.level != L) continue;
      const oracle_grid& g = P.g;
      const int G = g.ghost;
      for (int k = -G; k < g.n[2] + G; ++k)
        for (int j = -G; j < g.n[1] + G; ++j)
          for (int i = -G; i < g.n[0] + G; ++i) {
            if (i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2]) continue;
            const long gI[3] = {P.I0[0] + i, P.I0[1] + j, P.I0[2] + k};
            T* dst = st[p] + at(g, i, j, k);
            // same level
            int src = -1;
            for (size_t q = 0; q < H.size() && src < 0; ++q)
              if (q != p && H[q].level == L && in_interior(H[q], gI)) src = (int)q;
            if (src >= 0) {
              const HPatch& Q = H[src];
              const T* s = st[src] + at(Q.g, (int)(gI[0] - Q.I0[0]), (int)(gI[1] - Q.I0[1]), (int)(gI[2] - Q.I0[2]));
              for (int f = 0; f < NGF; ++f) dst[f * g.sf] = s[f * Q.g.sf];
              continue;
            }
            if (L == 0) continue;   // outer boundary
            // prolongation from level L-1: per axis the coarse taps
            long lo[3], hi[3];
            bool mid[3];
            for (int a = 0; a < 3; ++a) {
              // even global index: the coincident coarse point; odd: the
              // midpoint between coarse points (gI - 1)/2 and (gI + 1)/2
              // (exact divisions of even numbers, negative ones included)
              mid[a] = (gI[a] % 2 + 2) % 2 == 1;
              if (mid[a]) {
                const long left = (gI[a] - 1) / 2;
                lo[a] = left - m + 1;
                hi[a] = left + m;
              } else {
                lo[a] = hi[a] = gI[a] / 2;
              }
            }
            int cq = -1;
            for (size_t q = 0; q < H.size() && cq < 0; ++q) {
              if (H[q].level != L - 1) continue;
              bool ok = true;
              for (int a = 0; a < 3; ++a) ok = ok && in_stored_box(H[q], lo[a], hi[a], a);
              if (ok) cq = (int)q;
            }
            if (cq < 0) {
              ++bad;
              continue;
            }
            const HPatch& Q = H[cq];
            for (int f = 0; f < NGF; ++f) {
              T acc = T(0.0);
              for (long c2 = lo[2]; c2 <= hi[2]; ++c2)
                for (long c1 = lo[1]; c1 <= hi[1]; ++c1)
                  for (long c0 = lo[0]; c0 <= hi[0]; ++c0) {
                    const T w0 = mid[0] ? T(wmid[c0 - lo[0]]) : T(1.0);
                    const T w1 = mid[1] ? T(wmid[c1 - lo[1]]) : T(1.0);
                    const T w2 = mid[2] ? T(wmid[c2 - lo[2]]) : T(1.0);
                    const T v = st[cq][f * Q.g.sf + at(Q.g, (int)(c0 - Q.I0[0]), (int)(c1 - Q.I0[1]),
                                                      (int)(c2 - Q.I0[2]))];
                    acc = acc + w0 * w1 * w2 * v;
                  }
              dst[f * g.sf] = acc;
            }
          }
    }
  return bad ? -1 : 0;
}

// coarse interior points that coincide with a finer level's interior point
// take its value, finest level first
template <class T>
void restrict_levels(const std::vector<HPatch>& H, T* const* st) {
  int maxL = 0;
  for (const HPatch& q : H) maxL = std::max(maxL, q.level);
  for (int L = maxL; L >= 1; --L)
    for (size_t c = 0; c < H.size(); ++c) {
      const HPatch& C = H[c];
      if (C.level != L - 1) continue;
      for (int k = 0; k < C.g.n[2]; ++k)
        for (int j = 0; j < C.g.n[1]; ++j)
          for (int i = 0; i < C.g.n[0]; ++i) {
            const long fI[3] = {2 * (C.I0[0] + i), 2 * (C.I0[1] + j), 2 * (C.I0[2] + k)};
            for (size_t q = 0; q < H.size(); ++q) {
              if (H[q].level != L || !in_interior(H[q], fI)) continue;
              const HPatch& F = H[q];
              const T* s = st[q] + at(F.g, (int)(fI[0] - F.I0[0]), (int)(fI[1] - F.I0[1]), (int)(fI[2] - F.I0[2]));
              T* d = st[c] + at(C.g, i, j, k);
              for (int f = 0; f < NGF; ++f) d[f * C.g.sf] = s[f * F.g.sf];
              break;
            }
          }
    }
}

// nsteps RK4 (rk3 = false) or SSP RK3 steps of every patch with one dt,
// ghosts refilled after every stage, restriction and refill after every step
// (and once before the first)
template <class T>
int steps_synced(const oracle_params& P, const std::vector<HPatch>& H, T* const* u, double dt_in, int nsteps,
                 bool rk3) {
  const int np = (int)H.size();
  restrict_levels<T>(H, u);
  if (sync_ghosts<T>(H, P.fd_order, u)) return -1;
  const T dt = T(dt_in), half = T(0.5), two = T(2.0), sixth = dt / T(6.0);
  const T a2 = T(3.0) / T(4.0), b2 = T(1.0) / T(4.0), a3 = T(1.0) / T(3.0), b3 = T(2.0) / T(3.0);
  std::vector<std::vector<T>> k1(np), k2(np), k3(np), k4(np), s(np), s2(np);
  std::vector<T*> sp(np), s2p(np);
  for (int p = 0; p < np; ++p) {
    const size_t N = (size_t)H[p].g.sf * NGF;
    k1[p].assign(N, T(0.0));
    k2[p].assign(N, T(0.0));
    k3[p].assign(N, T(0.0));
    k4[p].assign(N, T(0.0));
    s[p].assign(N, T(0.0));
    s2[p].assign(N, T(0.0));
    sp[p] = s[p].data();
    s2p[p] = s2[p].data();
  }
  for (int step = 0; step < nsteps; ++step) {
    for (int p = 0; p < np; ++p) {
      const oracle_grid& g = H[p].g;
      const size_t N = (size_t)g.sf * NGF;
      std::copy(u[p], u[p] + N, s[p].begin());   // static ghosts of the stage inputs
      std::copy(u[p], u[p] + N, s2[p].begin());
      rhs_full<T>(P, g, u[p], k1[p].data());
      axpy_points<T>(P, g, u[p], rk3 ? dt : half * dt, k1[p].data(), s[p].data());
    }
    if (sync_ghosts<T>(H, P.fd_order, sp.data())) return -1;
    if (!rk3) {
      for (int p = 0; p < np; ++p) {
        rhs_full<T>(P, H[p].g, s[p].data(), k2[p].data());
        axpy_points<T>(P, H[p].g, u[p], half * dt, k2[p].data(), s[p].data());
      }
      if (sync_ghosts<T>(H, P.fd_order, sp.data())) return -1;
      for (int p = 0; p < np; ++p) {
        rhs_full<T>(P, H[p].g, s[p].data(), k3[p].data());
        axpy_points<T>(P, H[p].g, u[p], dt, k3[p].data(), s[p].data());
      }
      if (sync_ghosts<T>(H, P.fd_order, sp.data())) return -1;
      for (int p = 0; p < np; ++p) {
        const oracle_grid& g = H[p].g;
        rhs_full<T>(P, g, s[p].data(), k4[p].data());
        const int G = P.bc == 2 ? g.ghost : 0;
        for (int kz = -G; kz < g.n[2] + G; ++kz)
          for (int f = 0; f < NGF; ++f)
            for (int j = -G; j < g.n[1] + G; ++j)
              for (int i = -G; i < g.n[0] + G; ++i) {
                const long idx = f * g.sf + at(g, i, j, kz);
                u[p][idx] = u[p][idx] + sixth * (k1[p][idx] + two * k2[p][idx] + two * k3[p][idx] + k4[p][idx]);
              }
      }
    } else {
      for (int p = 0; p < np; ++p) {
        const oracle_grid& g = H[p].g;
        rhs_full<T>(P, g, s[p].data(), k2[p].data());
        const int G = P.bc == 2 ? g.ghost : 0;
        for (int kz = -G; kz < g.n[2] + G; ++kz)
          for (int f = 0; f < NGF; ++f)
            for (int j = -G; j < g.n[1] + G; ++j)
              for (int i = -G; i < g.n[0] + G; ++i) {
                const long idx = f * g.sf + at(g, i, j, kz);
                s2[p][idx] = a2 * u[p][idx] + b2 * (s[p][idx] + dt * k2[p][idx]);
              }
      }
      if (sync_ghosts<T>(H, P.fd_order, s2p.data())) return -1;
      for (int p = 0; p < np; ++p) {
        const oracle_grid& g = H[p].g;
        rhs_full<T>(P, g, s2[p].data(), k3[p].data());
        const int G = P.bc == 2 ? g.ghost : 0;
        for (int kz = -G; kz < g.n[2] + G; ++kz)
          for (int f = 0; f < NGF; ++f)
            for (int j = -G; j < g.n[1] + G; ++j)
              for (int i = -G; i < g.n[0] + G; ++i) {
                const long idx = f * g.sf + at(g, i, j, kz);
                u[p][idx] = a3 * u[p][idx] + b3 * (s2[p][idx] + dt * k3[p][idx]);
              }
      }
    }
    restrict_levels<T>(H, u);
    if (sync_ghosts<T>(H, P.fd_order, u)) return -1;
  }
  return 0;
}

}  // namespace

extern "C" {

int oracle_required_ghost(int order, int upwind, int ko_radius) {
  int need = order / 2;
  if (upwind && order / 2 + 1 > need) need = order / 2 + 1;
  return ko_radius > need ? ko_radius : need;
}

// Right-hand side at every interior point and, with the radiative boundary,
// at every ghost point; other entries of rhs (static or periodic ghosts, row
// padding) are untouched.
int oracle_rhs(const oracle_params* P, const oracle_grid* g, const double* u, double* rhs) {
  if (check(P, g) || !u || !rhs) return -1;
  set_threads(P);
  rhs_full<double>(*P, *g, u, rhs);
  return 0;
}

// nsteps classic RK4 steps, u advanced in place.  Stage inputs take their
// ghosts from u (static) or from periodic images (periodic).
int oracle_rk4(const oracle_params* P, const oracle_grid* g, double dt, int nsteps, double* u) {
  if (check(P, g) || !u || !(dt > 0.0) || nsteps < 0) return -1;
  set_threads(P);
  rk4<double>(*P, *g, dt, nsteps, u);
  return 0;
}

// oracle_rk4, with the wall time of the step loop (allocation of the stage
// vectors excluded) stored in *seconds: the timing of the CPU baseline.
int oracle_rk4_timed(const oracle_params* P, const oracle_grid* g, double dt, int nsteps, double* u,
                     double* seconds) {
  if (check(P, g) || !u || !(dt > 0.0) || nsteps < 0 || !seconds) return -1;
  set_threads(P);
  rk4<double>(*P, *g, dt, nsteps, u, seconds);
  return 0;
}

// nsteps third-order SSP Runge-Kutta steps (Shu-Osher), u advanced in place.
int oracle_rk3(const oracle_params* P, const oracle_grid* g, double dt, int nsteps, double* u) {
  if (check(P, g) || !u || !(dt > 0.0) || nsteps < 0) return -1;
  set_threads(P);
  rk3<double>(*P, *g, dt, nsteps, u);
  return 0;
}

// The same right-hand side and RK4 steps evaluated in x87 extended precision
// (inputs and outputs FP64): the reference for measuring FP64 rounding error.
int oracle_rhs_ext(const oracle_params* P, const oracle_grid* g, const double* u, double* rhs) {
  if (check(P, g) || !u || !rhs) return -1;
  set_threads(P);
  const size_t N = (size_t)g->sf * NGF;
  std::vector<long double> U(u, u + N), K(N, 0.0L);
  rhs_full<long double>(*P, *g, U.data(), K.data());
  const int G = P->bc == 2 ? g->ghost : 0;
  for (int kz = -G; kz < g->n[2] + G; ++kz)
    for (int f = 0; f < NGF; ++f)
      for (int j = -G; j < g->n[1] + G; ++j)
        for (int i = -G; i < g->n[0] + G; ++i) {
          const long idx = f * g->sf + at(*g, i, j, kz);
          rhs[idx] = (double)K[idx];
        }
  return 0;
}

// significand bits of the extended type (64 for x87)
int oracle_ext_mant_dig(void) { return LDBL_MANT_DIG; }

int oracle_rk4_ext(const oracle_params* P, const oracle_grid* g, double dt, int nsteps, double* u) {
  if (check(P, g) || !u || !(dt > 0.0) || nsteps < 0) return -1;
  set_threads(P);
  const size_t N = (size_t)g->sf * NGF;
  std::vector<long double> U(u, u + N);
  rk4<long double>(*P, *g, dt, nsteps, U.data());
  for (size_t i = 0; i < N; ++i) u[i] = (double)U[i];
  return 0;
}

int oracle_rk3_ext(const oracle_params* P, const oracle_grid* g, double dt, int nsteps, double* u) {
  if (check(P, g) || !u || !(dt > 0.0) || nsteps < 0) return -1;
  set_threads(P);
  const size_t N = (size_t)g->sf * NGF;
  std::vector<long double> U(u, u + N);
  rk3<long double>(*P, *g, dt, nsteps, U.data());
  for (size_t i = 0; i < N; ++i) u[i] = (double)U[i];
  return 0;
}

// Several patches (grids[p], states[p]): refill every ghost point from the
// patches of the same or the next coarser level (see sync_ghosts).  -1 if
// the spacings or origins do not form a hierarchy, or a refined patch has a
// ghost point neither source covers.
int oracle_sync_ghosts(const oracle_params* P, const oracle_grid* grids, double* const* states, int npatch) {
  if (!P || !grids || !states || npatch < 1) return -1;
  std::vector<HPatch> H;
  if (make_hierarchy(grids, npatch, H)) return -1;
  for (int p = 0; p < npatch; ++p)
    if (check(P, &grids[p]) || !states[p]) return -1;
  return sync_ghosts<double>(H, P->fd_order, states);
}

// Injection of finer interior points into coincident coarse interior points.
int oracle_restrict(const oracle_params* P, const oracle_grid* grids, double* const* states, int npatch) {
  if (!P || !grids || !states || npatch < 1) return -1;
  std::vector<HPatch> H;
  if (make_hierarchy(grids, npatch, H)) return -1;
  restrict_levels<double>(H, states);
  return 0;
}

// nsteps RK4 (integrator 4) or SSP RK3 (integrator 3) steps of all patches
// together with one dt: ghosts refilled after every stage, restriction and
// refill after every step and once before the first.  Periodic boundaries
// are not combined with several patches (-1).
int oracle_steps_synced(const oracle_params* P, const oracle_grid* grids, double* const* states, int npatch,
                        double dt, int nsteps, int integrator) {
  if (!P || !grids || !states || npatch < 1 || !(dt > 0.0) || nsteps < 0) return -1;
  if (P->bc == 1 || (integrator != 3 && integrator != 4)) return -1;
  std::vector<HPatch> H;
  if (make_hierarchy(grids, npatch, H)) return -1;
  for (int p = 0; p < npatch; ++p)
    if (check(P, &grids[p]) || !states[p]) return -1;
  set_threads(P);
  return steps_synced<double>(*P, H, states, dt, nsteps, integrator == 3);
}

int oracle_fill_periodic(const oracle_grid* g, double* u) {
  if (!g || !u) return -1;
  fill_periodic<double>(*g, u);
  return 0;
}

// Hamiltonian constraint at interior points into H (one GF with the grid's
// strides; ghost entries untouched).
int oracle_hamiltonian(const oracle_params* P, const oracle_grid* g, const double* u, double* H) {
  if (check(P, g) || !u || !H) return -1;
  set_threads(P);
  const Weights w = make_weights(P->fd_order);
  const oracle_grid G = *g;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < G.n[2]; ++k) {
    Point<double> pt;
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        const long idx = at(G, i, j, k);
        gather<double, double>(*P, G, w, u, idx, false, pt);
        H[idx] = ham_point<double>(pt.u, pt.d1, pt.d2);
      }
  }
  return 0;
}

// Momentum constraint M_i (three grid functions with the patch's strides,
// M[i * sf + idx]) at every interior point, from the centred first
// derivatives of the patch's finite-difference order.
int oracle_momentum(const oracle_params* P, const oracle_grid* g, const double* u, double* M) {
  if (check(P, g) || !u || !M) return -1;
  set_threads(P);
  const Weights w = make_weights(P->fd_order);
  const oracle_grid G = *g;
  const long st[3] = {1, G.sy, G.sz};
  const double inv_h = 1.0 / G.h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < G.n[2]; ++k) {
    double v[NGF], d1[NGF][3];
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        const long idx = at(G, i, j, k);
        // first derivatives of every grid function (the right-hand side's
        // gather skips those it does not need, At among them)
        for (int f = 0; f < NGF; ++f) {
          const double* q = u + f * G.sf + idx;
          v[f] = q[0];
          for (int a = 0; a < 3; ++a) d1[f][a] = op_d1<double>(q, st[a], w, inv_h);
        }
        double m[3];
        mom_point<double>(v, d1, m);
        for (int a = 0; a < 3; ++a) M[a * G.sf + idx] = m[a];
      }
  }
  return 0;
}

// Psi4 at every interior point into out[0 * sf + idx] (real part) and
// out[1 * sf + idx] (imaginary part), from centred first and second
// derivatives of the patch's order (the right-hand side's stencils) of
// chi, gt, K, At and Gt; coordinates from the grid's origin and spacing.
int oracle_psi4(const oracle_params* P, const oracle_grid* g, const double* u, double* out) {
  if (check(P, g) || !u || !out) return -1;
  set_threads(P);
  const Weights w = make_weights(P->fd_order);
  const oracle_grid G = *g;
  const long st[3] = {1, G.sy, G.sz};
  const double inv_h = 1.0 / G.h, inv_h2 = 1.0 / (G.h * G.h);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < G.n[2]; ++k) {
    double v[NGF], d1[NGF][3], d2[NGF][6];
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        const long idx = at(G, i, j, k);
        for (int f = 0; f < NGF; ++f) {
          const double* q = u + f * G.sf + idx;
          v[f] = q[0];
          for (int a = 0; a < 3; ++a) d1[f][a] = 0.0;
          for (int sl = 0; sl < 6; ++sl) d2[f][sl] = 0.0;
          if (f >= BETA || f == ALPHA) continue;   // the gauge does not enter
          for (int a = 0; a < 3; ++a) d1[f][a] = op_d1<double>(q, st[a], w, inv_h);
          if (f == CHI || (f >= GT && f < GT + 6))
            for (int sl = 0; sl < 6; ++sl) {
              const int a = PAIR[sl][0], b = PAIR[sl][1];
              d2[f][sl] = (a == b) ? op_d2<double>(q, st[a], w, inv_h2) : op_d11<double>(q, st[a], st[b], w, inv_h);
            }
        }
        const double xyz[3] = {G.origin[0] + i * G.h, G.origin[1] + j * G.h, G.origin[2] + k * G.h};
        Psi4Out<double> o;
        psi4_point<double>(v, d1, d2, xyz, o);
        out[idx] = o.re;
        out[G.sf + idx] = o.im;
      }
  }
  return 0;
}

// Psi4 at one point from caller-supplied values and derivatives (d1: 24x3,
// d2: 24x6 in slot order xx xy xz yy yz zz) and coordinates; res receives
// re, im, E (9, row-major), B (9) and the tetrad e_r, e_theta, e_phi (9).
int oracle_psi4_point(const double* u, const double* d1, const double* d2, const double* xyz, double* res) {
  if (!u || !d1 || !d2 || !xyz || !res) return -1;
  double D1[NGF][3], D2[NGF][6];
  std::memcpy(D1, d1, sizeof D1);
  std::memcpy(D2, d2, sizeof D2);
  Psi4Out<double> o;
  psi4_point<double>(u, D1, D2, xyz, o);
  res[0] = o.re;
  res[1] = o.im;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      res[2 + 3 * a + b] = o.E[a][b];
      res[11 + 3 * a + b] = o.B[a][b];
      res[20 + 3 * a + b] = o.tet[a][b];
    }
  return 0;
}

int oracle_mom_point(const double* u, const double* d1, double* M) {
  if (!u || !d1 || !M) return -1;
  double D1[NGF][3];
  std::memcpy(D1, d1, sizeof D1);
  mom_point<double>(u, D1, M);
  return 0;
}

// Algebraic constraints of the conformal variables: det(gt) = 1 and
// gt^ij At_ij = 0.  They are restored (the usual practice of moving-puncture
// BSSN codes; the paper does not spell it out) at every interior point by
//   gt_ij <- gt_ij / det(gt)^(1/3),   At_ij <- At_ij - 1/3 gt_ij (gt^kl At_kl)
// with gt and its inverse taken after the rescaling.  Periodic boundaries:
// the ghosts are refilled with the images; static ghosts are left alone.
int oracle_enforce_algebraic(const oracle_params* P, const oracle_grid* g, double* u) {
  if (check(P, g) || !u) return -1;
  set_threads(P);
  const oracle_grid G = *g;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < G.n[2]; ++k)
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        const long idx = at(G, i, j, k);
        double m[3][3], A[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            m[a][b] = u[(GT + SYM[a][b]) * G.sf + idx];
            A[a][b] = u[(AT + SYM[a][b]) * G.sf + idx];
          }
        const double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                           m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
        const double s = std::cbrt(det);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) m[a][b] = m[a][b] / s;
        // inverse of the rescaled metric: adjugate over its determinant
        const double dn = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                          m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                          m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
        double inv[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            const int a1 = (b + 1) % 3, a2 = (b + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
            inv[a][b] = (m[a1][b1] * m[a2][b2] - m[a1][b2] * m[a2][b1]) / dn;
          }
        double tr = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) tr = tr + inv[a][b] * A[a][b];
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) {
            u[(GT + SYM[a][b]) * G.sf + idx] = m[a][b];
            u[(AT + SYM[a][b]) * G.sf + idx] = A[a][b] - m[a][b] * tr / 3.0;
          }
      }
  if (P->bc == 1) fill_periodic<double>(G, u);
  return 0;
}

// Pointwise algebra with caller-supplied derivatives (d1: 24x3, d2: 24x6 in
// slot order xx xy xz yy yz zz, adv and diss: 24).
int oracle_rhs_point(const oracle_params* P, const double* u, const double* d1, const double* d2,
                     const double* adv, const double* diss, double* rhs) {
  if (!P || !u || !d1 || !d2 || !adv || !diss || !rhs) return -1;
  const Opts o = {P->lapse, P->shift, P->eta};
  double D1[NGF][3], D2[NGF][6];
  std::memcpy(D1, d1, sizeof D1);
  std::memcpy(D2, d2, sizeof D2);
  rhs_point<double>(o, u, D1, D2, adv, diss, rhs);
  return 0;
}

int oracle_ham_point(const double* u, const double* d1, const double* d2, double* H) {
  if (!u || !d1 || !d2 || !H) return -1;
  double D1[NGF][3], D2[NGF][6];
  std::memcpy(D1, d1, sizeof D1);
  std::memcpy(D2, d2, sizeof D2);
  *H = ham_point<double>(u, D1, D2);
  return 0;
}

// One operator on one grid function at every interior point (for pinning the
// stencils): op 0 = D1(axis a), 1 = D2(axis a), 2 = D_a D_b, 3 = lopsided
// (+), 4 = lopsided (-), 5 = Kreiss-Oliger(axis a, radius r, eps).
int oracle_apply_op(int op, int a, int b, int order, int r, double eps, const oracle_grid* g,
                    const double* f, double* out) {
  if (!g || !f || !out || (order != 4 && order != 8) || a < 0 || a > 2 || b < 0 || b > 2) return -1;
  const Weights w = make_weights(order);
  const oracle_grid G = *g;
  const long st[3] = {1, G.sy, G.sz};
  const double inv_h = 1.0 / G.h;
  for (int k = 0; k < G.n[2]; ++k)
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        const long idx = at(G, i, j, k);
        const double* p = f + idx;
        double v = 0.0;
        switch (op) {
          case 0: v = op_d1<double>(p, st[a], w, inv_h); break;
          case 1: v = op_d2<double>(p, st[a], w, inv_h * inv_h); break;
          case 2: v = op_d11<double>(p, st[a], st[b], w, inv_h); break;
          case 3: v = op_upwind<double>(p, st[a], w, true, inv_h); break;
          case 4: v = op_upwind<double>(p, st[a], w, false, inv_h); break;
          case 5: v = op_ko<double>(p, st[a], r, eps / G.h); break;
          default: return -1;
        }
        out[idx] = v;
      }
  return 0;
}

// Exact operation count of the right-hand side at one interior point
// (counts[0] = additions/subtractions, [1] = multiplications, [2] = divisions),
// counted by running the same code on a counting scalar.  Constants 1/h,
// 1/h^2, eps/h are per-grid and not counted.
int oracle_count_rhs_flops(const oracle_params* P, const oracle_grid* g, const double* u, int i, int j,
                           int k, long long* counts) {
  if (check(P, g) || !u || !counts) return -1;
  const Weights w = make_weights(P->fd_order);
  const Opts o = {P->lapse, P->shift, P->eta};
  Point<Counted> pt;
  Counted r[NGF];
  Counted::nadd = Counted::nmul = Counted::ndiv = 0;
  gather<Counted, double>(*P, *g, w, u, at(*g, i, j, k), true, pt);
  rhs_point<Counted>(o, pt.u, pt.d1, pt.d2, pt.adv, pt.diss, r);
  counts[0] = Counted::nadd;
  counts[1] = Counted::nmul;
  counts[2] = Counted::ndiv;
  return 0;
}

}  // extern "C"
