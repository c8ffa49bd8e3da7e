// stage_lds.hpp -- LDS-staged fused RK-stage kernel.
//
// A work-group owns a 64 x 4 tile of one z-plane (one wave per x-row).  The
// right-hand side is evaluated grid function by grid function in dependency
// order (beta, gt, chi, alpha, Gt, K, At, B).  Each grid function's stencil
// neighbourhood is staged into LDS by direct global->LDS loads (one
// buffer_load_dwordx4 ... lds per row of up to 128 doubles; no registers
// involved), double-buffered: the rows of the next grid function are in
// flight while the work-items evaluate the current one's stencils from LDS
// with compile-time immediate offsets.  One barrier per grid function.
//
// LDS layout per staged grid function (pitch P = 64 + 2R doubles):
//   plane dz = 0            rows y in [-R,  3+R]   (x and y stencils, xy mixed)
//   planes 1 <= |dz| <= RM  rows y in [-RM, 3+RM]  (xz / yz mixed, z stencils)
//   planes RM < |dz| <= R   rows y in [0, 3]       (z stencils only)
// with R the axis reach (upwind, Kreiss-Oliger) and RM the mixed reach.
// Grid functions that need no second derivatives stage only the axis cross.
#pragma once

#include "stage_kernel.hpp"

namespace chemora {

template <int R, int RM>
struct LdsLayout {
  static constexpr int TX = 64, TY = 4;
  static constexpr int P = TX + 2 * R;
  static constexpr int ROWS0 = TY + 2 * R, ROWS1 = TY + 2 * RM, ROWS2 = TY;
  static constexpr int SIZE = P * (ROWS0 + 2 * RM * ROWS1 + 2 * (R - RM) * ROWS2);
  // first row (y = -yhalo) of plane dz, in doubles
  __host__ __device__ static constexpr int plane(int dz) {
    const int a = dz < 0 ? -dz : dz;
    if (a == 0) return 0;
    if (a <= RM) return P * (ROWS0 + ((dz > 0 ? 2 * a - 1 : 2 * a) - 1) * ROWS1);
    return P * (ROWS0 + 2 * RM * ROWS1 + ((dz > 0 ? 2 * (a - RM) - 1 : 2 * (a - RM)) - 1) * ROWS2);
  }
  __host__ __device__ static constexpr int yhalo(int dz) {
    const int a = dz < 0 ? -dz : dz;
    return a == 0 ? R : (a <= RM ? RM : 0);
  }
  // offset (doubles) of tap (dx, dy, dz) from the work-item's anchor ty*P + tx
  __host__ __device__ static constexpr int off(int dx, int dy, int dz) {
    return plane(dz) + (dy + yhalo(dz)) * P + (dx + R);
  }
};

// One staged row: plane dz, tile-relative row y, x range [xlo, xhi].
struct RowDesc {
  int dz, y, xlo, xhi;
};

// Row r of the staging list of a grid function.  FULL lists (second-derivative
// GFs) hold the whole dz = 0 plane with halo R, the planes 1 <= |dz| <= RM with
// halo RM and the planes RM < |dz| <= R without halo; CROSS lists (axis
// stencils only) hold the dz = 0 plane as an x-cross plus y-halo columns and
// the other planes without halo.  Planes are ordered dz = 0, +1, -1, +2, -2, ...
// r is wave-uniform, so the decoding is scalar arithmetic.
template <int R, int RM, bool FULL>
struct RowList {
  static constexpr int TY = 4, TX = 64;
  __host__ __device__ static constexpr int plane_rows(int a) {
    return a == 0 ? TY + 2 * R : ((FULL && a <= RM) ? TY + 2 * RM : TY);
  }
  __host__ __device__ static constexpr int count() {
    int n = plane_rows(0);
    for (int a = 1; a <= R; ++a) n += 2 * plane_rows(a);
    return n;
  }
  __device__ __forceinline__ static RowDesc row(int r) {
    RowDesc d;
    if (r < plane_rows(0)) {
      const int y = r - R;
      const bool wide = FULL || (y >= 0 && y < TY);
      d.dz = 0;
      d.y = y;
      d.xlo = wide ? -R : 0;
      d.xhi = wide ? TX - 1 + R : TX - 1;
      return d;
    }
    r -= plane_rows(0);
#pragma unroll
    for (int a = 1; a <= R; ++a) {
      const int n = plane_rows(a);
      const int halo = (n - TY) / 2;
      if (r < 2 * n) {
        d.dz = r < n ? a : -a;
        d.y = (r < n ? r : r - n) - halo;
        d.xlo = -halo;
        d.xhi = TX - 1 + halo;
        return d;
      }
      r -= 2 * n;
    }
    d.dz = 0; d.y = 1 << 20; d.xlo = 0; d.xhi = -1;   // past the end: nothing to stage
    return d;
  }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

template <int ORDER, bool UPWIND, int R, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CHEMORA_WAVES_PER_EU)))
void stage_lds_kernel(StageArgs a) {
  using St = Stencil<ORDER>;
  constexpr int RM = ORDER / 2;
  using L = LdsLayout<R, RM>;
  __shared__ double buf0[L::SIZE];
  __shared__ double buf1[L::SIZE];

  const Geo G = a.geo;
  const int nblocks = a.tiles_x * a.tiles_y * G.nz;
  const int t = xcd_tile(blockIdx.x, nblocks);
  const int txi = t % a.tiles_x;
  const int tyi = (t / a.tiles_x) % a.tiles_y;
  const int k = t / (a.tiles_x * a.tiles_y);
  const int lane = threadIdx.x, wave = threadIdx.y;
  const int i0 = txi * TILE_X, j0 = tyi * TILE_Y;
  const bool valid = (i0 + lane < G.nx) && (j0 + wave < G.ny);
  // global accesses of work-items outside the interior use a clamped point
  const int ic = min(i0 + lane, G.nx - 1), jc = min(j0 + wave, G.ny - 1);

  // byte offsets are unsigned 32-bit (the host limits a state to 4 GiB)
  const unsigned sy = (unsigned)G.sy, sz = (unsigned)G.sz, sf = (unsigned)G.sf, gg = (unsigned)G.g;
  const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, G.sf);
  const unsigned vpt = (jc * sy + ic + gg) * 8u + XB * 8u;       // the point (pointwise buffers)
  const unsigned spt = ((k + gg) * sz + gg * sy) * 8u;          // its z plane / ghost offset
  auto val = [&](int f) __attribute__((always_inline)) { return bload(rin, vpt, spt + f * sf * 8u); };

  // ---- staging: every wave issues the rows r = wave, wave+4, ... of grid
  // function f into LDS buffer dst.  A row of W (even) doubles is one
  // dwordx4 direct-to-LDS load (lane l moves doubles 2l, 2l+1).  Columns past
  // the array end of a ragged tile are skipped; a lone last column is moved
  // through a register.
  const int xmax = G.nx - 1 + R - i0;       // last tile-relative x column inside the array
  const int ymax = G.ny - 1 + R - j0;
  auto issue = [&](int f, auto list, double* dst) __attribute__((always_inline)) {
    using List = decltype(list);
    constexpr int NR = List::count();
    constexpr int PER = (NR + 3) / 4;
#pragma unroll
    for (int n = 0; n < PER; ++n) {
      const int r = wave + 4 * n;
      if (r < NR) {
        const RowDesc d = List::row(r);
        if (d.y <= ymax) {
          double* row = dst + (L::plane(d.dz) + (d.y + L::yhalo(d.dz)) * L::P + R + d.xlo);
          const unsigned so =
              (f * sf + (k + gg + d.dz) * sz + (j0 + gg + d.y) * sy + i0 + gg + d.xlo) * 8u;
          const int w = min((int)(d.xhi - d.xlo + 1), xmax - d.xlo + 1);   // columns to move
          if (2 * lane + 1 < w)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr_t)row, 16, (XB + 2 * lane) * 8u, so, 0, 0);
          if (w > 0 && (w & 1) && 2 * lane + 1 == w)   // odd tail: one double
            row[w - 1] = bload(rin, (XB + w - 1) * 8u, so);
        }
      }
    }
  };
  auto issue_gf = [&](int f, bool full, double* dst) __attribute__((always_inline)) {
    if (full)
      issue(f, RowList<R, RM, true>{}, dst);
    else
      issue(f, RowList<R, RM, false>{}, dst);
  };
  auto sync = [&]() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };

  const int anchor = wave * L::P + lane;
  // stencil access into the buffer of the current phase
  auto make_ops = [&](const double* cur) __attribute__((always_inline)) {
    auto tap = [=](int dx, int dy, int dz) __attribute__((always_inline)) { return cur[anchor + L::off(dx, dy, dz)]; };
    return tap;
  };
  const double bet[3] = {val(gBETA), val(gBETA + 1), val(gBETA + 2)};
  auto D1 = [&](auto tap, int ax) __attribute__((always_inline)) {
    return St::first([&](int o) { return ax == 0 ? tap(o, 0, 0) : (ax == 1 ? tap(0, o, 0) : tap(0, 0, o)); }) *
           a.sc.d1;
  };
  auto D2 = [&](auto tap, int slot) __attribute__((always_inline)) {
    const int ai = SI(slot), bj = SJ(slot);
    auto along = [&](int o) __attribute__((always_inline)) { return ai == 0 ? tap(o, 0, 0) : (ai == 1 ? tap(0, o, 0) : tap(0, 0, o)); };
    if (ai == bj) return St::second(along) * a.sc.d2;
    const double v = St::first([&](int oa) {
      return St::first([&](int ob) {
        int d[3] = {0, 0, 0};
        d[ai] = oa;
        d[bj] = ob;
        return tap(d[0], d[1], d[2]);
      });
    });
    return v * a.sc.d11;
  };
  // advection + dissipation of the staged GF; rhs = (algebra + adv) + diss
  auto finish = [&](auto tap, double alg) __attribute__((always_inline)) {
    double adv = 0.0, diss = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      auto along = [&](int o) __attribute__((always_inline)) { return ax == 0 ? tap(o, 0, 0) : (ax == 1 ? tap(0, o, 0) : tap(0, 0, o)); };
      double d;
      if (UPWIND) {
        // both lopsided stencils from the same taps, then select by the sign of beta
        const double dp = St::lopsided(along, 1);
        const double dm = -St::lopsided([&](int o) { return along(-o); }, 1);
        d = (bet[ax] >= 0.0 ? dp : dm) * a.sc.up;
      } else {
        d = St::first(along) * a.sc.d1;
      }
      adv += bet[ax] * d;
      if (a.sc.ko_r > 0) {
        const double qd = ko_axis(along, a.sc.ko_r, a.sc.ko);
        diss = (ax == 0) ? qd : diss + qd;
      }
    }
    return (alg + adv) + diss;
  };
  auto emit = [&](int f, double kf) __attribute__((always_inline)) {
    if (!valid) return;
    const unsigned so = spt + f * sf * 8u;
    if (MODE == MODE_RHS) {
      bstore(state_rsrc(a.out, G.sf), vpt, so, kf);
    } else if (MODE == MODE_STAGE1) {
      const double u0 = val(f);
      bstore(state_rsrc(a.y, G.sf), vpt, so, u0 + a.cy * kf);
      bstore(state_rsrc(a.out, G.sf), vpt, so, u0 + a.cs * kf);
    } else if (MODE == MODE_STAGE23) {
      const double y0 = bload(state_rsrc(a.y, G.sf), vpt, so);
      const double u0 = bload(state_rsrc(a.un, G.sf), vpt, so);
      bstore(state_rsrc(a.y, G.sf), vpt, so, y0 + a.cy * kf);
      bstore(state_rsrc(a.out, G.sf), vpt, so, u0 + a.cs * kf);
    } else {
      const double y0 = bload(state_rsrc(a.y, G.sf), vpt, so);
      bstore(state_rsrc(a.out, G.sf), vpt, so, y0 + a.cy * kf);
    }
  };

  // staging sequence: 24 phases (B only with the Gamma-driver shift)
  const Gauge& gauge = a.gauge;
  const bool driver = gauge.shift == 0;
  auto seq_gf = [&](int p) __attribute__((always_inline)) -> int {
    // beta(3) gt(6) chi alpha Gt(3) K At(6) B(3)
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
  // phase p computes from buffer p&1 after issuing phase p+1 into the other
  auto begin = [&](int p) __attribute__((always_inline)) {
    if (p + 1 < nphase) issue_gf(seq_gf(p + 1), p + 1 < 11, ((p + 1) & 1) ? buf1 : buf0);
  };

  const double alpha = val(gALPHA), chi = val(gCHI), K = val(gK);
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
  // traceless extrinsic curvature, raised (point values only)
  double A[6], Au[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) A[s] = val(gAT + s);
  {
    double Am[3][3];
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

  issue_gf(seq_gf(0), true, buf0);
  sync();

  // ---- shift (phases 0-2)
  double db[3][3];
  double xts[3] = {0.0, 0.0, 0.0};
  double ddiv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    begin(c);
    auto tap = make_ops((c & 1) ? buf1 : buf0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) db[c][ax] = D1(tap, ax);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double dd = D2(tap, q);
      xts[c] += W(q) * gu[q] * dd;
      const int qi = SI(q), qj = SJ(q);
      if (qj == c) ddiv[qi] += dd;
      if (qi == c && qi != qj) ddiv[qj] += dd;
    }
    emit(gBETA + c, driver ? finish(tap, 0.75 * val(gB + c)) : 0.0);
    keep(db[c]);
    keep(xts);
    keep(ddiv);
    sync();
  }
  const double divb = db[0][0] + db[1][1] + db[2][2];

  // ---- conformal metric (phases 3-8)
  double Ric[6];
  double Gu[3][6];
  double Gd[3];
  {
    double dg[6][3];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int p = 3 + s;
      begin(p);
      auto tap = make_ops((p & 1) ? buf1 : buf0);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) dg[s][ax] = D1(tap, ax);
      double r = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) r += W(q) * gu[q] * D2(tap, q);
      Ric[s] = -0.5 * r;
      const int i = SI(s), jj = SJ(s);
      double lie = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) lie += g[S(i, kk)] * db[kk][jj] + g[S(jj, kk)] * db[kk][i];
      emit(gGT + s, finish(tap, -2.0 * alpha * A[s] + lie - (2.0 / 3.0) * g[s] * divb));
      keep(Ric[s]);
      keep(dg[s]);
      sync();
    }
    double Gl[3][6];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), jj = SJ(s);
        Gl[kk][s] = 0.5 * (dg[S(kk, i)][jj] + dg[S(kk, jj)][i] - dg[s][kk]);
      }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int s = 0; s < 6; ++s)
        Gu[kk][s] = gu[S(kk, 0)] * Gl[0][s] + gu[S(kk, 1)] * Gl[1][s] + gu[S(kk, 2)] * Gl[2][s];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < 6; ++s) acc += W(s) * gu[s] * Gu[kk][s];
      Gd[kk] = acc;
    }
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
          const double gmi = gu[S(0, m)] * Gu[kk][S(0, i)] + gu[S(1, m)] * Gu[kk][S(1, i)] +
                             gu[S(2, m)] * Gu[kk][S(2, i)];
          const double gmj = gu[S(0, m)] * Gu[kk][S(0, jj)] + gu[S(1, m)] * Gu[kk][S(1, jj)] +
                             gu[S(2, m)] * Gu[kk][S(2, jj)];
          r += gmi * (Gl[jj][S(kk, m)] + Gl[kk][S(m, jj)]) + gmj * Gl[i][S(kk, m)];
        }
      Ric[s] = r;
    }
  }
  // Gt^c_jk At^jk, the only later use of the Christoffel symbols besides chi/alpha
  double ga[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc += W(q) * Gu[c][q] * Au[q];
    ga[c] = acc;
  }
  keep(Gu);
  keep(Gd);
  keep(ga);
  keep(Ric);

  // ---- chi (phase 9)
  double dchi[3];
  const double ichi = 1.0 / chi;
  {
    begin(9);
    auto tap = make_ops(buf1);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) dchi[ax] = D1(tap, ax);
    double cdd[6];
#pragma unroll
    for (int s = 0; s < 6; ++s)
      cdd[s] = D2(tap, s) - (Gu[0][s] * dchi[0] + Gu[1][s] * dchi[1] + Gu[2][s] * dchi[2]);
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
    emit(gCHI, finish(tap, (2.0 / 3.0) * chi * (alpha * K - divb)));
    keep(Ric);
    keep(dchi);
    sync();
  }

  // ---- lapse (phase 10)
  double da[3];
  double DDa[6];
  {
    begin(10);
    auto tap = make_ops(buf0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) da[ax] = D1(tap, ax);
    double gudchi_da = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
      gudchi_da += (gu[S(kk, 0)] * dchi[0] + gu[S(kk, 1)] * dchi[1] + gu[S(kk, 2)] * dchi[2]) * da[kk];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = SI(s), jj = SJ(s);
      DDa[s] = D2(tap, s) - (Gu[0][s] * da[0] + Gu[1][s] * da[1] + Gu[2][s] * da[2]) -
               0.5 * ichi * (g[s] * gudchi_da - dchi[jj] * da[i] - dchi[i] * da[jj]);
    }
    keep(da);
    keep(DDa);
    if (gauge.lapse == 2)
      emit(gALPHA, 0.0);
    else
      emit(gALPHA, finish(tap, gauge.lapse == 0 ? -2.0 * alpha * K : -alpha * alpha * K));
    sync();
  }

  // ---- evolved Gt (phases 11-13)
  double xt_ad[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int p = 11 + c;
    begin(p);
    auto tap = make_ops((p & 1) ? buf1 : buf0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double d = D1(tap, ax);
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int i = SI(s), jj = SJ(s);
        if (jj == ax) Ric[s] += 0.5 * g[S(c, i)] * d;
        if (i == ax) Ric[s] += 0.5 * g[S(c, jj)] * d;
      }
    }
    xt_ad[c] = finish(tap, 0.0);
    keep(xt_ad[c]);
    keep(Ric);
    sync();
  }

  // ---- K (phase 14)
  double AA = 0.0;
  {
    double Am[3][3];
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
  double trDDa = 0.0, trRic = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    trDDa += W(s) * gu[s] * DDa[s];
    trRic += W(s) * gu[s] * Ric[s];
  }
  double xsrc[3];
  {
    begin(14);
    auto tap = make_ops(buf0);
    double dK[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) dK[ax] = D1(tap, ax);
    emit(gK, finish(tap, -chi * trDDa + alpha * (AA + K * K * (1.0 / 3.0))));
    // Gt source, complete now
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double r = xts[c];
      r += (1.0 / 3.0) * (gu[S(c, 0)] * ddiv[0] + gu[S(c, 1)] * ddiv[1] + gu[S(c, 2)] * ddiv[2]);
      r += (2.0 / 3.0) * Gd[c] * divb - (Gd[0] * db[c][0] + Gd[1] * db[c][1] + Gd[2] * db[c][2]);
      r -= 2.0 * (Au[S(c, 0)] * da[0] + Au[S(c, 1)] * da[1] + Au[S(c, 2)] * da[2]);
      const double adchi = Au[S(c, 0)] * dchi[0] + Au[S(c, 1)] * dchi[1] + Au[S(c, 2)] * dchi[2];
      const double gdK = gu[S(c, 0)] * dK[0] + gu[S(c, 1)] * dK[1] + gu[S(c, 2)] * dK[2];
      r += 2.0 * alpha * (ga[c] - 1.5 * ichi * adchi - (2.0 / 3.0) * gdK);
      xsrc[c] = r;
      emit(gXT + c, xt_ad[c] + r);
    }
    keep(xsrc);
    sync();
  }

  // ---- At (phases 15-20)
  const double trX = alpha * trRic - trDDa;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int p = 15 + s;
    begin(p);
    auto tap = make_ops((p & 1) ? buf1 : buf0);
    const int i = SI(s), jj = SJ(s);
    double la = 0.0, aa = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      la += A[S(i, kk)] * db[kk][jj] + A[S(jj, kk)] * db[kk][i];
      // At_ik At^k_j = At_ik gt^kl At_lj
      const double amkj = gu[S(kk, 0)] * A[S(0, jj)] + gu[S(kk, 1)] * A[S(1, jj)] + gu[S(kk, 2)] * A[S(2, jj)];
      aa += A[S(i, kk)] * amkj;
    }
    const double X = alpha * Ric[s] - DDa[s];
    emit(gAT + s, finish(tap, chi * (X - (1.0 / 3.0) * g[s] * trX) + alpha * (K * A[s] - 2.0 * aa) + la -
                              (2.0 / 3.0) * A[s] * divb));
    sync();
  }

  // ---- Gamma-driver B (phases 21-23)
  if (driver) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int p = 21 + c;
      begin(p);
      auto tap = make_ops((p & 1) ? buf1 : buf0);
      emit(gB + c, finish(tap, xsrc[c] - gauge.eta * val(gB + c)));
      sync();
    }
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) emit(gB + c, 0.0);
  }
}

}  // namespace chemora
