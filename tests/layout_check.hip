// Host-side check of the stage kernel's LDS staging layouts (the real header,
// compiled for the host): off() and decode() are inverse on every tap a
// work-item reads, every tap lies inside the staged buffer, and the clamped
// staging offsets of every tile of ragged patches stay inside the patch's
// stored box with each staged pair of doubles inside one row; the same for the
// cross layouts (order 8 with one buffer, order 4 at any tile depth).  Built and run
// by tests/test_layout_host.py; exit status 0 when no violation is found.
#include <cstdio>
#include <cstdlib>
#include "stage_kernel.hpp"
using namespace chemora;

template <int R, int RM, class SH>
int check(int nx, int ny, int nz, int g) {
  using L = LdsLayout<R, RM, SH>;
  int bad = 0;
  // taps read by a work-item at (xr, yr, tz): axis taps |d| <= R along each
  // axis, mixed taps (a, b) with |a|, |b| <= RM in each pair of axes; each
  // at the work-item's anchor plus the compile-time offset
  auto taps = [&](auto&& tap) {
    for (int d = -R; d <= R; ++d) { tap(d, 0, 0); tap(0, d, 0); tap(0, 0, d); }
    for (int a = -RM; a <= RM; ++a)
      for (int b = -RM; b <= RM; ++b) { tap(a, b, 0); tap(a, 0, b); tap(0, a, b); }
  };
  for (int tz = 0; tz < SH::TZ; ++tz)
    for (int yr = 0; yr < SH::TY; ++yr)
      for (int xr = 0; xr < SH::TX; ++xr)
        taps([&](int dx, int dy, int dz) {
          const int idx = L::anchor(xr, yr, tz) + L::off(dx, dy, dz);
          if (idx < 0 || idx >= L::SIZE) { ++bad; return; }
          int x, y, z;
          L::decode(idx, x, y, z);
          if (x != xr + dx || y != yr + dy || z != tz + dz) ++bad;
        });
  // staging offsets: clamped points inside the stored box, pairs inside a
  // row; on small patches also every tap of every valid work-item of every
  // tile reads an element its staging lane loaded unclamped
  const long sy = nx + 2 * g + (nx & 1), sz = sy * (ny + 2 * g);
  (void)sz;
  const int tx = (nx + SH::TX - 1) / SH::TX, ty = (ny + SH::TY - 1) / SH::TY, tzn = (nz + SH::TZ - 1) / SH::TZ;
  const bool small = (long)nx * ny * nz <= 40000;
  for (int kb = 0; kb < tzn; ++kb)
    for (int tyi = 0; tyi < ty; ++tyi)
      for (int txi = 0; txi < tx; ++txi) {
        const int i0 = txi * SH::TX, j0 = tyi * SH::TY, k0 = kb * SH::TZ;
        for (int c = 0; c < L::NCHUNK; ++c)
          for (int lane = 0; lane < 64; ++lane) {
            int x, y, dz;
            L::stage_point(c * L::CHUNK + 2 * lane, i0, j0, k0, nx, ny, nz, x, y, dz);
            const long gi = i0 + x + g, gj = j0 + y + g, gk = k0 + dz + g;
            if (gi < 0 || gi + 1 >= sy || gj < 0 || gj >= ny + 2 * g || gk < 0 || gk >= nz + 2 * g) ++bad;
          }
        if (!small) continue;
        for (int tz = 0; tz < SH::TZ; ++tz)
          for (int yr = 0; yr < SH::TY; ++yr)
            for (int xr = 0; xr < SH::TX; ++xr) {
              if (i0 + xr >= nx || j0 + yr >= ny || k0 + tz >= nz) continue;
              taps([&](int dx, int dy, int dz) {
                const int idx = L::anchor(xr, yr, tz) + L::off(dx, dy, dz);
                const int pair = idx & ~1;   // the lane's pair holds idx
                int x, y, z, ux, uy, uz;
                L::stage_point(pair, i0, j0, k0, nx, ny, nz, x, y, z);
                L::decode(pair, ux, uy, uz);
                if (x != ux || y != uy || z != uz) ++bad;
              });
            }
      }
  return bad;
}

// The cross layout (order 8 with one staging buffer, grid functions without
// mixed derivatives): every axis tap decodes back to its point inside the
// buffer (x and y taps at the full anchor, z taps at the column anchor);
// every staged element's clamped point lies inside the stored box with its
// pair in one row; the stage kernel's own column formula (one per-lane place
// per wave, the plane in the scalar offset) loads the same clamped points;
// and on small patches every tap of every valid work-item reads an element
// loaded unclamped.
template <int R, int RM, class SH>
int check_cross(int nx, int ny, int nz, int g) {
  using F = LdsLayout<R, RM, SH, 1>;
  using LC = CrossLayout<R, RM, SH>;
  int bad = 0;
  auto taps = [&](int xr, int yr, auto&& tap) {
    for (int d = -R; d <= R; ++d) {
      tap(F::anchor(xr, yr, 0) + F::off(d, 0, 0), d, 0, 0);
      tap(F::anchor(xr, yr, 0) + F::off(0, d, 0), 0, d, 0);
      if (d != 0) tap(LC::col_anchor(xr, yr) + LC::zoff(d), 0, 0, d);
    }
  };
  for (int yr = 0; yr < SH::TY; ++yr)
    for (int xr = 0; xr < SH::TX; ++xr)
      taps(xr, yr, [&](int idx, int dx, int dy, int dz) {
        if (idx < 0 || idx >= LC::SIZE) { ++bad; return; }
        int x, y, z;
        LC::decode(idx, x, y, z);
        if (x != xr + dx || y != yr + dy || z != dz) ++bad;
      });
  const long sy = nx + 2 * g + (nx & 1);
  const int tx = (nx + SH::TX - 1) / SH::TX, ty = (ny + SH::TY - 1) / SH::TY;
  const bool small = (long)nx * ny * nz <= 40000;
  for (int kb = 0; kb < nz; ++kb)
    for (int tyi = 0; tyi < ty; ++tyi)
      for (int txi = 0; txi < tx; ++txi) {
        const int i0 = txi * SH::TX, j0 = tyi * SH::TY, k0 = kb;
        for (int c = 0; c < LC::NCHUNK; ++c)
          for (int lane = 0; lane < 64; ++lane) {
            int x, y, dz;
            LC::stage_point(c * LC::CHUNK + 2 * lane, i0, j0, k0, nx, ny, nz, x, y, dz);
            const long gi = i0 + x + g, gj = j0 + y + g, gk = k0 + dz + g;
            if (gi < 0 || gi + 1 >= sy || gj < 0 || gj >= ny + 2 * g || gk < 0 || gk >= nz + 2 * g) ++bad;
            if (c < LC::NCHUNK0) continue;
            // the kernel's formula for a column chunk of wave c % WPG
            const int wave = c % SH::WPG;
            const int pos = ((wave - LC::NCHUNK0) % LC::CPP + LC::CPP) % LC::CPP;
            const int e = pos * LC::CHUNK + 2 * lane;
            int ky = e / SH::TX, kx = e - ky * SH::TX;
            const int xmax = nx - 1 + R - i0, ymax = ny - 1 + R - j0, zmax = nz - 1 + R - k0;
            ky = ky < ymax ? ky : ymax;
            if (kx >= xmax) kx = xmax - 1;
            const int j = (c - LC::NCHUNK0) / LC::CPP;
            int kz = (j & 1) ? -(j / 2 + 1) : j / 2 + 1;
            kz = kz < zmax ? kz : zmax;
            if (kx != x || ky != y || kz != dz || kz + R < 0) ++bad;
          }
        if (!small) continue;
        for (int yr = 0; yr < SH::TY; ++yr)
          for (int xr = 0; xr < SH::TX; ++xr) {
            if (i0 + xr >= nx || j0 + yr >= ny) continue;
            taps(xr, yr, [&](int idx, int, int, int) {
              const int pair = idx & ~1;
              int x, y, z, ux, uy, uz;
              LC::stage_point(pair, i0, j0, k0, nx, ny, nz, x, y, z);
              LC::decode(pair, ux, uy, uz);
              if (x != ux || y != uy || z != uz) ++bad;
            });
          }
      }
  return bad;
}

// the order-4 cross layout of any tile depth: x/y taps at the full layout's
// in-plane offsets from the cross anchor (as the kernel forms it), z taps
// from the column anchor; staging as the kernel issues it (tile-plane chunks
// with stage_point offsets, column chunks with one per-lane position per
// wave and the plane in the scalar part)
template <int R, int RM, class SH>
int check_crossz(int nx, int ny, int nz, int g) {
  using F = LdsLayout<R, RM, SH>;
  using LZ = CrossLayoutZ<R, SH>;
  static_assert(LZ::SIZE <= F::SIZEP, "the cross layout fits the full layout's buffer");
  int bad = 0;
  auto taps = [&](int xr, int yr, int tz, auto&& tap) {
    const int anc = LZ::anchor(xr, yr, tz) - (F::off(0, 0, 0) - LZ::off(0, 0));
    for (int d = -R; d <= R; ++d) {
      tap(anc + F::off(d, 0, 0), d, 0, 0);
      tap(anc + F::off(0, d, 0), 0, d, 0);
      tap(LZ::col_anchor(xr, yr, tz) + LZ::zoff(d), 0, 0, d);
    }
  };
  for (int tz = 0; tz < SH::TZ; ++tz)
    for (int yr = 0; yr < SH::TY; ++yr)
      for (int xr = 0; xr < SH::TX; ++xr)
        taps(xr, yr, tz, [&](int idx, int dx, int dy, int dz) {
          if (idx < 0 || idx >= LZ::SIZE) { ++bad; return; }
          int x, y, z;
          LZ::decode(idx, x, y, z);
          if (x != xr + dx || y != yr + dy || z != tz + dz) ++bad;
        });
  const long sy = nx + 2 * g + (nx & 1);
  const int tx = (nx + SH::TX - 1) / SH::TX, ty = (ny + SH::TY - 1) / SH::TY, tzn = (nz + SH::TZ - 1) / SH::TZ;
  const bool small = (long)nx * ny * nz <= 40000;
  for (int kb = 0; kb < tzn; ++kb)
    for (int tyi = 0; tyi < ty; ++tyi)
      for (int txi = 0; txi < tx; ++txi) {
        const int i0 = txi * SH::TX, j0 = tyi * SH::TY, k0 = kb * SH::TZ;
        for (int c = 0; c < LZ::NCHUNK; ++c)
          for (int lane = 0; lane < 64; ++lane) {
            int x, y, dz;
            LZ::stage_point(c * LZ::CHUNK + 2 * lane, i0, j0, k0, nx, ny, nz, x, y, dz);
            const long gi = i0 + x + g, gj = j0 + y + g, gk = k0 + dz + g;
            if (gi < 0 || gi + 1 >= sy || gj < 0 || gj >= ny + 2 * g || gk < 0 || gk >= nz + 2 * g) ++bad;
            if (c < LZ::NCHUNK0) continue;
            const int wave = c % SH::WPG;
            const int pos = ((wave - LZ::NCHUNK0) % LZ::CPP + LZ::CPP) % LZ::CPP;
            const int e = pos * LZ::CHUNK + 2 * lane;
            int ky = e / SH::TX, kx = e - ky * SH::TX;
            const int xmax = nx - 1 + R - i0, ymax = ny - 1 + R - j0, zmax = nz - 1 + R - k0;
            ky = ky < ymax ? ky : ymax;
            if (kx >= xmax) kx = xmax - 1;
            int kz = (c - LZ::NCHUNK0) / LZ::CPP - R;
            kz = kz < zmax ? kz : zmax;
            if (kx != x || ky != y || kz != dz || kz + R < 0) ++bad;
          }
        if (!small) continue;
        for (int tz = 0; tz < SH::TZ; ++tz)
          for (int yr = 0; yr < SH::TY; ++yr)
            for (int xr = 0; xr < SH::TX; ++xr) {
              if (i0 + xr >= nx || j0 + yr >= ny || k0 + tz >= nz) continue;
              taps(xr, yr, tz, [&](int idx, int, int, int) {
                const int pair = idx & ~1;
                int x, y, z, ux, uy, uz;
                LZ::stage_point(pair, i0, j0, k0, nx, ny, nz, x, y, z);
                LZ::decode(pair, ux, uy, uz);
                if (x != ux || y != uy || z != uz) ++bad;
              });
            }
      }
  return bad;
}

int main() {
  int bad = 0;
  const int shapes[][4] = {{70, 37, 19, 3}, {33, 9, 7, 3}, {128, 128, 128, 3}, {1, 1, 1, 3}, {65, 1, 2, 3},
                           {2, 33, 1, 3}, {21, 14, 11, 3}, {22, 13, 9, 4}, {26, 11, 8, 3}};
  for (auto& s : shapes) {
    const int g8 = 5 > s[3] ? 5 : s[3];
    bad += check<3, 2, Shape<32, 8, 2>>(s[0], s[1], s[2], s[3]);
    bad += check<3, 2, Shape<32, 8, 4>>(s[0], s[1], s[2], s[3]);
    bad += check<2, 2, Shape<32, 8, 2>>(s[0], s[1], s[2], s[3]);
    bad += check<2, 2, Shape<32, 8, 4>>(s[0], s[1], s[2], s[3]);
    bad += check<3, 2, Shape<32, 8, 1>>(s[0], s[1], s[2], s[3]);
    bad += check<3, 2, Shape<64, 4, 1>>(s[0], s[1], s[2], s[3]);
    bad += check<2, 2, Shape<32, 4, 1>>(s[0], s[1], s[2], s[3]);
    bad += check<3, 2, Shape<64, 8, 1>>(s[0], s[1], s[2], s[3]);
    bad += check<5, 4, Shape<32, 4, 1>>(s[0], s[1], s[2], g8);
    bad += check<5, 4, Shape<64, 4, 1>>(s[0], s[1], s[2], g8);
    bad += check<4, 4, Shape<32, 4, 1>>(s[0], s[1], s[2], g8);
    bad += check_cross<5, 4, Shape<32, 4, 1>>(s[0], s[1], s[2], g8);
    bad += check_cross<5, 4, Shape<64, 4, 1>>(s[0], s[1], s[2], g8);
    bad += check_cross<4, 4, Shape<32, 4, 1>>(s[0], s[1], s[2], g8);
    bad += check_crossz<3, 2, Shape<32, 8, 1>>(s[0], s[1], s[2], s[3]);
    bad += check_crossz<3, 2, Shape<32, 8, 2>>(s[0], s[1], s[2], s[3]);
    bad += check_crossz<3, 2, Shape<32, 8, 4>>(s[0], s[1], s[2], s[3]);
    bad += check_crossz<2, 2, Shape<32, 8, 2>>(s[0], s[1], s[2], s[3]);
    bad += check_crossz<3, 2, Shape<64, 8, 1>>(s[0], s[1], s[2], s[3]);
    bad += check_crossz<3, 2, Shape<64, 4, 1>>(s[0], s[1], s[2], s[3]);
    bad += check_crossz<3, 2, Shape<32, 4, 1>>(s[0], s[1], s[2], s[3]);
  }
  printf("layout check: %d violations\n", bad);
  return bad != 0;
}
