// fd_ops.hpp -- finite-difference operators for the gfx950 BSSN kernels.
//
// Every operator is written on differences of grid values (u_{+k} - u_{-k} or
// u_{+k} - u_0) with integer weights over a common denominator, and the
// 1/(D h) (or 1/(D h^2)) factor applied once at the end.  Constant data
// therefore gives exactly zero, and each derivative costs one multiply by a
// precomputed scale.  Weights:
//   order 4  D1: (8 d1 - d2) / 12h                      d_k = u_k - u_-k
//            D2: (16 s1 - s2) / 12h^2                   s_k = u_k + u_-k - 2u_0
//            lopsided (beta >= 0, offsets -1..3):
//                (-3 e_-1 + 18 e_1 - 6 e_2 + e_3) / 12h e_o = u_o - u_0
//   order 8  D1: (672 d1 - 168 d2 + 32 d3 - 3 d4) / 840h
//            D2: (8064 s1 - 1008 s2 + 128 s3 - 9 s4) / 5040h^2
//            lopsided (offsets -3..5):
//                (-5 e_-3 + 60 e_-2 - 420 e_-1 + 1050 e_1 - 420 e_2
//                 + 140 e_3 - 30 e_4 + 3 e_5) / 840h
//   Kreiss-Oliger radius r (Kreiss & Oliger 1973), dissipative sign, per axis:
//            r=2: (4 s1 - s2) * 2^-4 eps/h
//            r=3: (15 s1 - 6 s2 + s3) * 2^-6 eps/h
//            r=5: (210 s1 - 120 s2 + 45 s3 - 10 s4 + s5) * 2^-10 eps/h
// For beta < 0 the lopsided stencil is mirrored and negated.
// Split precision (order 4): the same differences, each formed in FP64 and
// rounded to FP32, combined with FP32 weights (first_f, second_f,
// lopsided_f, ko_axis_f).
// The mixed derivative D_a D_b is the outer D1 along a of inner D1's along b,
// both unscaled, divided by (12h)^2 or (840h)^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemora {

template <int ORDER>
struct Stencil;

template <>
struct Stencil<4> {
  static constexpr int R = 2;            // centred reach
  static constexpr double D1 = 12.0;     // denominators
  static constexpr double D2 = 12.0;
  static constexpr double DU = 12.0;
  template <class F>
  __device__ static __forceinline__ double first(F&& at) {
    return 8.0 * (at(1) - at(-1)) - (at(2) - at(-2));
  }
  template <class F>
  __device__ static __forceinline__ double second(F&& at) {
    const double c = at(0);
    return 16.0 * ((at(1) - c) + (at(-1) - c)) - ((at(2) - c) + (at(-2) - c));
  }
  // lopsided toward +axis; s = +1 or -1 mirrors the offsets, the caller
  // multiplies the result by s
  template <class F>
  __device__ static __forceinline__ double lopsided(F&& at, int s) {
    const double c = at(0);
    return -3.0 * (at(-s) - c) + 18.0 * (at(s) - c) - 6.0 * (at(2 * s) - c) + (at(3 * s) - c);
  }
  // The lopsided stencil toward +axis is (A + Q) / 2 and its mirror
  // (A - Q) / 2, with the antisymmetric part A = 21 b1 - 6 b2 + b3
  // (b_k = u_k - u_-k) and the symmetric part Q = 15 s1 - 6 s2 + s3
  // (s_k = (u_k - u_0) + (u_-k - u_0)), the sixth difference that
  // Kreiss-Oliger dissipation of radius 3 sums too.  So for either sign of
  // the advecting velocity, beta * lopsided = UA beta A + UQ |beta| Q.
  static constexpr int UR = 3;
  static constexpr double UA = 0.5, UQ = 0.5;
  static constexpr double USYM[5] = {15.0, -6.0, 1.0, 0.0, 0.0};
  template <class F>
  __device__ static __forceinline__ double upwind_anti(F&& at) {
    return 21.0 * (at(1) - at(-1)) - 6.0 * (at(2) - at(-2)) + (at(3) - at(-3));
  }
  // split precision: FP64 differences rounded to FP32, FP32 weights
  template <class F>
  __device__ static __forceinline__ float first_f(F&& at) {
    return 8.0f * (float)(at(1) - at(-1)) - (float)(at(2) - at(-2));
  }
  template <class F>
  __device__ static __forceinline__ float second_f(F&& at) {
    const double c = at(0);
    return 16.0f * (float)((at(1) - c) + (at(-1) - c)) - (float)((at(2) - c) + (at(-2) - c));
  }
  template <class F>
  __device__ static __forceinline__ float lopsided_f(F&& at, int s) {
    const double c = at(0);
    return -3.0f * (float)(at(-s) - c) + 18.0f * (float)(at(s) - c) - 6.0f * (float)(at(2 * s) - c) +
           (float)(at(3 * s) - c);
  }
};

template <>
struct Stencil<8> {
  static constexpr int R = 4;
  static constexpr double D1 = 840.0;
  static constexpr double D2 = 5040.0;
  static constexpr double DU = 840.0;
  template <class F>
  __device__ static __forceinline__ double first(F&& at) {
    return 672.0 * (at(1) - at(-1)) - 168.0 * (at(2) - at(-2)) + 32.0 * (at(3) - at(-3)) -
           3.0 * (at(4) - at(-4));
  }
  template <class F>
  __device__ static __forceinline__ double second(F&& at) {
    const double c = at(0);
    return 8064.0 * ((at(1) - c) + (at(-1) - c)) - 1008.0 * ((at(2) - c) + (at(-2) - c)) +
           128.0 * ((at(3) - c) + (at(-3) - c)) - 9.0 * ((at(4) - c) + (at(-4) - c));
  }
  template <class F>
  __device__ static __forceinline__ double lopsided(F&& at, int s) {
    const double c = at(0);
    return -5.0 * (at(-3 * s) - c) + 60.0 * (at(-2 * s) - c) - 420.0 * (at(-s) - c) +
           1050.0 * (at(s) - c) - 420.0 * (at(2 * s) - c) + 140.0 * (at(3 * s) - c) -
           30.0 * (at(4 * s) - c) + 3.0 * (at(5 * s) - c);
  }
  // lopsided (offsets -3..5) = A + 1.5 Q and its mirror A - 1.5 Q (in units
  // of 1/840h), A = 735 b1 - 240 b2 + 72.5 b3 - 15 b4 + 1.5 b5 and Q the
  // tenth difference 210 s1 - 120 s2 + 45 s3 - 10 s4 + s5 of Kreiss-Oliger
  // dissipation of radius 5
  static constexpr int UR = 5;
  static constexpr double UA = 1.0, UQ = 1.5;
  static constexpr double USYM[5] = {210.0, -120.0, 45.0, -10.0, 1.0};
  template <class F>
  __device__ static __forceinline__ double upwind_anti(F&& at) {
    return 735.0 * (at(1) - at(-1)) - 240.0 * (at(2) - at(-2)) + 72.5 * (at(3) - at(-3)) -
           15.0 * (at(4) - at(-4)) + 1.5 * (at(5) - at(-5));
  }
  // split-precision forms (the host builds split precision for order 4 only)
  template <class F>
  __device__ static __forceinline__ float first_f(F&& at) {
    return 672.0f * (float)(at(1) - at(-1)) - 168.0f * (float)(at(2) - at(-2)) + 32.0f * (float)(at(3) - at(-3)) -
           3.0f * (float)(at(4) - at(-4));
  }
  template <class F>
  __device__ static __forceinline__ float second_f(F&& at) {
    const double c = at(0);
    auto s = [&](int k) { return (float)((at(k) - c) + (at(-k) - c)); };
    return 8064.0f * s(1) - 1008.0f * s(2) + 128.0f * s(3) - 9.0f * s(4);
  }
  template <class F>
  __device__ static __forceinline__ float lopsided_f(F&& at, int s) {
    const double c = at(0);
    auto e = [&](int o) { return (float)(at(o) - c); };
    return -5.0f * e(-3 * s) + 60.0f * e(-2 * s) - 420.0f * e(-s) + 1050.0f * e(s) - 420.0f * e(2 * s) +
           140.0f * e(3 * s) - 30.0f * e(4 * s) + 3.0f * e(5 * s);
  }
};

// Kreiss-Oliger term along one axis for radius r <= RMAX (the reach of the
// caller's staged neighbourhood; ko_sum is the sum before the scale, which
// the upwind decomposition above reuses): the weighted sum of the symmetric
// differences s_k = (u_k - u_0) + (u_-k - u_0), accumulated from k = 1 upward
// with the integer weights w[k-1] of the radius (zero past it, so that the
// radius is data, not a branch), times scale = 2^(-2r) eps / h.  It is a
// 2r-th difference that cancels by many orders of magnitude on smooth data,
// so it is evaluated without FMA contraction in this fixed order: the result
// is then reproducible to the bit across compilers and independent of how
// the rest is scheduled.  A zero weight adds an exact zero.
template <int RMAX, class F>
__device__ __forceinline__ double ko_sum(F&& at, const double (&w)[5]) {
#pragma clang fp contract(off)
  static_assert(RMAX >= 1 && RMAX <= 5, "radius");
  const double c = at(0);
  auto s = [&](int k) { return (at(k) - c) + (at(-k) - c); };
  double acc = w[0] * s(1);
#pragma unroll
  for (int k = 2; k <= RMAX; ++k) acc = acc + w[k - 1] * s(k);
  return acc;
}

template <int RMAX, class F>
__device__ __forceinline__ double ko_axis(F&& at, const double (&w)[5], double scale) {
#pragma clang fp contract(off)
  return ko_sum<RMAX>(at, w) * scale;
}

// Split precision: the symmetric differences are formed in FP64 and rounded
// to FP32, weights and sum in FP32.
template <int RMAX, class F>
__device__ __forceinline__ float ko_axis_f(F&& at, const double (&w)[5], float scale) {
  static_assert(RMAX >= 1 && RMAX <= 5, "radius");
  const double c = at(0);
  auto s = [&](int k) { return (float)((at(k) - c) + (at(-k) - c)); };
  float acc = float(w[0]) * s(1);
#pragma unroll
  for (int k = 2; k <= RMAX; ++k) acc += float(w[k - 1]) * s(k);
  return acc * scale;
}

}  // namespace chemora
