// Device helpers shared by the libptk kernels.  All translation units are
// compiled with -ffp-contract=off: every binary64 operation below is rounded
// separately, in the order written.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

#include "launch.h"

namespace ptk {

// Positions accepted by the library: finite with |x| < 2^50.  Beyond that the
// binary64 wrap below can no longer bring x into [0, 2*pi) (the rounding error
// of L*q exceeds L), so such positions are reported as a domain error.
__device__ __forceinline__ bool in_domain(double x) { return fabs(x) < 0x1p50; }

// Steps 1-3 of the interpolation algorithm (Sec. 2.2) for one coordinate:
// periodic wrap, cell index and in-cell offset, by a fixed binary64 sequence.
// Returns the wrapped coordinate; *c in [0, N), *t in [0, 1).  A coordinate
// outside the domain is treated as 0 (the caller reports the error).
__device__ __forceinline__ double locate(double x, int N, double invd, int* c, double* t) {
  const double L = 6.283185307179586;
  if (!in_domain(x)) x = 0.0;
  double y;
  if (x >= 0.0 && x < L) {
    // the sequence below gives q = 0 here (x / L rounds below 1 for every
    // x < L: x <= L - 2^-50, so x / L <= 1 - 1.59 * 2^-53, which rounds to
    // 1 - 2^-52) and so y = x - 0 = x + 0: skip the division (x + 0.0 turns
    // -0 into +0 as the subtraction does)
    y = x + 0.0;
  } else {
    const double q = floor(x / L);
    y = x - L * q;
    if (y < 0.0) y = y + L;
    if (y >= L) y = 0.0;
  }
  double s = y * invd;
  double cf = floor(s);
  int ci = (int)cf;
  double tt = s - cf;
  if (ci >= N) {
    ci = 0;
    tt = 0.0;
  }
  *c = ci;
  *t = tt;
  return y;
}

__device__ __forceinline__ double wrap(double x) {
  const double L = 6.283185307179586;
  double q = floor(x / L);
  double y = x - L * q;
  if (y < 0.0) y = y + L;
  if (y >= L) y = 0.0;
  return y;
}

__device__ __forceinline__ bool in_domain3(double a, double b, double c) {
  return in_domain(a) && in_domain(b) && in_domain(c);
}

// Bin key of a cell: tile column (x2 tile slowest), then the x3 window --
// within a column, particles are ordered along x3 like the paper's slices.
__device__ __forceinline__ uint32_t bin_key(int c1, int c2, int c3, const BinGeom& g) {
  return (uint32_t)(((c2 / g.T) * g.ntx + c1 / g.T) * g.nw + c3 / g.W);
}

// bf16 <-> f32 (bit patterns in uint16).
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

// f32 -> f16 bit pattern, round to nearest even, subnormal results kept
// (integer arithmetic, so the result does not depend on a conversion
// instruction's denormal handling).  Values at or beyond 65520 become infinity.
__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
  const uint32_t x = __float_as_uint(f);
  const uint32_t sign = (x >> 16) & 0x8000u;
  const uint32_t a = x & 0x7FFFFFFFu;
  if (a >= 0x7F800000u) return (uint16_t)(sign | 0x7C00u | (a > 0x7F800000u ? 0x200u : 0u));
  const int e = (int)(a >> 23) - 127;
  const uint32_t m = a & 0x7FFFFFu;
  if (e > 15) return (uint16_t)(sign | 0x7C00u);
  if (e >= -14) {
    uint32_t r = ((uint32_t)(e + 15) << 10) | (m >> 13);
    const uint32_t rem = m & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (r & 1u))) ++r;  // a carry moves into the exponent
    return (uint16_t)(sign | r);
  }
  // subnormal half: the value in units of 2^-24 is (2^23 + m) * 2^(e+1)
  const int sh = -(e + 1);  // >= 14
  if (sh > 24) return (uint16_t)sign;
  const uint32_t mant = 0x800000u | m;
  uint32_t q = mant >> sh;
  const uint32_t rem = mant & ((1u << sh) - 1u), half = 1u << (sh - 1);
  if (rem > half || (rem == half && (q & 1u))) ++q;
  return (uint16_t)(sign | q);
}

}  // namespace ptk
