// Correctly rounded binary32 reciprocal and square root from the hardware
// approximations (v_rcp_f32, v_sqrt_f32) and fused multiply-adds.
//
// The render kernel's results must equal, bit for bit, those of a renderer
// that rounds every division and square root correctly; the compiler's
// correctly rounded sequences take 11 (division) and 16 (square root) vector
// instructions, these 5 and 9 (14 for the square root of any input).  Each
// function states the inputs on which it equals the correctly rounded
// operation, and prdpt_selftest_math checks every binary32 input of that
// domain on the device.  No function here branches: a guard on a computed
// value costs a divergent branch on every call, and the compiler may fold a
// class test of a computed value.
#pragma once
#include <hip/hip_runtime.h>

namespace prdpt {

// 1/x, correctly rounded, for x = +-0, +-inf, NaN and normal x with
// |x| <= 2^126.  One Newton step y + y (1 - x y), the residual fused, refines
// the hardware reciprocal y; where the residual is NaN (x = 0, inf, NaN) the
// hardware result is already the correctly rounded one.  Not for subnormal x
// or |x| > 2^126 (there the result is subnormal).
__device__ __forceinline__ float recip_nr(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, y, 1.0f);
  const float y1 = __builtin_fmaf(e, y, y);
  return e == e ? y1 : y;
}

// sqrt(x), correctly rounded, for |x| >= 2^-104 and for +-0, +inf and NaN:
// the hardware square root s is replaced by its lower neighbour when
// (s - ulp) s >= x and by its upper neighbour when (s + ulp) s < x, both
// residuals fused (negative x give NaN).  Not for 0 < |x| < 2^-104: the
// hardware square root takes subnormal inputs as zero and is less accurate
// near them.
__device__ __forceinline__ float sqrt_nr(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sm = __uint_as_float(__float_as_uint(s) - 1u);
  const float sp = __uint_as_float(__float_as_uint(s) + 1u);
  const float vm = __builtin_fmaf(-sm, s, x);
  const float vp = __builtin_fmaf(-sp, s, x);
  float r = vm <= 0.0f ? sm : s;
  r = vp > 0.0f ? sp : r;
  return r;
}

// sqrt(x), correctly rounded, for every binary32 x: x below 2^-96 (negative x
// too) is scaled by 2^32 into sqrt_nr's domain and its root scaled back by
// 2^-16; both scalings are exact (the root of a scaled subnormal is normal).
__device__ __forceinline__ float sqrt_cr(float x) {
  const bool small = x < 0x1p-96f;
  const float r = sqrt_nr(small ? x * 0x1p32f : x);
  return small ? r * 0x1p-16f : r;
}

}  // namespace prdpt
