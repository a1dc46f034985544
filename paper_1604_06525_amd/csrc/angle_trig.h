// Sine and cosine of an FP32 angle without branches, for energies that keep a
// rotation as its angle and form cos and sin where a row of the state is read.
//
// t = k (pi/2) + r with k the integer nearest to t (2/pi) and |r| <= pi/4
// (plus rounding): pi/2 is taken as the sum of two floats, the first the FP32
// rounding of pi/2 and the second the rest, each removed with a fused
// multiply-add (the classical two-constant reduction of Cody and Waite).  On
// that range the Taylor series of sin to r^9 and of cos to r^10 are each
// truncated below 3e-9, under the FP32 rounding of the result; the quadrant
// k mod 4 then picks and signs the two.  Accurate to about one unit in the last
// place for |t| up to a few thousand radians; far beyond that the reduction
// loses the angle.
//
// The header includes nothing: the library reads it after the HIP runtime
// header, and a CPU test defines the two function qualifiers empty.
#pragma once

namespace optmi {

__host__ __device__ inline void sincos_angle(float t, float* s, float* c) {
  const float kHalfPiHi = 1.57079637050628662109375f;       // pi/2 rounded to FP32
  const float kHalfPiLo = -4.37113900018624283e-8f;          // pi/2 - kHalfPiHi
  const float k = __builtin_rintf(t * 0.636619772367581343f);  // 2/pi
  float r = __builtin_fmaf(-k, kHalfPiHi, t);
  r = __builtin_fmaf(-k, kHalfPiLo, r);
  const float z = r * r;
  // sin r = r - r^3/3! + r^5/5! - r^7/7! + r^9/9!
  float ps = __builtin_fmaf(z, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = __builtin_fmaf(z, ps, 1.0f / 120.0f);
  ps = __builtin_fmaf(z, ps, -1.0f / 6.0f);
  const float sr = __builtin_fmaf(r * z, ps, r);
  // cos r = 1 - r^2/2! + r^4/4! - r^6/6! + r^8/8! - r^10/10!
  float pc = __builtin_fmaf(z, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = __builtin_fmaf(z, pc, -1.0f / 720.0f);
  pc = __builtin_fmaf(z, pc, 1.0f / 24.0f);
  pc = __builtin_fmaf(z, pc, -0.5f);
  const float cr = __builtin_fmaf(z, pc, 1.0f);
  // quadrant q = k mod 4 (exact in FP32): sin t, cos t = (sin r, cos r),
  // (cos r, -sin r), (-sin r, -cos r), (-cos r, sin r)
  const int q = (int)__builtin_fmaf(-4.0f, __builtin_floorf(k * 0.25f), k);
  const float a = (q & 1) ? cr : sr, b = (q & 1) ? sr : cr;
  *s = (q & 2) ? -a : a;
  *c = ((q + 1) & 2) ? -b : b;
}

}  // namespace optmi
