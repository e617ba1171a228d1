// Device helpers shared by the (de)gridding kernels and the image-level kernels:
// complex element types, the FP64-reduced phasor exp(2 pi i theta) and the radix-2/3/4/5
// DFT butterflies of the Stockham FFTs.
#ifndef AIDG_DEVICE_COMMON_H
#define AIDG_DEVICE_COMMON_H

#include <hip/hip_runtime.h>

namespace aidg {

template <typename R> struct C2;
template <> struct C2<float> { using T = float2; };
template <> struct C2<double> { using T = double2; };
template <typename R> struct C4;
template <> struct C4<float> { using T = float4; };
template <> struct C4<double> { using T = double4; };

template <typename R>
__device__ __forceinline__ typename C2<R>::T cmul(typename C2<R>::T a, typename C2<R>::T b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// (c, s) = (cos, sin) of an angle, rotated by qi quarter turns: swap for odd qi, then
// flip the sign bits (cos is negative for qi = 1, 2 mod 4 and sin for qi = 2, 3: bit 1
// of qi + 1 and of qi).
__device__ __forceinline__ float2 rotate_quarter(float c, float s, int qi) {
  const bool odd = qi & 1;
  const float cc = odd ? s : c, ss = odd ? c : s;
  const unsigned sign_c = ((unsigned)(qi + 1) << 30) & 0x80000000u, sign_s = ((unsigned)qi << 30) & 0x80000000u;
  return {__uint_as_float(__float_as_uint(cc) ^ sign_c), __uint_as_float(__float_as_uint(ss) ^ sign_s)};
}

// exp(2 pi i (t + qi / 4)) for |t| <= 1/8 turn, FP32: sin/cos(2 pi t) from their
// Taylor series to degree 9 and 10 (truncation < 2e-9 for |2 pi t| <= pi/4),
// evaluated by Horner in FP32, then a rotation by qi quarter turns.
__device__ __forceinline__ float2 phasor_quarter(float t, int qi) {
  const float t2 = t * t;
  float s = fmaf(t2, 42.058693944897634f, -76.70585975306136f);
  s = fmaf(t2, s, 81.60524927607504f);
  s = fmaf(t2, s, -41.341702240399755f);
  s = fmaf(t2, s, 6.283185307179586f);
  s = s * t;
  float c = fmaf(t2, -26.426256783374388f, 60.24464137187664f);
  c = fmaf(t2, c, -85.45681720669371f);
  c = fmaf(t2, c, 64.93939402266828f);
  c = fmaf(t2, c, -19.739208802178716f);
  c = fmaf(t2, c, 1.0f);
  return rotate_quarter(c, s, qi);
}

// exp(2 pi i theta) for a phase theta in turns, FP32 result.  The quarter-turn
// reduction happens in FP64 (theta = q/4 + t, |t| <= 1/8, exact) and t is rounded
// once to FP32.
__device__ __forceinline__ float2 phasor(double theta, float) {
  const double q = rint(4.0 * theta);
  const float t = (float)fma(q, -0.25, theta);
  return phasor_quarter(t, (int)q);  // |theta| is bounded by the grid size in turns
}

// exp(2 pi i theta) for a phase theta in turns, FP32 result: theta = q/4 + t with q the
// nearest integer to 4 theta and |t| <= 1/8, exact in FP64; t is rounded once to FP32
// (2^-28 turn at most, 2.3e-8 rad: the reduction to a quarter rather than a whole turn
// keeps this rounding 8x below that of a [-1/2, 1/2] argument), the transcendental unit's
// v_cos_f32 / v_sin_f32 (which take their argument in turns) give cos and sin of 2 pi t,
// and the result is rotated by q quarter turns.  On gfx950 the unit's absolute error is
// at most 1.3e-7 (rms 3.5e-8, phase rms 2.3e-8 rad), the size of FP32 rounding of a unit
// value; the whole phasor costs about 11 VALU operations where the Taylor form
// (phasor_quarter) takes about 20.
__device__ __forceinline__ float2 phasor_turns(double theta) {
  const double q = rint(4.0 * theta);
  const float t = (float)fma(q, -0.25, theta);
  return rotate_quarter(__builtin_amdgcn_cosf(t), __builtin_amdgcn_sinf(t), (int)q);
}

// A phasor that is raised to powers (a recurrence step) scaled back to unit magnitude:
// z (3 - |z|^2) / 2, the first Newton step of 1 / sqrt(|z|^2), exact to second order in
// |z|^2 - 1 (about 1e-7 here).  The transcendental unit's sine and cosine leave
// |z|^2 - 1 at -6.5e-8 on average (rms 8.6e-8), a bias that k steps of a recurrence
// would multiply by k; after the correction the magnitude error is FP32 rounding only.
__device__ __forceinline__ float2 unit_step(float2 z) {
  const float f = fmaf(-0.5f, fmaf(z.x, z.x, z.y * z.y), 1.5f);
  return {z.x * f, z.y * f};
}
__device__ __forceinline__ double2 unit_step(double2 z) { return z; }  // FP64: exact enough

// FP64 phasor of a phase in turns: reduction to [-1/2, 1/2] and the device library's sincospi.
__device__ __forceinline__ double2 phasor(double theta, double) {
  const double r = theta - rint(theta);
  double s, c;
  sincospi(2.0 * r, &s, &c);
  return {c, s};
}

// In-place DFT of R points: v[k] <- sum_j v[j] exp(DIR 2 pi i j k / R), DIR = -1
// (forward) or +1 (inverse), unnormalised.
template <typename V2, int R, int DIR>
__device__ __forceinline__ void butterfly(V2* v) {
  using Rt = decltype(v[0].x);
  if constexpr (R == 2) {
    const V2 a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    const V2 t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3];
    const V2 d = v[1] - v[3];
    const V2 t3 = {Rt(-DIR) * d.y, Rt(DIR) * d.x};  // (DIR i) d
    v[0] = t0 + t2;
    v[1] = t1 + t3;
    v[2] = t0 - t2;
    v[3] = t1 - t3;
  } else if constexpr (R == 3) {
    const Rt c = Rt(-0.5), dd = Rt(DIR) * Rt(0.86602540378443864676);
    const V2 t1 = v[1] + v[2], t2 = v[1] - v[2];
    const V2 m = v[0] + t1 * c;
    const V2 n = {-dd * t2.y, dd * t2.x};
    v[0] = v[0] + t1;
    v[1] = m + n;
    v[2] = m - n;
  } else if constexpr (R == 5) {
    // X_1 = a1 + (DIR i) b1, X_4 = a1 - (DIR i) b1, X_2 = a2 + (DIR i) b2, X_3 = a2 - (DIR i) b2
    // with c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5)
    const Rt c1 = Rt(0.30901699437494742410), c2 = Rt(-0.80901699437494742410);
    const Rt s1 = Rt(0.95105651629515357212), s2 = Rt(0.58778525229247312917);
    const V2 t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
    const V2 a1 = v[0] + t1 * c1 + t2 * c2, a2 = v[0] + t1 * c2 + t2 * c1;
    const V2 b1 = t3 * s1 + t4 * s2, b2 = t3 * s2 - t4 * s1;
    const V2 ib1 = {Rt(-DIR) * b1.y, Rt(DIR) * b1.x}, ib2 = {Rt(-DIR) * b2.y, Rt(DIR) * b2.x};
    v[0] = v[0] + t1 + t2;
    v[1] = a1 + ib1;
    v[4] = a1 - ib1;
    v[2] = a2 + ib2;
    v[3] = a2 - ib2;
  }
}

}  // namespace aidg

#endif  // AIDG_DEVICE_COMMON_H
