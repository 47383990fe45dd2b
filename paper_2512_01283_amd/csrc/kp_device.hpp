// kp_device.hpp -- device-side building blocks of the transport and imaging
// kernels for gfx950: counter-based RNG, Stokes reference bases, grain-frame
// quaternions, the signed basis-rotation angle, dipole extinction
// coefficients.  Everything is templated on the arithmetic type R (float for
// production transport, double for parity runs and for imaging).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

// ---------------------------------------------------------------------------
// precision-overloaded math (ROCm device libm)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float k_exp(float x) { return expf(x); }
__device__ __forceinline__ double k_exp(double x) { return exp(x); }
__device__ __forceinline__ float k_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double k_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float k_log(float x) { return logf(x); }
__device__ __forceinline__ double k_log(double x) { return log(x); }
__device__ __forceinline__ float k_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double k_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float k_sin(float x) { return sinf(x); }
__device__ __forceinline__ double k_sin(double x) { return sin(x); }
__device__ __forceinline__ float k_cos(float x) { return cosf(x); }
__device__ __forceinline__ double k_cos(double x) { return cos(x); }
__device__ __forceinline__ void k_sincospi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void k_sincospi(double x, double* s, double* c) { sincospi(x, s, c); }
template <typename R> __device__ __forceinline__ R k_inf();
template <> __device__ __forceinline__ float k_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double k_inf<double>() { return __builtin_huge_val(); }

// x^2 + y^2 at or below 2^-60 counts as the pole of the spherical basis
#define KP_POLE2 8.673617379884035e-19

// ---------------------------------------------------------------------------
// Philox4x64-10, the counter-based generator of Salmon, Moraes, Dror & Shaw
// (SC'11): ten rounds, each two 64x64->128 products, with the key bumped by
// the Weyl constants between rounds.  Stream of packet p, wavelength l:
// key (seed, l), block b at counter (p, b, 0, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = 0xD2E7470EE14C6C93ull, b = 0xCA5A826395121157ull;
    uint64_t hi0 = __umul64hi(a, x0), lo0 = a * x0;
    uint64_t hi1 = __umul64hi(b, x2), lo1 = b * x2;
    uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// 23 leading bits of a word as (k + 1/2) 2^-23: exact in float and double
template <typename R>
__device__ __forceinline__ R word_uniform(uint64_t w) {
  return (R)(uint32_t)(w >> 41) * (R)(1.0 / 8388608.0) + (R)(0.5 / 8388608.0);
}

// ---------------------------------------------------------------------------
// vectors, bases, quaternions
// ---------------------------------------------------------------------------
template <typename R> struct V3 { R x, y, z; };

template <typename R>
__device__ __forceinline__ R dot(const V3<R>& a, const V3<R>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ V3<R> cross(const V3<R>& a, const V3<R>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// azimuth cosine/sine of a direction, phi = 0 at the pole
template <typename R>
__device__ __forceinline__ void azimuth(const V3<R>& n, R& cp, R& sp, R& st) {
  R r2 = n.x * n.x + n.y * n.y;
  st = k_sqrt(r2);
  if (r2 <= (R)KP_POLE2) { cp = (R)1; sp = (R)0; }
  else { R inv = (R)1 / st; cp = n.x * inv; sp = n.y * inv; }
}

// Stokes reference basis (theta_hat, phi_hat) of a direction
template <typename R>
__device__ __forceinline__ void basis(const V3<R>& n, V3<R>& th, V3<R>& ph) {
  R cp, sp, st;
  azimuth(n, cp, sp, st);
  th = {n.z * cp, n.z * sp, -st};
  ph = {-sp, cp, (R)0};
}

// Unit quaternion (w, x, y, z) of the grain frame whose z axis is the
// alignment direction b: q = q_z(phi_B) q_y(theta_B), formed from the
// half-angle identities so that no trigonometric call is needed.
template <typename R> struct Quat { R w, x, y, z; };

template <typename R>
__device__ __forceinline__ Quat<R> grain_quat(V3<R> b) {
  R nb = k_sqrt(dot(b, b));
  R inv = (R)1 / nb;
  b = {b.x * inv, b.y * inv, b.z * inv};
  R r2 = b.x * b.x + b.y * b.y;
  R st = k_sqrt(r2);
  R ct2, st2;  // cos, sin of theta_B / 2 (both >= 0)
  if (b.z >= (R)0) { ct2 = k_sqrt((R)0.5 * ((R)1 + b.z)); st2 = st / ((R)2 * ct2); }
  else { st2 = k_sqrt((R)0.5 * ((R)1 - b.z)); ct2 = st / ((R)2 * st2); }
  R cp = (R)1, sp = (R)0;
  if (r2 > (R)KP_POLE2) { cp = b.x / st; sp = b.y / st; }
  R cp2, sp2;  // cos, sin of phi_B / 2 with phi_B in (-pi, pi]
  if (cp >= (R)0) { cp2 = k_sqrt((R)0.5 * ((R)1 + cp)); sp2 = sp / ((R)2 * cp2); }
  else {
    sp2 = k_sqrt((R)0.5 * ((R)1 - cp));
    if (sp < (R)0) sp2 = -sp2;
    cp2 = sp / ((R)2 * sp2);
  }
  return {cp2 * ct2, -sp2 * st2, cp2 * st2, sp2 * ct2};
}

// q^* (0, v) q : lab -> grain frame.  With q = (s, u): v + 2 u x (u x v) - 2 s u x v
template <typename R>
__device__ __forceinline__ V3<R> to_grain(const Quat<R>& q, const V3<R>& v) {
  V3<R> u{q.x, q.y, q.z};
  V3<R> t = cross(u, v);
  V3<R> t2 = cross(u, t);
  return {v.x + (R)2 * (t2.x - q.w * t.x), v.y + (R)2 * (t2.y - q.w * t.y),
          v.z + (R)2 * (t2.z - q.w * t.z)};
}
// q (0, v) q^* : grain -> lab frame
template <typename R>
__device__ __forceinline__ V3<R> from_grain(const Quat<R>& q, const V3<R>& v) {
  V3<R> u{q.x, q.y, q.z};
  V3<R> t = cross(u, v);
  V3<R> t2 = cross(u, t);
  return {v.x + (R)2 * (t2.x + q.w * t.x), v.y + (R)2 * (t2.y + q.w * t.y),
          v.z + (R)2 * (t2.z + q.w * t.z)};
}

// cos 2eta, sin 2eta for the basis change lab -> grain-frame natural basis of
// direction n (grain image ng): eta is the signed angle from the lab phi_hat
// carried into the grain frame to the natural phi_hat' of ng, positive about
// ng.  Stokes in the grain basis: Q' = c2 Q + s2 U, U' = -s2 Q + c2 U.
// phi_hat of a direction times sin(theta) (a positive factor), and phi_hat
// = (0, 1, 0) at the pole
template <typename R>
__device__ __forceinline__ V3<R> phi_scaled(const V3<R>& n) {
  const R r2 = n.x * n.x + n.y * n.y;
  return r2 <= (R)KP_POLE2 ? V3<R>{(R)0, (R)1, (R)0} : V3<R>{-n.y, n.x, (R)0};
}

template <typename R>
__device__ __forceinline__ void eta2(const Quat<R>& q, const V3<R>& n, const V3<R>& ng,
                                     R& c2, R& s2) {
  // cos and sin of eta up to one common positive factor (the two phi_hat
  // vectors are taken unnormalised), which cancels in cos 2 eta and sin 2 eta
  const V3<R> phg = to_grain(q, phi_scaled(n));
  const V3<R> php = phi_scaled(ng);
  const R c = dot(phg, php);
  const R s = dot(ng, cross(phg, php));
  const R ir = (R)1 / (c * c + s * s);
  c2 = (c * c - s * s) * ir;
  s2 = (R)2 * c * s * ir;
}

// 1 - e^{-x}  over x, i.e. (1 - e^{-x})/x with the x -> 0 limit
template <typename R>
__device__ __forceinline__ R phi1(R x) {
  return x == (R)0 ? (R)1 : -k_expm1(-x) / x;
}

}  // namespace kp
