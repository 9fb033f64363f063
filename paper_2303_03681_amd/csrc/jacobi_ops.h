// Algorithm 1's pair step on register-resident rows, shared by the Jacobi
// kernels: partial sums of (x^+x, y^+y, x^+y) per lane, the rotation of one
// pair from the reduced sums, and its application; plus the lane-exchange
// helpers used to reduce several pairs at once.
#pragma once

#include <hip/hip_runtime.h>

#include "wave_ops.h"

namespace mps {

template <int E>
__device__ __forceinline__ void pair_partials(const double2 (&x)[E], const double2 (&y)[E],
                                              double* acc) {
  double xx = 0.0, yy = 0.0, re = 0.0, im = 0.0;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const double2 a = x[k], b = y[k];
    xx += a.x * a.x + a.y * a.y;
    yy += b.x * b.x + b.y * b.y;
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  acc[0] = xx;
  acc[1] = yy;
  acc[2] = re;
  acc[3] = im;
}

struct Rot {
  double c, ar, ai, br, bi;  // x' = c x + (ar + i ai) y,  y' = c y + (br + i bi) x
};

// Algorithm 1's rotation from b_xx = x^+x, b_yy = y^+y and b_xy = x^+y of one
// pair, in this lane; the row with the lower index plays a_i.  Returns false
// when the pair is already orthogonal to the tolerance (|b_ij| <= eps
// sqrt(b_ii b_jj) or <= floor).  *dn receives t |b_ij|, by which b_ii grows
// and b_jj shrinks under the rotation.
// Algorithm 1's rotation test: |b_ij| > floor and |b_ij| > eps sqrt(b_ii
// b_jj), compared in squares (symmetric in the two rows).
__device__ __forceinline__ bool pair_needs_rot(double bxx, double byy, double br, double bi, double eps,
                                               double floor) {
  const double mag2 = br * br + bi * bi;
  return mag2 > floor * floor && mag2 > eps * eps * (bxx * byy);
}

// The rotation itself, for a pair that passed pair_needs_rot.
__device__ __forceinline__ void pair_rot_coeffs(double bxx, double byy, double br, double bi, bool x_is_i,
                                                Rot& rt, double* dn) {
  const double bii = x_is_i ? bxx : byy, bjj = x_is_i ? byy : bxx;
  const double mag2 = br * br + bi * bi;
  const double rinv = rsqrt(mag2);  // 1 / |b_ij|
  const double tau = (bii - bjj) * (0.5 * rinv);
  const double at = fabs(tau);
  const double sg = tau >= 0.0 ? 1.0 : -1.0;
  const double t = at > 1e100 ? sg * (0.5 / at) : sg / (at + sqrt(1.0 + tau * tau));
  const double c = rsqrt(1.0 + t * t);
  const double s = t * c;
  const double er = br * rinv, ei = x_is_i ? bi * rinv : -bi * rinv;
  // a_i' = c a_i + s conj(e) a_j,  a_j' = c a_j - s e a_i
  const double pr = s * er, pi = -s * ei, qr = -s * er, qi = -s * ei;
  rt.c = c;
  rt.ar = x_is_i ? pr : qr;
  rt.ai = x_is_i ? pi : qi;
  rt.br = x_is_i ? qr : pr;
  rt.bi = x_is_i ? qi : pi;
  if (dn) *dn = t * (mag2 * rinv);
}

__device__ __forceinline__ bool pair_rot_core(double bxx, double byy, double br, double bi, bool x_is_i,
                                              double eps, double floor, Rot& rt, double* dn) {
  if (!pair_needs_rot(bxx, byy, br, bi, eps, floor)) return false;
  pair_rot_coeffs(bxx, byy, br, bi, x_is_i, rt, dn);
  return true;
}

// The same from the reduced (x^+x, y^+y, Re x^+y, Im x^+y).
__device__ __forceinline__ bool pair_rot_lane(const double* acc, bool x_is_i, double eps,
                                              double floor, Rot& rt) {
  return pair_rot_core(acc[0], acc[1], acc[2], acc[3], x_is_i, eps, floor, rt, nullptr);
}

// Partial sums of Re and Im of x^+y over this lane's elements.
template <int E>
__device__ __forceinline__ void pair_partials_xy(const double2 (&x)[E], const double2 (&y)[E],
                                                 double& re, double& im) {
  re = 0.0;
  im = 0.0;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const double2 a = x[k], b = y[k];
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
}

template <int E>
__device__ __forceinline__ void pair_apply(double2 (&x)[E], double2 (&y)[E], const Rot& rt) {
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const double2 a = x[k], b = y[k];
    x[k] = make_double2(rt.c * a.x + (rt.ar * b.x - rt.ai * b.y), rt.c * a.y + (rt.ar * b.y + rt.ai * b.x));
    y[k] = make_double2(rt.c * b.x + (rt.br * a.x - rt.bi * a.y), rt.c * b.y + (rt.br * a.y + rt.bi * a.x));
  }
}

template <int PAT>
__device__ __forceinline__ double swizzle(double x) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), PAT);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), PAT);
  return __hiloint2double(hi, lo);
}
// ds_swizzle bit mode: lane' = ((lane & and) | or) ^ xor within 32 lanes
constexpr int swz(int x) { return 0x1F | (x << 10); }

__device__ __forceinline__ double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

}  // namespace mps
