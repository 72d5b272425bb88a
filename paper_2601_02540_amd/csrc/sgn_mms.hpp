// sgn_mms.hpp -- manufactured-solution source terms (Section 6.1.2).
//
// The manufactured fields are
//   b   = 0.08 (cos kx cos ky + 1/2 cos 2kx cos 2ky),       k = 2 pi
//   h   = 2 + 1/2 sin kx sin ky cos kt - b
//   u   = 0.3 sin kx sin kt,  v = 0.3 sin ky sin kt,  eta = h
//   w   = -h (u_x + v_y) + 3/2 (u b_x + v b_y).
// With eta = h the pressure-like terms of the hyperbolization vanish, and the
// system in the evolved variables reduces to
//   h_t + (h u)_x + (h v)_y            = S_h
//   u_t + u u_x + v u_y + g (h + b)_x  = S_u
//   v_t + u v_x + v v_y + g (h + b)_y  = S_v
//   w_t + u w_x + v w_y                = S_w
//   eta_t + u eta_x + v eta_y + 3/2 (u b_x + v b_y) - w = S_eta
// whose residuals are written out below from hand-derived derivatives
// (u_y = v_x = 0 for these fields).
#pragma once

#include <hip/hip_runtime.h>

namespace sgn {

// A real call, not inlined: inlined at every evaluation of a step tile, the five
// double-precision sincos evaluations took those kernels to 256 VGPRs plus
// 58-174 AGPRs at one wave per SIMD; called, they use 143-254 VGPRs, no AGPRs,
// a 48-byte call frame and two or three waves per SIMD.
__device__ inline __attribute__((noinline)) void mms_source(double x, double y, double t, double g, double S[5]) {
  const double k = 6.283185307179586476925286766559;
  const double k2 = k * k;
  double sx, cx, sy, cy, s2x, c2x, s2y, c2y, st, ct;
  sincos(k * x, &sx, &cx);
  sincos(k * y, &sy, &cy);
  sincos(2.0 * k * x, &s2x, &c2x);
  sincos(2.0 * k * y, &s2y, &c2y);
  sincos(k * t, &st, &ct);

  const double b_x = 0.08 * (-k * sx * cy - k * s2x * c2y);
  const double b_y = 0.08 * (-k * cx * sy - k * c2x * s2y);
  const double b_xx = 0.08 * (-k2 * cx * cy - 2.0 * k2 * c2x * c2y);
  const double b_yy = b_xx;
  const double b_xy = 0.08 * (k2 * sx * sy + 2.0 * k2 * s2x * s2y);
  const double b = 0.08 * (cx * cy + 0.5 * c2x * c2y);

  const double h = 2.0 + 0.5 * sx * sy * ct - b;
  const double h_t = -0.5 * k * sx * sy * st;
  const double h_x = 0.5 * k * cx * sy * ct - b_x;
  const double h_y = 0.5 * k * sx * cy * ct - b_y;

  const double u = 0.3 * sx * st;
  const double u_t = 0.3 * k * sx * ct;
  const double u_x = 0.3 * k * cx * st;
  const double u_xx = -0.3 * k2 * sx * st;
  const double u_xt = 0.3 * k2 * cx * ct;
  const double v = 0.3 * sy * st;
  const double v_t = 0.3 * k * sy * ct;
  const double v_y = 0.3 * k * cy * st;
  const double v_yy = -0.3 * k2 * sy * st;
  const double v_yt = 0.3 * k2 * cy * ct;

  const double div = u_x + v_y;
  const double w = -h * div + 1.5 * (u * b_x + v * b_y);
  const double w_t = -h_t * div - h * (u_xt + v_yt) + 1.5 * (u_t * b_x + v_t * b_y);
  const double w_x = -h_x * div - h * u_xx + 1.5 * (u_x * b_x + u * b_xx + v * b_xy);
  const double w_y = -h_y * div - h * v_yy + 1.5 * (u * b_xy + v_y * b_y + v * b_yy);

  S[0] = h_t + h_x * u + h * u_x + h_y * v + h * v_y;
  S[1] = u_t + u * u_x + g * (h_x + b_x);
  S[2] = v_t + v * v_y + g * (h_y + b_y);
  S[3] = w_t + u * w_x + v * w_y;
  S[4] = h_t + u * h_x + v * h_y + 1.5 * (u * b_x + v * b_y) - w;
}

}  // namespace sgn
