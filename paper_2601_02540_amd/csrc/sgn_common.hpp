// sgn_common.hpp -- shared definitions of the gfx950 kernels (device side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgn {

enum : int { BC_PERIODIC = 0, BC_REFLECTING = 1 };

// What a fused stage kernel does with the right-hand side k it evaluates at Y.
//   RHS:   out = k
//   FIRST: acc = Y + c_acc k,   out = Y  + c_y k     (Y is q_n)
//   MID:   acc = acc + c_acc k, out = qn + c_y k
//   LAST:  out = acc + c_acc k                       (out is q_{n+1})
enum : int { MODE_RHS = 0, MODE_FIRST = 1, MODE_MID = 2, MODE_LAST = 3 };

// Health flag bits raised by kernels.
enum : int { FLAG_NONPOS = 1, FLAG_NONFINITE = 2, FLAG_BADINDEX = 4 };

// Grid constants passed by value to every kernel.
struct GridConst {
  int nx, ny;
  int bc_x, bc_y;
  double dx, dy;          // spacing
  double inv2dx, inv2dy;  // 1/(2 dx), 1/(2 dy): interior central rows
  double invdx, invdy;    // 1/dx, 1/dy: reflecting closure rows
  double xmin, ymin;
  double g, lam;
};

// Quadrature weight of node i on an axis (diagonal of M): dx, or dx/2 at a wall.
__device__ __forceinline__ double axis_weight(int i, int n, int bc, double d) {
  return (bc == BC_REFLECTING && (i == 0 || i == n - 1)) ? 0.5 * d : d;
}

// Error-free transformation a + b = s + e (Knuth TwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated accumulator: value = s + c.
struct CSum {
  double s, c;
  __device__ __forceinline__ void init() { s = 0.0; c = 0.0; }
  __device__ __forceinline__ void add(double x) {
    double t, e;
    two_sum(s, x, t, e);
    s = t;
    c += e;
  }
  __device__ __forceinline__ void merge(double s2, double c2) {
    double t, e;
    two_sum(s, s2, t, e);
    s = t;
    c += c2 + e;
  }
};

// 1/h of a staged node: the hardware reciprocal estimate refined by Newton's
// iteration r <- r + r (1 - h r) (each step squares the relative error), two
// steps in FP64 and one in FP32, which leaves an error of about one unit in the
// last place against the six-instruction-longer IEEE division.  Every kernel
// stages 1/h through this function, so all step paths still form the same bits.
__device__ __forceinline__ double recip_staged(double h) {
  double r = __builtin_amdgcn_rcp(h);
  r = __builtin_fma(r, __builtin_fma(-h, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-h, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float recip_staged(float h) {
  const float r = __builtin_amdgcn_rcpf(h);
  return __builtin_fmaf(r, __builtin_fmaf(-h, r, 1.0f), r);
}

// `true` that the compiler cannot see through (an empty asm statement that
// claims to modify a VGPR; no instruction is emitted).  Used where a predicate
// that is constant for one boundary type would otherwise turn a guarded phase
// into straight-line code that the scheduler hoists across, at the price of
// doubling the kernel's register footprint.
__device__ __forceinline__ bool opaque_true() {
  int one = 1;
  asm volatile("" : "+v"(one));
  return one != 0;
}

// Blocks are dealt to the eight XCDs of the MI355X round-robin (block b runs on
// XCD b mod 8).  Give every XCD one contiguous range of tiles in row-major
// order so that the halo rows shared by vertically adjacent tiles are fetched
// into the same XCD's L2.  The map is a bijection on [0, ntiles).
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int xcd = b & 7;
  const int k = b >> 3;
  const int per = ntiles >> 3;
  const int rem = ntiles & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + k;
}

}  // namespace sgn
