// sgn_relax.hpp -- relaxation Runge-Kutta (fully discrete energy conservation).
//
// The semi-discretization conserves the total energy E = 1^T M E (Theorem 2);
// classical RK4 does not quite.  Relaxation in the incremental direction form
// takes the RK4 update d = q_RK4 - q_n, advances q_{n+1} = q_n + gam d and
// t_{n+1} = t_n + gam dt, with gam the root near 1 of E(q_n + gam d) = E(q_n);
// the method keeps its fourth order and conserves E to rounding.
//
// E(q_n + gam d) and E(q_n) agree in their leading digits (the potential
// energy dominates both), so their difference is not formed by subtraction.
// Per node, the change of each part of the energy density divided by gam is
// written out as a polynomial (a rational function for the lambda term) in gam
// whose coefficients are products of the node's values and increments:
//   kinetic   (h (u^2 + v^2)/2):  [dh (u^2 + v^2) + H (2u du + 2v dv + gam (du^2 + dv^2))] / 2
//   w term    (h w^2 / 6):        [dh w^2 + H (2w dw + gam dw^2)] / 6
//   potential (g h (h + 2b)/2):   g/2 dh (2h + 2b + gam dh)
//   lambda    (lam/6 (eta - h)^2 / h), A = eta - h, B = deta - dh:
//                                  lam/6 [h (2AB + gam B^2) - dh A^2] / (h H)
// with H = h + gam dh.  Their M-weighted sum s(gam) = (E(q_n + gam d) - E(q_n))/gam
// has no root at gam = 0; two Newton iterations from gam = 1, with s'(gam) from
// the same pass, find the relaxation root.  All of it in FP64 whatever the
// storage type, with compensated, deterministic reductions.
#pragma once

#include "sgn_fused.hpp"
#include "sgn_reduce.hpp"

namespace sgn {

// Per-block partial sums of s(gam) and s'(gam) (compensated: 4 doubles per
// block).  gam = 1 when `first`, else rs[0].
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void relax_partial(const GridConst gc, const T* __restrict__ q,
                                                             const T* __restrict__ qrk, const T* __restrict__ bplane,
                                                             const double* __restrict__ rs, int first,
                                                             double* __restrict__ partials) {
  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const double g = gc.g, lam = gc.lam;
  const double gam = first ? 1.0 : rs[0];
  CSum a[2];
  a[0].init();
  a[1].init();
  for (int j = blockIdx.x; j < ny; j += gridDim.x) {
    const double wy = axis_weight(j, ny, gc.bc_y, gc.dy);
    for (int i = threadIdx.x; i < nx; i += RED_THREADS) {
      const double M = axis_weight(i, nx, gc.bc_x, gc.dx) * wy;
      const size_t o = (size_t)j * nx + i;
      double x[5], dx[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        x[f] = (double)q[f * N + o];
        dx[f] = (double)qrk[f * N + o] - x[f];
      }
      double sv, dsv;
      relax_node_terms(x, dx, (double)bplane[o], g, lam, gam, sv, dsv);
      a[0].add(M * sv);
      a[1].add(M * dsv);
    }
  }
  block_merge<2>(a);
  if (threadIdx.x == 0) {
    partials[4 * blockIdx.x + 0] = a[0].s;
    partials[4 * blockIdx.x + 1] = a[0].c;
    partials[4 * blockIdx.x + 2] = a[1].s;
    partials[4 * blockIdx.x + 3] = a[1].c;
  }
}

// One block: s and s' from the partials (block order), one Newton update of
// gam in rs[0] (from 1 when `first`).  A step without a usable root (s' zero or
// not finite, or gam leaving [1/2, 3/2]) keeps gam = 1.  When `last`, the time
// in rs[1] advances by gam dt.
static __global__ __launch_bounds__(RED_THREADS) void relax_newton(const double* __restrict__ partials, int nparts,
                                                            double* __restrict__ rs, int first, int last,
                                                            double dt) {
  CSum a[2];
  a[0].init();
  a[1].init();
  // Thread t merges partials t, t + 256, t + 512, ... in that order; the loads
  // of eight of them are issued before the first merge (the step kernel leaves
  // one partial per tile, tens of thousands of them).
  constexpr int U = 8;
  for (int p0 = threadIdx.x; p0 < nparts; p0 += U * RED_THREADS) {
    double v[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * RED_THREADS;
#pragma unroll
      for (int k = 0; k < 4; ++k) v[u][k] = p < nparts ? partials[4 * p + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (p0 + u * RED_THREADS >= nparts) break;
      a[0].merge(v[u][0], v[u][1]);
      a[1].merge(v[u][2], v[u][3]);
    }
  }
  block_merge<2>(a);
  if (threadIdx.x == 0) {
    const double s = a[0].s + a[0].c, ds = a[1].s + a[1].c;
    const double gam = first ? 1.0 : rs[0];
    double next = gam;
    if (ds != 0.0 && isfinite(s) && isfinite(ds)) next = gam - s / ds;
    if (!(next >= 0.5 && next <= 1.5)) next = 1.0;
    rs[0] = next;
    if (last) rs[1] += next * dt;
  }
}

// rs[1] = t0 (the time accumulator of a relaxation run).
static __global__ void relax_set_time(double* __restrict__ rs, double t0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) rs[1] = t0;
}

// out <- q + gam (q_RK4 - q), elementwise over the five planes (out may be q).
template <typename T>
__global__ __launch_bounds__(256) void relax_update(size_t n5, T* out, const T* q, const T* __restrict__ qrk,
                                                    const double* __restrict__ rs) {
  const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n5) return;
  const T gam = T(rs[0]);
  const T x = q[k];
  out[k] = x + gam * (qrk[k] - x);
}

// One RK4 step of a relaxation run after its first: the step tile stages the
// relaxed state of the previous step, qa + gam (ra - qa), writes it out for
// its owned nodes (qbase) beside the RK4 result (qout), and reduces the first
// Newton iteration's sums per tile (EPI_RELAX), so no update pass runs between
// the steps.
template <typename T, int BCX, int BCY, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void relax_step_kernel(const GridConst gc, const T* __restrict__ qa,
                                                                   const T* __restrict__ bplane,
                                                                   T* __restrict__ qout, const RelaxIn<T> rx, T c6,
                                                                   T c3, T c2, T c1, double dt,
                                                                   int* __restrict__ flag,
                                                                   double* __restrict__ rpart) {
  constexpr int TX = StepGeom<TY>::TX;
  __shared__ StepSmem<T, TY, 1> s;
  const int ntx = (gc.nx + TX - 1) / TX;
  const int nty = (gc.ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  step_tile<T, BCX, BCY, false, TY, false, 1, EPI_RELAX, RK_RELAXED>(
      s, gc, (tile % ntx) * TX, (tile / ntx) * TY, qa, bplane, qout, c6, c3, c2, c1, 0.0, dt, flag, nullptr,
      rpart + 4 * tile, nullptr, &rx);
}

}  // namespace sgn
