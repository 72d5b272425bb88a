// sgn_stage.hpp -- the fused right-hand-side + Runge-Kutta stage kernel.
//
// One workgroup of 256 threads (four wave64s) owns a tile of 64 x TY nodes.
// It stages the tile plus a one-node halo of the six input planes
// (h, u, v, w, eta, b) and of 1/h in LDS, with the periodic wrap or the
// reflecting clamp applied while loading.  Each thread then evaluates the
// split-form rates of eq. (sd_periodic_2D_SGN) / eq. (semi_2D) for TY/4 nodes
// of one column, with the one-sided closure rows and the wall SATs of Remark
// "Concrete SBP operators and SATs" resolved per node, and applies the stage
// update in registers.  Products that are differentiated (h(h+b), u^2, hu,
// huv, eta^2/h, huw, ...) are formed at the two neighbours from LDS values, so
// only one reciprocal per node is computed.
#pragma once

#include "sgn_common.hpp"
#include "sgn_mms.hpp"

namespace sgn {

constexpr int TILE_X = 64;
constexpr int STAGE_THREADS = 256;
constexpr int THREAD_ROWS = STAGE_THREADS / TILE_X;  // 4

// Neighbour selection along one axis for node index i of n: the left/right
// LDS offsets (relative to the node) and the derivative scale.  Interior and
// periodic rows use (f[i+1] - f[i-1]) / (2 d); reflecting first/last rows use
// (f[1] - f[0]) / d and (f[n-1] - f[n-2]) / d.
template <int BC>
struct AxisStencil {
  int om, op;
  double scale;
  __device__ __forceinline__ AxisStencil(int i, int n, double inv2d, double invd) {
    om = -1;
    op = 1;
    scale = inv2d;
    if (BC == BC_REFLECTING) {
      if (i == 0) {
        om = 0;
        scale = invd;
      }
      if (i == n - 1) {
        op = 0;
        scale = invd;
      }
    }
  }
};

template <typename T>
struct Node {
  T h, u, v, w, eta, b, ih;  // ih = 1/h
};

template <typename T, int TY>
struct StageSmem {
  T f[7][TY + 2][TILE_X + 2];  // h u v w eta b 1/h
};

template <typename T, int TY>
__device__ __forceinline__ Node<T> lds_node(const StageSmem<T, TY>& s, int r, int c) {
  Node<T> n;
  n.h = s.f[0][r][c];
  n.u = s.f[1][r][c];
  n.v = s.f[2][r][c];
  n.w = s.f[3][r][c];
  n.eta = s.f[4][r][c];
  n.b = s.f[5][r][c];
  n.ih = s.f[6][r][c];
  return n;
}

// Rates of the five evolved variables at one node given its value, its four
// neighbours (already resolved for closures) and the derivative scales.
template <typename T>
struct Rates {
  T h, u, v, w, eta;
};

// Every derivative along one axis at a node carries the same scale (1/(2d) on
// interior and periodic rows, 1/d on a closure row), so the differences are
// formed unscaled, the x- and y-terms of each rate are summed separately and
// each sum is scaled once.  The wall SAT enters only on reflecting axes.
template <typename T, int BCX, int BCY>
__device__ __forceinline__ Rates<T> split_form_rates(const Node<T>& c, const Node<T>& xm, const Node<T>& xp,
                                                     const Node<T>& ym, const Node<T>& yp, T sx, T sy, T g, T lam,
                                                     T satx_coef, T saty_coef) {
  const T half = T(0.5);
  // x differences (12), unscaled
  const T dxh = xp.h - xm.h;
  const T dxu = xp.u - xm.u;
  const T dxv = xp.v - xm.v;
  const T dxw = xp.w - xm.w;
  const T dxeta = xp.eta - xm.eta;
  const T dxb = xp.b - xm.b;
  const T dxhH = xp.h * (xp.h + xp.b) - xm.h * (xm.h + xm.b);
  const T dxu2 = xp.u * xp.u - xm.u * xm.u;
  const T xphu = xp.h * xp.u, xmhu = xm.h * xm.u;
  const T dxhu = xphu - xmhu;
  const T dxhuv = xphu * xp.v - xmhu * xm.v;
  // D(eta^2/h) = D(h) + D((eta - h)(eta + h)/h): the second part is small
  // (eta stays close to h), so it is formed without cancellation
  const T dxe2c = (xp.eta - xp.h) * (xp.eta + xp.h) * xp.ih - (xm.eta - xm.h) * (xm.eta + xm.h) * xm.ih;
  const T dxhuw = xphu * xp.w - xmhu * xm.w;
  // y differences (12), unscaled
  const T dyh = yp.h - ym.h;
  const T dyu = yp.u - ym.u;
  const T dyv = yp.v - ym.v;
  const T dyw = yp.w - ym.w;
  const T dyeta = yp.eta - ym.eta;
  const T dyb = yp.b - ym.b;
  const T dyhH = yp.h * (yp.h + yp.b) - ym.h * (ym.h + ym.b);
  const T dyv2 = yp.v * yp.v - ym.v * ym.v;
  const T yphv = yp.h * yp.v, ymhv = ym.h * ym.v;
  const T dyhv = yphv - ymhv;
  const T dyhuv = yphv * yp.u - ymhv * ym.u;
  const T dye2c = (yp.eta - yp.h) * (yp.eta + yp.h) * yp.ih - (ym.eta - ym.h) * (ym.eta + ym.h) * ym.ih;
  const T dyhvw = yphv * yp.w - ymhv * ym.w;

  const T h = c.h, u = c.u, v = c.v, w = c.w, eta = c.eta;
  const T H = h + c.b;
  // r - 1 = (eta - h)/h and r^2 - 1 = (r - 1)(r + 1), formed from eta - h, so
  // that a state at rest (eta = h) gives exactly zero relaxation terms
  const T rm1 = (eta - h) * c.ih;
  const T omr = -rm1;
  const T r2m1 = rm1 * (rm1 + T(2));
  const T hu = h * u, hv = h * v, uv = u * v, hw = h * w;
  const T lam6 = lam * T(1.0 / 6.0), lam3 = lam * T(1.0 / 3.0), lam2 = lam * T(0.5);
  const T hsx = half * sx, hsy = half * sy;

  Rates<T> k;
  k.h = -(sx * (u * dxh + h * dxu) + sy * (v * dyh + h * dyv));
  if (BCX == BC_REFLECTING) k.h += satx_coef * hu;
  if (BCY == BC_REFLECTING) k.h += saty_coef * hv;

  // A = h u_t, B = h v_t (with the sign of the rates), C = the flux part of h w_t
  // lambda/6 (r^2 D h - D(eta^2/h)) = lambda/6 ((r^2 - 1) D h - D((eta - h)(eta + h)/h))
  const T Ax = g * (dxhH - H * dxh) + lam6 * (r2m1 * dxh - dxe2c) + lam3 * omr * dxeta + lam2 * omr * dxb;
  const T Ax2 = h * dxu2 - u * u * dxh + u * dxhu - hu * dxu;
  const T Ay2 = dyhuv - uv * dyh + hv * dyu - hu * dyv;
  const T A = sx * Ax + hsx * Ax2 + hsy * Ay2;
  const T By = g * (dyhH - H * dyh) + lam6 * (r2m1 * dyh - dye2c) + lam3 * omr * dyeta + lam2 * omr * dyb;
  const T By2 = h * dyv2 - v * v * dyh + v * dyhv - hv * dyv;
  const T Bx2 = dxhuv - uv * dxh + hu * dxv - hv * dxu;
  const T B = sy * By + hsy * By2 + hsx * Bx2;
  const T Cx = dxhuw + hu * dxw - u * w * dxh - hw * dxu;
  const T Cy = dyhvw + hv * dyw - v * w * dyh - hw * dyv;
  const T C = hsx * Cx + hsy * Cy;
  k.u = -A * c.ih;
  k.v = -B * c.ih;
  k.w = (lam * omr - C) * c.ih;
  k.eta = w - (sx * (u * dxeta + T(1.5) * u * dxb) + sy * (v * dyeta + T(1.5) * v * dyb));
  return k;
}

template <typename T, int BCX, int BCY, int MODE, bool SRC, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void stage_kernel(const GridConst gc, const T* __restrict__ Y,
                                                              const T* __restrict__ bplane,
                                                              const T* __restrict__ qn, T* __restrict__ acc,
                                                              T* __restrict__ out, T c_acc, T c_y, double t,
                                                              int* __restrict__ flag) {
  static_assert(TY % THREAD_ROWS == 0, "tile height must be a multiple of 4");
  constexpr int RPT = TY / THREAD_ROWS;
  constexpr int W = TILE_X + 2;
  constexpr int REGION = (TY + 2) * W;
  __shared__ StageSmem<T, TY> s;

  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const int ntx = (nx + TILE_X - 1) / TILE_X;
  const int nty = (ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  const int i0 = (tile % ntx) * TILE_X;
  const int j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;
  const int tx = tid & (TILE_X - 1);
  const int ty = tid >> 6;

  // Stage the tile and its halo.  Periodic axes wrap, reflecting axes clamp
  // (clamped halo values are never used: the closure rows are one-sided).
  for (int idx = tid; idx < REGION; idx += STAGE_THREADS) {
    const int rr = idx / W;
    const int cc = idx - rr * W;
    int gi = i0 - 1 + cc;
    int gj = j0 - 1 + rr;
    if (BCX == BC_PERIODIC) {
      if (gi < 0) gi += nx;
      while (gi >= nx) gi -= nx;
    } else {
      gi = gi < 0 ? 0 : (gi >= nx ? nx - 1 : gi);
    }
    if (BCY == BC_PERIODIC) {
      if (gj < 0) gj += ny;
      while (gj >= ny) gj -= ny;
    } else {
      gj = gj < 0 ? 0 : (gj >= ny ? ny - 1 : gj);
    }
    const size_t o = (size_t)gj * nx + gi;
    const T h = Y[o];
    s.f[0][rr][cc] = h;
    s.f[1][rr][cc] = Y[N + o];
    s.f[2][rr][cc] = Y[2 * N + o];
    s.f[3][rr][cc] = Y[3 * N + o];
    s.f[4][rr][cc] = Y[4 * N + o];
    s.f[5][rr][cc] = bplane[o];
    s.f[6][rr][cc] = recip_staged(h);
  }

  // Own-node operands of the stage update, fetched before the barrier so the
  // loads overlap the LDS staging.
  const int i = i0 + tx;
  T pre[RPT][5];
  T pacc[RPT][5];
  if (MODE == MODE_MID || MODE == MODE_LAST) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int j = j0 + ty + k * THREAD_ROWS;
      if (i < nx && j < ny) {
        const size_t o = (size_t)j * nx + i;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          pacc[k][f] = acc[f * N + o];
          if (MODE == MODE_MID) pre[k][f] = qn[f * N + o];
        }
      }
    }
  }
  __syncthreads();

  const T g = T(gc.g), lam = T(gc.lam);
  const AxisStencil<BCX> ax(i, nx, gc.inv2dx, gc.invdx);
  T satx = T(0);
  if (BCX == BC_REFLECTING) {
    if (i == 0) satx = T(-2.0 * gc.invdx);
    if (i == nx - 1) satx = T(2.0 * gc.invdx);
  }
  int health = 0;

#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = ty + k * THREAD_ROWS;
    const int j = j0 + lr;
    if (i >= nx || j >= ny) continue;
    const AxisStencil<BCY> ay(j, ny, gc.inv2dy, gc.invdy);
    T saty = T(0);
    if (BCY == BC_REFLECTING) {
      if (j == 0) saty = T(-2.0 * gc.invdy);
      if (j == ny - 1) saty = T(2.0 * gc.invdy);
    }
    const int r = lr + 1, cidx = tx + 1;
    const Node<T> c = lds_node(s, r, cidx);
    const Node<T> xm = lds_node(s, r, cidx + ax.om);
    const Node<T> xp = lds_node(s, r, cidx + ax.op);
    const Node<T> ym = lds_node(s, r + ay.om, cidx);
    const Node<T> yp = lds_node(s, r + ay.op, cidx);
    Rates<T> kk = split_form_rates<T, BCX, BCY>(c, xm, xp, ym, yp, T(ax.scale), T(ay.scale), g, lam, satx, saty);
    if (SRC) {
      double S[5];
      mms_source(gc.xmin + i * gc.dx, gc.ymin + j * gc.dy, t, gc.g, S);
      kk.h += T(S[0]);
      kk.u += T(S[1]);
      kk.v += T(S[2]);
      kk.w += T(S[3]);
      kk.eta += T(S[4]);
    }
    const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
    const T yv[5] = {c.h, c.u, c.v, c.w, c.eta};
    const size_t o = (size_t)j * nx + i;
    if (MODE == MODE_RHS) {
#pragma unroll
      for (int f = 0; f < 5; ++f) out[f * N + o] = kv[f];
    } else if (MODE == MODE_FIRST) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        acc[f * N + o] = yv[f] + c_acc * kv[f];
        out[f * N + o] = yv[f] + c_y * kv[f];
      }
    } else if (MODE == MODE_MID) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        acc[f * N + o] = pacc[k][f] + c_acc * kv[f];
        out[f * N + o] = pre[k][f] + c_y * kv[f];
      }
    } else {
      T nv[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        nv[f] = pacc[k][f] + c_acc * kv[f];
        out[f * N + o] = nv[f];
      }
      if (!(nv[0] > T(0))) health |= FLAG_NONPOS;
      const T sum = nv[0] + nv[1] + nv[2] + nv[3] + nv[4];
      if (!isfinite(sum)) health |= FLAG_NONFINITE;
    }
  }
  if (MODE == MODE_LAST && health) atomicOr(flag, health);
}

}  // namespace sgn
