// sgn_vjp.hpp -- vector-Jacobian product of the split-form right-hand side
// (discrete adjoint of eq. (sd_periodic_2D_SGN) / eq. (semi_2D)) and of the
// classical RK4 stages.
//
// Reverse of one node c.  Given the cotangent kb of the five rates at c, the
// reverse of split_form_rates yields cotangents of the node's own raw values
// and of the 24 derivative values D_x f(c), D_y f(c).  A derivative
// D f(c) = s (f(c+op) - f(c+om)) sends +s Dbar to the node c+op and -s Dbar
// to c+om (a one-sided closure row sends one of them to c itself); at the
// receiving node the product f (h(h+b), u^2, hu, huv, eta^2/h, ...) is chained
// back to that node's raw values.  The cotangent of node d is the sum of what
// d and its four neighbours send to it -- the transpose of the stencil.
//
// The cotangent a derivative D f(c) sends out, Dbar_f(c), depends only on node
// c's own state and rate cotangent (it is the factor multiplying D f in the
// rates, times the seed), not on any derivative.  The kernel therefore works
// in gather form, like the forward stencil: node d evaluates Dbar_f at its
// neighbours from their LDS values and applies the transposed operator column
//   (D^T Dbar)(d) = D[d-1][d] Dbar(d-1) + D[d][d] Dbar(d) + D[d+1][d] Dbar(d+1)
// (AxisTranspose below, closure rows included), then chains the amounts back
// through the products at d.  No value crosses threads except through LDS.
#pragma once

#include "sgn_stage.hpp"

namespace sgn {

// Reverse-mode stage roles.  Cotangent of the step output: Qb.
//   PLAIN: kb = Kin;           out = Ybar (5 planes), bout = bbar      (rhs VJP)
//   S4:    kb = a * Qb;        Kout = cq Qb + cy Ybar, Acc  = Ybar
//   S3/S2: kb = Kin;           Kout = cq Qb + cy Ybar, Acc += Ybar
//   S1:    kb = Kin;           Qb  = Qb + Acc + Ybar
// and every role but PLAIN adds the bathymetry cotangent into Bb.
enum : int { VJP_PLAIN = 0, VJP_S4 = 4, VJP_S3 = 3, VJP_S2 = 2, VJP_S1 = 1 };

template <typename T>
struct Cot {
  T h, u, v, w, eta, b;
  __device__ __forceinline__ void zero() { h = u = v = w = eta = b = T(0); }
  __device__ __forceinline__ void add(const Cot& o) {
    h += o.h;
    u += o.u;
    v += o.v;
    w += o.w;
    eta += o.eta;
    b += o.b;
  }
};

// Chain the derivative cotangents amounts a[0..11] of the x-quantities
// (h u v w eta b h(h+b) u^2 hu huv eta^2/h huw) at node n.
template <typename T>
__device__ __forceinline__ Cot<T> chain_x(const Node<T>& n, const T (&a)[12]) {
  Cot<T> c;
  const T e2 = n.eta * n.eta;
  c.h = a[0] + (T(2) * n.h + n.b) * a[6] + n.u * a[8] + n.u * n.v * a[9] - e2 * n.ih * n.ih * a[10] +
        n.u * n.w * a[11];
  c.u = a[1] + T(2) * n.u * a[7] + n.h * a[8] + n.h * n.v * a[9] + n.h * n.w * a[11];
  c.v = a[2] + n.h * n.u * a[9];
  c.w = a[3] + n.h * n.u * a[11];
  c.eta = a[4] + T(2) * n.eta * n.ih * a[10];
  c.b = a[5] + n.h * a[6];
  return c;
}

// Same for the y-quantities (h u v w eta b h(h+b) v^2 hv huv eta^2/h hvw).
template <typename T>
__device__ __forceinline__ Cot<T> chain_y(const Node<T>& n, const T (&a)[12]) {
  Cot<T> c;
  const T e2 = n.eta * n.eta;
  c.h = a[0] + (T(2) * n.h + n.b) * a[6] + n.v * a[8] + n.u * n.v * a[9] - e2 * n.ih * n.ih * a[10] +
        n.v * n.w * a[11];
  c.u = a[1] + n.h * n.v * a[9];
  c.v = a[2] + T(2) * n.v * a[7] + n.h * a[8] + n.h * n.u * a[9] + n.h * n.w * a[11];
  c.w = a[3] + n.h * n.v * a[11];
  c.eta = a[4] + T(2) * n.eta * n.ih * a[10];
  c.b = a[5] + n.h * a[6];
  return c;
}

// Reverse of split_form_rates at one node.  Outputs the cotangent of the node's
// own raw values (center) and the derivative cotangents dX[12], dY[12] (of the
// derivative values themselves, before the stencil scale).
template <typename T>
__device__ __forceinline__ void split_form_reverse(const Node<T>& c, const Node<T>& xm, const Node<T>& xp,
                                                   const Node<T>& ym, const Node<T>& yp, T sx, T sy, T g, T lam,
                                                   T satx, T saty, const T (&kb)[5], Cot<T>& cen, T (&dX)[12],
                                                   T (&dY)[12]) {
  const T half = T(0.5);
  // forward values
  const T Dxh = sx * (xp.h - xm.h), Dxu = sx * (xp.u - xm.u), Dxv = sx * (xp.v - xm.v), Dxw = sx * (xp.w - xm.w);
  const T Dxeta = sx * (xp.eta - xm.eta), Dxb = sx * (xp.b - xm.b);
  const T DxhH = sx * (xp.h * (xp.h + xp.b) - xm.h * (xm.h + xm.b));
  const T Dxu2 = sx * (xp.u * xp.u - xm.u * xm.u);
  const T xphu = xp.h * xp.u, xmhu = xm.h * xm.u;
  const T Dxhu = sx * (xphu - xmhu);
  const T Dxhuv = sx * (xphu * xp.v - xmhu * xm.v);
  const T Dxe2h = sx * (xp.eta * xp.eta * xp.ih - xm.eta * xm.eta * xm.ih);
  const T Dxhuw = sx * (xphu * xp.w - xmhu * xm.w);
  const T Dyh = sy * (yp.h - ym.h), Dyu = sy * (yp.u - ym.u), Dyv = sy * (yp.v - ym.v), Dyw = sy * (yp.w - ym.w);
  const T Dyeta = sy * (yp.eta - ym.eta), Dyb = sy * (yp.b - ym.b);
  const T DyhH = sy * (yp.h * (yp.h + yp.b) - ym.h * (ym.h + ym.b));
  const T Dyv2 = sy * (yp.v * yp.v - ym.v * ym.v);
  const T yphv = yp.h * yp.v, ymhv = ym.h * ym.v;
  const T Dyhv = sy * (yphv - ymhv);
  const T Dyhuv = sy * (yphv * yp.u - ymhv * ym.u);
  const T Dye2h = sy * (yp.eta * yp.eta * yp.ih - ym.eta * ym.eta * ym.ih);
  const T Dyhvw = sy * (yphv * yp.w - ymhv * ym.w);
  const T h = c.h, u = c.u, v = c.v, w = c.w, eta = c.eta, ih = c.ih;
  const T H = h + c.b;
  const T r = eta * ih;
  const T omr = T(1) - r;
  const T hu = h * u, hv = h * v, uv = u * v, hw = h * w, uw = u * w, vw = v * w;
  const T lam6 = lam * T(1.0 / 6.0), lam3 = lam * T(1.0 / 3.0), lam2 = lam * T(0.5);
  const T A = g * (DxhH - H * Dxh) +
              half * (h * Dxu2 - u * u * Dxh + u * Dxhu - hu * Dxu + Dyhuv - uv * Dyh + hv * Dyu - hu * Dyv) +
              lam6 * (r * r * Dxh - Dxe2h) + lam3 * omr * Dxeta + lam2 * omr * Dxb;
  const T B = g * (DyhH - H * Dyh) +
              half * (h * Dyv2 - v * v * Dyh + v * Dyhv - hv * Dyv + Dxhuv - uv * Dxh + hu * Dxv - hv * Dxu) +
              lam6 * (r * r * Dyh - Dye2h) + lam3 * omr * Dyeta + lam2 * omr * Dyb;
  const T C = half * (Dxhuw + hu * Dxw - u * w * Dxh - hw * Dxu + Dyhvw + hv * Dyw - v * w * Dyh - hw * Dyv);

  const T ah = kb[0], au = kb[1], av = kb[2], aw = kb[3], ae = kb[4];
  for (int k = 0; k < 12; ++k) {
    dX[k] = T(0);
    dY[k] = T(0);
  }
  const T Ab = -au * ih, Bb = -av * ih, Cb = -aw * ih;
  T ihb = -au * A - av * B + aw * (lam * omr - C);
  T omrb = lam * aw * ih;
  T hb, ub, vb, wb, etab, Hb, hub, hvb, uvb, hwb, uwb, vwb, rb;
  // k_eta = w - (u Dxeta + v Dyeta + 3/2 (u Dxb + v Dyb))
  wb = ae;
  ub = -ae * (Dxeta + T(1.5) * Dxb);
  vb = -ae * (Dyeta + T(1.5) * Dyb);
  dX[4] = -ae * u;
  dY[4] = -ae * v;
  dX[5] = -T(1.5) * ae * u;
  dY[5] = -T(1.5) * ae * v;
  // k_h = -(u Dxh + h Dxu + v Dyh + h Dyv) + satx hu + saty hv
  ub += -ah * Dxh;
  dX[0] = -ah * u;
  hb = -ah * (Dxu + Dyv);
  dX[1] = -ah * h;
  vb += -ah * Dyh;
  dY[0] = -ah * v;
  dY[2] = -ah * h;
  hub = ah * satx;
  hvb = ah * saty;
  // A
  dX[6] += g * Ab;
  Hb = -g * Ab * Dxh;
  dX[0] += -g * Ab * H;
  hb += half * Ab * Dxu2;
  dX[7] += half * Ab * h;
  ub += -Ab * u * Dxh;
  dX[0] += -half * Ab * u * u;
  ub += half * Ab * Dxhu;
  dX[8] += half * Ab * u;
  hub += -half * Ab * Dxu;
  dX[1] += -half * Ab * hu;
  dY[9] += half * Ab;
  uvb = -half * Ab * Dyh;
  dY[0] += -half * Ab * uv;
  hvb += half * Ab * Dyu;
  dY[1] += half * Ab * hv;
  hub += -half * Ab * Dyv;
  dY[2] += -half * Ab * hu;
  rb = lam3 * Ab * r * Dxh;
  dX[0] += lam6 * Ab * r * r;
  dX[10] += -lam6 * Ab;
  omrb += lam3 * Ab * Dxeta + lam2 * Ab * Dxb;
  dX[4] += lam3 * Ab * omr;
  dX[5] += lam2 * Ab * omr;
  // B
  dY[6] += g * Bb;
  Hb += -g * Bb * Dyh;
  dY[0] += -g * Bb * H;
  hb += half * Bb * Dyv2;
  dY[7] += half * Bb * h;
  vb += -Bb * v * Dyh;
  dY[0] += -half * Bb * v * v;
  vb += half * Bb * Dyhv;
  dY[8] += half * Bb * v;
  hvb += -half * Bb * Dyv;
  dY[2] += -half * Bb * hv;
  dX[9] += half * Bb;
  uvb += -half * Bb * Dxh;
  dX[0] += -half * Bb * uv;
  hub += half * Bb * Dxv;
  dX[2] += half * Bb * hu;
  hvb += -half * Bb * Dxu;
  dX[1] += -half * Bb * hv;
  rb += lam3 * Bb * r * Dyh;
  dY[0] += lam6 * Bb * r * r;
  dY[10] += -lam6 * Bb;
  omrb += lam3 * Bb * Dyeta + lam2 * Bb * Dyb;
  dY[4] += lam3 * Bb * omr;
  dY[5] += lam2 * Bb * omr;
  // C
  dX[11] += half * Cb;
  hub += half * Cb * Dxw;
  dX[3] += half * Cb * hu;
  uwb = -half * Cb * Dxh;
  dX[0] += -half * Cb * uw;
  hwb = -half * Cb * Dxu;
  dX[1] += -half * Cb * hw;
  dY[11] += half * Cb;
  hvb += half * Cb * Dyw;
  dY[3] += half * Cb * hv;
  vwb = -half * Cb * Dyh;
  dY[0] += -half * Cb * vw;
  hwb += -half * Cb * Dyv;
  dY[2] += -half * Cb * hw;
  // center products
  rb += -omrb;
  hb += Hb;
  T bb = Hb;
  hb += u * hub;
  ub += h * hub;
  hb += v * hvb;
  vb += h * hvb;
  ub += v * uvb;
  vb += u * uvb;
  hb += w * hwb;
  wb += h * hwb;
  ub += w * uwb;
  wb += u * uwb;
  vb += w * vwb;
  wb += v * vwb;
  etab = rb * ih;
  ihb += rb * eta;
  hb += -ih * ih * ihb;
  cen.h = hb;
  cen.u = ub;
  cen.v = vb;
  cen.w = wb;
  cen.eta = etab;
  cen.b = bb;
}

// Column d of the 1D operator: weights of Dbar(d-1), Dbar(d), Dbar(d+1) in
// (D^T Dbar)(d).  Interior/periodic rows are (-1, 0, 1)/(2 delta); the
// reflecting first and last rows are (-2, 2)/(2 delta) (n >= 4 assumed).
template <typename T, int BC>
struct AxisTranspose {
  T wl, wc, wr;
  __device__ __forceinline__ AxisTranspose(int i, int n, double inv2d, double invd) {
    wl = T(inv2d);
    wc = T(0);
    wr = T(-inv2d);
    if (BC == BC_REFLECTING) {
      if (i == 0) {
        wl = T(0);
        wc = T(-invd);
      } else if (i == 1) {
        wl = T(invd);
      }
      if (i == n - 1) {
        wr = T(0);
        wc = T(invd);
      } else if (i == n - 2) {
        wr = T(-invd);
      }
    }
  }
};

template <typename T>
struct Seed {
  T h, u, v, w, eta;  // cotangent of the five rates at one node
};

// Dbar of the 12 x-quantities (h u v w eta b h(h+b) u^2 hu huv eta^2/h huw) at
// a node from its own state n and seed a: the factor of each D_x f in the
// rates of eq. (sd_periodic_2D_SGN), times the seed of that rate.
template <typename T>
__device__ __forceinline__ void dbar_x(const Node<T>& n, const Seed<T>& a, T g, T lam, T (&q)[12]) {
  const T half = T(0.5);
  const T ih = n.ih;
  const T Ab = -a.u * ih, Bb = -a.v * ih, Cb = -a.w * ih;
  const T H = n.h + n.b, r = n.eta * ih, omr = T(1) - r;
  const T hu = n.h * n.u, hv = n.h * n.v, hw = n.h * n.w;
  q[0] = -g * Ab * H - half * Ab * n.u * n.u + lam * T(1.0 / 6.0) * Ab * r * r - half * Bb * n.u * n.v -
         half * Cb * n.u * n.w - a.h * n.u;
  q[1] = -half * Ab * hu - half * Bb * hv - half * Cb * hw - a.h * n.h;
  q[2] = half * Bb * hu;
  q[3] = half * Cb * hu;
  q[4] = lam * T(1.0 / 3.0) * Ab * omr - a.eta * n.u;
  q[5] = lam * T(0.5) * Ab * omr - T(1.5) * a.eta * n.u;
  q[6] = g * Ab;
  q[7] = half * Ab * n.h;
  q[8] = half * Ab * n.u;
  q[9] = half * Bb;
  q[10] = -lam * T(1.0 / 6.0) * Ab;
  q[11] = half * Cb;
}

// Same for the 12 y-quantities (h u v w eta b h(h+b) v^2 hv huv eta^2/h hvw).
template <typename T>
__device__ __forceinline__ void dbar_y(const Node<T>& n, const Seed<T>& a, T g, T lam, T (&q)[12]) {
  const T half = T(0.5);
  const T ih = n.ih;
  const T Ab = -a.u * ih, Bb = -a.v * ih, Cb = -a.w * ih;
  const T H = n.h + n.b, r = n.eta * ih, omr = T(1) - r;
  const T hu = n.h * n.u, hv = n.h * n.v, hw = n.h * n.w;
  q[0] = -g * Bb * H - half * Bb * n.v * n.v + lam * T(1.0 / 6.0) * Bb * r * r - half * Ab * n.u * n.v -
         half * Cb * n.v * n.w - a.h * n.v;
  q[1] = half * Ab * hv;
  q[2] = -half * Bb * hv - half * Ab * hu - half * Cb * hw - a.h * n.h;
  q[3] = half * Cb * hv;
  q[4] = lam * T(1.0 / 3.0) * Bb * omr - a.eta * n.v;
  q[5] = lam * T(0.5) * Bb * omr - T(1.5) * a.eta * n.v;
  q[6] = g * Bb;
  q[7] = half * Bb * n.h;
  q[8] = half * Bb * n.v;
  q[9] = half * Ab;
  q[10] = -lam * T(1.0 / 6.0) * Bb;
  q[11] = half * Cb;
}

template <typename T, int TY>
struct VjpSmem {
  T f[12][TY + 2][TILE_X + 2];  // h u v w eta b 1/h | seeds of h u v w eta
};

template <typename T, int TY>
__device__ __forceinline__ void vjp_lds(const VjpSmem<T, TY>& s, int r, int c, Node<T>& n, Seed<T>& a) {
  n.h = s.f[0][r][c];
  n.u = s.f[1][r][c];
  n.v = s.f[2][r][c];
  n.w = s.f[3][r][c];
  n.eta = s.f[4][r][c];
  n.b = s.f[5][r][c];
  n.ih = s.f[6][r][c];
  a.h = s.f[7][r][c];
  a.u = s.f[8][r][c];
  a.v = s.f[9][r][c];
  a.w = s.f[10][r][c];
  a.eta = s.f[11][r][c];
}

// One reverse-mode stage (role ROLE) on a 64 x TY tile per workgroup.
template <typename T, int BCX, int BCY, int ROLE, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void vjp_kernel(const GridConst gc, const T* __restrict__ Y,
                                                            const T* __restrict__ bplane, const T* Kin, T* Qb,
                                                            T* __restrict__ Kout, T* __restrict__ Acc,
                                                            T* __restrict__ Bb, T a_in, T cq, T cy) {
  static_assert(TY % THREAD_ROWS == 0, "tile height must be a multiple of 4");
  constexpr int RPT = TY / THREAD_ROWS;
  constexpr int W = TILE_X + 2;
  constexpr int REGION = (TY + 2) * W;
  __shared__ VjpSmem<T, TY> s;
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
#pragma unroll
    for (int f = 0; f < 5; ++f) s.f[7 + f][rr][cc] = a_in * Kin[f * N + o];
  }
  __syncthreads();

  const T g = T(gc.g), lam = T(gc.lam);
  const int i = i0 + tx;
  const AxisStencil<BCX> ax(i, nx, gc.inv2dx, gc.invdx);
  const AxisTranspose<T, BCX> tx_(i, nx, gc.inv2dx, gc.invdx);
  T satx = T(0);
  if (BCX == BC_REFLECTING) {
    if (i == 0) satx = T(-2.0 * gc.invdx);
    if (i == nx - 1) satx = T(2.0 * gc.invdx);
  }

#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = ty + k * THREAD_ROWS;
    const int j = j0 + lr;
    if (i >= nx || j >= ny) continue;
    const AxisStencil<BCY> ay(j, ny, gc.inv2dy, gc.invdy);
    const AxisTranspose<T, BCY> ty_(j, ny, gc.inv2dy, gc.invdy);
    T saty = T(0);
    if (BCY == BC_REFLECTING) {
      if (j == 0) saty = T(-2.0 * gc.invdy);
      if (j == ny - 1) saty = T(2.0 * gc.invdy);
    }
    const int r = lr + 1, c = tx + 1;
    Node<T> nc, nxm, nxp, nym, nyp;
    Seed<T> ac, axm, axp, aym, ayp;
    vjp_lds(s, r, c, nc, ac);
    vjp_lds(s, r, c - 1, nxm, axm);
    vjp_lds(s, r, c + 1, nxp, axp);
    vjp_lds(s, r - 1, c, nym, aym);
    vjp_lds(s, r + 1, c, nyp, ayp);
    // local part: reverse of this node's own rates (stencil neighbours with closures)
    const Node<T>& sxm = ax.om == 0 ? nc : nxm;
    const Node<T>& sxp = ax.op == 0 ? nc : nxp;
    const Node<T>& sym = ay.om == 0 ? nc : nym;
    const Node<T>& syp = ay.op == 0 ? nc : nyp;
    const T kb[5] = {ac.h, ac.u, ac.v, ac.w, ac.eta};
    Cot<T> out;
    T dX[12], dY[12];
    split_form_reverse<T>(nc, sxm, sxp, sym, syp, T(ax.scale), T(ay.scale), g, lam, satx, saty, kb, out, dX, dY);
    // transpose part: Dbar of the neighbours (and of this node on closure columns)
    T qa[12], qb[12], amt[12];
    dbar_x(nxm, axm, g, lam, qa);
    dbar_x(nxp, axp, g, lam, qb);
#pragma unroll
    for (int m = 0; m < 12; ++m) amt[m] = tx_.wl * qa[m] + tx_.wc * dX[m] + tx_.wr * qb[m];
    out.add(chain_x(nc, amt));
    dbar_y(nym, aym, g, lam, qa);
    dbar_y(nyp, ayp, g, lam, qb);
#pragma unroll
    for (int m = 0; m < 12; ++m) amt[m] = ty_.wl * qa[m] + ty_.wc * dY[m] + ty_.wr * qb[m];
    out.add(chain_y(nc, amt));

    const size_t od = (size_t)j * nx + i;
    const T yb[5] = {out.h, out.u, out.v, out.w, out.eta};
    if (ROLE == VJP_PLAIN) {
#pragma unroll
      for (int f = 0; f < 5; ++f) Kout[f * N + od] = yb[f];
      Bb[od] = out.b;
    } else {
      if (ROLE == VJP_S4) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const T q = Qb[f * N + od];
          Kout[f * N + od] = cq * q + cy * yb[f];
          Acc[f * N + od] = yb[f];
        }
      } else if (ROLE == VJP_S3 || ROLE == VJP_S2) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const T q = Qb[f * N + od];
          Kout[f * N + od] = cq * q + cy * yb[f];
          Acc[f * N + od] = Acc[f * N + od] + yb[f];
        }
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f) Qb[f * N + od] = Qb[f * N + od] + Acc[f * N + od] + yb[f];
      }
      Bb[od] = Bb[od] + out.b;
    }
  }
}

}  // namespace sgn
