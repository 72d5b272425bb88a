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
// The diagonal D[d][d] vanishes except on the first and last row of a
// reflecting axis, so only those nodes evaluate their own Dbar; the reverse of
// a node's own rates (split_form_reverse) therefore stops at its raw values.
#pragma once

#include "sgn_fused.hpp"
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

// Reverse of split_form_rates at one node, through the node's own values: the
// cotangent of the node's raw values (center) from the seed kb of its rates.
// The cotangents of the node's derivative values, dbar_x and dbar_y of the node
// itself (below), reach the node's own values only through the diagonal of
// the operator, i.e. on the reflecting closure rows.
template <typename T>
__device__ __forceinline__ void split_form_reverse(const Node<T>& c, const Node<T>& xm, const Node<T>& xp,
                                                   const Node<T>& ym, const Node<T>& yp, T sx, T sy, T g, T lam,
                                                   T satx, T saty, const T (&kb)[5], Cot<T>& cen) {
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
  const T Ab = -au * ih, Bb = -av * ih, Cb = -aw * ih;
  T ihb = -au * A - av * B + aw * (lam * omr - C);
  T omrb = lam * aw * ih;
  T hb, ub, vb, wb, etab, Hb, hub, hvb, uvb, hwb, uwb, vwb, rb;
  // k_eta = w - (u Dxeta + v Dyeta + 3/2 (u Dxb + v Dyb))
  wb = ae;
  ub = -ae * (Dxeta + T(1.5) * Dxb);
  vb = -ae * (Dyeta + T(1.5) * Dyb);
  // k_h = -(u Dxh + h Dxu + v Dyh + h Dyv) + satx hu + saty hv
  ub += -ah * Dxh;
  hb = -ah * (Dxu + Dyv);
  vb += -ah * Dyh;
  hub = ah * satx;
  hvb = ah * saty;
  // A
  Hb = -g * Ab * Dxh;
  hb += half * Ab * Dxu2;
  ub += -Ab * u * Dxh;
  ub += half * Ab * Dxhu;
  hub += -half * Ab * Dxu;
  uvb = -half * Ab * Dyh;
  hvb += half * Ab * Dyu;
  hub += -half * Ab * Dyv;
  rb = lam3 * Ab * r * Dxh;
  omrb += lam3 * Ab * Dxeta + lam2 * Ab * Dxb;
  // B
  Hb += -g * Bb * Dyh;
  hb += half * Bb * Dyv2;
  vb += -Bb * v * Dyh;
  vb += half * Bb * Dyhv;
  hvb += -half * Bb * Dyv;
  uvb += -half * Bb * Dxh;
  hub += half * Bb * Dxv;
  hvb += -half * Bb * Dxu;
  rb += lam3 * Bb * r * Dyh;
  omrb += lam3 * Bb * Dyeta + lam2 * Bb * Dyb;
  // C
  hub += half * Cb * Dxw;
  uwb = -half * Cb * Dxh;
  hwb = -half * Cb * Dxu;
  hvb += half * Cb * Dyw;
  vwb = -half * Cb * Dyh;
  hwb += -half * Cb * Dyv;
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

template <typename T>
__device__ __forceinline__ Seed<T> opaque_seed(Seed<T> a) {
  asm volatile("" : "+v"(a.h), "+v"(a.u), "+v"(a.v), "+v"(a.w), "+v"(a.eta));
  return a;
}

template <typename T, int TY>
struct VjpSmem {
  T f[12][TY + 2][TILE_X + 2];  // h u v w eta b 1/h | seeds of h u v w eta
};

// With SCALE, the seed planes hold unscaled values and the seeds are formed as
// sc * plane here (the same product the role kernels store when staging).
template <typename T, bool SCALE = false, class Smem>
__device__ __forceinline__ void vjp_lds(const Smem& s, int r, int c, Node<T>& n, Seed<T>& a, T sc = T(1)) {
  n.h = s.f[0][r][c];
  n.u = s.f[1][r][c];
  n.v = s.f[2][r][c];
  n.w = s.f[3][r][c];
  n.eta = s.f[4][r][c];
  n.b = s.f[5][r][c];
  n.ih = s.f[6][r][c];
  a.h = SCALE ? sc * s.f[7][r][c] : s.f[7][r][c];
  a.u = SCALE ? sc * s.f[8][r][c] : s.f[8][r][c];
  a.v = SCALE ? sc * s.f[9][r][c] : s.f[9][r][c];
  a.w = SCALE ? sc * s.f[10][r][c] : s.f[10][r][c];
  a.eta = SCALE ? sc * s.f[11][r][c] : s.f[11][r][c];
}

// Cotangent of the raw values of node (i, j), in the domain: the reverse of
// its own rates plus what its neighbours' derivatives send it (the gathered
// transpose), from a staging s that holds Y, b, 1/h and the seeds (planes
// 0..11) around the node's position (r, c).
template <typename T, int BCX, int BCY, bool SCALE = false, class Smem>
__device__ __forceinline__ Cot<T> vjp_node(const Smem& s, int r, int c, int i, int j, const GridConst& gc,
                                           T sc = T(1)) {
  const int nx = gc.nx, ny = gc.ny;
  const T g = T(gc.g), lam = T(gc.lam);
  const AxisStencil<BCX> ax(i, nx, gc.inv2dx, gc.invdx);
  const AxisTranspose<T, BCX> tx_(i, nx, gc.inv2dx, gc.invdx);
  T satx = T(0);
  if (BCX == BC_REFLECTING) {
    if (i == 0) satx = T(-2.0 * gc.invdx);
    if (i == nx - 1) satx = T(2.0 * gc.invdx);
  }
  const AxisStencil<BCY> ay(j, ny, gc.inv2dy, gc.invdy);
  const AxisTranspose<T, BCY> ty_(j, ny, gc.inv2dy, gc.invdy);
  T saty = T(0);
  if (BCY == BC_REFLECTING) {
    if (j == 0) saty = T(-2.0 * gc.invdy);
    if (j == ny - 1) saty = T(2.0 * gc.invdy);
  }
  Node<T> nc, nxm, nxp, nym, nyp;
  Seed<T> ac, axm, axp, aym, ayp;
  vjp_lds<T, SCALE>(s, r, c, nc, ac, sc);
  vjp_lds<T, SCALE>(s, r, c - 1, nxm, axm, sc);
  vjp_lds<T, SCALE>(s, r, c + 1, nxp, axp, sc);
  vjp_lds<T, SCALE>(s, r - 1, c, nym, aym, sc);
  vjp_lds<T, SCALE>(s, r + 1, c, nyp, ayp, sc);
  // Opaque copies: where one thread evaluates neighbouring nodes, the compiler
  // would otherwise share loads and products between the evaluations and fuse
  // the arithmetic differently; every evaluation rounds as a lone one does.
  nc = opaque_node(nc);
  nxm = opaque_node(nxm);
  nxp = opaque_node(nxp);
  nym = opaque_node(nym);
  nyp = opaque_node(nyp);
  ac = opaque_seed(ac);
  axm = opaque_seed(axm);
  axp = opaque_seed(axp);
  aym = opaque_seed(aym);
  ayp = opaque_seed(ayp);
  // local part: reverse of this node's own rates (stencil neighbours with closures)
  const Node<T>& sxm = ax.om == 0 ? nc : nxm;
  const Node<T>& sxp = ax.op == 0 ? nc : nxp;
  const Node<T>& sym = ay.om == 0 ? nc : nym;
  const Node<T>& syp = ay.op == 0 ? nc : nyp;
  const T kb[5] = {ac.h, ac.u, ac.v, ac.w, ac.eta};
  Cot<T> out;
  split_form_reverse<T>(nc, sxm, sxp, sym, syp, T(ax.scale), T(ay.scale), g, lam, satx, saty, kb, out);
  // transpose part: Dbar of the neighbours, and of this node itself where
  // the operator's diagonal is nonzero (the closure rows of a reflecting axis)
  T qa[12], qb[12], amt[12];
  dbar_x(nxm, axm, g, lam, qa);
  dbar_x(nxp, axp, g, lam, qb);
#pragma unroll
  for (int m = 0; m < 12; ++m) amt[m] = tx_.wl * qa[m] + tx_.wr * qb[m];
  if (BCX == BC_REFLECTING && (i == 0 || i == nx - 1)) {
    dbar_x(nc, ac, g, lam, qa);
#pragma unroll
    for (int m = 0; m < 12; ++m) amt[m] += tx_.wc * qa[m];
  }
  out.add(chain_x(nc, amt));
  dbar_y(nym, aym, g, lam, qa);
  dbar_y(nyp, ayp, g, lam, qb);
#pragma unroll
  for (int m = 0; m < 12; ++m) amt[m] = ty_.wl * qa[m] + ty_.wr * qb[m];
  if (BCY == BC_REFLECTING && (j == 0 || j == ny - 1)) {
    dbar_y(nc, ac, g, lam, qa);
#pragma unroll
    for (int m = 0; m < 12; ++m) amt[m] += ty_.wc * qa[m];
  }
  out.add(chain_y(nc, amt));
  return out;
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

  // Stage Y, b and the scaled seeds with a one-node halo.  Every load of the
  // region is issued before the first LDS write waits for one, so each
  // workgroup keeps the whole region in flight.
  {
    constexpr int ITER = (REGION + STAGE_THREADS - 1) / STAGE_THREADS;
    T v[ITER][11];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * STAGE_THREADS;
      if (idx < REGION) {
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
#pragma unroll
        for (int f = 0; f < 5; ++f) v[it][f] = Y[f * N + o];
        v[it][5] = bplane[o];
#pragma unroll
        for (int f = 0; f < 5; ++f) v[it][6 + f] = Kin[f * N + o];
      }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * STAGE_THREADS;
      if (idx < REGION) {
        const int rr = idx / W;
        const int cc = idx - rr * W;
#pragma unroll
        for (int f = 0; f < 6; ++f) s.f[f][rr][cc] = v[it][f];
        s.f[6][rr][cc] = recip_staged(v[it][0]);
#pragma unroll
        for (int f = 0; f < 5; ++f) s.f[7 + f][rr][cc] = a_in * v[it][6 + f];
      }
    }
  }
  __syncthreads();

  const int i = i0 + tx;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = ty + k * THREAD_ROWS;
    const int j = j0 + lr;
    if (i >= nx || j >= ny) continue;
    // this node's qbar and bbar, loaded before the evaluation so that their
    // latency overlaps it (the sum Acc is read at the end: loaded here too it
    // takes the reflecting instances past 256 registers)
    const size_t od = (size_t)j * nx + i;
    T qv[5], bv = T(0);
    if (ROLE != VJP_PLAIN) {
#pragma unroll
      for (int f = 0; f < 5; ++f) qv[f] = Qb[f * N + od];
      bv = Bb[od];
    }
    const Cot<T> out = vjp_node<T, BCX, BCY>(s, lr + 1, tx + 1, i, j, gc);
    const T yb[5] = {out.h, out.u, out.v, out.w, out.eta};
    if (ROLE == VJP_PLAIN) {
#pragma unroll
      for (int f = 0; f < 5; ++f) Kout[f * N + od] = yb[f];
      Bb[od] = out.b;
    } else {
      if (ROLE == VJP_S4) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          Kout[f * N + od] = cq * qv[f] + cy * yb[f];
          Acc[f * N + od] = yb[f];
        }
      } else if (ROLE == VJP_S3 || ROLE == VJP_S2) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          Kout[f * N + od] = cq * qv[f] + cy * yb[f];
          Acc[f * N + od] = Acc[f * N + od] + yb[f];
        }
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f) Qb[f * N + od] = qv[f] + Acc[f * N + od] + yb[f];
      }
      Bb[od] = bv + out.b;
    }
  }
}

// Two consecutive reverse stages in one launch, the reverse counterpart of the
// step kernel's temporal blocking: PAIR = 2 runs roles S4 and S3, PAIR = 1
// roles S2 and S1, over the step kernel's TX x (512 / TX) tiles.  The first
// evaluation (state YA and seed aA * KinA, staged with a two-node halo) runs
// on the tile and on the ring of nodes around it; there its stage cotangent
// YbarA gives the second evaluation's seed kbB = cqA qbar + cyA YbarA, which
// replaces the first seed in LDS beside the second state YB (one-node halo),
// and the second evaluation runs on the tile:
//   PAIR 2: KinA = qbar, aA = dt/6 (the seed planes hold qbar itself and the
//           seeds aA qbar are formed as they are read, so kbB takes qbar from
//           LDS), YA = Y4, YB = Y3, (cqA, cyA) = (dt/3, dt),
//           Kout = cqB qbar + cyB YbarB with (cqB, cyB) = (dt/3, dt/2),
//           Acc = YbarA + YbarB (YbarA written after the first evaluation)
//   PAIR 1: KinA = the seed of S2, aA = 1, YA = Y2, YB = Y1 = q_n,
//           (cqA, cyA) = (dt/6, dt/2), QbOut = qbar + (Acc + YbarA) + YbarB
//           (a buffer other than Qb: neighbouring tiles still read qbar on
//           their rings while this one writes)
//   both:   bbar = (bbar + bbarA) + bbarB, the first sum written after the
//           first evaluation.
// Node by node this is the arithmetic of the two role kernels (the compiler
// fuses the multiply-adds of the separately built kernels differently, so the
// results agree to rounding), and the results do not depend on the tile
// shape.  Algorithmic traffic per node: 28 values for S4 + S3
// (role kernels: 56) and 33 for S2 + S1 (61), plus the sums written between
// the evaluations and read back (6 values each way, mostly served by L2); the
// price is the ring of first evaluations (1 + 2 (TX + 2 + TY) / 512 of them
// per owned node).
// The reverse kernels use the 512-node step tiles: 32 x 16 or 64 x 8.
template <int TX>
using VjpGeom = StepGeom<TX == 64 ? 8 : 16>;

template <typename T, int TX>
struct VjpPairSmem {
  T f[12][VjpGeom<TX>::TY + 4][TX + 4];  // h u v w eta b 1/h | seeds of h u v w eta
};

template <typename T, int BCX, int BCY, int PAIR, int TX>
__global__ __launch_bounds__(STAGE_THREADS, 2) void vjp_pair_kernel(const GridConst gc, const T* __restrict__ YA,
                                                                 const T* __restrict__ YB,
                                                                 const T* __restrict__ bplane, const T* KinA,
                                                                 const T* Qb, T* __restrict__ QbOut,
                                                                 T* __restrict__ Kout, T* __restrict__ Acc,
                                                                 T* __restrict__ Bb, T aA, T cqA, T cyA, T cqB,
                                                                 T cyB) {
  static_assert(PAIR == 1 || PAIR == 2, "PAIR is 2 (S4 + S3) or 1 (S2 + S1)");
  using G = VjpGeom<TX>;
  static_assert(G::TX == TX, "32 x 16 or 64 x 8 tiles");
  constexpr int TY = G::TY;
  constexpr int H = 2;  // LDS position of tile node (0, 0)
  constexpr int RXA = TX + 2 * H, REGA = RXA * (TY + 2 * H);
  constexpr int RXB = TX + 2, REGB = RXB * (TY + 2);
  __shared__ VjpPairSmem<T, TX> s;
  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const int ntx = (nx + TX - 1) / TX;
  const int nty = (ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  const int i0 = (tile % ntx) * TX;
  const int j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;

  // 1. YA, b and aA * KinA with a two-node halo; all loads issued first
  {
    constexpr int ITER = (REGA + STAGE_THREADS - 1) / STAGE_THREADS;
    T v[ITER][11];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * STAGE_THREADS;
      if (idx < REGA) {
        const int rr = idx / RXA;
        const int cc = idx - rr * RXA;
        const size_t o = (size_t)wrap_or_clamp<BCY>(j0 - H + rr, ny) * nx + wrap_or_clamp<BCX>(i0 - H + cc, nx);
#pragma unroll
        for (int f = 0; f < 5; ++f) v[it][f] = YA[f * N + o];
        v[it][5] = bplane[o];
#pragma unroll
        for (int f = 0; f < 5; ++f) v[it][6 + f] = KinA[f * N + o];
      }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * STAGE_THREADS;
      if (idx < REGA) {
        const int rr = idx / RXA;
        const int cc = idx - rr * RXA;
#pragma unroll
        for (int f = 0; f < 6; ++f) s.f[f][rr][cc] = v[it][f];
        s.f[6][rr][cc] = recip_staged(v[it][0]);
#pragma unroll
        for (int f = 0; f < 5; ++f) s.f[7 + f][rr][cc] = PAIR == 2 ? v[it][6 + f] : aA * v[it][6 + f];
      }
    }
  }

  // Slots of this thread: slot 0 the ring node tid (if any), slots 1 and 2 the
  // tile nodes (lx, ly0) and (lx, ly0 + 1); positions relative to the tile.
  const int lx = tid % TX;
  const int ly0 = 2 * (tid / TX);
  int pr[3], pc[3];
  bool slot[3], ev[3];
  slot[0] = tid < G::RING1;
  pr[0] = 0;
  pc[0] = 0;
  if (slot[0]) ring_node<TY>(tid, pr[0], pc[0]);
  pr[1] = ly0;
  pc[1] = lx;
  pr[2] = ly0 + 1;
  pc[2] = lx;
  slot[1] = slot[2] = true;
#pragma unroll
  for (int q = 0; q < 3; ++q)
    ev[q] = slot[q] && on_axis<BCX>(i0 + pc[q], nx) && on_axis<BCY>(j0 + pr[q], ny);
  __syncthreads();

  // 2. First evaluation on the ring and the tile (periodic images of nodes
  //    past a ragged edge included): the seeds of the second one.
  //    The owned nodes' sums go to memory as the role kernels write them
  //    (Acc, bbar; read back after the second evaluation, from L2).
  T kbB[3][5];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    __builtin_amdgcn_sched_barrier(0);
    if (!ev[q]) continue;
    const int iw = wrap_or_clamp<BCX>(i0 + pc[q], nx), jw = wrap_or_clamp<BCY>(j0 + pr[q], ny);
    const size_t o = (size_t)jw * nx + iw;
    // PAIR 2: the seed planes hold qbar itself (KinA = qbar), scaled by aA as it is read
    const Cot<T> out = vjp_node<T, BCX, BCY, PAIR == 2>(s, pr[q] + H, pc[q] + H, iw, jw, gc, aA);
    const T yb[5] = {out.h, out.u, out.v, out.w, out.eta};
#pragma unroll
    for (int f = 0; f < 5; ++f)
      kbB[q][f] = cqA * (PAIR == 2 ? s.f[7 + f][pr[q] + H][pc[q] + H] : Qb[f * N + o]) + cyA * yb[f];
    if (q > 0 && i0 + pc[q] < nx && j0 + pr[q] < ny) {
      if (PAIR == 2) {
#pragma unroll
        for (int f = 0; f < 5; ++f) Acc[f * N + o] = yb[f];
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f) Acc[f * N + o] = Acc[f * N + o] + yb[f];
      }
      Bb[o] = Bb[o] + out.b;
    }
  }
  // the second state, loaded while the other waves finish their evaluations
  constexpr int ITB = (REGB + STAGE_THREADS - 1) / STAGE_THREADS;
  T w[ITB][5];
#pragma unroll
  for (int it = 0; it < ITB; ++it) {
    const int idx = tid + it * STAGE_THREADS;
    if (idx < REGB) {
      const int rr = idx / RXB;
      const int cc = idx - rr * RXB;
      const size_t o = (size_t)wrap_or_clamp<BCY>(j0 - 1 + rr, ny) * nx + wrap_or_clamp<BCX>(i0 - 1 + cc, nx);
#pragma unroll
      for (int f = 0; f < 5; ++f) w[it][f] = YB[f * N + o];
    }
  }
  __syncthreads();

  // 3. YB and its 1/h over the one-node halo (b stays), the new seeds on the
  //    tile and ring.  Positions outside a reflecting wall then take the seed
  //    of the wall node they copy, as the role kernels stage them.
#pragma unroll
  for (int it = 0; it < ITB; ++it) {
    const int idx = tid + it * STAGE_THREADS;
    if (idx < REGB) {
      const int rr = idx / RXB + H - 1;
      const int cc = idx - (idx / RXB) * RXB + H - 1;
#pragma unroll
      for (int f = 0; f < 5; ++f) s.f[f][rr][cc] = w[it][f];
      s.f[6][rr][cc] = recip_staged(w[it][0]);
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (!ev[q]) continue;
#pragma unroll
    for (int f = 0; f < 5; ++f) s.f[7 + f][pr[q] + H][pc[q] + H] = kbB[q][f];
  }
  if (BCX == BC_REFLECTING || BCY == BC_REFLECTING) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (!slot[q] || ev[q]) continue;
      // the reflecting axis clamps; on a periodic axis the position is its own
      const int ic = BCX == BC_REFLECTING ? wrap_or_clamp<BC_REFLECTING>(i0 + pc[q], nx) - i0 : pc[q];
      const int jc = BCY == BC_REFLECTING ? wrap_or_clamp<BC_REFLECTING>(j0 + pr[q], ny) - j0 : pr[q];
#pragma unroll
      for (int f = 0; f < 5; ++f) s.f[7 + f][pr[q] + H][pc[q] + H] = s.f[7 + f][jc + H][ic + H];
    }
  }
  __syncthreads();

  // 4. Second evaluation on the owned nodes in the domain, and the outputs.
  const int i = i0 + lx;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    __builtin_amdgcn_sched_barrier(0);
    const int j = j0 + ly0 + k;
    if (i >= nx || j >= ny) continue;
    const size_t od = (size_t)j * nx + i;
    T qv[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) qv[f] = Qb[f * N + od];
    const T bv = Bb[od];
    const Cot<T> out = vjp_node<T, BCX, BCY>(s, ly0 + k + H, lx + H, i, j, gc);
    const T yb[5] = {out.h, out.u, out.v, out.w, out.eta};
    if (PAIR == 2) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        Kout[f * N + od] = cqB * qv[f] + cyB * yb[f];
        Acc[f * N + od] = Acc[f * N + od] + yb[f];
      }
    } else {
#pragma unroll
      for (int f = 0; f < 5; ++f) QbOut[f * N + od] = qv[f] + Acc[f * N + od] + yb[f];
    }
    Bb[od] = bv + out.b;
  }
}

}  // namespace sgn
