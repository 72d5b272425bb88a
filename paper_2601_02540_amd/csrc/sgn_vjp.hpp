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
// Layout of the work: a wavefront owns a strip of 64 consecutive columns and
// walks down a block of rows.  Lane L holds column c0 - 2 + L; lanes 1..62
// reverse their node, lanes 2..61 own the 60 output columns.  Row-wise
// contributions cross lanes by shuffles; column-wise ones stay in the lane's
// registers from one row to the next (rows j-1, j, j+1 of raw values are kept
// in a rolling window), so no LDS is needed.
#pragma once

#include "sgn_stage.hpp"

namespace sgn {

constexpr int VJP_STRIP = 60;  // output columns per wavefront
constexpr int VJP_WAVES = 4;   // wavefronts per workgroup (independent strips)

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

template <typename T>
__device__ __forceinline__ T shfl_from_left(T x) {  // value of lane L-1
  return __shfl_up(x, 1, 64);
}
template <typename T>
__device__ __forceinline__ T shfl_from_right(T x) {  // value of lane L+1
  return __shfl_down(x, 1, 64);
}
template <typename T>
__device__ __forceinline__ Node<T> shfl_node_left(const Node<T>& n) {
  Node<T> o;
  o.h = shfl_from_left(n.h);
  o.u = shfl_from_left(n.u);
  o.v = shfl_from_left(n.v);
  o.w = shfl_from_left(n.w);
  o.eta = shfl_from_left(n.eta);
  o.b = shfl_from_left(n.b);
  o.ih = shfl_from_left(n.ih);
  return o;
}
template <typename T>
__device__ __forceinline__ Node<T> shfl_node_right(const Node<T>& n) {
  Node<T> o;
  o.h = shfl_from_right(n.h);
  o.u = shfl_from_right(n.u);
  o.v = shfl_from_right(n.v);
  o.w = shfl_from_right(n.w);
  o.eta = shfl_from_right(n.eta);
  o.b = shfl_from_right(n.b);
  o.ih = shfl_from_right(n.ih);
  return o;
}

template <int BC>
__device__ __forceinline__ int vjp_wrap(int g, int n) {
  if (BC == BC_PERIODIC) {
    if (g < 0) g += n;
    while (g >= n) g -= n;
    return g;
  }
  return g < 0 ? 0 : (g >= n ? n - 1 : g);
}

template <typename T, int BCX, int BCY>
__device__ __forceinline__ Node<T> vjp_load(const T* __restrict__ Y, const T* __restrict__ bplane, size_t N, int nx,
                                            int gi, int gj) {
  const size_t o = (size_t)gj * nx + gi;
  Node<T> n;
  n.h = Y[o];
  n.u = Y[N + o];
  n.v = Y[2 * N + o];
  n.w = Y[3 * N + o];
  n.eta = Y[4 * N + o];
  n.b = bplane[o];
  n.ih = T(1) / n.h;
  return n;
}

// One reverse-mode stage (role ROLE) over the whole grid.  ROWS output rows per
// wavefront work item.
template <typename T, int BCX, int BCY, int ROLE, int ROWS>
__global__ __launch_bounds__(64 * VJP_WAVES) void vjp_kernel(const GridConst gc, const T* __restrict__ Y,
                                                             const T* __restrict__ bplane,
                                                             const T* Kin, T* Qb,
                                                             T* __restrict__ Kout, T* __restrict__ Acc,
                                                             T* __restrict__ Bb, T a_in, T cq, T cy) {
  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const int lane = threadIdx.x & 63;
  const int nsx = (nx + VJP_STRIP - 1) / VJP_STRIP;
  const int nsy = (ny + ROWS - 1) / ROWS;
  const int item = blockIdx.x * VJP_WAVES + (threadIdx.x >> 6);
  if (item >= nsx * nsy) return;  // whole wavefront leaves together
  const int sxi = item % nsx, syi = item / nsx;
  const int c0 = sxi * VJP_STRIP;
  const int jstart = syi * ROWS;
  const int jend = min(jstart + ROWS, ny);

  const int col = c0 - 2 + lane;  // unwrapped column of this lane
  const bool col_in = BCX == BC_PERIODIC || (col >= 0 && col < nx);
  const int gi = vjp_wrap<BCX>(col, nx);
  const bool reverse_lane = lane >= 1 && lane <= 62 && col_in;
  const bool out_lane = lane >= 2 && lane <= 61 && col >= c0 && col < c0 + VJP_STRIP && col < nx;
  // x stencil of this lane's node
  int omx = -1, opx = 1;
  T sx = T(gc.inv2dx), satx = T(0);
  if (BCX == BC_REFLECTING) {
    if (col == 0) {
      omx = 0;
      sx = T(gc.invdx);
      satx = T(-2.0 * gc.invdx);
    }
    if (col == nx - 1) {
      opx = 0;
      sx = T(gc.invdx);
      satx = T(2.0 * gc.invdx);
    }
  }
  const T g = T(gc.g), lam = T(gc.lam);

  // rolling window of raw rows j-1, j, j+1 (and j+2 in flight) and partial
  // cotangents of rows j-1, j; the rate cotangents of row j+1 are also fetched
  // one row ahead, so every load has a row of work to hide behind.
  Node<T> Rm = vjp_load<T, BCX, BCY>(Y, bplane, N, nx, gi, vjp_wrap<BCY>(jstart - 2, ny));
  Node<T> R0 = vjp_load<T, BCX, BCY>(Y, bplane, N, nx, gi, vjp_wrap<BCY>(jstart - 1, ny));
  Node<T> Rn = vjp_load<T, BCX, BCY>(Y, bplane, N, nx, gi, vjp_wrap<BCY>(jstart, ny));
  T kbn[5];
  {
    const int j = jstart - 1;
    const bool row_in = BCY == BC_PERIODIC || (j >= 0 && j < ny);
    const size_t o = (size_t)vjp_wrap<BCY>(j, ny) * nx + gi;
#pragma unroll
    for (int f = 0; f < 5; ++f) kbn[f] = (reverse_lane && row_in) ? a_in * Kin[f * N + o] : T(0);
  }
  Cot<T> Pm, P0;
  Pm.zero();
  P0.zero();

  for (int j = jstart - 1; j <= jend; ++j) {
    const Node<T> Rp = Rn;
    T kb[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) kb[f] = kbn[f];
    if (j + 1 <= jend) {
      Rn = vjp_load<T, BCX, BCY>(Y, bplane, N, nx, gi, vjp_wrap<BCY>(j + 2, ny));
      const bool nrow_in = BCY == BC_PERIODIC || (j + 1 >= 0 && j + 1 < ny);
      const size_t o = (size_t)vjp_wrap<BCY>(j + 1, ny) * nx + gi;
#pragma unroll
      for (int f = 0; f < 5; ++f) kbn[f] = (reverse_lane && nrow_in) ? a_in * Kin[f * N + o] : T(0);
    }
    const bool row_in = BCY == BC_PERIODIC || (j >= 0 && j < ny);
    // x neighbours of this row (all lanes take part in the shuffles)
    const Node<T> XM = shfl_node_left(R0);
    const Node<T> XP = shfl_node_right(R0);
    Cot<T> cen, sendL, sendR, toUp, toDown;
    cen.zero();
    sendL.zero();
    sendR.zero();
    toUp.zero();
    toDown.zero();
    if (reverse_lane && row_in) {
      int omy = -1, opy = 1;
      T sy = T(gc.inv2dy), saty = T(0);
      if (BCY == BC_REFLECTING) {
        if (j == 0) {
          omy = 0;
          sy = T(gc.invdy);
          saty = T(-2.0 * gc.invdy);
        }
        if (j == ny - 1) {
          opy = 0;
          sy = T(gc.invdy);
          saty = T(2.0 * gc.invdy);
        }
      }
      const Node<T>& xm = omx == 0 ? R0 : XM;
      const Node<T>& xp = opx == 0 ? R0 : XP;
      const Node<T>& ym = omy == 0 ? R0 : Rm;
      const Node<T>& yp = opy == 0 ? R0 : Rp;
      T dX[12], dY[12];
      split_form_reverse<T>(R0, xm, xp, ym, yp, sx, sy, g, lam, satx, saty, kb, cen, dX, dY);
      T ax[12], ay[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        ax[k] = sx * dX[k];
        ay[k] = sy * dY[k];
      }
      const Cot<T> cxp = chain_x(xp, ax);  // +s Dbar to the right target
      const Cot<T> cyp = chain_y(yp, ay);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        ax[k] = -ax[k];
        ay[k] = -ay[k];
      }
      const Cot<T> cxm = chain_x(xm, ax);  // -s Dbar to the left target
      const Cot<T> cym = chain_y(ym, ay);
      if (opx == 0) cen.add(cxp); else sendR = cxp;
      if (omx == 0) cen.add(cxm); else sendL = cxm;
      if (opy == 0) cen.add(cyp); else toDown = cyp;
      if (omy == 0) cen.add(cym); else toUp = cym;
    }
    // what the neighbours in this row send to this lane
    Cot<T> recv;
    recv.h = shfl_from_left(sendR.h) + shfl_from_right(sendL.h);
    recv.u = shfl_from_left(sendR.u) + shfl_from_right(sendL.u);
    recv.v = shfl_from_left(sendR.v) + shfl_from_right(sendL.v);
    recv.w = shfl_from_left(sendR.w) + shfl_from_right(sendL.w);
    recv.eta = shfl_from_left(sendR.eta) + shfl_from_right(sendL.eta);
    recv.b = shfl_from_left(sendR.b) + shfl_from_right(sendL.b);
    P0.add(cen);
    P0.add(recv);
    Pm.add(toUp);
    // row j-1 is complete
    const int jd = j - 1;
    if (out_lane && jd >= jstart && jd < jend) {
      const size_t od = (size_t)jd * nx + col;
      const T yb[5] = {Pm.h, Pm.u, Pm.v, Pm.w, Pm.eta};
      if (ROLE == VJP_PLAIN) {
#pragma unroll
        for (int f = 0; f < 5; ++f) Kout[f * N + od] = yb[f];
        Bb[od] = Pm.b;
      } else {
        if (ROLE == VJP_S4) {
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            const T qb = Qb[f * N + od];
            Kout[f * N + od] = cq * qb + cy * yb[f];
            Acc[f * N + od] = yb[f];
          }
        } else if (ROLE == VJP_S3 || ROLE == VJP_S2) {
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            const T qb = Qb[f * N + od];
            Kout[f * N + od] = cq * qb + cy * yb[f];
            Acc[f * N + od] = Acc[f * N + od] + yb[f];
          }
        } else {
#pragma unroll
          for (int f = 0; f < 5; ++f) Qb[f * N + od] = Qb[f * N + od] + Acc[f * N + od] + yb[f];
        }
        Bb[od] = Bb[od] + Pm.b;
      }
    }
    Pm = P0;
    P0 = toDown;
    Rm = R0;
    R0 = Rp;
  }
}

}  // namespace sgn
