// sgn_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow CPU evaluation of the energy-conserving split-form SBP
// semi-discretization of the two-dimensional hyperbolized Serre-Green-Naghdi
// equations with variable bathymetry (arXiv 2601.02540, Section 4).  It exists
// so that the tests, the smoke check and the benchmark's CPU-baseline leg can
// check the HIP path against something written independently from the paper.
// The product path never links, loads or calls this file.  It shares no code,
// header, constant or table with paper_2601_02540_amd/csrc.
//
// Conventions (all from the paper unless marked "reading"):
//  * state q = five planes [h, u, v, w, eta], each ny*nx row-major, x fastest;
//    bathymetry b is one more plane.  Node (i, j) is x_i, y_j.
//  * 1D operators of Remark "Concrete SBP operators and SATs" (Section 4.2):
//      periodic:   D = circ(-1, 0, 1)/(2 dx), M = dx I,
//      reflecting: interior central, first/last rows (-2, 2)/(2 dx),
//                  M = dx diag(1/2, 1, ..., 1, 1/2), BN = e_R e_R^T - e_L e_L^T.
//    Reading of the node placement: periodic dx = L/N with the right end point
//    excluded (so that M = dx I integrates the period exactly); reflecting
//    dx = L/(N-1) with both end points on the grid.
//  * 2D operators are tensor products (Section 2.2): D_x acts along i, D_y
//    along j, M_ij = wx_i * wy_j, and M^{-1} R^T B N_x R = (Mx^{-1} BN_x) (x) I.
//  * Rates: periodic semi-discretization eq. (sd_periodic_2D_SGN, Section 4.1);
//    reflecting one eq. (semi_2D, Section 4.2), whose only change is the SAT
//    pair in the h equation.  The u, v, w rows are printed multiplied by h;
//    the oracle divides by h.
//  * Energy E and its gradient d_q E: Theorem 1 proof (Section 4.1).
//  * Auxiliary initialization eq. (initialization), Section 6.
//  * Time integration: classical four-stage RK4 with a fixed step (the paper
//    itself uses an adaptive five-stage FSAL method; see the design notes).
//
// Arithmetic is evaluated in the order the equations are printed; build with
// -O2 -ffp-contract=off so that no fused multiply-add reorders it.
// The OpenMP pragmas only matter for the threaded timing build (-fopenmp):
// they split loops whose iterations write disjoint outputs, so every value is
// formed by the same operations in the same order as in the serial build (a
// test checks that both builds agree bit for bit); the reductions stay serial.
// Every function is templated on the scalar so that the same source evaluates
// in double (reference), float (to bound single-precision runs) and
// std::complex<double> (complex-step directional derivatives for the adjoint
// and manufactured-solution pins).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t nx, ny;
  double xmin, xmax, ymin, ymax;
  int32_t bc_x, bc_y;  // 0 = periodic, 1 = reflecting
  double g, lambda;
} orc_grid;

}  // extern "C"

namespace {

using cplx = std::complex<double>;

// ---------------------------------------------------------------------------
// One-dimensional SBP operator (Remark "Concrete SBP operators and SATs").
// D is stored as an explicit list of matrix entries (row, col, value) taken
// straight from the printed matrices; M and BN are diagonals.
struct Op1D {
  int n = 0;
  int bc = 0;
  double delta = 0;
  std::vector<int> row, col;
  std::vector<double> val;
  std::vector<double> w;   // diagonal of the mass matrix M
  std::vector<double> bn;  // diagonal of B N = e_R e_R^T - e_L e_L^T (zero if periodic)

  void add(int r, int c, double v) {
    row.push_back(r);
    col.push_back(c);
    val.push_back(v);
  }
};

Op1D make_op(int n, int bc, double lo, double hi) {
  Op1D op;
  op.n = n;
  op.bc = bc;
  op.w.assign(n, 0.0);
  op.bn.assign(n, 0.0);
  if (bc == 0) {
    op.delta = (hi - lo) / n;
    const double c = 1.0 / (2.0 * op.delta);
    for (int i = 0; i < n; ++i) {
      op.add(i, (i - 1 + n) % n, -c);
      op.add(i, (i + 1) % n, c);
      op.w[i] = op.delta;
    }
  } else {
    op.delta = (hi - lo) / (n - 1);
    const double c = 1.0 / (2.0 * op.delta);
    op.add(0, 0, -2.0 * c);
    op.add(0, 1, 2.0 * c);
    for (int i = 1; i < n - 1; ++i) {
      op.add(i, i - 1, -c);
      op.add(i, i + 1, c);
    }
    op.add(n - 1, n - 2, -2.0 * c);
    op.add(n - 1, n - 1, 2.0 * c);
    for (int i = 0; i < n; ++i) op.w[i] = op.delta;
    op.w[0] = 0.5 * op.delta;
    op.w[n - 1] = 0.5 * op.delta;
    op.bn[0] = -1.0;
    op.bn[n - 1] = 1.0;
  }
  return op;
}

struct Ops {
  Op1D x, y;
  int nx, ny;
  size_t N;
};

Ops make_ops(const orc_grid& g) {
  Ops o;
  o.x = make_op(g.nx, g.bc_x, g.xmin, g.xmax);
  o.y = make_op(g.ny, g.bc_y, g.ymin, g.ymax);
  o.nx = g.nx;
  o.ny = g.ny;
  o.N = (size_t)g.nx * (size_t)g.ny;
  return o;
}

// out = D_x f : D acting on the x index of every row j.
template <class T>
void apply_dx(const Ops& o, const T* f, T* out) {
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < o.N; ++k) out[k] = T(0);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < o.ny; ++j)
    for (size_t e = 0; e < o.x.val.size(); ++e)
      out[(size_t)j * o.nx + o.x.row[e]] += T(o.x.val[e]) * f[(size_t)j * o.nx + o.x.col[e]];
}

// out = D_y f : D acting on the y index of every column i.
template <class T>
void apply_dy(const Ops& o, const T* f, T* out) {
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < o.N; ++k) out[k] = T(0);
  // (threaded build: a static schedule gives every thread the same columns i
  // for every entry e, so each output still sums its entries in order e)
#pragma omp parallel
  for (size_t e = 0; e < o.y.val.size(); ++e)
#pragma omp for schedule(static) nowait
    for (int i = 0; i < o.nx; ++i)
      out[(size_t)o.y.row[e] * o.nx + i] += T(o.y.val[e]) * f[(size_t)o.y.col[e] * o.nx + i];
}

// out += D_x^T f  (transpose: every entry scatters from its row to its column).
template <class T>
void add_dxT(const Ops& o, const T* f, T* out) {
  for (int j = 0; j < o.ny; ++j)
    for (size_t e = 0; e < o.x.val.size(); ++e)
      out[(size_t)j * o.nx + o.x.col[e]] += T(o.x.val[e]) * f[(size_t)j * o.nx + o.x.row[e]];
}

template <class T>
void add_dyT(const Ops& o, const T* f, T* out) {
  for (size_t e = 0; e < o.y.val.size(); ++e)
    for (int i = 0; i < o.nx; ++i)
      out[(size_t)o.y.col[e] * o.nx + i] += T(o.y.val[e]) * f[(size_t)o.y.row[e] * o.nx + i];
}

// Neumaier-compensated sum, row-major order.
struct Neumaier {
  double s = 0, c = 0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// ---------------------------------------------------------------------------
// Manufactured solution (Section 6.1.2) and its source terms.
//
// The fields are the printed b, h, u, v, eta = h, w = -h (u_x + v_y) +
// 3/2 (u b_x + v b_y).  The sources are the residuals of the continuous system
// eq. (2D_hyperbolic_SGN) as printed (conservative form), with every partial
// derivative taken by the complex step, and then converted to the primitive
// unknowns evolved by the semi-discretization:
//   S_h = R_h,  S_u = (R_hu - u R_h)/h,  S_v = (R_hv - v R_h)/h,
//   S_w = (R_hw - w R_h)/h,  S_eta = (R_heta - eta R_h)/h,
// which follows from (h q)_t = h q_t + q h_t.  The first derivatives u_x, v_y,
// b_x, b_y inside w are written out from the printed formulas.
template <class T>
struct MmsFields {
  T b, h, u, v, eta, w;
};

template <class T>
MmsFields<T> mms_fields(T x, T y, T t) {
  const double pi = M_PI;
  const double k = 2.0 * pi;
  MmsFields<T> f;
  f.b = 0.08 * (std::cos(k * x) * std::cos(k * y) + 0.5 * std::cos(2.0 * k * x) * std::cos(2.0 * k * y));
  f.h = 2.0 + 0.5 * std::sin(k * x) * std::sin(k * y) * std::cos(k * t) - f.b;
  f.u = 0.3 * std::sin(k * x) * std::sin(k * t);
  f.v = 0.3 * std::sin(k * y) * std::sin(k * t);
  f.eta = f.h;
  T ux = 0.3 * k * std::cos(k * x) * std::sin(k * t);
  T vy = 0.3 * k * std::cos(k * y) * std::sin(k * t);
  T bx = 0.08 * (-k * std::sin(k * x) * std::cos(k * y) - 0.5 * 2.0 * k * std::sin(2.0 * k * x) * std::cos(2.0 * k * y));
  T by = 0.08 * (-k * std::cos(k * x) * std::sin(k * y) - 0.5 * 2.0 * k * std::cos(2.0 * k * x) * std::sin(2.0 * k * y));
  f.w = -f.h * (ux + vy) + 1.5 * (f.u * bx + f.v * by);
  return f;
}

const double CS_EPS = 1e-30;

// Conserved quantities and fluxes of eq. (2D_hyperbolic_SGN) built from the
// fields, with p(h, eta) = lambda/3 (eta/h) (1 - eta/h).
template <class T>
struct MmsFluxes {
  T h, hu, hv, heta, hw;      // conserved variables
  T fxx, fyy, huv;            // momentum fluxes: h u^2 + g h^2/2 + h p, h v^2 + g h^2/2 + h p, h u v
  T hetau, hetav, hwu, hwv;   // fluxes of h eta and h w
  T b;
};

template <class T>
MmsFluxes<T> mms_fluxes(const MmsFields<T>& f, double g, double lam) {
  MmsFluxes<T> F;
  const T p = lam / 3.0 * (f.eta / f.h) * (1.0 - f.eta / f.h);
  F.h = f.h;
  F.hu = f.h * f.u;
  F.hv = f.h * f.v;
  F.heta = f.h * f.eta;
  F.hw = f.h * f.w;
  F.fxx = f.h * f.u * f.u + 0.5 * g * f.h * f.h + f.h * p;
  F.fyy = f.h * f.v * f.v + 0.5 * g * f.h * f.h + f.h * p;
  F.huv = f.h * f.u * f.v;
  F.hetau = f.h * f.eta * f.u;
  F.hetav = f.h * f.eta * f.v;
  F.hwu = f.h * f.w * f.u;
  F.hwv = f.h * f.w * f.v;
  F.b = f.b;
  return F;
}

// Returns the five primitive sources [S_h, S_u, S_v, S_w, S_eta] at (x, y, t).
// Each partial derivative of a flux is the imaginary part of that flux built
// from fields evaluated at a complex-perturbed x, y or t, divided by the step.
void mms_source_point(double g, double lam, double x, double y, double t, double S[5]) {
  const MmsFluxes<cplx> Fx = mms_fluxes(mms_fields(cplx(x, CS_EPS), cplx(y, 0), cplx(t, 0)), g, lam);
  const MmsFluxes<cplx> Fy = mms_fluxes(mms_fields(cplx(x, 0), cplx(y, CS_EPS), cplx(t, 0)), g, lam);
  const MmsFluxes<cplx> Ft = mms_fluxes(mms_fields(cplx(x, 0), cplx(y, 0), cplx(t, CS_EPS)), g, lam);
  auto dx = [&](cplx MmsFluxes<cplx>::*m) { return std::imag(Fx.*m) / CS_EPS; };
  auto dy = [&](cplx MmsFluxes<cplx>::*m) { return std::imag(Fy.*m) / CS_EPS; };
  auto dt = [&](cplx MmsFluxes<cplx>::*m) { return std::imag(Ft.*m) / CS_EPS; };
  using F = MmsFluxes<cplx>;

  const MmsFields<double> f = mms_fields<double>(x, y, t);
  const double bx = dx(&F::b);
  const double by = dy(&F::b);
  const double p = lam / 3.0 * (f.eta / f.h) * (1.0 - f.eta / f.h);

  const double Rh = dt(&F::h) + dx(&F::hu) + dy(&F::hv);
  const double Rhu = dt(&F::hu) + dx(&F::fxx) + dy(&F::huv) + (g * f.h + 1.5 * (f.h / f.eta) * p) * bx;
  const double Rhv = dt(&F::hv) + dx(&F::huv) + dy(&F::fyy) + (g * f.h + 1.5 * (f.h / f.eta) * p) * by;
  const double Rheta = dt(&F::heta) + dx(&F::hetau) + dy(&F::hetav) + 1.5 * f.h * (f.u * bx + f.v * by) - f.h * f.w;
  const double Rhw = dt(&F::hw) + dx(&F::hwu) + dy(&F::hwv) - lam * (1.0 - f.eta / f.h);

  S[0] = Rh;
  S[1] = (Rhu - f.u * Rh) / f.h;
  S[2] = (Rhv - f.v * Rh) / f.h;
  S[3] = (Rhw - f.w * Rh) / f.h;
  S[4] = (Rheta - f.eta * Rh) / f.h;
}

double node_x(const Ops& o, const orc_grid& g, int i) { return g.xmin + i * o.x.delta; }
double node_y(const Ops& o, const orc_grid& g, int j) { return g.ymin + j * o.y.delta; }

// ---------------------------------------------------------------------------
// Right-hand side of the semi-discretization.
template <class T>
void rhs_impl(const orc_grid& gr, const Ops& o, const T* q, const T* b, double t, int src, T* dq) {
  const size_t N = o.N;
  const T* h = q;
  const T* u = q + N;
  const T* v = q + 2 * N;
  const T* w = q + 3 * N;
  const T* eta = q + 4 * N;
  const T g = T(gr.g);
  const T lam = T(gr.lambda);
  const T half = T(0.5);

  // Pointwise (componentwise) products.
  std::vector<T> H(N), hH(N), u2(N), v2(N), hu(N), hv(N), huv(N), uv(N), e2h(N), huw(N), hvw(N), uw(N), vw(N), hw(N);
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < N; ++k) {
    H[k] = h[k] + b[k];
    hH[k] = h[k] * H[k];
    u2[k] = u[k] * u[k];
    v2[k] = v[k] * v[k];
    hu[k] = h[k] * u[k];
    hv[k] = h[k] * v[k];
    huv[k] = h[k] * u[k] * v[k];
    uv[k] = u[k] * v[k];
    e2h[k] = eta[k] * eta[k] / h[k];
    huw[k] = h[k] * u[k] * w[k];
    hvw[k] = h[k] * v[k] * w[k];
    uw[k] = u[k] * w[k];
    vw[k] = v[k] * w[k];
    hw[k] = h[k] * w[k];
  }

  // First derivatives.
  std::vector<T> Dxh(N), Dxu(N), Dxv(N), Dxw(N), Dxeta(N), Dxb(N), DxhH(N), Dxu2(N), Dxhu(N), Dxhuv(N), Dxe2h(N), Dxhuw(N);
  std::vector<T> Dyh(N), Dyu(N), Dyv(N), Dyw(N), Dyeta(N), Dyb(N), DyhH(N), Dyv2(N), Dyhv(N), Dyhuv(N), Dye2h(N), Dyhvw(N);
  apply_dx(o, h, Dxh.data());
  apply_dx(o, u, Dxu.data());
  apply_dx(o, v, Dxv.data());
  apply_dx(o, w, Dxw.data());
  apply_dx(o, eta, Dxeta.data());
  apply_dx(o, b, Dxb.data());
  apply_dx(o, hH.data(), DxhH.data());
  apply_dx(o, u2.data(), Dxu2.data());
  apply_dx(o, hu.data(), Dxhu.data());
  apply_dx(o, huv.data(), Dxhuv.data());
  apply_dx(o, e2h.data(), Dxe2h.data());
  apply_dx(o, huw.data(), Dxhuw.data());
  apply_dy(o, h, Dyh.data());
  apply_dy(o, u, Dyu.data());
  apply_dy(o, v, Dyv.data());
  apply_dy(o, w, Dyw.data());
  apply_dy(o, eta, Dyeta.data());
  apply_dy(o, b, Dyb.data());
  apply_dy(o, hH.data(), DyhH.data());
  apply_dy(o, v2.data(), Dyv2.data());
  apply_dy(o, hv.data(), Dyhv.data());
  apply_dy(o, huv.data(), Dyhuv.data());
  apply_dy(o, e2h.data(), Dye2h.data());
  apply_dy(o, hvw.data(), Dyhvw.data());

#pragma omp parallel for schedule(static)
  for (int j = 0; j < o.ny; ++j) {
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      // SATs, eq. (semi_2D): M^{-1} R^T B N_x R (h u) and the same in y.
      T satx = T(0), saty = T(0);
      if (gr.bc_x == 1) satx = T(o.x.bn[i] / o.x.w[i]) * hu[k];
      if (gr.bc_y == 1) saty = T(o.y.bn[j] / o.y.w[j]) * hv[k];

      // h equation
      const T ht = -(u[k] * Dxh[k] + h[k] * Dxu[k] + v[k] * Dyh[k] + h[k] * Dyv[k]) + satx + saty;

      // h u_t + A = 0
      const T r = eta[k] / h[k];
      const T r2 = (eta[k] * eta[k]) / (h[k] * h[k]);
      const T A = g * DxhH[k] - g * H[k] * Dxh[k] + half * h[k] * Dxu2[k] - half * u2[k] * Dxh[k] +
                  half * u[k] * Dxhu[k] - half * hu[k] * Dxu[k] + half * Dyhuv[k] - half * uv[k] * Dyh[k] +
                  half * hv[k] * Dyu[k] - half * hu[k] * Dyv[k] + lam / T(6) * r2 * Dxh[k] + lam / T(3) * Dxeta[k] -
                  lam / T(3) * r * Dxeta[k] - lam / T(6) * Dxe2h[k] + lam / T(2) * (T(1) - r) * Dxb[k];
      // h v_t + B = 0
      const T B = g * DyhH[k] - g * H[k] * Dyh[k] + half * h[k] * Dyv2[k] - half * v2[k] * Dyh[k] +
                  half * v[k] * Dyhv[k] - half * hv[k] * Dyv[k] + half * Dxhuv[k] - half * uv[k] * Dxh[k] +
                  half * hu[k] * Dxv[k] - half * hv[k] * Dxu[k] + lam / T(6) * r2 * Dyh[k] + lam / T(3) * Dyeta[k] -
                  lam / T(3) * r * Dyeta[k] - lam / T(6) * Dye2h[k] + lam / T(2) * (T(1) - r) * Dyb[k];
      // h w_t + C = lambda (1 - eta/h)
      const T C = half * Dxhuw[k] + half * hu[k] * Dxw[k] - half * uw[k] * Dxh[k] - half * hw[k] * Dxu[k] +
                  half * Dyhvw[k] + half * hv[k] * Dyw[k] - half * vw[k] * Dyh[k] - half * hw[k] * Dyv[k];
      // eta_t + (...) = w
      const T et = w[k] - (u[k] * Dxeta[k] + v[k] * Dyeta[k] + T(1.5) * u[k] * Dxb[k] + T(1.5) * v[k] * Dyb[k]);

      dq[k] = ht;
      dq[N + k] = -A / h[k];
      dq[2 * N + k] = -B / h[k];
      dq[3 * N + k] = (lam * (T(1) - r) - C) / h[k];
      dq[4 * N + k] = et;
    }
  }

  if (src == 1) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < o.ny; ++j)
      for (int i = 0; i < o.nx; ++i) {
        double S[5];
        mms_source_point(gr.g, gr.lambda, node_x(o, gr, i), node_y(o, gr, j), t, S);
        const size_t k = (size_t)j * o.nx + i;
        for (int f = 0; f < 5; ++f) dq[f * N + k] += T(S[f]);
      }
  }
}

// Classical RK4 with a fixed step, one step.
template <class T>
void rk4_step_impl(const orc_grid& gr, const Ops& o, T* q, const T* b, double dt, double t, int src) {
  const size_t M = 5 * o.N;
  std::vector<T> k1(M), k2(M), k3(M), k4(M), Y(M);
  const T Tdt = T(dt);
  rhs_impl(gr, o, q, b, t, src, k1.data());
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < M; ++k) Y[k] = q[k] + Tdt / T(2) * k1[k];
  rhs_impl(gr, o, Y.data(), b, t + dt / 2, src, k2.data());
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < M; ++k) Y[k] = q[k] + Tdt / T(2) * k2[k];
  rhs_impl(gr, o, Y.data(), b, t + dt / 2, src, k3.data());
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < M; ++k) Y[k] = q[k] + Tdt * k3[k];
  rhs_impl(gr, o, Y.data(), b, t + dt, src, k4.data());
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < M; ++k) q[k] = q[k] + Tdt * (k1[k] + T(2) * k2[k] + T(2) * k3[k] + k4[k]) / T(6);
}

// ---------------------------------------------------------------------------
// Adaptive Runge-Kutta pair of the kind the paper integrates with (Section
// "Numerical Experiments": explicit, third order, five stages, first same as
// last, an embedded error estimator driving the step size, relative and
// absolute tolerances 1e-6).  The paper names the method by citation only, so
// the coefficients are this project's reading, a pair of that shape:
//   * main method, order 3, five stages, stages chained through the
//     subdiagonal only: Y_{i+1} = y_n + h c_{i+1} k_i, with
//     c = (0, 1/3, 3/4, 4/5, 3071/3720) and the weights b below, which make
//     the stability polynomial 1 + z + z^2/2 + z^3/6 + z^4/31 + z^5/163 (stable
//     on the imaginary axis up to |y| ~ 3.9, where the conservative
//     semi-discretization's spectrum lies);
//   * embedded method, order 2, on the five stages and the first-same-as-last
//     stage k6 = f(y_{n+1}) (abscissa 1, row b): weights bh below;
//   * error estimate y_{n+1} - yh_{n+1} = h sum_i (b_i - bh_i) k_i, measured in
//     the root-mean-square norm over all 5N values, each scaled by
//     atol + rtol max(|y_n|, |y_{n+1}|);
//   * PI step-size control (Hairer-Wanner, Solving ODEs II, Section IV.2):
//     accepted when err <= 1, next step h 0.9 err^(-0.7/3) errp^(0.4/3)
//     limited to [0.2, 5] h (to [0.2, 1] h right after a rejection), errp the
//     last accepted err (at least 1e-4, 1 at the start); rejected steps are
//     retried with h max(0.2, 0.9 err^(-1/3)); the last step is cut (or
//     stretched by at most a relative 1e-10) to end at t_end exactly.
struct Fsal35 {
  double c[6];
  double a[6][6];
  double b[6];   // main weights (b[5] = 0: the last stage only serves the estimate)
  double bh[6];  // embedded weights
};

Fsal35 fsal35_tableau() {
  Fsal35 t{};
  const double c[6] = {0.0, 1.0 / 3.0, 3.0 / 4.0, 4.0 / 5.0, 3071.0 / 3720.0, 1.0};
  const double b[6] = {7200668.0 / 46553289.0, 1701.0 / 5053.0, 6098.0 / 15159.0, 350.0 / 5053.0,
                       18600.0 / 500573.0, 0.0};
  const double bh[6] = {7502453.0 / 46553289.0, 1701.0 / 5053.0, 6098.0 / 15159.0, 350.0 / 5053.0, 0.0,
                        15355.0 / 500573.0};
  for (int i = 0; i < 6; ++i) {
    t.c[i] = c[i];
    t.b[i] = b[i];
    t.bh[i] = bh[i];
  }
  for (int i = 1; i < 5; ++i) t.a[i][i - 1] = c[i];  // Y_{i+1} = y_n + h c_{i+1} k_i
  for (int j = 0; j < 5; ++j) t.a[5][j] = b[j];      // the FSAL stage is f(y_{n+1})
  return t;
}

// Runs the pair from t0 to t_end (or for max_attempts attempts).  adaptive = 0:
// fixed steps h = dt0 (the last one cut to reach t_end), every step accepted
// (the estimate is still formed and recorded).  rec (may be NULL) receives
// (h, err, accepted) per attempt.  Returns the number of attempts.
int64_t fsal35_run(const orc_grid& gr, const Ops& o, double* y, const double* b, double t0, double t_end,
                   double dt0, double rtol, double atol, int adaptive, int64_t max_attempts, double* rec,
                   double* t_out, int64_t* n_acc, int64_t* n_rej) {
  const Fsal35 tb = fsal35_tableau();
  const size_t M = 5 * o.N;
  std::vector<std::vector<double>> k(6, std::vector<double>(M));
  std::vector<double> Y(M), ynew(M);
  rhs_impl(gr, o, y, b, t0, 0, k[0].data());
  double t = t0, dt = dt0, errp = 1.0;
  bool after_reject = false;
  int64_t att = 0, acc = 0, rej = 0;
  const double safety = 0.9, facmin = 0.2, facmax = 5.0, kexp = 3.0;
  while (t < t_end && att < max_attempts) {
    // the last step ends exactly at t_end (also when rounding left it a hair longer than dt)
    const double h = (t_end - t <= dt * (1.0 + 1e-10)) ? t_end - t : dt;
    for (int i = 1; i < 5; ++i) {
      for (size_t m = 0; m < M; ++m) {
        double sum = 0.0;
        for (int j = 0; j < i; ++j) sum += tb.a[i][j] * k[j][m];
        Y[m] = y[m] + h * sum;
      }
      rhs_impl(gr, o, Y.data(), b, t + tb.c[i] * h, 0, k[i].data());
    }
    for (size_t m = 0; m < M; ++m) {
      double sum = 0.0;
      for (int j = 0; j < 5; ++j) sum += tb.b[j] * k[j][m];
      ynew[m] = y[m] + h * sum;
    }
    rhs_impl(gr, o, ynew.data(), b, t + h, 0, k[5].data());
    Neumaier sq;
    for (size_t m = 0; m < M; ++m) {
      double e = 0.0;
      for (int j = 0; j < 6; ++j) e += (tb.b[j] - tb.bh[j]) * k[j][m];
      e *= h;
      const double scale = atol + rtol * std::max(std::fabs(y[m]), std::fabs(ynew[m]));
      sq.add((e / scale) * (e / scale));
    }
    const double err = std::sqrt(sq.value() / (double)M);
    const bool ok = !adaptive || err <= 1.0;
    if (rec) {
      rec[3 * att + 0] = h;
      rec[3 * att + 1] = err;
      rec[3 * att + 2] = ok ? 1.0 : 0.0;
    }
    ++att;
    if (ok) {
      std::memcpy(y, ynew.data(), M * sizeof(double));
      std::swap(k[0], k[5]);  // first same as last
      t = (h == t_end - t) ? t_end : t + h;
      ++acc;
      if (adaptive) {
        double fac = safety * std::pow(err, -0.7 / kexp) * std::pow(errp, 0.4 / kexp);
        fac = std::min(fac, after_reject ? 1.0 : facmax);
        fac = std::max(fac, facmin);
        dt = h * fac;
        errp = std::max(err, 1e-4);
      }
      after_reject = false;
    } else {
      ++rej;
      dt = h * std::max(facmin, safety * std::pow(err, -1.0 / kexp));
      after_reject = true;
    }
  }
  *t_out = t;
  *n_acc = acc;
  *n_rej = rej;
  return att;
}

// Energy density E = h ((u^2+v^2)/2 + e), e = w^2/6 + g/2 (h + 2b) + lambda/6 (eta/h - 1)^2.
double energy_density(double g, double lam, double h, double u, double v, double w, double eta, double b) {
  const double e = w * w / 6.0 + g / 2.0 * (h + 2.0 * b) + lam / 6.0 * (eta / h - 1.0) * (eta / h - 1.0);
  return h * ((u * u + v * v) / 2.0 + e);
}

// E(q + gam d) - E(q), the change of the total energy along an update
// direction d, accumulated in extended precision (long double) so that the
// difference of two totals that agree in their leading digits keeps its own.
long double energy_change(const orc_grid& gr, const Ops& o, const double* q, const double* d, const double* b,
                          long double gam) {
  const size_t N = o.N;
  const long double g = gr.g, lam = gr.lambda;
  long double sum = 0.0L, comp = 0.0L;  // Neumaier
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      long double x0[5], x1[5];
      for (int f = 0; f < 5; ++f) {
        x0[f] = q[f * N + k];
        x1[f] = x0[f] + gam * (long double)d[f * N + k];
      }
      const long double bk = b[k];
      long double e[2];
      const long double* xs[2] = {x0, x1};
      for (int m = 0; m < 2; ++m) {
        const long double h = xs[m][0], u = xs[m][1], v = xs[m][2], w = xs[m][3], eta = xs[m][4];
        const long double r = eta / h - 1.0L;
        e[m] = h * ((u * u + v * v) / 2.0L + w * w / 6.0L + g / 2.0L * (h + 2.0L * bk) + lam / 6.0L * r * r);
      }
      const long double x = (long double)o.x.w[i] * (long double)o.y.w[j] * (e[1] - e[0]);
      const long double t = sum + x;
      comp += std::fabs(sum) >= std::fabs(x) ? (sum - t) + x : (x - t) + sum;
      sum = t;
    }
  return sum + comp;
}

template <class T>
void init_aux_impl(const Ops& o, T* q, const T* b) {
  const size_t N = o.N;
  T* h = q;
  T* u = q + N;
  T* v = q + 2 * N;
  T* w = q + 3 * N;
  T* eta = q + 4 * N;
  std::vector<T> Dxu(N), Dyv(N), Dxb(N), Dyb(N);
  apply_dx(o, u, Dxu.data());
  apply_dy(o, v, Dyv.data());
  apply_dx(o, b, Dxb.data());
  apply_dy(o, b, Dyb.data());
  for (size_t k = 0; k < N; ++k) {
    eta[k] = h[k];
    w[k] = -h[k] * (Dxu[k] + Dyv[k]) + T(1.5) * (u[k] * Dxb[k] + v[k] * Dyb[k]);
  }
}

// ---------------------------------------------------------------------------
// Discrete adjoint (discretize, then differentiate): (q_bar, b_bar) += J^T a
// for the Jacobian J of the right-hand side with respect to (q, b).  Written
// term by term against rhs_impl: a term  c * X * D(Y)  of a rate with
// cotangent abar contributes  X_bar += c abar D(Y)  and  Y_bar += D^T(c abar X),
// and every pointwise product is then chained back to h, u, v, w, eta, b.
void rhs_vjp_impl(const orc_grid& gr, const Ops& o, const double* q, const double* b, const double* a,
                  double* qbar, double* bbar) {
  const size_t N = o.N;
  const double* h = q;
  const double* u = q + N;
  const double* v = q + 2 * N;
  const double* w = q + 3 * N;
  const double* eta = q + 4 * N;
  const double g = gr.g, lam = gr.lambda;
  using vec = std::vector<double>;

  // forward intermediates (as in rhs_impl)
  vec H(N), hH(N), u2(N), v2(N), hu(N), hv(N), huv(N), uv(N), e2h(N), huw(N), hvw(N), uw(N), vw(N), hw(N), r(N), r2(N);
  for (size_t k = 0; k < N; ++k) {
    H[k] = h[k] + b[k];
    hH[k] = h[k] * H[k];
    u2[k] = u[k] * u[k];
    v2[k] = v[k] * v[k];
    hu[k] = h[k] * u[k];
    hv[k] = h[k] * v[k];
    huv[k] = h[k] * u[k] * v[k];
    uv[k] = u[k] * v[k];
    e2h[k] = eta[k] * eta[k] / h[k];
    huw[k] = h[k] * u[k] * w[k];
    hvw[k] = h[k] * v[k] * w[k];
    uw[k] = u[k] * w[k];
    vw[k] = v[k] * w[k];
    hw[k] = h[k] * w[k];
    r[k] = eta[k] / h[k];
    r2[k] = (eta[k] * eta[k]) / (h[k] * h[k]);
  }
  auto Dx = [&](const double* f) { vec out(N); apply_dx(o, f, out.data()); return out; };
  auto Dy = [&](const double* f) { vec out(N); apply_dy(o, f, out.data()); return out; };
  const vec Dxh = Dx(h), Dxu = Dx(u), Dxv = Dx(v), Dxw = Dx(w), Dxeta = Dx(eta), Dxb = Dx(b);
  const vec Dyh = Dy(h), Dyu = Dy(u), Dyv = Dy(v), Dyw = Dy(w), Dyeta = Dy(eta), Dyb = Dy(b);
  const vec DxhH = Dx(hH.data()), Dxu2 = Dx(u2.data()), Dxhu = Dx(hu.data()), Dxhuv = Dx(huv.data()),
            Dxe2h = Dx(e2h.data()), Dxhuw = Dx(huw.data());
  const vec DyhH = Dy(hH.data()), Dyv2 = Dy(v2.data()), Dyhv = Dy(hv.data()), Dyhuv = Dy(huv.data()),
            Dye2h = Dy(e2h.data()), Dyhvw = Dy(hvw.data());

  // the bracketed sums A (h u_t + A = 0), B (h v_t + B = 0), C (h w_t + C = lam (1 - r))
  vec A(N), B(N), C(N);
  for (size_t k = 0; k < N; ++k) {
    A[k] = g * DxhH[k] - g * H[k] * Dxh[k] + 0.5 * h[k] * Dxu2[k] - 0.5 * u2[k] * Dxh[k] + 0.5 * u[k] * Dxhu[k] -
           0.5 * hu[k] * Dxu[k] + 0.5 * Dyhuv[k] - 0.5 * uv[k] * Dyh[k] + 0.5 * hv[k] * Dyu[k] -
           0.5 * hu[k] * Dyv[k] + lam / 6 * r2[k] * Dxh[k] + lam / 3 * Dxeta[k] - lam / 3 * r[k] * Dxeta[k] -
           lam / 6 * Dxe2h[k] + lam / 2 * (1 - r[k]) * Dxb[k];
    B[k] = g * DyhH[k] - g * H[k] * Dyh[k] + 0.5 * h[k] * Dyv2[k] - 0.5 * v2[k] * Dyh[k] + 0.5 * v[k] * Dyhv[k] -
           0.5 * hv[k] * Dyv[k] + 0.5 * Dxhuv[k] - 0.5 * uv[k] * Dxh[k] + 0.5 * hu[k] * Dxv[k] -
           0.5 * hv[k] * Dxu[k] + lam / 6 * r2[k] * Dyh[k] + lam / 3 * Dyeta[k] - lam / 3 * r[k] * Dyeta[k] -
           lam / 6 * Dye2h[k] + lam / 2 * (1 - r[k]) * Dyb[k];
    C[k] = 0.5 * Dxhuw[k] + 0.5 * hu[k] * Dxw[k] - 0.5 * uw[k] * Dxh[k] - 0.5 * hw[k] * Dxu[k] +
           0.5 * Dyhvw[k] + 0.5 * hv[k] * Dyw[k] - 0.5 * vw[k] * Dyh[k] - 0.5 * hw[k] * Dyv[k];
  }

  // cotangents of the rates
  const double* ah = a;
  const double* au = a + N;
  const double* av = a + 2 * N;
  const double* aw = a + 3 * N;
  const double* aeta = a + 4 * N;
  vec hb(N, 0), ub(N, 0), vb(N, 0), wb(N, 0), etab(N, 0), bb(N, 0);
  vec Hb(N, 0), hHb(N, 0), u2b(N, 0), v2b(N, 0), hub(N, 0), hvb(N, 0), huvb(N, 0), uvb(N, 0), e2hb(N, 0),
      huwb(N, 0), hvwb(N, 0), uwb(N, 0), vwb(N, 0), hwb(N, 0), rb(N, 0), r2b(N, 0);
  // seeds of A, B, C: u_t = -A/h, v_t = -B/h, w_t = (lam (1 - r) - C)/h
  vec Ab(N), Bb(N), Cb(N);
  for (size_t k = 0; k < N; ++k) {
    Ab[k] = -au[k] / h[k];
    Bb[k] = -av[k] / h[k];
    Cb[k] = -aw[k] / h[k];
    hb[k] += au[k] * A[k] / (h[k] * h[k]) + av[k] * B[k] / (h[k] * h[k]) -
             aw[k] * (lam * (1 - r[k]) - C[k]) / (h[k] * h[k]);
    rb[k] += -lam * aw[k] / h[k];
  }
  // term c * X * D(Y): X_bar += c abar DY ; Y_bar += D^T(c abar X)   (X == nullptr means 1)
  vec tmp(N);
  auto term = [&](double c, const vec& abar, const vec* X, vec* Xb, const vec& DY, vec& Yb, bool xdir) {
    for (size_t k = 0; k < N; ++k) {
      if (Xb) (*Xb)[k] += c * abar[k] * DY[k];
      tmp[k] = c * abar[k] * (X ? (*X)[k] : 1.0);
    }
    if (xdir)
      add_dxT(o, tmp.data(), Yb.data());
    else
      add_dyT(o, tmp.data(), Yb.data());
  };
  const vec hv_(h, h + N), uv_(u, u + N), vv_(v, v + N), wv_(w, w + N), etav_(eta, eta + N);
  vec omr(N), ones(N, 1.0);
  for (size_t k = 0; k < N; ++k) omr[k] = 1 - r[k];
  vec omrb(N, 0);

  // A
  term(g, Ab, nullptr, nullptr, DxhH, hHb, true);
  term(-g, Ab, &H, &Hb, Dxh, hb, true);
  term(0.5, Ab, &hv_, &hb, Dxu2, u2b, true);
  term(-0.5, Ab, &u2, &u2b, Dxh, hb, true);
  term(0.5, Ab, &uv_, &ub, Dxhu, hub, true);
  term(-0.5, Ab, &hu, &hub, Dxu, ub, true);
  term(0.5, Ab, nullptr, nullptr, Dyhuv, huvb, false);
  term(-0.5, Ab, &uv, &uvb, Dyh, hb, false);
  term(0.5, Ab, &hv, &hvb, Dyu, ub, false);
  term(-0.5, Ab, &hu, &hub, Dyv, vb, false);
  term(lam / 6, Ab, &r2, &r2b, Dxh, hb, true);
  term(lam / 3, Ab, nullptr, nullptr, Dxeta, etab, true);
  term(-lam / 3, Ab, &r, &rb, Dxeta, etab, true);
  term(-lam / 6, Ab, nullptr, nullptr, Dxe2h, e2hb, true);
  term(lam / 2, Ab, &omr, &omrb, Dxb, bb, true);
  // B
  term(g, Bb, nullptr, nullptr, DyhH, hHb, false);
  term(-g, Bb, &H, &Hb, Dyh, hb, false);
  term(0.5, Bb, &hv_, &hb, Dyv2, v2b, false);
  term(-0.5, Bb, &v2, &v2b, Dyh, hb, false);
  term(0.5, Bb, &vv_, &vb, Dyhv, hvb, false);
  term(-0.5, Bb, &hv, &hvb, Dyv, vb, false);
  term(0.5, Bb, nullptr, nullptr, Dxhuv, huvb, true);
  term(-0.5, Bb, &uv, &uvb, Dxh, hb, true);
  term(0.5, Bb, &hu, &hub, Dxv, vb, true);
  term(-0.5, Bb, &hv, &hvb, Dxu, ub, true);
  term(lam / 6, Bb, &r2, &r2b, Dyh, hb, false);
  term(lam / 3, Bb, nullptr, nullptr, Dyeta, etab, false);
  term(-lam / 3, Bb, &r, &rb, Dyeta, etab, false);
  term(-lam / 6, Bb, nullptr, nullptr, Dye2h, e2hb, false);
  term(lam / 2, Bb, &omr, &omrb, Dyb, bb, false);
  // C
  term(0.5, Cb, nullptr, nullptr, Dxhuw, huwb, true);
  term(0.5, Cb, &hu, &hub, Dxw, wb, true);
  term(-0.5, Cb, &uw, &uwb, Dxh, hb, true);
  term(-0.5, Cb, &hw, &hwb, Dxu, ub, true);
  term(0.5, Cb, nullptr, nullptr, Dyhvw, hvwb, false);
  term(0.5, Cb, &hv, &hvb, Dyw, wb, false);
  term(-0.5, Cb, &vw, &vwb, Dyh, hb, false);
  term(-0.5, Cb, &hw, &hwb, Dyv, vb, false);
  // h_t = -(u Dxh + h Dxu + v Dyh + h Dyv) + SATs
  vec ahv(ah, ah + N);
  term(-1.0, ahv, &uv_, &ub, Dxh, hb, true);
  term(-1.0, ahv, &hv_, &hb, Dxu, ub, true);
  term(-1.0, ahv, &vv_, &vb, Dyh, hb, false);
  term(-1.0, ahv, &hv_, &hb, Dyv, vb, false);
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      if (gr.bc_x == 1) hub[k] += o.x.bn[i] / o.x.w[i] * ah[k];
      if (gr.bc_y == 1) hvb[k] += o.y.bn[j] / o.y.w[j] * ah[k];
    }
  // eta_t = w - (u Dxeta + v Dyeta + 1.5 u Dxb + 1.5 v Dyb)
  vec aev(aeta, aeta + N);
  for (size_t k = 0; k < N; ++k) wb[k] += aeta[k];
  term(-1.0, aev, &uv_, &ub, Dxeta, etab, true);
  term(-1.0, aev, &vv_, &vb, Dyeta, etab, false);
  term(-1.5, aev, &uv_, &ub, Dxb, bb, true);
  term(-1.5, aev, &vv_, &vb, Dyb, bb, false);

  // chain the pointwise products back to h, u, v, w, eta, b
  for (size_t k = 0; k < N; ++k) {
    rb[k] -= omrb[k];
    hb[k] += H[k] * hHb[k];
    Hb[k] += h[k] * hHb[k];
    hb[k] += Hb[k];
    bb[k] += Hb[k];
    ub[k] += 2 * u[k] * u2b[k];
    vb[k] += 2 * v[k] * v2b[k];
    hb[k] += u[k] * hub[k];
    ub[k] += h[k] * hub[k];
    hb[k] += v[k] * hvb[k];
    vb[k] += h[k] * hvb[k];
    hb[k] += u[k] * v[k] * huvb[k];
    ub[k] += h[k] * v[k] * huvb[k];
    vb[k] += h[k] * u[k] * huvb[k];
    ub[k] += v[k] * uvb[k];
    vb[k] += u[k] * uvb[k];
    etab[k] += 2 * eta[k] / h[k] * e2hb[k];
    hb[k] += -eta[k] * eta[k] / (h[k] * h[k]) * e2hb[k];
    hb[k] += u[k] * w[k] * huwb[k];
    ub[k] += h[k] * w[k] * huwb[k];
    wb[k] += h[k] * u[k] * huwb[k];
    hb[k] += v[k] * w[k] * hvwb[k];
    vb[k] += h[k] * w[k] * hvwb[k];
    wb[k] += h[k] * v[k] * hvwb[k];
    ub[k] += w[k] * uwb[k];
    wb[k] += u[k] * uwb[k];
    vb[k] += w[k] * vwb[k];
    wb[k] += v[k] * vwb[k];
    hb[k] += w[k] * hwb[k];
    wb[k] += h[k] * hwb[k];
    etab[k] += rb[k] / h[k];
    hb[k] += -eta[k] / (h[k] * h[k]) * rb[k];
    etab[k] += 2 * eta[k] / (h[k] * h[k]) * r2b[k];
    hb[k] += -2 * eta[k] * eta[k] / (h[k] * h[k] * h[k]) * r2b[k];
  }
  for (size_t k = 0; k < N; ++k) {
    qbar[k] += hb[k];
    qbar[N + k] += ub[k];
    qbar[2 * N + k] += vb[k];
    qbar[3 * N + k] += wb[k];
    qbar[4 * N + k] += etab[k];
    if (bbar) bbar[k] += bb[k];
  }
}

// Reverse of one classical RK4 step from q_n: on entry qbar is the cotangent of
// q_{n+1}, on exit that of q_n; bbar accumulates the bathymetry cotangent.
//   kb4 = dt/6 qb;            Yb4 = J(Y4)^T kb4
//   kb3 = dt/3 qb + dt Yb4;   Yb3 = J(Y3)^T kb3
//   kb2 = dt/3 qb + dt/2 Yb3; Yb2 = J(Y2)^T kb2
//   kb1 = dt/6 qb + dt/2 Yb2; Yb1 = J(Y1)^T kb1
//   qb_n = qb + Yb1 + Yb2 + Yb3 + Yb4
void rk4_vjp_impl(const orc_grid& gr, const Ops& o, const double* q, const double* b, double dt, double* qbar,
                  double* bbar) {
  const size_t M = 5 * o.N;
  std::vector<double> k1(M), k2(M), k3(M), Y2(M), Y3(M), Y4(M);
  rhs_impl<double>(gr, o, q, b, 0.0, 0, k1.data());
  for (size_t k = 0; k < M; ++k) Y2[k] = q[k] + dt / 2 * k1[k];
  rhs_impl<double>(gr, o, Y2.data(), b, 0.0, 0, k2.data());
  for (size_t k = 0; k < M; ++k) Y3[k] = q[k] + dt / 2 * k2[k];
  rhs_impl<double>(gr, o, Y3.data(), b, 0.0, 0, k3.data());
  for (size_t k = 0; k < M; ++k) Y4[k] = q[k] + dt * k3[k];
  std::vector<double> kb(M), Yb4(M, 0), Yb3(M, 0), Yb2(M, 0), Yb1(M, 0);
  for (size_t k = 0; k < M; ++k) kb[k] = dt / 6 * qbar[k];
  rhs_vjp_impl(gr, o, Y4.data(), b, kb.data(), Yb4.data(), bbar);
  for (size_t k = 0; k < M; ++k) kb[k] = dt / 3 * qbar[k] + dt * Yb4[k];
  rhs_vjp_impl(gr, o, Y3.data(), b, kb.data(), Yb3.data(), bbar);
  for (size_t k = 0; k < M; ++k) kb[k] = dt / 3 * qbar[k] + dt / 2 * Yb3[k];
  rhs_vjp_impl(gr, o, Y2.data(), b, kb.data(), Yb2.data(), bbar);
  for (size_t k = 0; k < M; ++k) kb[k] = dt / 6 * qbar[k] + dt / 2 * Yb2[k];
  rhs_vjp_impl(gr, o, q, b, kb.data(), Yb1.data(), bbar);
  for (size_t k = 0; k < M; ++k) qbar[k] = qbar[k] + Yb1[k] + Yb2[k] + Yb3[k] + Yb4[k];
}

// Gauge-misfit loss of a rollout:  L = 1/2 sum_{n=1..nsteps} sum_g (zeta_g^n - target_{n-1,g})^2,
// zeta = h + b at gauge nodes, from h0 = zeta0 - b, u0 = v0 = 0 and the
// auxiliary initialization.  Templated for the complex-step pin.
template <class T>
T gauge_loss_impl(const orc_grid& gr, const Ops& o, const T* zeta0, const T* b, double dt, int64_t nsteps,
                  const int64_t* gidx, int ng, const double* target) {
  const size_t N = o.N;
  std::vector<T> q(5 * N, T(0));
  for (size_t k = 0; k < N; ++k) q[k] = zeta0[k] - b[k];
  init_aux_impl<T>(o, q.data(), b);
  T L = T(0);
  for (int64_t n = 1; n <= nsteps; ++n) {
    rk4_step_impl<T>(gr, o, q.data(), b, dt, 0.0, 0);
    for (int gi = 0; gi < ng; ++gi) {
      const T m = q[gidx[gi]] + b[gidx[gi]] - T(target[(n - 1) * ng + gi]);
      L += T(0.5) * m * m;
    }
  }
  return L;
}

}  // namespace

// ===========================================================================
// C entry points used by the Python test harness (ctypes).  All pointers are
// host pointers; q is 5*nx*ny values, b is nx*ny values.
extern "C" {

// Grid spacing along each axis (reading of the node placement above).
void orc_spacing(const orc_grid* g, double* dx, double* dy) {
  Ops o = make_ops(*g);
  *dx = o.x.delta;
  *dy = o.y.delta;
}

// The 1D operator as a dense n x n matrix (row-major), its mass diagonal and
// the diagonal of B N.
void orc_op1d_dense(int n, int bc, double lo, double hi, double* D, double* w, double* bn) {
  Op1D op = make_op(n, bc, lo, hi);
  for (int k = 0; k < n * n; ++k) D[k] = 0.0;
  for (size_t e = 0; e < op.val.size(); ++e) D[(size_t)op.row[e] * n + op.col[e]] += op.val[e];
  for (int i = 0; i < n; ++i) {
    w[i] = op.w[i];
    bn[i] = op.bn[i];
  }
}

void orc_apply_dx(const orc_grid* g, const double* f, double* out) {
  Ops o = make_ops(*g);
  apply_dx(o, f, out);
}
void orc_apply_dy(const orc_grid* g, const double* f, double* out) {
  Ops o = make_ops(*g);
  apply_dy(o, f, out);
}

void orc_rhs(const orc_grid* g, const double* q, const double* b, double t, int src, double* dq) {
  Ops o = make_ops(*g);
  rhs_impl<double>(*g, o, q, b, t, src, dq);
}

void orc_rhs_f32(const orc_grid* g, const float* q, const float* b, double t, int src, float* dq) {
  Ops o = make_ops(*g);
  rhs_impl<float>(*g, o, q, b, t, src, dq);
}

// Directional derivative of the right-hand side by the complex step:
// out = d/de rhs(q + e dq_dir, b + e db_dir) at e = 0, exact to rounding.
void orc_rhs_jvp(const orc_grid* g, const double* q, const double* b, const double* dq_dir, const double* db_dir,
                 double* out) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  std::vector<cplx> qc(5 * N), bc(N), dqc(5 * N);
  for (size_t k = 0; k < 5 * N; ++k) qc[k] = cplx(q[k], CS_EPS * dq_dir[k]);
  for (size_t k = 0; k < N; ++k) bc[k] = cplx(b[k], db_dir ? CS_EPS * db_dir[k] : 0.0);
  rhs_impl<cplx>(*g, o, qc.data(), bc.data(), 0.0, 0, dqc.data());
  for (size_t k = 0; k < 5 * N; ++k) out[k] = std::imag(dqc[k]) / CS_EPS;
}

void orc_rk4(const orc_grid* g, double* q, const double* b, double dt, double t0, int64_t nsteps, int src) {
  Ops o = make_ops(*g);
  for (int64_t s = 0; s < nsteps; ++s) rk4_step_impl<double>(*g, o, q, b, dt, t0 + s * dt, src);
}

void orc_rk4_f32(const orc_grid* g, float* q, const float* b, double dt, double t0, int64_t nsteps, int src) {
  Ops o = make_ops(*g);
  for (int64_t s = 0; s < nsteps; ++s) rk4_step_impl<float>(*g, o, q, b, dt, t0 + s * dt, src);
}

// Relaxation RK4 in the incremental direction form (the fully discrete energy
// conservation the paper names as an extension): each step computes the
// classical RK4 update d = q_RK4 - q_n, then q_{n+1} = q_n + gam_n d and
// t_{n+1} = t_n + gam_n dt, with gam_n the root in [1/2, 3/2] of
// E(q_n + gam d) = E(q_n) (the other root is gam = 0), found by bisection on the
// extended-precision energy change.  Without a sign change (d = 0) gam_n = 1.
// gammas[n] receives gam_n; *t_end the final time.
void orc_rk4_relax(const orc_grid* g, double* q, const double* b, double dt, double t0, int64_t nsteps,
                   double* t_end, double* gammas) {
  Ops o = make_ops(*g);
  const size_t M = 5 * o.N;
  std::vector<double> qrk(M), d(M);
  double t = t0;
  for (int64_t s = 0; s < nsteps; ++s) {
    std::memcpy(qrk.data(), q, M * sizeof(double));
    rk4_step_impl<double>(*g, o, qrk.data(), b, dt, t, 0);
    for (size_t k = 0; k < M; ++k) d[k] = qrk[k] - q[k];
    long double lo = 0.5L, hi = 1.5L;
    long double rlo = energy_change(*g, o, q, d.data(), b, lo);
    const long double rhi = energy_change(*g, o, q, d.data(), b, hi);
    double gam = 1.0;
    if ((rlo < 0.0L && rhi > 0.0L) || (rlo > 0.0L && rhi < 0.0L)) {
      for (int it = 0; it < 80; ++it) {
        const long double mid = 0.5L * (lo + hi);
        if (mid == lo || mid == hi) break;
        const long double rm = energy_change(*g, o, q, d.data(), b, mid);
        if (rm == 0.0L) {
          lo = hi = mid;
          break;
        }
        if ((rm < 0.0L) == (rlo < 0.0L)) {
          lo = mid;
          rlo = rm;
        } else {
          hi = mid;
        }
      }
      gam = (double)(0.5L * (lo + hi));
    }
    for (size_t k = 0; k < M; ++k) q[k] = q[k] + gam * d[k];
    t = t + gam * dt;
    if (gammas) gammas[s] = gam;
  }
  *t_end = t;
}

void orc_init_aux(const orc_grid* g, double* q, const double* b) {
  Ops o = make_ops(*g);
  init_aux_impl<double>(o, q, b);
}

// Total mass 1^T M h and total energy 1^T M E (Theorems 1 and 2).
void orc_mass_energy(const orc_grid* g, const double* q, const double* b, double* mass, double* energy) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  Neumaier sm, se;
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      const double Mk = o.x.w[i] * o.y.w[j];
      sm.add(Mk * q[k]);
      se.add(Mk * energy_density(g->g, g->lambda, q[k], q[N + k], q[2 * N + k], q[3 * N + k], q[4 * N + k], b[k]));
    }
  *mass = sm.value();
  *energy = se.value();
}

// Same totals for a single-precision state, accumulated in double.
void orc_mass_energy_f32(const orc_grid* g, const float* q, const float* b, double* mass, double* energy) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  Neumaier sm, se;
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      const double Mk = o.x.w[i] * o.y.w[j];
      sm.add(Mk * (double)q[k]);
      se.add(Mk * energy_density(g->g, g->lambda, q[k], q[N + k], q[2 * N + k], q[3 * N + k], q[4 * N + k], b[k]));
    }
  *mass = sm.value();
  *energy = se.value();
}

// Semi-discrete rates: mass_rate = 1^T M h_t, energy_rate = <d_q E, q_t>_M with
// d_h E = u^2/2 + v^2/2 + w^2/6 + g h + g b + lambda/6 (1 - eta^2/h^2),
// d_u E = h u, d_v E = h v, d_w E = h w / 3, d_eta E = -lambda/3 (1 - eta/h).
// scale[0] = sum M |h_t|, scale[1] = sum M (|d_h E h_t| + ... + |d_eta E eta_t|).
void orc_rates(const orc_grid* g, const double* q, const double* b, double* mass_rate, double* energy_rate,
               double* scale) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  std::vector<double> dq(5 * N);
  rhs_impl<double>(*g, o, q, b, 0.0, 0, dq.data());
  Neumaier sm, se, am, ae;
  const double G = g->g, lam = g->lambda;
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      const double Mk = o.x.w[i] * o.y.w[j];
      const double h = q[k], u = q[N + k], v = q[2 * N + k], w = q[3 * N + k], eta = q[4 * N + k];
      const double dEh = 0.5 * u * u + 0.5 * v * v + w * w / 6.0 + G * h + G * b[k] +
                         lam / 6.0 * (1.0 - (eta * eta) / (h * h));
      const double dEu = h * u, dEv = h * v, dEw = h * w / 3.0, dEeta = -lam / 3.0 * (1.0 - eta / h);
      const double t1 = dEh * dq[k], t2 = dEu * dq[N + k], t3 = dEv * dq[2 * N + k], t4 = dEw * dq[3 * N + k],
                   t5 = dEeta * dq[4 * N + k];
      sm.add(Mk * dq[k]);
      se.add(Mk * t1);
      se.add(Mk * t2);
      se.add(Mk * t3);
      se.add(Mk * t4);
      se.add(Mk * t5);
      am.add(Mk * std::fabs(dq[k]));
      ae.add(Mk * (std::fabs(t1) + std::fabs(t2) + std::fabs(t3) + std::fabs(t4) + std::fabs(t5)));
    }
  *mass_rate = sm.value();
  *energy_rate = se.value();
  scale[0] = am.value();
  scale[1] = ae.value();
}

// Time step from the characteristic speeds of the hyperbolic system (reading:
// c^2 = g h + lambda eta^2 / (3 h^2) from the x-flux Jacobian in primitive
// variables), dt = cfl / max_ij [(|u|+c)/dx + (|v|+c)/dy].
double orc_cfl_dt(const orc_grid* g, const double* q, double cfl) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  double m = 0.0;
  for (size_t k = 0; k < N; ++k) {
    const double h = q[k], u = q[N + k], v = q[2 * N + k], eta = q[4 * N + k];
    const double c = std::sqrt(g->g * h + g->lambda * eta * eta / (3.0 * h * h));
    const double s = (std::fabs(u) + c) / o.x.delta + (std::fabs(v) + c) / o.y.delta;
    if (s > m) m = s;
  }
  return cfl / m;
}

// Manufactured solution sampled on the grid at time t: q (5 planes) and b.
void orc_mms_fields(const orc_grid* g, double t, double* q, double* b) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      const size_t k = (size_t)j * o.nx + i;
      MmsFields<double> f = mms_fields<double>(node_x(o, *g, i), node_y(o, *g, j), t);
      q[k] = f.h;
      q[N + k] = f.u;
      q[2 * N + k] = f.v;
      q[3 * N + k] = f.w;
      q[4 * N + k] = f.eta;
      b[k] = f.b;
    }
}

void orc_mms_source(const orc_grid* g, double t, double* S) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  for (int j = 0; j < o.ny; ++j)
    for (int i = 0; i < o.nx; ++i) {
      double s[5];
      mms_source_point(g->g, g->lambda, node_x(o, *g, i), node_y(o, *g, j), t, s);
      for (int f = 0; f < 5; ++f) S[f * N + (size_t)j * o.nx + i] = s[f];
    }
}

void orc_rhs_vjp(const orc_grid* g, const double* q, const double* b, const double* a, double* qbar, double* bbar) {
  Ops o = make_ops(*g);
  rhs_vjp_impl(*g, o, q, b, a, qbar, bbar);
}

void orc_rk4_vjp(const orc_grid* g, const double* q, const double* b, double dt, double* qbar, double* bbar) {
  Ops o = make_ops(*g);
  rk4_vjp_impl(*g, o, q, b, dt, qbar, bbar);
}

// Directional derivative of one RK4 step along (dq, db) by the complex step.
void orc_rk4_jvp(const orc_grid* g, const double* q, const double* b, double dt, const double* dq, const double* db,
                 double* out) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  std::vector<cplx> qc(5 * N), bc(N);
  for (size_t k = 0; k < 5 * N; ++k) qc[k] = cplx(q[k], CS_EPS * dq[k]);
  for (size_t k = 0; k < N; ++k) bc[k] = cplx(b[k], db ? CS_EPS * db[k] : 0.0);
  rk4_step_impl<cplx>(*g, o, qc.data(), bc.data(), dt, 0.0, 0);
  for (size_t k = 0; k < 5 * N; ++k) out[k] = std::imag(qc[k]) / CS_EPS;
}

// Gauge-misfit loss and its directional derivative along (dzeta0, db) by the
// complex step (the whole rollout in complex arithmetic).
void orc_gauge_loss(const orc_grid* g, const double* zeta0, const double* b, double dt, int64_t nsteps,
                    const int64_t* gidx, int ng, const double* target, const double* dzeta0, const double* db,
                    double* loss, double* dloss) {
  Ops o = make_ops(*g);
  const size_t N = o.N;
  std::vector<cplx> zc(N), bc(N);
  for (size_t k = 0; k < N; ++k) {
    zc[k] = cplx(zeta0[k], dzeta0 ? CS_EPS * dzeta0[k] : 0.0);
    bc[k] = cplx(b[k], db ? CS_EPS * db[k] : 0.0);
  }
  const cplx L = gauge_loss_impl<cplx>(*g, o, zc.data(), bc.data(), dt, nsteps, gidx, ng, target);
  *loss = std::real(L);
  if (dloss) *dloss = std::imag(L) / CS_EPS;
}

// Gradient of the gauge-misfit loss by the discrete adjoint: every state of the
// rollout is kept, then the steps are reversed with orc_rk4_vjp-equivalent
// sweeps, and the initialization h0 = zeta0 - b, eta0 = h0, w0(h0, u0 = 0,
// v0 = 0, b) is reversed last.
void orc_gauge_loss_grad(const orc_grid* g, const double* zeta0, const double* b, double dt, int64_t nsteps,
                         const int64_t* gidx, int ng, const double* target, double* loss, double* grad_zeta0,
                         double* grad_b) {
  Ops o = make_ops(*g);
  const size_t N = o.N, M = 5 * N;
  std::vector<std::vector<double>> states;
  std::vector<double> q(M, 0.0);
  for (size_t k = 0; k < N; ++k) q[k] = zeta0[k] - b[k];
  init_aux_impl<double>(o, q.data(), b);
  double L = 0.0;
  std::vector<double> mis((size_t)nsteps * ng);
  for (int64_t n = 1; n <= nsteps; ++n) {
    states.push_back(q);
    rk4_step_impl<double>(*g, o, q.data(), b, dt, 0.0, 0);
    for (int gi = 0; gi < ng; ++gi) {
      const double m = q[gidx[gi]] + b[gidx[gi]] - target[(n - 1) * ng + gi];
      mis[(n - 1) * ng + gi] = m;
      L += 0.5 * m * m;
    }
  }
  *loss = L;
  std::vector<double> qb(M, 0.0), bb(N, 0.0);
  for (int64_t n = nsteps; n >= 1; --n) {
    for (int gi = 0; gi < ng; ++gi) {
      qb[gidx[gi]] += mis[(n - 1) * ng + gi];
      bb[gidx[gi]] += mis[(n - 1) * ng + gi];
    }
    rk4_vjp_impl(*g, o, states[n - 1].data(), b, dt, qb.data(), bb.data());
  }
  // initialization: eta0 = h0, w0 = -h0 (D_x u0 + D_y v0) + 3/2 (u0 D_x b + v0 D_y b) with u0 = v0 = 0:
  // w0 does not depend on h0 or b, so h0_bar = qb_h + qb_eta.
  for (size_t k = 0; k < N; ++k) {
    const double h0b = qb[k] + qb[4 * N + k];
    grad_zeta0[k] = h0b;
    grad_b[k] = bb[k] - h0b;
  }
}

// The adaptive pair (see fsal35_run): q is advanced in place.
int64_t orc_fsal35(const orc_grid* g, double* q, const double* b, double t0, double t_end, double dt0, double rtol,
                   double atol, int adaptive, int64_t max_attempts, double* rec, double* t_out, int64_t* n_acc,
                   int64_t* n_rej) {
  Ops o = make_ops(*g);
  return fsal35_run(*g, o, q, b, t0, t_end, dt0, rtol, atol, adaptive, max_attempts, rec, t_out, n_acc, n_rej);
}

// The pair's coefficients: c[6], a[36] (row-major), b[6], bh[6].
void orc_fsal35_tableau(double* c, double* a, double* b, double* bh) {
  const Fsal35 t = fsal35_tableau();
  for (int i = 0; i < 6; ++i) {
    c[i] = t.c[i];
    b[i] = t.b[i];
    bh[i] = t.bh[i];
    for (int j = 0; j < 6; ++j) a[6 * i + j] = t.a[i][j];
  }
}

// Threads the build runs its loops on (1 for the serial build).
int orc_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
