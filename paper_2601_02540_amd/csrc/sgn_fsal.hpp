// sgn_fsal.hpp -- the adaptive five-stage, third-order FSAL Runge-Kutta pair.
//
// The paper integrates with an explicit third-order, five-stage Runge-Kutta
// method whose last stage is the first of the next step (FSAL), with an
// embedded error estimate driving the step size (Section "Numerical
// Experiments"; relative and absolute tolerances 1e-6).  The paper names the
// method only by citation; the pair here has that shape:
//   Y_1 = y_n,  Y_{i+1} = y_n + h c_{i+1} k_i  (k_i = f(Y_i)),
//   c = (0, 1/3, 3/4, 4/5, 3071/3720),
//   y_{n+1} = y_n + h (b_1 k_1 + ... + b_5 k_5),
//   b = (7200668/46553289, 1701/5053, 6098/15159, 350/5053, 18600/500573),
// third order with stability polynomial 1 + z + z^2/2 + z^3/6 + z^4/31 +
// z^5/163 (imaginary-axis stability interval ~3.9).  With k_6 = f(y_{n+1})
// (the next step's k_1) the embedded second-order solution differs from
// y_{n+1} by
//   e = h b_5 (k_5 - (1 - c_5) k_1 - c_5 k_6),
// i.e. the rate at c_5 against the linear interpolation of the rates at the
// ends of the step.  err = RMS over all 5N values of
// e / (atol + rtol max(|y_n|, |y_{n+1}|)); err <= 1 accepts.  The PI
// controller (Hairer-Wanner, Section IV.2) sets the next step to
// h 0.9 err^(-0.7/3) errp^(0.4/3), limited to [0.2, 5] h ([0.2, 1] h right
// after a rejection; errp = the last accepted err, at least 1e-4); a rejected
// step is retried with h max(0.2, 0.9 err^(-1/3)); the last step ends at t_end.
//
// On the four-stage and pair step paths one attempt is five launches over
// 64 x TY tiles with a one-node halo (the layout and right-hand side of the
// stage kernel) and a one-block controller:
//   S2:   stages Y_2 = y + h c_2 k_1 (formed while staging from y and k_1),
//         writes acc = y + h b_1 k_1 + h b_2 k_2 into the other state buffer
//         and Y_3 = y + h c_3 k_2                               21 values/node
//   S3:   Y_3 -> acc += h b_3 k_3, Y_4 = y + h c_4 k_3           26
//   S4:   Y_4 -> acc += h b_4 k_4, Y_5 = y + h c_5 k_4           26
//   S5:   Y_5 -> y_{n+1} = acc + h b_5 k_5,
//         e' = h b_5 (k_5 - (1 - c_5) k_1)                       26
//   FSAL: y_{n+1} -> k_6 (the next k_1), e = e' - h b_5 c_5 k_6, per-tile
//         compensated sums of the scaled squares, health check   21
//   control: merges the tile sums in tile order, accepts or rejects, updates
//         t, h, the counters and the buffer selector in device memory.
// On the default (fused) step path S2 .. S5 are one launch of the step tile
// (fsal_step_kernel): 21 + 21 values per node and attempt instead of 120.
// The state buffer holding y_n and the one holding k_1 are selected by a
// device-side index that flips on acceptance, so a rejected attempt leaves
// y_n and k_1 untouched and no copy is needed.  Every kernel returns at once
// once the run is done, so graphs of several attempts can be replayed past
// the end.
#pragma once

#include "sgn_fused.hpp"
#include "sgn_reduce.hpp"
#include "sgn_stage.hpp"

namespace sgn {

struct Fsal35 {
  static constexpr double c2 = 1.0 / 3.0, c3 = 3.0 / 4.0, c4 = 4.0 / 5.0, c5 = 3071.0 / 3720.0;
  static constexpr double b1 = 7200668.0 / 46553289.0, b2 = 1701.0 / 5053.0, b3 = 6098.0 / 15159.0,
                          b4 = 350.0 / 5053.0, b5 = 18600.0 / 500573.0;
};

// Run state in device memory (written by the control kernel only).
struct AdaptCtl {
  double t, h, t_end, errp, err;
  double rtol, atol;
  long long attempts, accepted, rejected, max_attempts;
  int cur;           // y_n in q[cur], k_1 in k[cur]
  int done;          // 0 running, 1 reached t_end, 2 attempt limit, 3 non-finite error,
                     // 4 an accepted state failed the health check
  int after_reject;  // the last attempt was rejected
  int adaptive;      // 0: fixed steps h, all accepted
  int att_health;    // health bits of the current attempt's y_{n+1} (FLAG_*)
};

template <typename T>
struct FsalArgs {
  T* q[2];
  T* k[2];
  T* ya;
  T* yb;
  T* e;
  const T* b;
  double* part;  // FSAL role: 2 doubles per tile
  AdaptCtl* ctl;
};

enum : int { FS_S2 = 2, FS_S3 = 3, FS_S4 = 4, FS_S5 = 5, FS_FSAL = 6 };

template <typename T, int BCX, int BCY, int ROLE, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void fsal_kernel(const GridConst gc, const FsalArgs<T> a) {
  static_assert(TY % THREAD_ROWS == 0, "tile height must be a multiple of 4");
  constexpr int RPT = TY / THREAD_ROWS;
  constexpr int W = TILE_X + 2;
  constexpr int REGION = (TY + 2) * W;
  __shared__ StageSmem<T, TY> s;

  AdaptCtl* ctl = a.ctl;
  if (ctl->done) return;  // the same for the whole grid
  const int cur = ctl->cur;
  const double h = ctl->h;
  const T* y = a.q[cur];
  T* ynew = a.q[cur ^ 1];
  const T* k1 = a.k[cur];
  T* knext = a.k[cur ^ 1];
  const T* Yin = ROLE == FS_S2 ? y : (ROLE == FS_S3 || ROLE == FS_S5) ? a.ya : ROLE == FS_S4 ? a.yb : ynew;
  T* Yout = ROLE == FS_S2 ? a.ya : ROLE == FS_S3 ? a.yb : a.ya;
  using C = Fsal35;
  const T cin = T(h * C::c2);  // S2: Y_2 = y + h c_2 k_1
  const T c1a = T(h * C::b1);
  const T cacc = T(h * (ROLE == FS_S2 ? C::b2 : ROLE == FS_S3 ? C::b3 : ROLE == FS_S4 ? C::b4 : C::b5));
  const T cy = T(h * (ROLE == FS_S2 ? C::c3 : ROLE == FS_S3 ? C::c4 : C::c5));
  const T ce1 = T(h * C::b5 * (1.0 - C::c5));  // S5: e' = h b5 k5 - h b5 (1 - c5) k1
  const T ce6 = T(h * C::b5 * C::c5);          // FSAL: e = e' - h b5 c5 k6

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
    T v[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) v[f] = ROLE == FS_S2 ? Yin[f * N + o] + cin * k1[f * N + o] : Yin[f * N + o];
#pragma unroll
    for (int f = 0; f < 5; ++f) s.f[f][rr][cc] = v[f];
    s.f[5][rr][cc] = a.b[o];
    s.f[6][rr][cc] = recip_staged(v[0]);
  }

  // own-node operands, fetched before the barrier
  const int i = i0 + tx;
  T pa[RPT][5], pb[RPT][5];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int j = j0 + ty + k * THREAD_ROWS;
    if (i < nx && j < ny) {
      const size_t o = (size_t)j * nx + i;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        if (ROLE == FS_S2) {
          pa[k][f] = y[f * N + o];
          pb[k][f] = k1[f * N + o];
        } else if (ROLE == FS_S3 || ROLE == FS_S4) {
          pa[k][f] = y[f * N + o];
          pb[k][f] = ynew[f * N + o];
        } else if (ROLE == FS_S5) {
          pa[k][f] = k1[f * N + o];
          pb[k][f] = ynew[f * N + o];
        } else {
          pa[k][f] = y[f * N + o];
          pb[k][f] = a.e[f * N + o];
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
  CSum sq;
  sq.init();
  const double atol = ctl->atol, rtol = ctl->rtol;

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
    const Rates<T> kk =
        split_form_rates<T, BCX, BCY>(c, xm, xp, ym, yp, T(ax.scale), T(ay.scale), g, lam, satx, saty);
    const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
    const T yv[5] = {c.h, c.u, c.v, c.w, c.eta};
    const size_t o = (size_t)j * nx + i;
    if (ROLE == FS_S2) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        ynew[f * N + o] = pa[k][f] + c1a * pb[k][f] + cacc * kv[f];
        Yout[f * N + o] = pa[k][f] + cy * kv[f];
      }
    } else if (ROLE == FS_S3 || ROLE == FS_S4) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        ynew[f * N + o] = pb[k][f] + cacc * kv[f];
        Yout[f * N + o] = pa[k][f] + cy * kv[f];
      }
    } else if (ROLE == FS_S5) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        ynew[f * N + o] = pb[k][f] + cacc * kv[f];
        a.e[f * N + o] = cacc * kv[f] - ce1 * pa[k][f];
      }
    } else {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        knext[f * N + o] = kv[f];
        const double ef = (double)pb[k][f] - (double)ce6 * (double)kv[f];
        const double sc = atol + rtol * fmax(fabs((double)pa[k][f]), fabs((double)yv[f]));
        const double z = ef / sc;
        sq.add(z * z);
      }
      if (!(yv[0] > T(0))) health |= FLAG_NONPOS;
      const T sum = yv[0] + yv[1] + yv[2] + yv[3] + yv[4];
      if (!isfinite(sum)) health |= FLAG_NONFINITE;
    }
  }
  if (ROLE == FS_FSAL) {
    if (health) atomicOr(&ctl->att_health, health);
    CSum arr[1] = {sq};
    block_merge<1>(arr);
    if (tid == 0) {
      a.part[2 * tile + 0] = arr[0].s;
      a.part[2 * tile + 1] = arr[0].c;
    }
  }
}

// S2 .. S5 of one attempt in one launch (the default step path): the step
// tile in its RK_FSAL mode over TX x TY tiles (StepGeom) with a four-node halo.
// Reads y, k_1 and b, writes y_{n+1} and e'; the intermediate stages Y_2 .. Y_5
// stay in LDS (the rings around each tile are evaluated redundantly).  21
// values per node instead of the 99 of the four role kernels.  Same arithmetic
// as the roles node by node, so the same bits.
template <typename T, int BCX, int BCY, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void fsal_step_kernel(const GridConst gc, const FsalArgs<T> a) {
  constexpr int TX = StepGeom<TY>::TX;
  __shared__ StepSmem<T, TY, 1> s;
  const AdaptCtl* ctl = a.ctl;
  if (ctl->done) return;  // the same for the whole grid
  const int cur = ctl->cur;
  const double h = ctl->h;
  using C = Fsal35;
  FsalStage<T> fx;
  fx.k1 = a.k[cur];
  fx.e = a.e;
  fx.cin = T(h * C::c2);
  fx.c1a = T(h * C::b1);
  fx.cy[0] = T(h * C::c3);
  fx.cy[1] = T(h * C::c4);
  fx.cy[2] = T(h * C::c5);
  fx.ca[0] = T(h * C::b2);
  fx.ca[1] = T(h * C::b3);
  fx.ca[2] = T(h * C::b4);
  fx.ca[3] = T(h * C::b5);
  fx.ce1 = T(h * C::b5 * (1.0 - C::c5));
  const int ntx = (gc.nx + TX - 1) / TX;
  const int nty = (gc.ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  step_tile<T, BCX, BCY, false, TY, false, 1, EPI_NONE, RK_FSAL>(s, gc, (tile % ntx) * TX, (tile / ntx) * TY,
                                                                 a.q[cur], a.b, a.q[cur ^ 1], T(0), T(0), T(0),
                                                                 T(0), 0.0, 0.0, nullptr, nullptr, nullptr, &fx);
}

// One block: merges the tile sums in tile order into err and applies the
// controller.  rec (may be NULL): (h, err, accepted) of attempt n at
// rec[3n .. 3n+2] while n < rec_cap.
// An accepted y_{n+1} that failed the health check ends the run (done = 4)
// and raises its bits in flag; a rejected one is simply retried.
static __global__ __launch_bounds__(RED_THREADS) void fsal_control(AdaptCtl* __restrict__ ctl,
                                                                    const double* __restrict__ part, int nparts,
                                                                    double inv_count, double* __restrict__ rec,
                                                                    long long rec_cap, int* __restrict__ flag) {
  if (ctl->done) return;
  CSum a[1];
  a[0].init();
  for (int p = threadIdx.x; p < nparts; p += RED_THREADS) a[0].merge(part[2 * p], part[2 * p + 1]);
  block_merge<1>(a);
  if (threadIdx.x != 0) return;
  const double err = sqrt((a[0].s + a[0].c) * inv_count);
  const double h = ctl->h, t = ctl->t, t_end = ctl->t_end;
  const long long n = ctl->attempts;
  const bool ok = !ctl->adaptive || err <= 1.0;
  if (rec && n < rec_cap) {
    rec[3 * n + 0] = h;
    rec[3 * n + 1] = err;
    rec[3 * n + 2] = ok ? 1.0 : 0.0;
  }
  ctl->attempts = n + 1;
  ctl->err = err;
  const int health = ctl->att_health;
  ctl->att_health = 0;
  if (!isfinite(err)) {
    atomicOr(flag, health | FLAG_NONFINITE);
    ctl->done = 3;
    return;
  }
  if (ok && health) {
    atomicOr(flag, health);
    ctl->done = 4;
    return;
  }
  double dt = h;
  double tn = t;
  if (ok) {
    tn = (h == t_end - t) ? t_end : t + h;
    ctl->t = tn;
    ctl->cur ^= 1;
    ctl->accepted += 1;
    if (ctl->adaptive) {
      double fac = 0.9 * pow(err, -0.7 / 3.0) * pow(ctl->errp, 0.4 / 3.0);
      fac = fmin(fac, ctl->after_reject ? 1.0 : 5.0);
      fac = fmax(fac, 0.2);
      dt = h * fac;
      ctl->errp = fmax(err, 1e-4);
    }
    ctl->after_reject = 0;
  } else {
    ctl->rejected += 1;
    dt = h * fmax(0.2, 0.9 * pow(err, -1.0 / 3.0));
    ctl->after_reject = 1;
  }
  if (!(tn < t_end)) {
    ctl->done = 1;
    ctl->h = dt;
    return;
  }
  // the last step ends exactly at t_end (also when rounding left it a hair longer than dt)
  ctl->h = (t_end - tn <= dt * (1.0 + 1e-10)) ? t_end - tn : dt;
  if (ctl->attempts >= ctl->max_attempts) ctl->done = 2;
}

static __global__ void fsal_init(AdaptCtl* __restrict__ ctl, double t0, double h0, double t_end, double rtol,
                                 double atol, long long max_attempts, int adaptive) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctl->t = t0;
  ctl->h = h0;
  ctl->t_end = t_end;
  ctl->errp = 1.0;
  ctl->err = 0.0;
  ctl->rtol = rtol;
  ctl->atol = atol;
  ctl->attempts = 0;
  ctl->accepted = 0;
  ctl->rejected = 0;
  ctl->max_attempts = max_attempts;
  ctl->cur = 0;
  ctl->done = t0 < t_end ? 0 : 1;
  ctl->after_reject = 0;
  ctl->adaptive = adaptive;
  ctl->att_health = 0;
}

}  // namespace sgn
