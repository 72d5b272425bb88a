// sgn_fused.hpp -- one classical RK4 step in one kernel.
//
// Each workgroup owns a tile of TX x TY nodes (32 x 24 by default, or 32 x 16
// or 64 x 8) and stages the state q with a four-node halo of
// (h, u, v, w, eta, b, 1/h) in LDS.  The four right-hand
// sides of the step are evaluated on shrinking regions, since each evaluation
// reaches one node further than the stage it reads:
//   k1 = f(q)   on the tile and the rings at distance 1..3,  Y2 = q + dt/2 k1
//   k2 = f(Y2)  on the tile and the rings at distance 1..2,  Y3 = q + dt/2 k2
//   k3 = f(Y3)  on the tile and the ring at distance 1,      Y4 = q + dt k3
//   k4 = f(Y4)  on the tile:  q_new = acc + dt/6 k4,
// with acc = q + dt/6 k1 + dt/3 k2 + dt/3 k3 kept in registers for the owned
// nodes.  Each intermediate stage overwrites the previous one in LDS (b is
// kept).  Only q and b are read and q_new written: 11 values per node and
// step from HBM, against 37 for the two pair kernels and 84 for four stage
// kernels.  The price is the ring evaluations: 1.24 right-hand sides per owned
// node and stage for a 32 x 24 tile, 1.31 for 32 x 16 and 1.42 for 64 x 8.
//
// Thread map: thread t owns the NO = TX TY / 256 tile nodes
// (t mod TX, NO floor(t / TX) + k), k < NO (three for 32 x 24, two for the
// others), in every stage, so their q and acc stay in registers; each node
// shares y-neighbours with the one below it.  Ring nodes are numbered by distance (all of
// ring 1 first, then ring 2, then ring 3); thread t evaluates ring nodes t and
// t + 256 in every stage whose region contains them, so the q of a ring node is
// read from LDS once, in the first stage.
//
// The output buffer must not alias the input (neighbouring tiles read the
// halo of q); sgn_step alternates between the caller's buffer and the
// context's accumulator buffer.
#pragma once

#include "sgn_pair.hpp"
#include "sgn_reduce.hpp"

namespace sgn {

constexpr int STEP_HALO = 4;  // one node per right-hand side of the step

// Tile shapes of the step kernel: TX x TY with TY = 24 (32 wide, three owned
// nodes per thread), 16 (32 wide) or 8 (64 wide; both two per thread).
template <int TY_>
struct StepGeom {
  static constexpr int TY = TY_;
  static constexpr int TX = TY == 8 ? 64 : 32;
  static constexpr int NO = TX * TY / STAGE_THREADS;  // owned nodes per thread
  static constexpr int RX = TX + 2 * STEP_HALO;
  static constexpr int RY = TY + 2 * STEP_HALO;
  // nodes of the ring at distance d around the tile
  static constexpr int ring(int d) { return 2 * (TX + 2 * d) + 2 * (TY + 2 * d - 2); }
  static constexpr int RING1 = ring(1);
  static constexpr int RING2 = RING1 + ring(2);
  static constexpr int RING3 = RING2 + ring(3);
  static_assert(TY == 8 || TY == 16 || TY == 24, "tile shapes 64 x 8, 32 x 16, 32 x 24");
  static_assert(NO * STAGE_THREADS == TX * TY && (NO == 2 || NO == 3), "two or three owned nodes per thread");
  static_assert(RING3 <= 2 * STAGE_THREADS, "two ring slots per thread");
};

// Rows are padded to an odd number of elements (PAD = 1) so that the ring
// columns, which lanes read down a column, spread over the LDS banks.  The
// manufactured-source instantiations (the heaviest, with the source evaluated
// inline) keep unpadded rows (PAD = 0): their reflecting variant returned wrong
// values near the x-walls with padded rows, a failure not explained by the
// source; unpadded they agree bit for bit with the four-stage path.
template <typename T, int TY, int PAD>
struct StepSmem {
  T f[7][StepGeom<TY>::RY][StepGeom<TY>::RX + PAD];  // h u v w eta b 1/h, then the current stage (b kept)
};

// The node's values behind an empty asm statement: the compiler can no longer
// identify them with the values they were copied from, so it neither merges
// arithmetic on them with earlier arithmetic nor changes how that arithmetic
// is fused.
template <typename T>
__device__ __forceinline__ Node<T> opaque_node(Node<T> n) {
  asm volatile("" : "+v"(n.h), "+v"(n.u), "+v"(n.v), "+v"(n.w), "+v"(n.eta), "+v"(n.b), "+v"(n.ih));
  return n;
}

// Which Runge-Kutta method a step tile runs.  RK_CLASSIC: one classical RK4
// step from q.  RK_FSAL: evaluations 2 to 5 of one attempt of the adaptive
// five-stage pair (sgn_fsal.hpp): the tile stages Y_2 = y + h c_2 k_1 (from
// the input y and the attempt's k_1), evaluates k_2 .. k_5 on the shrinking
// regions, and writes y_{n+1} = y + h (b_1 k_1 + ... + b_5 k_5) and the partial
// error estimate e' = h b_5 (k_5 - (1 - c_5) k_1) of the owned nodes.  The
// tile first stages y, from which the owned and ring nodes keep their y in
// registers (as the classical step keeps q), then overwrites it with Y_2; k_1
// of the owned nodes is read again from global memory (L2).
// RK_RELAXED: one classical RK4 step from the relaxed state of the previous
// relaxation step, q = qa + gam (ra - qa), formed while staging (the arithmetic
// of relax_update, so the same bits), which the tile also writes out for its
// owned nodes (RelaxIn).
enum : int { RK_CLASSIC = 0, RK_FSAL = 1, RK_RELAXED = 2 };

// Operands of an RK_RELAXED tile: q (the step's input pointer) is qa.
template <typename T>
struct RelaxIn {
  const T* ra;             // the previous step's RK4 result
  const double* rs;        // rs[0] = gam of the previous step
  T* qbase;                // out: the relaxed state of the owned nodes
};

// Coefficients and extra operands of an RK_FSAL tile (h already applied).
template <typename T>
struct FsalStage {
  const T* k1;  // k_1 of the attempt
  T* e;         // out: e' of the owned nodes
  T cin;        // h c_2
  T c1a;        // h b_1
  T cy[3];      // evaluation s = k_{s+1}: Y_{s+2} = y + cy[s-1] k_{s+1}  (s = 1, 2, 3)
  T ca[4];      // acc += ca[s-1] k_{s+1}                                  (s = 1 .. 4)
  T ce1;        // h b_5 (1 - c_5)
};

// Position (r, c), relative to the tile origin, of ring node m (0 <= m < RING3).
template <int TY>
__device__ __forceinline__ void ring_node(int m, int& r, int& c) {
  using G = StepGeom<TY>;
  constexpr int TX = G::TX;
  int d;
  if (m < G::RING1) {
    d = 1;
  } else if (m < G::RING2) {
    d = 2;
    m -= G::RING1;
  } else {
    d = 3;
    m -= G::RING2;
  }
  const int w = TX + 2 * d;          // top and bottom rows
  const int hs = G::TY + 2 * d - 2;  // left and right columns without the corners
  if (m < w) {
    r = -d;
    c = m - d;
  } else if (m < 2 * w) {
    r = G::TY - 1 + d;
    c = m - w - d;
  } else if (m < 2 * w + hs) {
    r = m - 2 * w - d + 1;
    c = -d;
  } else {
    r = m - 2 * w - hs - d + 1;
    c = TX - 1 + d;
  }
}

// One tile (origin i0, j0) of one RK4 step, executed by a whole workgroup.
// SAVE (the adjoint's recomputation): also write the intermediate stages
// Y2, Y3, Y4 of the owned nodes to ysave, three consecutive states.
// EPI (EPI_RELAX or EPI_TOTALS): also reduce the tile's two sums (see the
// enum; from the step's input and output values held in registers) into
// rpart[0..3].
// The caller synchronizes the workgroup before reusing `s` for another tile.
// RK = RK_FSAL (no source, no stage saving, no epilogue): q is the attempt's
// y_n, qout receives y_{n+1}, *fx supplies k_1, the coefficients and the e'
// output; c6 .. c1, t0, dt and flag are unused (the health of y_{n+1} is
// checked by the attempt's FSAL evaluation).
template <typename T, int BCX, int BCY, bool SRC, int TY, bool SAVE, int PAD, int EPI = EPI_NONE,
          int RK = RK_CLASSIC>
__device__ __forceinline__ void step_tile(StepSmem<T, TY, PAD>& s, const GridConst& gc, int i0, int j0,
                                          const T* __restrict__ q, const T* __restrict__ bplane,
                                          T* __restrict__ qout, T c6, T c3, T c2, T c1, double t0, double dt,
                                          int* __restrict__ flag, T* __restrict__ ysave,
                                          double* __restrict__ rpart = nullptr,
                                          const FsalStage<T>* __restrict__ fx = nullptr,
                                          const RelaxIn<T>* __restrict__ rx = nullptr) {
  static_assert(RK != RK_FSAL || (!SRC && !SAVE && EPI == EPI_NONE), "the FSAL tile has no extras");
  static_assert(RK != RK_RELAXED || (!SRC && !SAVE), "the relaxed tile has no source or stage saving");
  using G = StepGeom<TY>;
  constexpr int TX = G::TX, NO = G::NO;
  constexpr int RX = G::RX;
  constexpr int REGION = G::RX * G::RY;

  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const int tid = threadIdx.x;

  // 1. Stage q and b with the four-node halo (periodic wrap or wall clamp).
  //    Every load of the region is issued before the first one is waited
  //    for: the step kernel reads little per unit of work, so its bandwidth
  //    is set by how many bytes each workgroup keeps in flight.
  constexpr int NF = RK == RK_FSAL ? 1 : 0;
  T yown[NF ? NO : 1][5], yring[NF ? 2 : 1][5];  // RK_FSAL: y of the owned and ring nodes
  {
    constexpr int ITER = (REGION + STAGE_THREADS - 1) / STAGE_THREADS;
    T v[ITER][6];
    T kst[RK != RK_CLASSIC ? ITER : 1][5];
    // The staging waves take the issue priority until the barrier: their loads
    // and LDS writes go out ahead of the other workgroup's evaluation on the
    // same SIMDs (measured: FP32 2% and FP64 0.3-0.5% faster, same bits).
    __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * STAGE_THREADS;
      if (idx < REGION) {
        const int rr = idx / RX;
        const int cc = idx - rr * RX;
        const int gi = wrap_or_clamp<BCX>(i0 - STEP_HALO + cc, nx);
        const int gj = wrap_or_clamp<BCY>(j0 - STEP_HALO + rr, ny);
        const size_t o = (size_t)gj * nx + gi;
#pragma unroll
        for (int f = 0; f < 5; ++f) v[it][f] = q[f * N + o];
        v[it][5] = bplane[o];
        if constexpr (RK == RK_FSAL) {
#pragma unroll
          for (int f = 0; f < 5; ++f) kst[it][f] = fx->k1[f * N + o];
        }
        if constexpr (RK == RK_RELAXED) {
#pragma unroll
          for (int f = 0; f < 5; ++f) kst[it][f] = rx->ra[f * N + o];
        }
      }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * STAGE_THREADS;
      if (idx < REGION) {
        const int rr = idx / RX;
        const int cc = idx - rr * RX;
        if constexpr (RK == RK_RELAXED) {
          const T gam = T(rx->rs[0]);
#pragma unroll
          for (int f = 0; f < 5; ++f) v[it][f] = v[it][f] + gam * (kst[it][f] - v[it][f]);
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) s.f[f][rr][cc] = v[it][f];
        if constexpr (RK != RK_FSAL) s.f[6][rr][cc] = recip_staged(v[it][0]);
      }
    }
    if constexpr (RK == RK_FSAL) {
      __syncthreads();
      // LDS holds y: the owned and ring nodes take their y from it (the ring's
      // periodic images and clamped wall copies included), then Y_2 =
      // y + h c_2 k_1 and its 1/h replace it
      const int lx_ = tid % TX, ly_ = NO * (tid / TX);
#pragma unroll
      for (int k = 0; k < NO; ++k) {
#pragma unroll
        for (int f = 0; f < 5; ++f) yown[k][f] = s.f[f][ly_ + k + STEP_HALO][lx_ + STEP_HALO];
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int m = tid + k * STAGE_THREADS;
        if (m < G::RING3) {
          int r_, c_;
          ring_node<TY>(m, r_, c_);
#pragma unroll
          for (int f = 0; f < 5; ++f) yring[k][f] = s.f[f][r_ + STEP_HALO][c_ + STEP_HALO];
        }
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const int idx = tid + it * STAGE_THREADS;
        if (idx < REGION) {
          const int rr = idx / RX;
          const int cc = idx - rr * RX;
          T y2[5];
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            y2[f] = v[it][f] + fx->cin * kst[it][f];
            s.f[f][rr][cc] = y2[f];
          }
          s.f[6][rr][cc] = recip_staged(y2[0]);
        }
      }
    }
  }

  __builtin_amdgcn_s_setprio(0);
  // Owned nodes (lx, ly0 + k), k < NO, and ring slots of this thread.
  const int lx = tid % TX;
  const int ly0 = NO * (tid / TX);
  const int i = i0 + lx;
  bool own_dom[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int j = j0 + ly0 + k;
    own_dom[k] = on_axis<BCX>(i, nx) && on_axis<BCY>(j, ny);
  }
  int ring_r[2], ring_c[2];
  bool ring_ok[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int m = tid + k * STAGE_THREADS;
    ring_r[k] = 0;
    ring_c[k] = 0;
    ring_ok[k] = false;
    if (m < G::RING3) {
      ring_node<TY>(m, ring_r[k], ring_c[k]);
      ring_ok[k] = on_axis<BCX>(i0 + ring_c[k], nx) && on_axis<BCY>(j0 + ring_r[k], ny);
    }
  }
  __syncthreads();

  T qo[NO][5], acc[NO][5], qr[2][5];
  T k1o[NF ? NO : 1][5];  // RK_FSAL: k_1 of the owned nodes
  if constexpr (RK == RK_FSAL) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (tid + k * STAGE_THREADS < G::RING3) {
#pragma unroll
        for (int f = 0; f < 5; ++f) qr[k][f] = yring[k][f];
      }
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) {
#pragma unroll
      for (int f = 0; f < 5; ++f) qo[k][f] = yown[k][f];
      if (own_dom[k]) {
        const size_t ow = (size_t)wrap_or_clamp<BCY>(j0 + ly0 + k, ny) * nx + wrap_or_clamp<BCX>(i, nx);
#pragma unroll
        for (int f = 0; f < 5; ++f) k1o[k][f] = fx->k1[f * N + ow];
      }
    }
  }
  int health = 0;
  CSum rsum[2];
  if (EPI != EPI_NONE) {
    rsum[0].init();
    rsum[1].init();
  }
#pragma unroll
  for (int st = 1; st <= 4; ++st) {
    T cy = st == 3 ? c1 : c2;             // Y_{st+1} = q + cy k_st
    T ca = st == 1 || st == 4 ? c6 : c3;  // acc += ca k_st
    if constexpr (RK == RK_FSAL) {
      cy = st < 4 ? fx->cy[st - 1] : T(0);
      ca = fx->ca[st - 1];
    }
    const double ts = t0 + (st == 1 ? 0.0 : (st == 4 ? dt : 0.5 * dt));
    const int ring_lim = st == 1 ? G::RING3 : (st == 2 ? G::RING2 : G::RING1);
    T ro[NO][5], rr[2][5];
    // Owned nodes.  Node k lies just above node k - 1 in y, so whenever node k
    // is in the domain (then j0 + ly0 + k - 1 is neither the first row nor
    // beyond the last) its lower y-neighbour is node k - 1's centre, and node
    // 1's centre is node 0's upper y-neighbour: the pair reads 8 nodes from
    // LDS, not 10, and three nodes read 12, not 15.
    const auto finish = [&](int k, const Rates<T>& kk, const Node<T>& cn) {
      const int j = j0 + ly0 + k;
      const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
      if constexpr (RK == RK_FSAL) {
        if (st == 1) {
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            acc[k][f] = qo[k][f] + fx->c1a * k1o[k][f] + ca * kv[f];
            ro[k][f] = qo[k][f] + cy * kv[f];
          }
        } else if (st < 4) {
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            acc[k][f] = acc[k][f] + ca * kv[f];
            ro[k][f] = qo[k][f] + cy * kv[f];
          }
        }
      } else if (st == 1) {
        const T yv[5] = {cn.h, cn.u, cn.v, cn.w, cn.eta};
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          qo[k][f] = yv[f];
          acc[k][f] = yv[f] + ca * kv[f];
          ro[k][f] = yv[f] + cy * kv[f];
        }
        if constexpr (RK == RK_RELAXED) {
          if (i < nx && j < ny) {
            const size_t o = (size_t)j * nx + i;
#pragma unroll
            for (int f = 0; f < 5; ++f) rx->qbase[f * N + o] = yv[f];
          }
        }
      } else if (st < 4) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          acc[k][f] = acc[k][f] + ca * kv[f];
          ro[k][f] = qo[k][f] + cy * kv[f];
        }
      }
      if (SAVE && st < 4 && i < nx && j < ny) {
        T* ys = ysave + (size_t)(st - 1) * 5 * N + (size_t)j * nx + i;
#pragma unroll
        for (int f = 0; f < 5; ++f) ys[f * N] = ro[k][f];
      }
      if (st == 4) {
        const size_t o = (size_t)j * nx + i;
        T nv[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          nv[f] = acc[k][f] + ca * kv[f];
          qout[f * N + o] = nv[f];
        }
        if constexpr (RK == RK_FSAL) {
#pragma unroll
          for (int f = 0; f < 5; ++f) fx->e[f * N + o] = ca * kv[f] - fx->ce1 * k1o[k][f];
        } else {
          if (!(nv[0] > T(0))) health |= FLAG_NONPOS;
          const T sum = nv[0] + nv[1] + nv[2] + nv[3] + nv[4];
          if (!isfinite(sum)) health |= FLAG_NONFINITE;
        }
        if (EPI == EPI_TOTALS) {
          const double M = axis_weight(i, nx, gc.bc_x, gc.dx) * axis_weight(j, ny, gc.bc_y, gc.dy);
          const double bb = (double)s.f[5][ly0 + k + STEP_HALO][lx + STEP_HALO];
          rsum[0].add(M * (double)nv[0]);
          rsum[1].add(M * energy_density((double)nv[0], (double)nv[1], (double)nv[2], (double)nv[3], (double)nv[4],
                                         bb, gc.g, gc.lam));
        }
        if (EPI == EPI_RELAX) {
          double x[5], d[5];
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            x[f] = (double)qo[k][f];
            d[f] = (double)nv[f] - x[f];
          }
          double sv, dsv;
          relax_node_terms(x, d, (double)s.f[5][ly0 + k + STEP_HALO][lx + STEP_HALO], gc.g, gc.lam, 1.0, sv, dsv);
          const double M = axis_weight(i, nx, gc.bc_x, gc.dx) * axis_weight(j, ny, gc.bc_y, gc.dy);
          rsum[0].add(M * sv);
          rsum[1].add(M * dsv);
        }
      }
    };
    {
      __builtin_amdgcn_sched_barrier(0);
      const int j = j0 + ly0;
      // node 1 in the domain implies node 0 in the domain
      const bool run0 = st < 4 ? own_dom[0] : (i < nx && j < ny);
      const bool run1 = st < 4 ? own_dom[1] : (i < nx && j + 1 < ny);
      if (run0) {
        const int r = ly0 + STEP_HALO, c = lx + STEP_HALO;
        const AxisStencil<BCX> ax(i, nx, gc.inv2dx, gc.invdx);
        const AxisStencil<BCY> ay0(j, ny, gc.inv2dy, gc.invdy);
        const Node<T> c0 = lds_load<T>(s, r, c);
        const Node<T> up = lds_load<T>(s, r + ay0.op, c);
        {
          const Node<T> xm = lds_load<T>(s, r, c + ax.om);
          const Node<T> xp = lds_load<T>(s, r, c + ax.op);
          const Node<T> dn = lds_load<T>(s, r + ay0.om, c);
          finish(0, node_rates<T, BCX, BCY, SRC>(c0, xm, xp, dn, up, ax, ay0, i, j, gc, ts), c0);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (run1) {
          // Node 1 re-enters the shared nodes as opaque values: products of
          // them formed for node 0 are formed again, rounded exactly as every
          // other evaluation of the right-hand side rounds them.
          const Node<T> c0n = opaque_node(c0), upn = opaque_node(up);
          const AxisStencil<BCY> ay1(j + 1, ny, gc.inv2dy, gc.invdy);
          const Node<T> xm = lds_load<T>(s, r + 1, c + ax.om);
          const Node<T> xp = lds_load<T>(s, r + 1, c + ax.op);
          const Node<T> up1 = lds_load<T>(s, r + 1 + ay1.op, c);
          finish(1, node_rates<T, BCX, BCY, SRC>(upn, xm, xp, c0n, up1, ax, ay1, i, j + 1, gc, ts), upn);
          if constexpr (NO == 3) {
            __builtin_amdgcn_sched_barrier(0);
            const bool run2 = st < 4 ? own_dom[2] : (i < nx && j + 2 < ny);
            if (run2) {
              // node 1's centre re-enters as an opaque value; node 2's own
              // centre is read again (taking it from node 1's upper neighbour
              // changes how node 1's arithmetic is fused)
              const Node<T> c1n = opaque_node(upn);
              const AxisStencil<BCY> ay2(j + 2, ny, gc.inv2dy, gc.invdy);
              const Node<T> c2 = lds_load<T>(s, r + 2, c);
              const Node<T> xm2 = lds_load<T>(s, r + 2, c + ax.om);
              const Node<T> xp2 = lds_load<T>(s, r + 2, c + ax.op);
              const Node<T> up2 = lds_load<T>(s, r + 2 + ay2.op, c);
              finish(2, node_rates<T, BCX, BCY, SRC>(c2, xm2, xp2, c1n, up2, ax, ay2, i, j + 2, gc, ts), c2);
            }
          }
        }
      }
    }
    if (st == 4) break;
    // ring nodes inside this stage's region
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      __builtin_amdgcn_sched_barrier(0);
      const int m = tid + k * STAGE_THREADS;
      if (m >= ring_lim || !ring_ok[k]) continue;
      Node<T> cn;
      const Rates<T> kk = tile_eval<T, BCX, BCY, SRC>(s, ring_r[k] + STEP_HALO, ring_c[k] + STEP_HALO,
                                                      i0 + ring_c[k], j0 + ring_r[k], gc, ts, cn);
      const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
      if constexpr (RK != RK_FSAL) {
        if (st == 1) {
          qr[k][0] = cn.h;
          qr[k][1] = cn.u;
          qr[k][2] = cn.v;
          qr[k][3] = cn.w;
          qr[k][4] = cn.eta;
        }
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) rr[k][f] = qr[k][f] + cy * kv[f];
    }
    __syncthreads();
    // the stage just formed replaces the one read
#pragma unroll
    for (int k = 0; k < NO; ++k) {
      if (!own_dom[k]) continue;
      const int r = ly0 + k + STEP_HALO, c = lx + STEP_HALO;
#pragma unroll
      for (int f = 0; f < 5; ++f) s.f[f][r][c] = ro[k][f];
      s.f[6][r][c] = recip_staged(ro[k][0]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int m = tid + k * STAGE_THREADS;
      if (m >= ring_lim || !ring_ok[k]) continue;
      const int r = ring_r[k] + STEP_HALO, c = ring_c[k] + STEP_HALO;
#pragma unroll
      for (int f = 0; f < 5; ++f) s.f[f][r][c] = rr[k][f];
      s.f[6][r][c] = recip_staged(rr[k][0]);
    }
    __syncthreads();
  }
  if constexpr (RK != RK_FSAL) {
    if (health) atomicOr(flag, health);
  }
  if (EPI != EPI_NONE) {
    block_merge<2>(rsum);
    if (tid == 0) {
      rpart[0] = rsum[0].s;
      rpart[1] = rsum[0].c;
      rpart[2] = rsum[1].s;
      rpart[3] = rsum[1].c;
    }
  }
}

// EPI != EPI_NONE: rpart holds 4 doubles per tile, in tile order.
template <typename T, int BCX, int BCY, bool SRC, int TY, bool SAVE = false, int EPI = EPI_NONE>
__global__ __launch_bounds__(STAGE_THREADS) void step_kernel(const GridConst gc, const T* __restrict__ q,
                                                             const T* __restrict__ bplane, T* __restrict__ qout,
                                                             T c6, T c3, T c2, T c1, double t0, double dt,
                                                             int* __restrict__ flag, T* __restrict__ ysave,
                                                             double* __restrict__ rpart) {
  constexpr int TX = StepGeom<TY>::TX;
  __shared__ StepSmem<T, TY, SRC ? 0 : 1> s;
  const int ntx = (gc.nx + TX - 1) / TX;
  const int nty = (gc.ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  step_tile<T, BCX, BCY, SRC, TY, SAVE, SRC ? 0 : 1, EPI>(s, gc, (tile % ntx) * TX, (tile / ntx) * TY, q, bplane,
                                                          qout, c6, c3, c2, c1, t0, dt, flag, ysave,
                                                          EPI != EPI_NONE ? rpart + 4 * tile : nullptr);
}

}  // namespace sgn
