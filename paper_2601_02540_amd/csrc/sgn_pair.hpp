// sgn_pair.hpp -- two Runge-Kutta stages fused in one kernel.
//
// The classical RK4 step is split into two launches, each evaluating two
// right-hand sides:
//   pair 1:  k1 = f(q)  on the tile plus a one-node ring,  Ya = q + dt/2 k1
//            k2 = f(Ya) on the tile:  acc = q + dt/6 k1 + dt/3 k2,  Yb = q + dt/2 k2
//   pair 2:  k3 = f(Yb) on the tile plus ring,  Ya = q + dt k3
//            k4 = f(Ya) on the tile:  q_new = acc + dt/3 k3 + dt/6 k4
// The intermediate stage Ya never leaves LDS.  A workgroup stages its
// 64 x TY tile with a two-node halo of (h, u, v, w, eta, b, 1/h); after the
// first evaluation the intermediate values overwrite the input planes in place
// (b is kept), and the second evaluation reads them.  HBM traffic per step is
// 37 values per node instead of 84 for four separate stage kernels.
//
// Buffer rotation: pair 2 writes q_new over acc (each node reads its own acc
// before writing it), so the state alternates between two buffers and returns
// to the caller's buffer after every second step.
#pragma once

#include "sgn_stage.hpp"

namespace sgn {

template <typename T, int TY>
struct PairSmem {
  T f[7][TY + 4][TILE_X + 4];  // h u v w eta b 1/h  (later: the intermediate stage, b kept)
};

template <int BC>
__device__ __forceinline__ int wrap_or_clamp(int g, int n) {
  if (BC == BC_PERIODIC) {
    // g lies in [-4, n + 66] (a tile origin below n, the tile's extent and a
    // halo of at most four nodes) and n >= 4: one addition or a few
    // subtractions wrap it (more than one only on axes shorter than the tile).
    if (g < 0) g += n;
    while (g >= n) g -= n;
  } else {
    g = g < 0 ? 0 : (g >= n ? n - 1 : g);
  }
  return g;
}

// Is global index g (unwrapped) a node of the axis?  Periodic images always are.
template <int BC>
__device__ __forceinline__ bool on_axis(int g, int n) {
  if (BC == BC_PERIODIC) return opaque_true();
  return g >= 0 && g < n;
}

// The seven staged values of LDS position (r, c).  `Smem` holds the planes
// h u v w eta b 1/h as f[7][rows][cols].
template <typename T, class Smem>
__device__ __forceinline__ Node<T> lds_load(const Smem& s, int r, int c) {
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

// Right-hand side at node (i, j) (unwrapped indices) from its value and its four
// neighbours as the stencils ax, ay select them (closure rows included).
template <typename T, int BCX, int BCY, bool SRC>
__device__ __forceinline__ Rates<T> node_rates(const Node<T>& center, const Node<T>& xm, const Node<T>& xp,
                                               const Node<T>& ym, const Node<T>& yp, const AxisStencil<BCX>& ax,
                                               const AxisStencil<BCY>& ay, int i, int j, const GridConst& gc,
                                               double t) {
  T satx = T(0), saty = T(0);
  if (BCX == BC_REFLECTING) {
    if (i == 0) satx = T(-2.0 * gc.invdx);
    if (i == gc.nx - 1) satx = T(2.0 * gc.invdx);
  }
  if (BCY == BC_REFLECTING) {
    if (j == 0) saty = T(-2.0 * gc.invdy);
    if (j == gc.ny - 1) saty = T(2.0 * gc.invdy);
  }
  Rates<T> k = split_form_rates<T, BCX, BCY>(center, xm, xp, ym, yp, T(ax.scale), T(ay.scale), T(gc.g), T(gc.lam),
                                             satx, saty);
  if (SRC) {
    const int gi = wrap_or_clamp<BCX>(i, gc.nx), gj = wrap_or_clamp<BCY>(j, gc.ny);
    double S[5];
    mms_source(gc.xmin + gi * gc.dx, gc.ymin + gj * gc.dy, t, gc.g, S);
    k.h += T(S[0]);
    k.u += T(S[1]);
    k.v += T(S[2]);
    k.w += T(S[3]);
    k.eta += T(S[4]);
  }
  return k;
}

// Right-hand side at LDS position (r, c) of node (i, j) (unwrapped indices).
template <typename T, int BCX, int BCY, bool SRC, class Smem>
__device__ __forceinline__ Rates<T> tile_eval(const Smem& s, int r, int c, int i, int j, const GridConst& gc, double t,
                                              Node<T>& center) {
  const AxisStencil<BCX> ax(i, gc.nx, gc.inv2dx, gc.invdx);
  const AxisStencil<BCY> ay(j, gc.ny, gc.inv2dy, gc.invdy);
  center = lds_load<T>(s, r, c);
  const Node<T> xm = lds_load<T>(s, r, c + ax.om);
  const Node<T> xp = lds_load<T>(s, r, c + ax.op);
  const Node<T> ym = lds_load<T>(s, r + ay.om, c);
  const Node<T> yp = lds_load<T>(s, r + ay.op, c);
  return node_rates<T, BCX, BCY, SRC>(center, xm, xp, ym, yp, ax, ay, i, j, gc, t);
}

// One tile (origin i0, j0) of a stage pair, executed by a whole workgroup.
// PAIR = 1: Yin = q (state), writes acc_io = acc and yb_out = Yb.
// PAIR = 2: Yin = Yb, qn = q (state), acc_io holds acc on entry and q_new on exit.
// The caller synchronizes the workgroup before reusing `s` for another tile.
// SAVE (adjoint recomputation): also write the intermediate stage of owned
// nodes to ysave (pair 1: Y2 = q + dt/2 k1; pair 2: Y4 = q + dt k3), and in
// pair 2 write q_new to qout instead of over acc.
template <typename T, int BCX, int BCY, int PAIR, bool SRC, int TY, bool SAVE = false>
__device__ __forceinline__ void pair_tile(PairSmem<T, TY>& s, const GridConst& gc, int i0, int j0,
                                          const T* __restrict__ Yin, const T* __restrict__ bplane,
                                          const T* __restrict__ qn, T* acc_io, T* __restrict__ yb_out, T c1_acc,
                                          T c1_y, T c2_acc, T c2_y, double t1, double t2, int* __restrict__ flag,
                                          T* __restrict__ ysave = nullptr, T* __restrict__ qout = nullptr) {
  static_assert(TY % THREAD_ROWS == 0, "tile height must be a multiple of 4");
  constexpr int RPT = TY / THREAD_ROWS;
  constexpr int W2 = TILE_X + 4;
  constexpr int REGION = (TY + 4) * W2;
  constexpr int RING = 2 * (TILE_X + 2) + 2 * TY;
  static_assert(RING <= STAGE_THREADS, "ring must fit one pass");

  const int nx = gc.nx, ny = gc.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const int tid = threadIdx.x;
  const int tx = tid & (TILE_X - 1);
  const int ty = tid >> 6;

  // 1. Stage the input state with a two-node halo.
#pragma unroll 1
  for (int idx = tid; idx < REGION; idx += STAGE_THREADS) {
    const int rr = idx / W2;
    const int cc = idx - rr * W2;
    const int gi = wrap_or_clamp<BCX>(i0 - 2 + cc, nx);
    const int gj = wrap_or_clamp<BCY>(j0 - 2 + rr, ny);
    const size_t o = (size_t)gj * nx + gi;
    const T h = Yin[o];
    s.f[0][rr][cc] = h;
    s.f[1][rr][cc] = Yin[N + o];
    s.f[2][rr][cc] = Yin[2 * N + o];
    s.f[3][rr][cc] = Yin[3 * N + o];
    s.f[4][rr][cc] = Yin[4 * N + o];
    s.f[5][rr][cc] = bplane[o];
    s.f[6][rr][cc] = recip_staged(h);
  }

  // Own-node operands fetched before the barrier.
  const int i = i0 + tx;
  T base[RPT][5];  // pair 1: unused (taken from LDS); pair 2: q at the node
  T accr[RPT][5];  // pair 2: acc at the node
  if (PAIR == 2) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int j = j0 + ty + k * THREAD_ROWS;
      // q is needed at every node whose intermediate stage is formed, including
      // periodic images past a ragged tile edge; acc only at owned nodes.
      if (on_axis<BCX>(i, nx) && on_axis<BCY>(j, ny)) {
        const size_t ow = (size_t)wrap_or_clamp<BCY>(j, ny) * nx + wrap_or_clamp<BCX>(i, nx);
#pragma unroll
        for (int f = 0; f < 5; ++f) base[k][f] = qn[f * N + ow];
      }
      if (i < nx && j < ny) {
        const size_t o = (size_t)j * nx + i;
#pragma unroll
        for (int f = 0; f < 5; ++f) accr[k][f] = acc_io[f * N + o];
      }
    }
  }
  // Ring node handled by this thread (if any) and, for pair 2, its q.
  int ring_r = -1, ring_c = -1, ring_i = 0, ring_j = 0;
  bool ring_valid = false;
  if (tid < RING) {
    int r1, c1;
    if (tid < TILE_X + 2) {
      r1 = 0;
      c1 = tid;
    } else if (tid < 2 * (TILE_X + 2)) {
      r1 = TY + 1;
      c1 = tid - (TILE_X + 2);
    } else {
      const int qd = tid - 2 * (TILE_X + 2);
      if (qd < TY) {
        r1 = qd + 1;
        c1 = 0;
      } else {
        r1 = qd - TY + 1;
        c1 = TILE_X + 1;
      }
    }
    ring_r = r1 + 1;
    ring_c = c1 + 1;
    ring_i = i0 - 1 + c1;
    ring_j = j0 - 1 + r1;
    ring_valid = on_axis<BCX>(ring_i, nx) && on_axis<BCY>(ring_j, ny);
  }
  T ring_base[5];
  if (PAIR == 2 && ring_valid) {
    const size_t o = (size_t)wrap_or_clamp<BCY>(ring_j, ny) * nx + wrap_or_clamp<BCX>(ring_i, nx);
#pragma unroll
    for (int f = 0; f < 5; ++f) ring_base[f] = qn[f * N + o];
  }
  __syncthreads();

  // 2. First evaluation on the tile and the ring; keep the intermediate stage
  //    in registers until every thread is done reading the input planes.
  T mid[RPT][5];
  bool in_dom[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    // keep the evaluations of different rows apart: interleaving them costs
    // more registers than it hides latency
    __builtin_amdgcn_sched_barrier(0);
    const int lr = ty + k * THREAD_ROWS;
    const int j = j0 + lr;
    in_dom[k] = on_axis<BCX>(i, nx) && on_axis<BCY>(j, ny);
    if (!in_dom[k]) continue;
    Node<T> cnode;
    const Rates<T> kk = tile_eval<T, BCX, BCY, SRC>(s, lr + 2, tx + 2, i, j, gc, t1, cnode);
    const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
    if (PAIR == 1) {
      const T yv[5] = {cnode.h, cnode.u, cnode.v, cnode.w, cnode.eta};
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        base[k][f] = yv[f];
        accr[k][f] = yv[f] + c1_acc * kv[f];
        mid[k][f] = yv[f] + c1_y * kv[f];
      }
    } else {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        accr[k][f] = accr[k][f] + c1_acc * kv[f];
        mid[k][f] = base[k][f] + c1_y * kv[f];
      }
    }
  }
  T ring_mid[5];
  __builtin_amdgcn_sched_barrier(0);
  if (ring_valid) {
    Node<T> cnode;
    const Rates<T> kk = tile_eval<T, BCX, BCY, SRC>(s, ring_r, ring_c, ring_i, ring_j, gc, t1, cnode);
    const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
    const T yv[5] = {cnode.h, cnode.u, cnode.v, cnode.w, cnode.eta};
#pragma unroll
    for (int f = 0; f < 5; ++f) ring_mid[f] = (PAIR == 1 ? yv[f] : ring_base[f]) + c1_y * kv[f];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    if (!in_dom[k]) continue;
    const int r = ty + k * THREAD_ROWS + 2, c = tx + 2;
    if (SAVE) {
      const int j = j0 + ty + k * THREAD_ROWS;
      if (i < nx && j < ny) {
#pragma unroll
        for (int f = 0; f < 5; ++f) ysave[f * N + (size_t)j * nx + i] = mid[k][f];
      }
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) s.f[f][r][c] = mid[k][f];
    s.f[6][r][c] = recip_staged(mid[k][0]);
  }
  if (ring_valid) {
#pragma unroll
    for (int f = 0; f < 5; ++f) s.f[f][ring_r][ring_c] = ring_mid[f];
    s.f[6][ring_r][ring_c] = recip_staged(ring_mid[0]);
  }
  __syncthreads();

  // 3. Second evaluation on the tile and the outputs.
  int health = 0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    __builtin_amdgcn_sched_barrier(0);
    const int lr = ty + k * THREAD_ROWS;
    const int j = j0 + lr;
    if (i >= nx || j >= ny) continue;
    Node<T> cnode;
    const Rates<T> kk = tile_eval<T, BCX, BCY, SRC>(s, lr + 2, tx + 2, i, j, gc, t2, cnode);
    const T kv[5] = {kk.h, kk.u, kk.v, kk.w, kk.eta};
    const size_t o = (size_t)j * nx + i;
    if (PAIR == 1) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        acc_io[f * N + o] = accr[k][f] + c2_acc * kv[f];
        yb_out[f * N + o] = base[k][f] + c2_y * kv[f];
      }
    } else {
      T nv[5];
      T* dst = SAVE ? qout : acc_io;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        nv[f] = accr[k][f] + c2_acc * kv[f];
        dst[f * N + o] = nv[f];
      }
      if (!(nv[0] > T(0))) health |= FLAG_NONPOS;
      const T sum = nv[0] + nv[1] + nv[2] + nv[3] + nv[4];
      if (!isfinite(sum)) health |= FLAG_NONFINITE;
    }
  }
  if (PAIR == 2 && health) atomicOr(flag, health);
}

template <typename T, int BCX, int BCY, int PAIR, bool SRC, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void pair_kernel(const GridConst gc, const T* __restrict__ Yin,
                                                             const T* __restrict__ bplane, const T* __restrict__ qn,
                                                             T* acc_io, T* __restrict__ yb_out, T c1_acc, T c1_y,
                                                             T c2_acc, T c2_y, double t1, double t2,
                                                             int* __restrict__ flag) {
  __shared__ PairSmem<T, TY> s;
  const int ntx = (gc.nx + TILE_X - 1) / TILE_X;
  const int nty = (gc.ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  pair_tile<T, BCX, BCY, PAIR, SRC, TY>(s, gc, (tile % ntx) * TILE_X, (tile / ntx) * TY, Yin, bplane, qn, acc_io,
                                        yb_out, c1_acc, c1_y, c2_acc, c2_y, t1, t2, flag);
}

// Pair kernel of the adjoint's segment recomputation (no source terms): the
// same tile code with the intermediate stages saved (see pair_tile, SAVE).
template <typename T, int BCX, int BCY, int PAIR, int TY>
__global__ __launch_bounds__(STAGE_THREADS) void pair_save_kernel(const GridConst gc, const T* __restrict__ Yin,
                                                                  const T* __restrict__ bplane,
                                                                  const T* __restrict__ qn, T* acc_io,
                                                                  T* __restrict__ yb_out, T* __restrict__ ysave,
                                                                  T* __restrict__ qout, T c1_acc, T c1_y, T c2_acc,
                                                                  T c2_y, int* __restrict__ flag) {
  __shared__ PairSmem<T, TY> s;
  const int ntx = (gc.nx + TILE_X - 1) / TILE_X;
  const int nty = (gc.ny + TY - 1) / TY;
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  pair_tile<T, BCX, BCY, PAIR, false, TY, true>(s, gc, (tile % ntx) * TILE_X, (tile / ntx) * TY, Yin, bplane, qn,
                                                acc_io, yb_out, c1_acc, c1_y, c2_acc, c2_y, 0.0, 0.0, flag, ysave,
                                                qout);
}

}  // namespace sgn
