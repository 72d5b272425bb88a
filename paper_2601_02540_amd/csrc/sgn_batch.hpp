// sgn_batch.hpp -- an ensemble of independent problems in one launch per RK4
// step (step tiles) or per stage pair (pair tiles).
//
// Every instance has its own grid size, boundary types, spacing, g, lambda and
// time step.  The tiles of all instances form one work list (instance-major,
// row-major tiles within an instance), cut into eight contiguous ranges, one per
// XCD, so tiles of the same instance (and their shared halo rows) stay in one
// L2.  Each work item runs the same tile code as the single-problem kernels,
// with the boundary variant chosen per instance at run time (uniform per
// workgroup).  A launch has either one workgroup per work item or a persistent
// grid of workgroups that walks the list.
#pragma once

#include "sgn_fused.hpp"
#include "sgn_pair.hpp"

namespace sgn {

struct InstDesc {
  GridConst gc;
  double dt;
  int tile_base;  // first work item of this instance
  int ntx, nty;   // tiles per axis
  int pad;
  void* q;        // caller's state
  void* acc;      // scratch state (second buffer of the ping-pong)
  void* yb;       // scratch stage plane set
  const void* b;  // bathymetry copy
};

template <typename T, int PAIR, int TY, int BCX, int BCY>
__device__ __forceinline__ void batch_tile(PairSmem<T, TY>& s, const InstDesc& d, int i0, int j0, int parity,
                                           int* flag) {
  T* q = (T*)d.q;
  T* acc = (T*)d.acc;
  T* cur = parity ? acc : q;
  T* oth = parity ? q : acc;
  const T* b = (const T*)d.b;
  T* yb = (T*)d.yb;
  const double dt = d.dt;
  if (PAIR == 1)
    pair_tile<T, BCX, BCY, 1, false, TY>(s, d.gc, i0, j0, cur, b, nullptr, oth, yb, T(dt / 6.0), T(dt / 2.0),
                                         T(dt / 3.0), T(dt / 2.0), 0.0, 0.0, flag);
  else
    pair_tile<T, BCX, BCY, 2, false, TY>(s, d.gc, i0, j0, yb, b, cur, oth, nullptr, T(dt / 3.0), T(dt),
                                         T(dt / 6.0), T(0.0), 0.0, 0.0, flag);
}

// Work item w of a stage pair.
template <typename T, int PAIR, int TY>
__device__ __forceinline__ void batch_pair_item(PairSmem<T, TY>& s, const InstDesc* __restrict__ desc,
                                                const int* __restrict__ work_inst, int w, int parity,
                                                int* __restrict__ flags) {
  const int inst = work_inst[w];
  const InstDesc d = desc[inst];
  const int t = w - d.tile_base;
  const int i0 = (t % d.ntx) * TILE_X;
  const int j0 = (t / d.ntx) * TY;
  switch (d.gc.bc_x * 2 + d.gc.bc_y) {
    case 0: batch_tile<T, PAIR, TY, 0, 0>(s, d, i0, j0, parity, flags + inst); break;
    case 1: batch_tile<T, PAIR, TY, 0, 1>(s, d, i0, j0, parity, flags + inst); break;
    case 2: batch_tile<T, PAIR, TY, 1, 0>(s, d, i0, j0, parity, flags + inst); break;
    default: batch_tile<T, PAIR, TY, 1, 1>(s, d, i0, j0, parity, flags + inst); break;
  }
}

// parity 0: state in q, written to acc; parity 1: state in acc, written to q.
// PERSIST: a persistent grid (a multiple of 8 workgroups) walks the list, one
// contiguous range per XCD.  Otherwise one workgroup per work item (a grid of
// nwork), dealt to the XCDs in the same contiguous ranges; such a kernel holds
// no loop-invariant state across tiles, so it needs fewer registers and runs
// at a higher occupancy.
template <typename T, int PAIR, int TY, bool PERSIST>
__global__ __launch_bounds__(STAGE_THREADS) void batch_pair_kernel(const InstDesc* __restrict__ desc,
                                                                   const int* __restrict__ work_inst, int nwork,
                                                                   int parity, int* __restrict__ flags) {
  __shared__ PairSmem<T, TY> s;
  if (!PERSIST) {
    batch_pair_item<T, PAIR, TY>(s, desc, work_inst, xcd_tile(blockIdx.x, nwork), parity, flags);
    return;
  }
  const int xcd = blockIdx.x & 7;
  const int k = blockIdx.x >> 3;
  const int blocks_per_xcd = gridDim.x >> 3;
  const int start = (int)((long long)nwork * xcd / 8);
  const int end = (int)((long long)nwork * (xcd + 1) / 8);
  for (int w = start + k; w < end; w += blocks_per_xcd) {
    batch_pair_item<T, PAIR, TY>(s, desc, work_inst, w, parity, flags);
    __syncthreads();
  }
}

// Work item w of one RK4 step by the step tile (tiles of TX x TY, StepGeom).
template <typename T, int TY>
__device__ __forceinline__ void batch_step_item(StepSmem<T, TY, 1>& s, const InstDesc* __restrict__ desc,
                                                const int* __restrict__ work_inst, int w, int parity,
                                                int* __restrict__ flags) {
  constexpr int TX = StepGeom<TY>::TX;
  const int inst = work_inst[w];
  const InstDesc d = desc[inst];
  const int t = w - d.tile_base;
  const int i0 = (t % d.ntx) * TX;
  const int j0 = (t / d.ntx) * TY;
  const T* cur = (const T*)(parity ? d.acc : d.q);
  T* oth = (T*)(parity ? d.q : d.acc);
  const T* b = (const T*)d.b;
  const double dt = d.dt;
  const T c6 = T(dt / 6.0), c3 = T(dt / 3.0), c2 = T(dt / 2.0), c1 = T(dt);
  switch (d.gc.bc_x * 2 + d.gc.bc_y) {
    case 0: step_tile<T, 0, 0, false, TY, false>(s, d.gc, i0, j0, cur, b, oth, c6, c3, c2, c1, 0.0, dt, flags + inst, nullptr); break;
    case 1: step_tile<T, 0, 1, false, TY, false>(s, d.gc, i0, j0, cur, b, oth, c6, c3, c2, c1, 0.0, dt, flags + inst, nullptr); break;
    case 2: step_tile<T, 1, 0, false, TY, false>(s, d.gc, i0, j0, cur, b, oth, c6, c3, c2, c1, 0.0, dt, flags + inst, nullptr); break;
    default: step_tile<T, 1, 1, false, TY, false>(s, d.gc, i0, j0, cur, b, oth, c6, c3, c2, c1, 0.0, dt, flags + inst, nullptr); break;
  }
}

// One RK4 step of every instance.  parity and PERSIST as for batch_pair_kernel.
template <typename T, int TY, bool PERSIST>
__global__ __launch_bounds__(STAGE_THREADS) void batch_step_kernel(const InstDesc* __restrict__ desc,
                                                                   const int* __restrict__ work_inst, int nwork,
                                                                   int parity, int* __restrict__ flags) {
  __shared__ StepSmem<T, TY, 1> s;
  if (!PERSIST) {
    batch_step_item<T, TY>(s, desc, work_inst, xcd_tile(blockIdx.x, nwork), parity, flags);
    return;
  }
  const int xcd = blockIdx.x & 7;
  const int k = blockIdx.x >> 3;
  const int blocks_per_xcd = gridDim.x >> 3;  // the grid is a multiple of 8
  const int start = (int)((long long)nwork * xcd / 8);
  const int end = (int)((long long)nwork * (xcd + 1) / 8);
  for (int w = start + k; w < end; w += blocks_per_xcd) {
    batch_step_item<T, TY>(s, desc, work_inst, w, parity, flags);
    __syncthreads();
  }
}

}  // namespace sgn
