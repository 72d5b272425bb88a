// sgn_lib.hip -- C ABI of include/sgn.h: context, validation, launches, graphs.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sgn.h"
#include "sgn_internal.hpp"
#include "sgn_reduce.hpp"
#include "sgn_fused.hpp"
#include "sgn_pair.hpp"
#include "sgn_stage.hpp"

namespace {

thread_local std::string g_create_error;

// Steps captured per graph replay (even, so the pair path returns to q).
constexpr int GRAPH_STEPS = 8;

using sgn_host::GraphCache;

}  // namespace

namespace sgn_host {

sgn_status fail(sgn_ctx* c, sgn_status st, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return st;
}

sgn_status hip_fail(sgn_ctx* c, hipError_t e, const char* what) {
  return fail(c, SGN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace sgn_host

namespace {

using sgn_host::fail;
using sgn_host::hip_fail;

#define HIPCHK(c, expr) SGN_HIPCHK(c, expr)

double axis_spacing(int n, double lo, double hi, int bc) {
  return bc == SGN_PERIODIC ? (hi - lo) / n : (hi - lo) / (n - 1);
}

void destroy_graphs(sgn_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = GraphCache{};
  }
  if (c->relax_graph.exec) (void)hipGraphExecDestroy(c->relax_graph.exec);
  c->relax_graph = GraphCache{};
  if (c->totals_graph.exec) (void)hipGraphExecDestroy(c->totals_graph.exec);
  c->totals_graph = GraphCache{};
  c->totals_series = nullptr;
  if (c->fs.graph.exec) (void)hipGraphExecDestroy(c->fs.graph.exec);
  c->fs.graph = GraphCache{};
}

int reduce_blocks(const sgn_ctx* c) { return c->p.ny < sgn::RED_MAX_BLOCKS ? c->p.ny : sgn::RED_MAX_BLOCKS; }

// ---------------------------------------------------------------------------
// Stage launches

template <typename T, int MODE, int TY>
hipError_t launch_stage_ty(const sgn_ctx* c, hipStream_t s, const void* Y, const void* qn, void* acc, void* out,
                           double c_acc, double c_y, double t) {
  const int ntx = (c->p.nx + sgn::TILE_X - 1) / sgn::TILE_X;
  const int nty = (c->p.ny + TY - 1) / TY;
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
  const bool src = c->p.source == SGN_SRC_MMS;
  const T* Yp = (const T*)Y;
  const T* bp = (const T*)c->b;
  const T* qp = (const T*)qn;
  T* ap = (T*)acc;
  T* op = (T*)out;
#define SGN_LAUNCH(BX, BY, S)                                                                             \
  hipLaunchKernelGGL((sgn::stage_kernel<T, BX, BY, MODE, S, TY>), grid, block, 0, s, c->gc, Yp, bp, qp, ap, op, \
                     (T)c_acc, (T)c_y, t, c->flag)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (!src) {
    if (bx == 0 && by == 0) SGN_LAUNCH(0, 0, false);
    else if (bx == 0 && by == 1) SGN_LAUNCH(0, 1, false);
    else if (bx == 1 && by == 0) SGN_LAUNCH(1, 0, false);
    else SGN_LAUNCH(1, 1, false);
  } else {
    if (bx == 0 && by == 0) SGN_LAUNCH(0, 0, true);
    else if (bx == 0 && by == 1) SGN_LAUNCH(0, 1, true);
    else if (bx == 1 && by == 0) SGN_LAUNCH(1, 0, true);
    else SGN_LAUNCH(1, 1, true);
  }
#undef SGN_LAUNCH
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_stage(const sgn_ctx* c, hipStream_t s, const void* Y, const void* qn, void* acc, void* out,
                        double c_acc, double c_y, double t) {
  if (c->p.dtype == SGN_F64) {
    if (c->tile_y == 16) return launch_stage_ty<double, MODE, 16>(c, s, Y, qn, acc, out, c_acc, c_y, t);
    return launch_stage_ty<double, MODE, 8>(c, s, Y, qn, acc, out, c_acc, c_y, t);
  }
  if (c->tile_y == 16) return launch_stage_ty<float, MODE, 16>(c, s, Y, qn, acc, out, c_acc, c_y, t);
  return launch_stage_ty<float, MODE, 8>(c, s, Y, qn, acc, out, c_acc, c_y, t);
}

template <typename T, int PAIR, int TY>
hipError_t launch_pair_ty(const sgn_ctx* c, hipStream_t s, const void* Yin, const void* qn, void* acc_io, void* yb,
                          double c1_acc, double c1_y, double c2_acc, double c2_y, double t1, double t2) {
  const int ntx = (c->p.nx + sgn::TILE_X - 1) / sgn::TILE_X;
  const int nty = (c->p.ny + TY - 1) / TY;
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
  const bool src = c->p.source == SGN_SRC_MMS;
  const T* Yp = (const T*)Yin;
  const T* bp = (const T*)c->b;
  const T* qp = (const T*)qn;
  T* ap = (T*)acc_io;
  T* yp = (T*)yb;
#define SGN_LAUNCH(BX, BY, S)                                                                                 \
  hipLaunchKernelGGL((sgn::pair_kernel<T, BX, BY, PAIR, S, TY>), grid, block, 0, s, c->gc, Yp, bp, qp, ap, yp, \
                     (T)c1_acc, (T)c1_y, (T)c2_acc, (T)c2_y, t1, t2, c->flag)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (!src) {
    if (bx == 0 && by == 0) SGN_LAUNCH(0, 0, false);
    else if (bx == 0 && by == 1) SGN_LAUNCH(0, 1, false);
    else if (bx == 1 && by == 0) SGN_LAUNCH(1, 0, false);
    else SGN_LAUNCH(1, 1, false);
  } else {
    if (bx == 0 && by == 0) SGN_LAUNCH(0, 0, true);
    else if (bx == 0 && by == 1) SGN_LAUNCH(0, 1, true);
    else if (bx == 1 && by == 0) SGN_LAUNCH(1, 0, true);
    else SGN_LAUNCH(1, 1, true);
  }
#undef SGN_LAUNCH
  return hipGetLastError();
}

template <int PAIR>
hipError_t launch_pair(const sgn_ctx* c, hipStream_t s, const void* Yin, const void* qn, void* acc_io, void* yb,
                       double c1_acc, double c1_y, double c2_acc, double c2_y, double t1, double t2) {
  if (c->p.dtype == SGN_F64) {
    if (c->tile_y == 16) return launch_pair_ty<double, PAIR, 16>(c, s, Yin, qn, acc_io, yb, c1_acc, c1_y, c2_acc, c2_y, t1, t2);
    return launch_pair_ty<double, PAIR, 8>(c, s, Yin, qn, acc_io, yb, c1_acc, c1_y, c2_acc, c2_y, t1, t2);
  }
  if (c->tile_y == 16) return launch_pair_ty<float, PAIR, 16>(c, s, Yin, qn, acc_io, yb, c1_acc, c1_y, c2_acc, c2_y, t1, t2);
  return launch_pair_ty<float, PAIR, 8>(c, s, Yin, qn, acc_io, yb, c1_acc, c1_y, c2_acc, c2_y, t1, t2);
}

template <typename T, int TY>
hipError_t launch_fused_ty(const sgn_ctx* c, hipStream_t s, const void* qin, void* qout, double dt, double t0,
                           void* ysave, double* rpart, int epi) {
  constexpr int TX = sgn::StepGeom<TY>::TX;
  const int ntx = (c->p.nx + TX - 1) / TX;
  const int nty = (c->p.ny + TY - 1) / TY;
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
  const bool src = c->p.source == SGN_SRC_MMS;
  const T* qp = (const T*)qin;
  const T* bp = (const T*)c->b;
  T* op = (T*)qout;
  T* ys = (T*)ysave;
#define SGN_LAUNCH_K(BX, BY, S, SV, RX)                                                                         \
  do {                                                                                                         \
    if (c->prof_start)                                                                                         \
      hipExtLaunchKernelGGL((sgn::step_kernel<T, BX, BY, S, TY, SV, RX>), grid, block, 0, s, c->prof_start,    \
                            c->prof_stop, 0, c->gc, qp, bp, op, (T)(dt / 6.0), (T)(dt / 3.0), (T)(dt / 2.0),  \
                            (T)dt, t0, dt, c->flag, ys, rpart);                                               \
    else                                                                                                       \
      hipLaunchKernelGGL((sgn::step_kernel<T, BX, BY, S, TY, SV, RX>), grid, block, 0, s, c->gc, qp, bp, op,   \
                         (T)(dt / 6.0), (T)(dt / 3.0), (T)(dt / 2.0), (T)dt, t0, dt, c->flag, ys, rpart);     \
  } while (0)
#define SGN_LAUNCH(BX, BY, S) SGN_LAUNCH_K(BX, BY, S, false, sgn::EPI_NONE)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (rpart && epi == sgn::EPI_RELAX) {  // relaxation sums (no source terms, no stage saving)
    if (bx == 0 && by == 0) SGN_LAUNCH_K(0, 0, false, false, sgn::EPI_RELAX);
    else if (bx == 0 && by == 1) SGN_LAUNCH_K(0, 1, false, false, sgn::EPI_RELAX);
    else if (bx == 1 && by == 0) SGN_LAUNCH_K(1, 0, false, false, sgn::EPI_RELAX);
    else SGN_LAUNCH_K(1, 1, false, false, sgn::EPI_RELAX);
  } else if (rpart) {  // mass and energy of the new state (no source terms, no stage saving)
    if (bx == 0 && by == 0) SGN_LAUNCH_K(0, 0, false, false, sgn::EPI_TOTALS);
    else if (bx == 0 && by == 1) SGN_LAUNCH_K(0, 1, false, false, sgn::EPI_TOTALS);
    else if (bx == 1 && by == 0) SGN_LAUNCH_K(1, 0, false, false, sgn::EPI_TOTALS);
    else SGN_LAUNCH_K(1, 1, false, false, sgn::EPI_TOTALS);
  } else if (ys) {  // stage saving (no source terms; not on 32 x 24 tiles)
    if constexpr (TY != 24) {
      if (bx == 0 && by == 0) SGN_LAUNCH_K(0, 0, false, true, sgn::EPI_NONE);
      else if (bx == 0 && by == 1) SGN_LAUNCH_K(0, 1, false, true, sgn::EPI_NONE);
      else if (bx == 1 && by == 0) SGN_LAUNCH_K(1, 0, false, true, sgn::EPI_NONE);
      else SGN_LAUNCH_K(1, 1, false, true, sgn::EPI_NONE);
    }
  } else if (!src) {
    if (bx == 0 && by == 0) SGN_LAUNCH(0, 0, false);
    else if (bx == 0 && by == 1) SGN_LAUNCH(0, 1, false);
    else if (bx == 1 && by == 0) SGN_LAUNCH(1, 0, false);
    else SGN_LAUNCH(1, 1, false);
  } else if constexpr (TY != 24) {  // source terms (not on 32 x 24 tiles)
    if (bx == 0 && by == 0) SGN_LAUNCH(0, 0, true);
    else if (bx == 0 && by == 1) SGN_LAUNCH(0, 1, true);
    else if (bx == 1 && by == 0) SGN_LAUNCH(1, 0, true);
    else SGN_LAUNCH(1, 1, true);
  }
#undef SGN_LAUNCH
#undef SGN_LAUNCH_K
  return hipGetLastError();
}

// One RK4 step in one kernel, from state buffer `qin` into `qout` (distinct);
// with `ysave`, also the stage states Y2, Y3, Y4 (three consecutive states);
// with `rpart`, also the epilogue sums `epi` (sgn::EPI_*) of every tile.
// Stage saving and source terms run on 32 x 16 tiles where the context's
// step tile is 32 x 24 (their 32 x 24 instances reach the register limit);
// every tile shape forms the same values.
hipError_t launch_fused(const sgn_ctx* c, hipStream_t s, const void* qin, void* qout, double dt, double t0,
                        void* ysave = nullptr, double* rpart = nullptr, int epi = sgn::EPI_NONE) {
  const int ty = c->step_tile == 24 && (ysave || c->p.source == SGN_SRC_MMS) ? 16 : c->step_tile;
  if (c->p.dtype == SGN_F64) {
    if (ty == 24) return launch_fused_ty<double, 24>(c, s, qin, qout, dt, t0, ysave, rpart, epi);
    if (ty == 16) return launch_fused_ty<double, 16>(c, s, qin, qout, dt, t0, ysave, rpart, epi);
    return launch_fused_ty<double, 8>(c, s, qin, qout, dt, t0, ysave, rpart, epi);
  }
  if (ty == 24) return launch_fused_ty<float, 24>(c, s, qin, qout, dt, t0, ysave, rpart, epi);
  if (ty == 16) return launch_fused_ty<float, 16>(c, s, qin, qout, dt, t0, ysave, rpart, epi);
  return launch_fused_ty<float, 8>(c, s, qin, qout, dt, t0, ysave, rpart, epi);
}

// Two RK4 steps on the fused path: q -> acc -> q.
hipError_t enqueue_fused_double_step(const sgn_ctx* c, hipStream_t s, void* q, double dt, double t) {
  hipError_t e = launch_fused(c, s, q, c->acc, dt, t);
  if (e) return e;
  return launch_fused(c, s, c->acc, q, dt, t + dt);
}

// One RK4 step with two fused stage pairs, from state buffer `cur` into `oth`
// (which also carries acc between the two launches).
hipError_t enqueue_pair_step(const sgn_ctx* c, hipStream_t s, void* cur, void* oth, double dt, double t) {
  hipError_t e = launch_pair<1>(c, s, cur, nullptr, oth, c->yb, dt / 6.0, dt / 2.0, dt / 3.0, dt / 2.0, t, t + dt / 2.0);
  if (e) return e;
  return launch_pair<2>(c, s, c->yb, cur, oth, nullptr, dt / 3.0, dt, dt / 6.0, 0.0, t + dt / 2.0, t + dt);
}

// Two RK4 steps on the pair path: q -> acc -> q.
hipError_t enqueue_pair_double_step(const sgn_ctx* c, hipStream_t s, void* q, double dt, double t) {
  hipError_t e = enqueue_pair_step(c, s, q, c->acc, dt, t);
  if (e) return e;
  return enqueue_pair_step(c, s, c->acc, q, dt, t + dt);
}

// One classical RK4 step in three-register form (q, acc, and two stage planes):
//   k1 = f(q),  acc = q + dt/6 k1,   Ya = q + dt/2 k1
//   k2 = f(Ya), acc += dt/3 k2,      Yb = q + dt/2 k2
//   k3 = f(Yb), acc += dt/3 k3,      Ya = q + dt k3
//   k4 = f(Ya), q = acc + dt/6 k4
hipError_t enqueue_step(const sgn_ctx* c, hipStream_t s, void* q, double dt, double t) {
  hipError_t e;
  if ((e = launch_stage<sgn::MODE_FIRST>(c, s, q, nullptr, c->acc, c->ya, dt / 6.0, dt / 2.0, t))) return e;
  if ((e = launch_stage<sgn::MODE_MID>(c, s, c->ya, q, c->acc, c->yb, dt / 3.0, dt / 2.0, t + dt / 2.0))) return e;
  if ((e = launch_stage<sgn::MODE_MID>(c, s, c->yb, q, c->acc, c->ya, dt / 3.0, dt, t + dt / 2.0))) return e;
  return launch_stage<sgn::MODE_LAST>(c, s, c->ya, nullptr, c->acc, q, dt / 6.0, 0.0, t + dt);
}

// Two RK4 steps that leave the state in q, on the pair or the fused path.
hipError_t enqueue_double_step(const sgn_ctx* c, hipStream_t s, void* q, double dt, double t) {
  if (c->step_path == SGN_PATH_FUSED) return enqueue_fused_double_step(c, s, q, dt, t);
  return enqueue_pair_double_step(c, s, q, dt, t);
}

bool double_steps(const sgn_ctx* c) { return c->step_path == SGN_PATH_PAIRS || c->step_path == SGN_PATH_FUSED; }

// Enqueues `steps` RK4 steps on the context's step path (an even count on the
// pair and fused paths).
hipError_t enqueue_steps(const sgn_ctx* c, hipStream_t s, void* q, double dt, int steps, double t0) {
  hipError_t e = hipSuccess;
  if (double_steps(c)) {
    for (int k = 0; k + 1 < steps && e == hipSuccess; k += 2) e = enqueue_double_step(c, s, q, dt, t0 + k * dt);
  } else {
    for (int k = 0; k < steps && e == hipSuccess; ++k) e = enqueue_step(c, s, q, dt, t0 + k * dt);
  }
  return e;
}

sgn_status get_graph(sgn_ctx* c, int slot, void* q, double dt, int steps, hipGraphExec_t* out) {
  GraphCache& g = c->graphs[slot];
  if (g.exec && g.q == q && g.dt == dt && g.steps == steps && g.path == c->step_path && g.tile_y == c->tile_y &&
      g.step_tile == c->step_tile) {
    *out = g.exec;
    return SGN_OK;
  }
  if (g.exec) {
    (void)hipGraphExecDestroy(g.exec);
    g = GraphCache{};
  }
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = enqueue_steps(c, c->cap_stream, q, dt, steps, 0.0);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(c, le, "stage launch during capture");
  }
  if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
  g.exec = exec;
  g.q = q;
  g.dt = dt;
  g.steps = steps;
  g.path = c->step_path;
  g.tile_y = c->tile_y;
  g.step_tile = c->step_tile;
  *out = exec;
  return SGN_OK;
}

}  // namespace

namespace sgn_host {

// Copies the health flag and `nres` result doubles to host, synchronizes, and
// converts a raised flag into a status (clearing it).
sgn_status sync_results(sgn_ctx* c, int nres) {
  if (nres > 0) HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, nres * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->host_flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int f = *c->host_flag;
  if (f) {
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f & sgn::FLAG_BADINDEX) return fail(c, SGN_E_ARG, "a gauge index lies outside the grid");
    if (f & sgn::FLAG_NONFINITE) return fail(c, SGN_E_NONFINITE, "a step produced a non-finite value");
    return fail(c, SGN_E_NONPOS_DEPTH, "a step produced h <= 0 (the method has no wetting/drying)");
  }
  return SGN_OK;
}

sgn_status check_ctx(sgn_ctx* c, bool need_b) {
  if (!c) return SGN_E_ARG;
  if (need_b && !c->b_set) return fail(c, SGN_E_STATE, "bathymetry not set (call sgn_set_bathymetry first)");
  return SGN_OK;
}

hipError_t launch_stage_mode(const sgn_ctx* c, hipStream_t s, int mode, const void* Y, const void* qn, void* acc,
                             void* out, double c_acc, double c_y, double t) {
  switch (mode) {
    case sgn::MODE_RHS: return launch_stage<sgn::MODE_RHS>(c, s, Y, qn, acc, out, c_acc, c_y, t);
    case sgn::MODE_FIRST: return launch_stage<sgn::MODE_FIRST>(c, s, Y, qn, acc, out, c_acc, c_y, t);
    case sgn::MODE_MID: return launch_stage<sgn::MODE_MID>(c, s, Y, qn, acc, out, c_acc, c_y, t);
    default: return launch_stage<sgn::MODE_LAST>(c, s, Y, qn, acc, out, c_acc, c_y, t);
  }
}

hipError_t enqueue_step_into(const sgn_ctx* c, hipStream_t s, const void* cur, void* oth, double dt, double t,
                             void* ysave, double* rpart, int epi) {
  return ::launch_fused(c, s, cur, oth, dt, t, ysave, rpart, epi);
}

int step_tiles(const sgn_ctx* c) {
  const int ty = c->step_tile;
  const int tx = ty == 8 ? sgn::StepGeom<8>::TX : sgn::StepGeom<16>::TX;
  return ((c->p.nx + tx - 1) / tx) * ((c->p.ny + ty - 1) / ty);
}

sgn_status ensure_tile_partials(sgn_ctx* c) {
  // room for the largest tile count of the tile shapes (32 x 24 has the fewest tiles)
  const size_t nx = (size_t)c->p.nx, ny = (size_t)c->p.ny;
  const size_t tiles = std::max(((nx + 31) / 32) * ((ny + 15) / 16), ((nx + 63) / 64) * ((ny + 7) / 8));
  if (c->tile_partials_cap >= 4 * tiles) return SGN_OK;
  SGN_HIPCHK(c, hipStreamSynchronize(c->stream));  // earlier steps may still write the old buffer
  if (c->tile_partials) (void)hipFree(c->tile_partials);
  c->tile_partials = nullptr;
  c->tile_partials_cap = 0;
  destroy_graphs(c);  // captured graphs hold the old address
  if (hipMalloc((void**)&c->tile_partials, 4 * tiles * sizeof(double)) != hipSuccess)
    return fail(c, SGN_E_ALLOC, "per-tile partial sums");
  c->tile_partials_cap = 4 * tiles;
  return SGN_OK;
}

hipError_t enqueue_pair_step(const sgn_ctx* c, hipStream_t s, void* cur, void* oth, double dt, double t) {
  return ::enqueue_pair_step(c, s, cur, oth, dt, t);
}

sgn_status check_params(const sgn_params* p) {
  if (!p) return fail(nullptr, SGN_E_ARG, "params is NULL");
  if (p->nx < 4 || p->ny < 4) return fail(nullptr, SGN_E_SHAPE, "each axis needs at least 4 nodes");
  if (!(std::isfinite(p->xmin) && std::isfinite(p->xmax) && p->xmax > p->xmin && std::isfinite(p->ymin) &&
        std::isfinite(p->ymax) && p->ymax > p->ymin))
    return fail(nullptr, SGN_E_SHAPE, "domain bounds must be finite with max > min");
  if ((p->bc_x != SGN_PERIODIC && p->bc_x != SGN_REFLECTING) || (p->bc_y != SGN_PERIODIC && p->bc_y != SGN_REFLECTING))
    return fail(nullptr, SGN_E_ARG, "unknown boundary type");
  if (!(std::isfinite(p->g) && p->g > 0.0)) return fail(nullptr, SGN_E_ARG, "g must be finite and > 0");
  if (!(std::isfinite(p->lambda) && p->lambda >= 0.0)) return fail(nullptr, SGN_E_ARG, "lambda must be finite and >= 0");
  if (p->dtype != SGN_F64 && p->dtype != SGN_F32) return fail(nullptr, SGN_E_ARG, "unknown dtype");
  if (p->source != SGN_SRC_NONE && p->source != SGN_SRC_MMS) return fail(nullptr, SGN_E_ARG, "unknown source");
  const size_t N = (size_t)p->nx * (size_t)p->ny;
  if (N > ((size_t)1 << 40)) return fail(nullptr, SGN_E_SHAPE, "grid too large");
  return SGN_OK;
}

sgn::GridConst grid_const(const sgn_params& p) {
  sgn::GridConst gc{};
  gc.nx = p.nx;
  gc.ny = p.ny;
  gc.bc_x = p.bc_x;
  gc.bc_y = p.bc_y;
  gc.dx = axis_spacing(p.nx, p.xmin, p.xmax, p.bc_x);
  gc.dy = axis_spacing(p.ny, p.ymin, p.ymax, p.bc_y);
  gc.inv2dx = 1.0 / (2.0 * gc.dx);
  gc.inv2dy = 1.0 / (2.0 * gc.dy);
  gc.invdx = 1.0 / gc.dx;
  gc.invdy = 1.0 / gc.dy;
  gc.xmin = p.xmin;
  gc.ymin = p.ymin;
  gc.g = p.g;
  gc.lam = p.lambda;
  return gc;
}

}  // namespace sgn_host

namespace {

using sgn_host::sync_results;
using sgn_host::check_ctx;

template <typename T>
hipError_t launch_totals(const sgn_ctx* c, const void* q, const void* dq, int what) {
  const int nb = reduce_blocks(c);
  if (what == 0)
    hipLaunchKernelGGL((sgn::totals_partial<T, 0>), dim3(nb), dim3(sgn::RED_THREADS), 0, c->stream, c->gc,
                       (const T*)q, (const T*)c->b, (const T*)nullptr, c->partials);
  else
    hipLaunchKernelGGL((sgn::totals_partial<T, 1>), dim3(nb), dim3(sgn::RED_THREADS), 0, c->stream, c->gc,
                       (const T*)q, (const T*)c->b, (const T*)dq, c->partials);
  hipLaunchKernelGGL(sgn::totals_final, dim3(1), dim3(sgn::RED_THREADS), 0, c->stream, c->partials, nb, c->result);
  return hipGetLastError();
}


}  // namespace

extern "C" {

const char* sgn_status_string(int32_t s) {
  switch (s) {
    case SGN_OK: return "SGN_OK";
    case SGN_E_ARG: return "SGN_E_ARG";
    case SGN_E_SHAPE: return "SGN_E_SHAPE";
    case SGN_E_UNSUPPORTED: return "SGN_E_UNSUPPORTED";
    case SGN_E_HIP: return "SGN_E_HIP";
    case SGN_E_NONPOS_DEPTH: return "SGN_E_NONPOS_DEPTH";
    case SGN_E_NONFINITE: return "SGN_E_NONFINITE";
    case SGN_E_ALLOC: return "SGN_E_ALLOC";
    case SGN_E_STATE: return "SGN_E_STATE";
    default: return "SGN_E_UNKNOWN";
  }
}

const char* sgn_last_error(const sgn_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

sgn_status sgn_create(const sgn_params* p, void* stream, sgn_ctx** out) {
  if (!out) return fail(nullptr, SGN_E_ARG, "out is NULL");
  *out = nullptr;
  sgn_status pst = sgn_host::check_params(p);
  if (pst) return pst;
  const size_t N = (size_t)p->nx * (size_t)p->ny;

  sgn_ctx* c = new sgn_ctx();
  c->p = *p;
  c->N = N;
  c->esize = p->dtype == SGN_F64 ? sizeof(double) : sizeof(float);
  c->tile_y = p->dtype == SGN_F64 ? 8 : 16;  // measured best on MI355X at 4096^2
  // the step kernel's 32 x 24 tile (measured best on MI355X) once the grid has
  // enough of them to fill the GPU (four workgroups per CU); 32 x 16 below that
  c->step_tile = ((p->nx + 31) / 32) * ((p->ny + 23) / 24) >= 1024 ? 24 : 16;
  c->stream = (hipStream_t)stream;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "hipGetDevice");
  }
  c->gc = sgn_host::grid_const(*p);

  const size_t plane = N * c->esize;
  bool ok = hipMalloc(&c->b, plane) == hipSuccess && hipMalloc(&c->acc, 5 * plane) == hipSuccess &&
            hipMalloc(&c->ya, 5 * plane) == hipSuccess && hipMalloc(&c->yb, 5 * plane) == hipSuccess &&
            hipMalloc((void**)&c->partials, 4 * sgn::RED_MAX_BLOCKS * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&c->result, 8 * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&c->flag, sizeof(int)) == hipSuccess &&
            hipHostMalloc((void**)&c->host_result, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&c->host_flag, sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    sgn_destroy(c);
    return fail(nullptr, SGN_E_ALLOC, "device allocation failed");
  }
  if (hipMemsetAsync(c->flag, 0, sizeof(int), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    sgn_destroy(c);
    return fail(nullptr, SGN_E_HIP, "initial flag clear failed");
  }
  *out = c;
  return SGN_OK;
}

sgn_status sgn_destroy(sgn_ctx* c) {
  if (!c) return SGN_OK;
  (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  sgn_host::free_adjoint(c);
  sgn_host::free_fsal(c);
  if (c->b) (void)hipFree(c->b);
  if (c->acc) (void)hipFree(c->acc);
  if (c->ya) (void)hipFree(c->ya);
  if (c->yb) (void)hipFree(c->yb);
  if (c->partials) (void)hipFree(c->partials);
  if (c->tile_partials) (void)hipFree(c->tile_partials);
  if (c->series_counter) (void)hipFree(c->series_counter);
  if (c->result) (void)hipFree(c->result);
  if (c->flag) (void)hipFree(c->flag);
  if (c->host_result) (void)hipHostFree(c->host_result);
  if (c->host_flag) (void)hipHostFree(c->host_flag);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return SGN_OK;
}

sgn_status sgn_set_stream(sgn_ctx* c, void* stream) {
  if (!c) return SGN_E_ARG;
  c->stream = (hipStream_t)stream;
  destroy_graphs(c);
  return SGN_OK;
}

sgn_status sgn_spacing(const sgn_ctx* c, double* dx, double* dy) {
  if (!c || !dx || !dy) return SGN_E_ARG;
  *dx = c->gc.dx;
  *dy = c->gc.dy;
  return SGN_OK;
}

sgn_status sgn_set_bathymetry(sgn_ctx* c, const void* b) {
  if (!c) return SGN_E_ARG;
  if (!b) return fail(c, SGN_E_ARG, "b is NULL");
  HIPCHK(c, hipMemcpyAsync(c->b, b, c->N * c->esize, hipMemcpyDeviceToDevice, c->stream));
  c->b_set = true;
  return SGN_OK;
}

sgn_status sgn_init_aux(sgn_ctx* c, void* q) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  const dim3 grid((c->p.nx + 63) / 64, (c->p.ny + 3) / 4), block(256);
  if (c->p.dtype == SGN_F64)
    hipLaunchKernelGGL(sgn::init_aux_kernel<double>, grid, block, 0, c->stream, c->gc, (double*)q, (const double*)c->b);
  else
    hipLaunchKernelGGL(sgn::init_aux_kernel<float>, grid, block, 0, c->stream, c->gc, (float*)q, (const float*)c->b);
  HIPCHK(c, hipGetLastError());
  return SGN_OK;
}

sgn_status sgn_rhs(sgn_ctx* c, const void* q, void* dq, double t) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q || !dq) return fail(c, SGN_E_ARG, "q or dq is NULL");
  if (q == dq) return fail(c, SGN_E_ARG, "q and dq must not overlap");
  if (!std::isfinite(t)) return fail(c, SGN_E_ARG, "t must be finite");
  HIPCHK(c, launch_stage<sgn::MODE_RHS>(c, c->stream, q, nullptr, nullptr, dq, 0.0, 0.0, t));
  return SGN_OK;
}

sgn_status sgn_step(sgn_ctx* c, void* q, double dt, int64_t nsteps, double t0) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, SGN_E_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(c, SGN_E_ARG, "nsteps must be >= 0");
  if (!std::isfinite(t0)) return fail(c, SGN_E_ARG, "t0 must be finite");
  if (nsteps == 0) return SGN_OK;
  if (c->p.source != SGN_SRC_NONE) {
    // Stage times matter: launch directly (pairs of steps, then a single one).
    int64_t s = 0;
    if (double_steps(c))
      for (; s + 1 < nsteps; s += 2) HIPCHK(c, enqueue_double_step(c, c->stream, q, dt, t0 + (double)s * dt));
    for (; s < nsteps; ++s) HIPCHK(c, enqueue_step(c, c->stream, q, dt, t0 + (double)s * dt));
    return SGN_OK;
  }
  int64_t left = nsteps;
  if (left >= GRAPH_STEPS) {
    hipGraphExec_t ge;
    if ((st = get_graph(c, 0, q, dt, GRAPH_STEPS, &ge))) return st;
    for (; left >= GRAPH_STEPS; left -= GRAPH_STEPS) HIPCHK(c, hipGraphLaunch(ge, c->stream));
  }
  const int small = double_steps(c) ? 2 : 1;
  if (left >= small) {
    hipGraphExec_t g1;
    if ((st = get_graph(c, 1, q, dt, small, &g1))) return st;
    for (; left >= small; left -= small) HIPCHK(c, hipGraphLaunch(g1, c->stream));
  }
  // An odd final step on the pair or fused path runs as four single-stage kernels in place.
  if (left > 0) HIPCHK(c, enqueue_step(c, c->stream, q, dt, 0.0));
  return SGN_OK;
}

sgn_status sgn_prepare_step(sgn_ctx* c, void* q, double dt, int64_t nsteps) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, SGN_E_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(c, SGN_E_ARG, "nsteps must be >= 0");
  if (nsteps == 0 || c->p.source != SGN_SRC_NONE) return SGN_OK;
  // the same split as sgn_step: 8-step replays, then 1- or 2-step replays
  hipGraphExec_t ge;
  if (nsteps >= GRAPH_STEPS && (st = get_graph(c, 0, q, dt, GRAPH_STEPS, &ge))) return st;
  const int small = double_steps(c) ? 2 : 1;
  if (nsteps % GRAPH_STEPS >= small && (st = get_graph(c, 1, q, dt, small, &ge))) return st;
  return SGN_OK;
}

sgn_status sgn_set_option(sgn_ctx* c, int32_t option, int64_t value) {
  if (!c) return SGN_E_ARG;
  if (option == SGN_OPT_STEP_PATH) {
    if (value != SGN_PATH_PAIRS && value != SGN_PATH_STAGES && value != SGN_PATH_FUSED)
      return fail(c, SGN_E_ARG, "unknown step path");
    c->step_path = (int)value;
  } else if (option == SGN_OPT_TILE_Y) {
    if (value != 8 && value != 16 && value != 24) return fail(c, SGN_E_UNSUPPORTED, "tile height must be 8, 16 or 24");
    c->tile_y = value == 24 ? 16 : (int)value;
    c->step_tile = (int)value;
  } else if (option == SGN_OPT_ADJOINT_STORE) {
    if (value < 0) return fail(c, SGN_E_ARG, "adjoint storage must be >= 0 bytes");
    c->adj_store_bytes = value;
  } else {
    return fail(c, SGN_E_ARG, "unknown option");
  }
  destroy_graphs(c);
  return SGN_OK;
}

sgn_status sgn_mass_energy(sgn_ctx* c, const void* q, double* mass, double* energy) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  hipError_t e = c->p.dtype == SGN_F64 ? launch_totals<double>(c, q, nullptr, 0) : launch_totals<float>(c, q, nullptr, 0);
  HIPCHK(c, e);
  if ((st = sync_results(c, 2))) return st;
  if (mass) *mass = c->host_result[0];
  if (energy) *energy = c->host_result[1];
  return SGN_OK;
}

sgn_status sgn_mass(sgn_ctx* c, const void* q, double* out) {
  if (!out) return c ? fail(c, SGN_E_ARG, "out is NULL") : SGN_E_ARG;
  return sgn_mass_energy(c, q, out, nullptr);
}

sgn_status sgn_energy(sgn_ctx* c, const void* q, double* out) {
  if (!out) return c ? fail(c, SGN_E_ARG, "out is NULL") : SGN_E_ARG;
  return sgn_mass_energy(c, q, nullptr, out);
}

sgn_status sgn_rates(sgn_ctx* c, const void* q, double* mass_rate, double* energy_rate) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  if (c->p.source != SGN_SRC_NONE) return fail(c, SGN_E_UNSUPPORTED, "rates are defined without source terms");
  HIPCHK(c, launch_stage<sgn::MODE_RHS>(c, c->stream, q, nullptr, nullptr, c->acc, 0.0, 0.0, 0.0));
  hipError_t e = c->p.dtype == SGN_F64 ? launch_totals<double>(c, q, c->acc, 1) : launch_totals<float>(c, q, c->acc, 1);
  HIPCHK(c, e);
  if ((st = sync_results(c, 2))) return st;
  if (mass_rate) *mass_rate = c->host_result[0];
  if (energy_rate) *energy_rate = c->host_result[1];
  return SGN_OK;
}

sgn_status sgn_cfl_dt(sgn_ctx* c, const void* q, double cfl, double* dt) {
  sgn_status st = check_ctx(c, false);
  if (st) return st;
  if (!q || !dt) return fail(c, SGN_E_ARG, "q or dt is NULL");
  if (!(std::isfinite(cfl) && cfl > 0.0)) return fail(c, SGN_E_ARG, "cfl must be finite and > 0");
  const int nb = reduce_blocks(c);
  if (c->p.dtype == SGN_F64)
    hipLaunchKernelGGL(sgn::speed_partial<double>, dim3(nb), dim3(sgn::RED_THREADS), 0, c->stream, c->gc,
                       (const double*)q, c->partials);
  else
    hipLaunchKernelGGL(sgn::speed_partial<float>, dim3(nb), dim3(sgn::RED_THREADS), 0, c->stream, c->gc,
                       (const float*)q, c->partials);
  hipLaunchKernelGGL(sgn::speed_final, dim3(1), dim3(sgn::RED_THREADS), 0, c->stream, c->partials, nb, c->result);
  HIPCHK(c, hipGetLastError());
  if ((st = sync_results(c, 1))) return st;
  const double m = c->host_result[0];
  if (!(std::isfinite(m) && m > 0.0)) return fail(c, SGN_E_NONFINITE, "characteristic speed is not finite and positive");
  *dt = cfl / m;
  return SGN_OK;
}

sgn_status sgn_profile_stages(sgn_ctx* c, void* q, double dt, int64_t nsteps, double* ms) {
  sgn_status st = check_ctx(c, true);
  if (st) return st;
  if (!q || !ms) return fail(c, SGN_E_ARG, "q or ms is NULL");
  if (!(std::isfinite(dt) && dt > 0.0) || nsteps <= 0) return fail(c, SGN_E_ARG, "dt must be > 0 and nsteps > 0");
  if (nsteps > 1024) return fail(c, SGN_E_ARG, "nsteps must be <= 1024");
  const bool pairs = c->step_path == SGN_PATH_PAIRS;
  const bool fused = c->step_path == SGN_PATH_FUSED;
  if ((pairs || fused) && (nsteps & 1)) ++nsteps;  // whole double steps, so the state ends in q
  const int nk = fused ? 0 : 4;                      // events between the launches of a profiled unit
  const int64_t units = (pairs || fused) ? nsteps / 2 : nsteps;
  // Pair and four-stage paths: one event between consecutive launches.  Fused
  // path: a start and a stop event bound to each step kernel itself
  // (hipExtLaunchKernelGGL), so nothing is enqueued between the launches.  All
  // launches go in before the first wait, so the kernels run back to back as in
  // a timed run; with more than one unit the first (warm-up) unit is left out
  // of the means.
  std::vector<hipEvent_t> ev(fused ? (size_t)(4 * units + 1) : (size_t)(units * nk + 1), nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (!e) e = hipEventCreate(&x);
  int n = 0;
  if (!e) e = hipEventRecord(ev[n++], c->stream);
  for (int64_t u = 0; u < units && e == hipSuccess; ++u) {
    const double t = (double)u * ((pairs || fused) ? 2.0 : 1.0) * dt;
    if (fused) {
      // two consecutive steps (q -> acc -> q), each timed by its own events
      c->prof_start = ev[(size_t)(4 * u + 1)];
      c->prof_stop = ev[(size_t)(4 * u + 2)];
      e = launch_fused(c, c->stream, q, c->acc, dt, t);
      c->prof_start = ev[(size_t)(4 * u + 3)];
      c->prof_stop = ev[(size_t)(4 * u + 4)];
      if (!e) e = launch_fused(c, c->stream, c->acc, q, dt, t + dt);
      c->prof_start = c->prof_stop = nullptr;
      n = (int)(4 * u + 5);
    } else if (pairs) {
      // pair 1 and pair 2 of two consecutive steps (q -> acc -> q)
      e = launch_pair<1>(c, c->stream, q, nullptr, c->acc, c->yb, dt / 6.0, dt / 2.0, dt / 3.0, dt / 2.0, t, t + dt / 2.0);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
      if (!e) e = launch_pair<2>(c, c->stream, c->yb, q, c->acc, nullptr, dt / 3.0, dt, dt / 6.0, 0.0, t + dt / 2.0, t + dt);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
      if (!e) e = launch_pair<1>(c, c->stream, c->acc, nullptr, q, c->yb, dt / 6.0, dt / 2.0, dt / 3.0, dt / 2.0, t + dt, t + 1.5 * dt);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
      if (!e) e = launch_pair<2>(c, c->stream, c->yb, c->acc, q, nullptr, dt / 3.0, dt, dt / 6.0, 0.0, t + 1.5 * dt, t + 2.0 * dt);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
    } else {
      e = launch_stage<sgn::MODE_FIRST>(c, c->stream, q, nullptr, c->acc, c->ya, dt / 6.0, dt / 2.0, t);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
      if (!e) e = launch_stage<sgn::MODE_MID>(c, c->stream, c->ya, q, c->acc, c->yb, dt / 3.0, dt / 2.0, t + dt / 2.0);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
      if (!e) e = launch_stage<sgn::MODE_MID>(c, c->stream, c->yb, q, c->acc, c->ya, dt / 3.0, dt, t + dt / 2.0);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
      if (!e) e = launch_stage<sgn::MODE_LAST>(c, c->stream, c->ya, nullptr, c->acc, q, dt / 6.0, 0.0, t + dt);
      if (!e) e = hipEventRecord(ev[n++], c->stream);
    }
  }
  if (!e) e = hipEventSynchronize(ev[n - 1]);
  double acc_ms[4] = {0, 0, 0, 0};
  const int64_t first = units > 1 ? 1 : 0;
  for (int64_t u = first; u < units && !e && fused; ++u)
    for (int k = 0; k < 2 && !e; ++k) {
      float m = 0.f;
      e = hipEventElapsedTime(&m, ev[(size_t)(4 * u + 1 + 2 * k)], ev[(size_t)(4 * u + 2 + 2 * k)]);
      acc_ms[0] += m;
    }
  for (int64_t u = first; u < units && !e && !fused; ++u)
    for (int k = 0; k < nk && !e; ++k) {
      float m = 0.f;
      e = hipEventElapsedTime(&m, ev[(size_t)(u * nk + k)], ev[(size_t)(u * nk + k + 1)]);
      acc_ms[k] += m;
    }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(c, e, "profiled step");
  const double used = (double)(units - first);
  if (fused) {
    // ms[0] = one fused step (mean over both steps of each unit)
    ms[0] = acc_ms[0] / (2.0 * used);
    ms[1] = ms[2] = ms[3] = 0.0;
  } else if (pairs) {
    // ms[0] = pair 1, ms[1] = pair 2 (means over both steps of each unit)
    ms[0] = (acc_ms[0] + acc_ms[2]) / (2.0 * used);
    ms[1] = (acc_ms[1] + acc_ms[3]) / (2.0 * used);
    ms[2] = 0.0;
    ms[3] = 0.0;
  } else {
    for (int k = 0; k < 4; ++k) ms[k] = acc_ms[k] / used;
  }
  return sync_results(c, 0);
}

sgn_status sgn_check(sgn_ctx* c) {
  if (!c) return SGN_E_ARG;
  return sync_results(c, 0);
}

}  // extern "C"
