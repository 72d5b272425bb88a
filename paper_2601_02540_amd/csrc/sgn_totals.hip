// sgn_totals.hip -- C ABI of RK4 stepping with the total mass and energy of
// every step recorded on the device (sgn_step_totals).
//
// Each step runs the step kernel with its totals epilogue: every tile reduces
// M h and M E of the state it writes, from the values it holds in registers,
// so the series costs no pass over the state.  Two small kernels reduce the
// per-tile partials (in a fixed order: deterministic) into the next slot of
// the caller's series, whose index lives in device memory, so that the steps
// replay from one captured graph.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sgn.h"
#include "sgn_internal.hpp"
#include "sgn_reduce.hpp"

namespace {

using sgn_host::fail;
using sgn_host::hip_fail;

#define HIPCHK(c, expr) SGN_HIPCHK(c, expr)

// Steps captured per graph replay (even: the state returns to the caller's buffer).
constexpr int TOTALS_GRAPH_STEPS = 8;

// One step from `cur` into `oth` and the totals of the new state into the series.
hipError_t enqueue_step_with_totals(const sgn_ctx* c, hipStream_t s, void* cur, void* oth, double dt,
                                    double* series) {
  hipError_t e = sgn_host::enqueue_step_into(c, s, cur, oth, dt, 0.0, nullptr, c->tile_partials, sgn::EPI_TOTALS);
  if (e) return e;
  const int tiles = sgn_host::step_tiles(c);
  const int per_min = sgn::RED_THREADS;
  int nb = (tiles + per_min - 1) / per_min;
  if (nb > sgn::RED_MAX_BLOCKS) nb = sgn::RED_MAX_BLOCKS;
  const int per = (tiles + nb - 1) / nb;
  hipLaunchKernelGGL(sgn::partials_merge, dim3(nb), dim3(sgn::RED_THREADS), 0, s, (const double*)c->tile_partials,
                     tiles, per, c->partials);
  hipLaunchKernelGGL(sgn::series_final, dim3(1), dim3(sgn::RED_THREADS), 0, s, (const double*)c->partials, nb,
                     series, c->series_counter);
  return hipGetLastError();
}

// `steps` steps starting from the caller's buffer q (the state ends in q when
// steps is even, in the scratch buffer otherwise).
hipError_t enqueue_steps_with_totals(const sgn_ctx* c, hipStream_t s, void* q, double dt, int steps, int first,
                                     double* series) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < steps && e == hipSuccess; ++k) {
    const bool from_q = ((first + k) % 2) == 0;
    e = enqueue_step_with_totals(c, s, from_q ? q : c->acc, from_q ? c->acc : q, dt, series);
  }
  return e;
}

}  // namespace

extern "C" {

sgn_status sgn_step_totals(sgn_ctx* c, void* q, double dt, int64_t nsteps, double* series) {
  sgn_status st = sgn_host::check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, SGN_E_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(c, SGN_E_ARG, "nsteps must be >= 0");
  if (nsteps > (int64_t)0x3fffffff) return fail(c, SGN_E_ARG, "nsteps too large for one series");
  if (c->p.source != SGN_SRC_NONE)
    return fail(c, SGN_E_UNSUPPORTED, "recorded totals need the semi-discretization without source terms");
  if (nsteps == 0) return SGN_OK;
  if (!series) return fail(c, SGN_E_ARG, "series is NULL");
  if ((st = sgn_host::ensure_tile_partials(c))) return st;
  if (!c->series_counter && hipMalloc((void**)&c->series_counter, sizeof(int)) != hipSuccess) {
    c->series_counter = nullptr;
    return fail(c, SGN_E_ALLOC, "series counter");
  }
  hipLaunchKernelGGL(sgn::counter_reset, dim3(1), dim3(64), 0, c->stream, c->series_counter);
  HIPCHK(c, hipGetLastError());
  int64_t left = nsteps;
  if (left >= TOTALS_GRAPH_STEPS) {
    auto& g = c->totals_graph;
    if (!(g.exec && g.q == q && g.dt == dt && g.step_tile == c->step_tile && c->totals_series == series)) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g = sgn_host::GraphCache{};
      c->totals_series = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = enqueue_steps_with_totals(c, c->cap_stream, q, dt, TOTALS_GRAPH_STEPS, 0, series);
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
      if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(c, le, "step launch during capture");
      }
      if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
      hipGraphExec_t exec = nullptr;
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
      g.exec = exec;
      g.q = q;
      g.dt = dt;
      g.steps = TOTALS_GRAPH_STEPS;
      g.path = c->step_path;
      g.tile_y = c->tile_y;
      g.step_tile = c->step_tile;
      c->totals_series = series;
    }
    for (; left >= TOTALS_GRAPH_STEPS; left -= TOTALS_GRAPH_STEPS) HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
  }
  if (left > 0) {
    HIPCHK(c, enqueue_steps_with_totals(c, c->stream, q, dt, (int)left, 0, series));
    if (left % 2)  // the state is in the scratch buffer
      HIPCHK(c, hipMemcpyAsync(q, c->acc, 5 * c->N * c->esize, hipMemcpyDeviceToDevice, c->stream));
  }
  return SGN_OK;
}

}  // extern "C"
