// sgn_relax.hip -- C ABI of the relaxation RK4 step (sgn_step_relaxation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "sgn.h"
#include "sgn_internal.hpp"
#include "sgn_relax.hpp"

namespace {

using sgn_host::fail;
using sgn_host::hip_fail;

#define HIPCHK(c, expr) SGN_HIPCHK(c, expr)

// Steps captured per graph replay.
constexpr int RELAX_GRAPH_STEPS = 8;

// Device scalars of the relaxation: rs[0] = gam, rs[1] = t.  They live in the
// context's result slots 4 and 5 (slots 0..3 serve the synchronizing totals).
double* relax_scalars(const sgn_ctx* c) { return c->result + 4; }

int reduce_blocks(const sgn_ctx* c) { return c->p.ny < sgn::RED_MAX_BLOCKS ? c->p.ny : sgn::RED_MAX_BLOCKS; }

template <typename T>
hipError_t enqueue_relaxed_step_t(const sgn_ctx* c, hipStream_t s, void* q, double dt) {
  // Classical RK4 update into acc: pair kernels on the pair path; otherwise
  // the step kernel, which also forms the sums of the first Newton iteration
  // (gam = 1) per tile from the values it holds, saving that pass over q, acc, b.
  const bool fused = c->step_path != SGN_PATH_PAIRS;
  hipError_t e = fused ? sgn_host::enqueue_step_into(c, s, q, c->acc, dt, 0.0, nullptr, c->tile_partials,
                                                     sgn::EPI_RELAX)
                       : sgn_host::enqueue_pair_step(c, s, q, c->acc, dt, 0.0);
  if (e) return e;
  const int nb = reduce_blocks(c);
  double* rs = relax_scalars(c);
  for (int it = 0; it < 2; ++it) {
    if (it == 0 && fused) {
      hipLaunchKernelGGL(sgn::relax_newton, dim3(1), dim3(sgn::RED_THREADS), 0, s, (const double*)c->tile_partials,
                         sgn_host::step_tiles(c), rs, 1, 0, dt);
      continue;
    }
    hipLaunchKernelGGL(sgn::relax_partial<T>, dim3(nb), dim3(sgn::RED_THREADS), 0, s, c->gc, (const T*)q,
                       (const T*)c->acc, (const T*)c->b, (const double*)rs, it == 0 ? 1 : 0, c->partials);
    hipLaunchKernelGGL(sgn::relax_newton, dim3(1), dim3(sgn::RED_THREADS), 0, s, (const double*)c->partials, nb,
                       rs, it == 0 ? 1 : 0, it == 1 ? 1 : 0, dt);
  }
  const size_t n5 = 5 * c->N;
  hipLaunchKernelGGL(sgn::relax_update<T>, dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, s, n5, (T*)q,
                     (const T*)c->acc, (const double*)rs);
  return hipGetLastError();
}

hipError_t enqueue_relaxed_steps(const sgn_ctx* c, hipStream_t s, void* q, double dt, int steps) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < steps && e == hipSuccess; ++k)
    e = c->p.dtype == SGN_F64 ? enqueue_relaxed_step_t<double>(c, s, q, dt) : enqueue_relaxed_step_t<float>(c, s, q, dt);
  return e;
}

}  // namespace

extern "C" {

sgn_status sgn_step_relaxation(sgn_ctx* c, void* q, double dt, int64_t nsteps, double t0, double* t_end) {
  sgn_status st = sgn_host::check_ctx(c, true);
  if (st) return st;
  if (!q) return fail(c, SGN_E_ARG, "q is NULL");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, SGN_E_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(c, SGN_E_ARG, "nsteps must be >= 0");
  if (!std::isfinite(t0)) return fail(c, SGN_E_ARG, "t0 must be finite");
  if (c->p.source != SGN_SRC_NONE)
    return fail(c, SGN_E_UNSUPPORTED, "relaxation needs the energy-conserving semi-discretization (no source terms)");
  if (c->step_path != SGN_PATH_PAIRS && (st = sgn_host::ensure_tile_partials(c))) return st;
  // the time accumulator starts at t0
  hipLaunchKernelGGL(sgn::relax_set_time, dim3(1), dim3(64), 0, c->stream, relax_scalars(c), t0);
  HIPCHK(c, hipGetLastError());
  int64_t left = nsteps;
  if (left >= RELAX_GRAPH_STEPS) {
    auto& g = c->relax_graph;
    if (!(g.exec && g.q == q && g.dt == dt && g.path == c->step_path && g.tile_y == c->tile_y &&
          g.step_tile == c->step_tile)) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g = sgn_host::GraphCache{};
      HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = enqueue_relaxed_steps(c, c->cap_stream, q, dt, RELAX_GRAPH_STEPS);
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
      if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(c, le, "relaxation launch during capture");
      }
      if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
      hipGraphExec_t exec = nullptr;
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
      g.exec = exec;
      g.q = q;
      g.dt = dt;
      g.steps = RELAX_GRAPH_STEPS;
      g.path = c->step_path;
      g.tile_y = c->tile_y;
      g.step_tile = c->step_tile;
    }
    for (; left >= RELAX_GRAPH_STEPS; left -= RELAX_GRAPH_STEPS) HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
  }
  if (left > 0) HIPCHK(c, enqueue_relaxed_steps(c, c->stream, q, dt, (int)left));
  if (!t_end) return SGN_OK;
  HIPCHK(c, hipMemcpyAsync(c->host_result + 5, relax_scalars(c) + 1, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  if ((st = sgn_host::sync_results(c, 0))) return st;
  *t_end = c->host_result[5];
  return SGN_OK;
}

}  // extern "C"
