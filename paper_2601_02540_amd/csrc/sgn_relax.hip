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

// The Newton iterations for gam after an RK4 update base -> rk: the first from
// the step kernel's per-tile sums (fused) or a pass of its own (pairs), the
// second from a pass over (base, rk, b); rs[0] = gam, rs[1] += gam dt.
template <typename T>
void enqueue_newton(const sgn_ctx* c, hipStream_t s, const void* base, const void* rk, bool fused, double dt) {
  const int nb = reduce_blocks(c);
  double* rs = relax_scalars(c);
  for (int it = 0; it < 2; ++it) {
    if (it == 0 && fused) {
      hipLaunchKernelGGL(sgn::relax_newton, dim3(1), dim3(sgn::RED_THREADS), 0, s, (const double*)c->tile_partials,
                         sgn_host::step_tiles(c), rs, 1, 0, dt);
      continue;
    }
    hipLaunchKernelGGL(sgn::relax_partial<T>, dim3(nb), dim3(sgn::RED_THREADS), 0, s, c->gc, (const T*)base,
                       (const T*)rk, (const T*)c->b, (const double*)rs, it == 0 ? 1 : 0, c->partials);
    hipLaunchKernelGGL(sgn::relax_newton, dim3(1), dim3(sgn::RED_THREADS), 0, s, (const double*)c->partials, nb,
                       rs, it == 0 ? 1 : 0, it == 1 ? 1 : 0, dt);
  }
}

template <typename T>
hipError_t launch_update(const sgn_ctx* c, hipStream_t s, void* out, const void* base, const void* rk) {
  const size_t n5 = 5 * c->N;
  hipLaunchKernelGGL(sgn::relax_update<T>, dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, s, n5, (T*)out,
                     (const T*)base, (const T*)rk, (const double*)relax_scalars(c));
  return hipGetLastError();
}

template <typename T, int TY>
hipError_t launch_relax_step(const sgn_ctx* c, hipStream_t s, const void* qa, const void* ra, void* qbase, void* rk,
                             double dt) {
  constexpr int TX = sgn::StepGeom<TY>::TX;
  const int ntx = (c->p.nx + TX - 1) / TX, nty = (c->p.ny + TY - 1) / TY;
  const sgn::RelaxIn<T> rx{(const T*)ra, relax_scalars(c), (T*)qbase};
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
#define SGN_RLX(BX, BY)                                                                                             \
  hipLaunchKernelGGL((sgn::relax_step_kernel<T, BX, BY, TY>), grid, block, 0, s, c->gc, (const T*)qa, (const T*)c->b, \
                     (T*)rk, rx, (T)(dt / 6.0), (T)(dt / 3.0), (T)(dt / 2.0), (T)dt, dt, c->flag, c->tile_partials)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (bx == 0 && by == 0) SGN_RLX(0, 0);
  else if (bx == 0 && by == 1) SGN_RLX(0, 1);
  else if (bx == 1 && by == 0) SGN_RLX(1, 0);
  else SGN_RLX(1, 1);
#undef SGN_RLX
  return hipGetLastError();
}

// `steps` relaxed steps of q in place.  Pair path: per step the RK4 update into
// acc, the two Newton iterations and the update pass.  Step-kernel paths: the
// first step updates q into acc; every later one stages the previous step's
// relaxed state on the fly (relax_step_kernel), alternating between the buffer
// pairs (q, acc) and (ya, yb); one update pass at the end writes q.
template <typename T>
hipError_t enqueue_relaxed_steps_t(const sgn_ctx* c, hipStream_t s, void* q, double dt, int steps) {
  if (steps <= 0) return hipSuccess;
  const bool fused = c->step_path != SGN_PATH_PAIRS;
  if (!fused) {
    for (int k = 0; k < steps; ++k) {
      hipError_t e = sgn_host::enqueue_pair_step(c, s, q, c->acc, dt, 0.0);
      if (e) return e;
      enqueue_newton<T>(c, s, q, c->acc, false, dt);
      if ((e = launch_update<T>(c, s, q, q, c->acc))) return e;
    }
    return hipSuccess;
  }
  void* base[2] = {q, c->ya};
  void* rk[2] = {c->acc, c->yb};
  hipError_t e = sgn_host::enqueue_step_into(c, s, q, c->acc, dt, 0.0, nullptr, c->tile_partials, sgn::EPI_RELAX);
  if (e) return e;
  enqueue_newton<T>(c, s, q, c->acc, true, dt);
  for (int k = 1; k < steps; ++k) {
    const int a = (k - 1) & 1, b = k & 1;
    e = c->step_tile == 24 ? launch_relax_step<T, 24>(c, s, base[a], rk[a], base[b], rk[b], dt)
        : c->step_tile == 16 ? launch_relax_step<T, 16>(c, s, base[a], rk[a], base[b], rk[b], dt)
                             : launch_relax_step<T, 8>(c, s, base[a], rk[a], base[b], rk[b], dt);
    if (e) return e;
    enqueue_newton<T>(c, s, base[b], rk[b], true, dt);
  }
  const int l = (steps - 1) & 1;
  return launch_update<T>(c, s, q, base[l], rk[l]);
}

hipError_t enqueue_relaxed_steps(const sgn_ctx* c, hipStream_t s, void* q, double dt, int steps) {
  return c->p.dtype == SGN_F64 ? enqueue_relaxed_steps_t<double>(c, s, q, dt, steps)
                               : enqueue_relaxed_steps_t<float>(c, s, q, dt, steps);
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
