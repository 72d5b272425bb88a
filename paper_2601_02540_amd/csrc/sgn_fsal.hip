// sgn_fsal.hip -- C ABI of the adaptive five-stage FSAL pair (sgn_step_adaptive).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "sgn.h"
#include "sgn_fsal.hpp"
#include "sgn_internal.hpp"

namespace {

using sgn_host::fail;
using sgn_host::hip_fail;

#define HIPCHK(c, expr) SGN_HIPCHK(c, expr)

// Attempts captured per graph replay, and replays between two looks at the
// run state from the host.
constexpr int FSAL_GRAPH_ATTEMPTS = 8;
constexpr int FSAL_REPLAYS_PER_CHECK = 4;

int fsal_tiles(const sgn_ctx* c) {
  const int ntx = (c->p.nx + sgn::TILE_X - 1) / sgn::TILE_X;
  const int nty = (c->p.ny + c->tile_y - 1) / c->tile_y;
  return ntx * nty;
}

sgn_status ensure_buffers(sgn_ctx* c) {
  auto& f = c->fs;
  const size_t state = 5 * c->N * c->esize;
  const size_t part = 2 * (size_t)std::max(((c->p.nx + 63) / 64) * ((c->p.ny + 7) / 8), 1);
  bool ok = true;
  for (void** p : {&f.k[0], &f.k[1], &f.e})
    if (!*p) ok = ok && hipMalloc(p, state) == hipSuccess;
  if (ok && f.part_cap < part) {
    if (f.part) (void)hipFree(f.part);
    f.part = nullptr;
    f.part_cap = 0;
    ok = hipMalloc((void**)&f.part, part * sizeof(double)) == hipSuccess;
    if (ok) f.part_cap = part;
    if (f.graph.exec) (void)hipGraphExecDestroy(f.graph.exec);
    f.graph = sgn_host::GraphCache{};
  }
  if (ok && !f.ctl) ok = hipMalloc(&f.ctl, sizeof(sgn::AdaptCtl)) == hipSuccess;
  if (ok && !f.host_ctl) ok = hipHostMalloc(&f.host_ctl, sizeof(sgn::AdaptCtl), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    sgn_host::free_fsal(c);
    return fail(c, SGN_E_ALLOC, "buffers of the adaptive pair");
  }
  return SGN_OK;
}

template <typename T, int TY>
hipError_t enqueue_attempt_ty(const sgn_ctx* c, hipStream_t s, void* q, double* rec, long long rec_cap) {
  const int ntx = (c->p.nx + sgn::TILE_X - 1) / sgn::TILE_X;
  const int nty = (c->p.ny + TY - 1) / TY;
  const int nt = ntx * nty;
  const dim3 grid((unsigned)nt), block(sgn::STAGE_THREADS);
  const auto& f = c->fs;
  sgn::FsalArgs<T> a;
  a.q[0] = (T*)q;
  a.q[1] = (T*)c->acc;
  a.k[0] = (T*)f.k[0];
  a.k[1] = (T*)f.k[1];
  a.ya = (T*)c->ya;  // the stage states of the role kernels: the context's own
  a.yb = (T*)c->yb;
  a.e = (T*)f.e;
  a.b = (const T*)c->b;
  a.part = f.part;
  a.ctl = (sgn::AdaptCtl*)f.ctl;
  const int bx = c->p.bc_x, by = c->p.bc_y;
#define SGN_ROLE(R)                                                                                           \
  do {                                                                                                        \
    if (bx == 0 && by == 0) hipLaunchKernelGGL((sgn::fsal_kernel<T, 0, 0, R, TY>), grid, block, 0, s, c->gc, a); \
    else if (bx == 0 && by == 1) hipLaunchKernelGGL((sgn::fsal_kernel<T, 0, 1, R, TY>), grid, block, 0, s, c->gc, a); \
    else if (bx == 1 && by == 0) hipLaunchKernelGGL((sgn::fsal_kernel<T, 1, 0, R, TY>), grid, block, 0, s, c->gc, a); \
    else hipLaunchKernelGGL((sgn::fsal_kernel<T, 1, 1, R, TY>), grid, block, 0, s, c->gc, a);                \
  } while (0)
  if (c->step_path == SGN_PATH_FUSED) {
    // S2 .. S5 in one launch of the step tile; with the context's 32 x 24 step
    // tile, 32 x 24 on periodic grids and 32 x 16 otherwise (the attempt's
    // 32 x 24 instances with a wall reach the register limit)
    const int ty = c->step_tile == 8 ? 8 : (c->step_tile == 24 && bx == 0 && by == 0 ? 24 : 16);
    const int tx = ty == 8 ? sgn::StepGeom<8>::TX : sgn::StepGeom<16>::TX;
    const int sx = (c->p.nx + tx - 1) / tx, sy = (c->p.ny + ty - 1) / ty;
    const dim3 sgrid((unsigned)(sx * sy));
#define SGN_FSTEP(TY_)                                                                                             \
  do {                                                                                                             \
    if (bx == 0 && by == 0) hipLaunchKernelGGL((sgn::fsal_step_kernel<T, 0, 0, TY_>), sgrid, block, 0, s, c->gc, a);      \
    else if (bx == 0 && by == 1) hipLaunchKernelGGL((sgn::fsal_step_kernel<T, 0, 1, TY_>), sgrid, block, 0, s, c->gc, a); \
    else if (bx == 1 && by == 0) hipLaunchKernelGGL((sgn::fsal_step_kernel<T, 1, 0, TY_>), sgrid, block, 0, s, c->gc, a); \
    else hipLaunchKernelGGL((sgn::fsal_step_kernel<T, 1, 1, TY_>), sgrid, block, 0, s, c->gc, a);                   \
  } while (0)
    if (ty == 24) hipLaunchKernelGGL((sgn::fsal_step_kernel<T, 0, 0, 24>), sgrid, block, 0, s, c->gc, a);
    else if (ty == 16) SGN_FSTEP(16);
    else SGN_FSTEP(8);
#undef SGN_FSTEP
  } else {
    SGN_ROLE(sgn::FS_S2);
    SGN_ROLE(sgn::FS_S3);
    SGN_ROLE(sgn::FS_S4);
    SGN_ROLE(sgn::FS_S5);
  }
  SGN_ROLE(sgn::FS_FSAL);
#undef SGN_ROLE
  hipLaunchKernelGGL(sgn::fsal_control, dim3(1), dim3(sgn::RED_THREADS), 0, s, (sgn::AdaptCtl*)f.ctl, f.part, nt,
                     1.0 / (5.0 * (double)c->N), rec, rec_cap, c->flag);
  return hipGetLastError();
}

hipError_t enqueue_attempt(const sgn_ctx* c, hipStream_t s, void* q, double* rec, long long rec_cap) {
  if (c->p.dtype == SGN_F64)
    return c->tile_y == 16 ? enqueue_attempt_ty<double, 16>(c, s, q, rec, rec_cap)
                           : enqueue_attempt_ty<double, 8>(c, s, q, rec, rec_cap);
  return c->tile_y == 16 ? enqueue_attempt_ty<float, 16>(c, s, q, rec, rec_cap)
                         : enqueue_attempt_ty<float, 8>(c, s, q, rec, rec_cap);
}

sgn_status get_graph(sgn_ctx* c, void* q, double* rec, long long rec_cap, hipGraphExec_t* out) {
  auto& f = c->fs;
  auto& g = f.graph;
  if (g.exec && g.q == q && g.tile_y == c->tile_y && g.path == c->step_path && g.step_tile == c->step_tile &&
      f.graph_rec == rec && f.graph_rec_cap == rec_cap) {
    *out = g.exec;
    return SGN_OK;
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g = sgn_host::GraphCache{};
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int a = 0; a < FSAL_GRAPH_ATTEMPTS && le == hipSuccess; ++a) le = enqueue_attempt(c, c->cap_stream, q, rec, rec_cap);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(c, le, "adaptive attempt launch during capture");
  }
  if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
  g.exec = exec;
  g.q = q;
  g.tile_y = c->tile_y;
  g.path = c->step_path;
  g.step_tile = c->step_tile;
  f.graph_rec = rec;
  f.graph_rec_cap = rec_cap;
  *out = exec;
  return SGN_OK;
}

}  // namespace

namespace sgn_host {

void free_fsal(sgn_ctx* c) {
  auto& f = c->fs;
  if (f.graph.exec) (void)hipGraphExecDestroy(f.graph.exec);
  for (void* p : {f.k[0], f.k[1], f.e, f.ctl})
    if (p) (void)hipFree(p);
  if (f.part) (void)hipFree(f.part);
  if (f.host_ctl) (void)hipHostFree(f.host_ctl);
  f = FsalBuffers{};
}

}  // namespace sgn_host

extern "C" {

sgn_status sgn_step_adaptive(sgn_ctx* c, void* q, double t0, double t_end, double dt0, double rtol, double atol,
                             int32_t adaptive, int64_t max_attempts, double* record, int64_t record_cap,
                             sgn_adaptive_result* out) {
  sgn_status st = sgn_host::check_ctx(c, true);
  if (st) return st;
  if (!q || !out) return fail(c, SGN_E_ARG, "q or out is NULL");
  if (c->p.source != SGN_SRC_NONE) return fail(c, SGN_E_UNSUPPORTED, "the adaptive pair runs without source terms");
  if (!(std::isfinite(t0) && std::isfinite(t_end) && t_end >= t0)) return fail(c, SGN_E_ARG, "need finite t0 <= t_end");
  if (!(std::isfinite(dt0) && dt0 > 0.0)) return fail(c, SGN_E_ARG, "dt0 must be finite and > 0");
  if (!(std::isfinite(rtol) && std::isfinite(atol) && rtol >= 0.0 && atol >= 0.0 && rtol + atol > 0.0))
    return fail(c, SGN_E_ARG, "tolerances must be finite, >= 0 and not both 0");
  if (max_attempts < 1) return fail(c, SGN_E_ARG, "max_attempts must be >= 1");
  if (record_cap < 0 || (record_cap > 0 && !record)) return fail(c, SGN_E_ARG, "record is NULL with record_cap > 0");
  std::memset(out, 0, sizeof(*out));
  if ((st = ensure_buffers(c))) return st;
  auto& f = c->fs;
  if ((size_t)fsal_tiles(c) * 2 > f.part_cap) return fail(c, SGN_E_STATE, "partial sums too small for the tiling");
  double* rec = record_cap > 0 ? record : nullptr;

  // k_1 = f(q) at t0 into k[0]; the run state
  HIPCHK(c, sgn_host::launch_stage_mode(c, c->stream, sgn::MODE_RHS, q, nullptr, nullptr, f.k[0], 0.0, 0.0, t0));
  const double h0 = (t_end - t0 <= dt0 * (1.0 + 1e-10)) ? t_end - t0 : dt0;
  hipLaunchKernelGGL(sgn::fsal_init, dim3(1), dim3(1), 0, c->stream, (sgn::AdaptCtl*)f.ctl, t0, h0, t_end, rtol, atol,
                     (long long)max_attempts, adaptive ? 1 : 0);
  HIPCHK(c, hipGetLastError());
  hipGraphExec_t ge;
  if ((st = get_graph(c, q, rec, record_cap, &ge))) return st;
  sgn::AdaptCtl* hc = (sgn::AdaptCtl*)f.host_ctl;
  const int64_t max_replays = max_attempts / FSAL_GRAPH_ATTEMPTS + 2;
  for (int64_t r = 0;;) {
    for (int k = 0; k < FSAL_REPLAYS_PER_CHECK && r < max_replays; ++k, ++r) HIPCHK(c, hipGraphLaunch(ge, c->stream));
    HIPCHK(c, hipMemcpyAsync(hc, f.ctl, sizeof(sgn::AdaptCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (hc->done || r >= max_replays) break;
  }
  // the final state lives in the buffer the selector names
  if (hc->cur == 1) HIPCHK(c, hipMemcpyAsync(q, c->acc, 5 * c->N * c->esize, hipMemcpyDeviceToDevice, c->stream));
  out->t = hc->t;
  out->h_next = hc->h;
  out->last_err = hc->err;
  out->attempts = hc->attempts;
  out->accepted = hc->accepted;
  out->rejected = hc->rejected;
  out->reached_end = hc->done == 1 ? 1 : 0;
  if ((st = sgn_check(c))) return st;  // synchronizes; reports the health flag
  if (hc->done == 3) return fail(c, SGN_E_NONFINITE, "non-finite error estimate");
  if (hc->done == 4) return fail(c, SGN_E_NONPOS_DEPTH, "an accepted step left a non-positive depth");
  return SGN_OK;
}

}  // extern "C"
