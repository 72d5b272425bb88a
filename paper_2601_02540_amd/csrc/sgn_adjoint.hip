// sgn_adjoint.hip -- discrete adjoint entry points: RHS and RK4-step VJPs and a
// gauge-misfit loss gradient with sqrt(T) checkpointing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "sgn.h"
#include "sgn_internal.hpp"
#include "sgn_reduce.hpp"
#include "sgn_pair.hpp"
#include "sgn_vjp.hpp"

namespace {

using sgn_host::fail;
using sgn_host::hip_fail;
#define HIPCHK(c, expr) SGN_HIPCHK(c, expr)

constexpr int VJP_TY = 8;

template <typename T, int ROLE>
hipError_t launch_vjp_t(const sgn_ctx* c, hipStream_t s, const void* Y, const void* Kin, void* Qb, void* Kout,
                        void* Acc, void* Bb, double a_in, double cq, double cy) {
  const int ntx = (c->p.nx + sgn::TILE_X - 1) / sgn::TILE_X;
  const int nty = (c->p.ny + VJP_TY - 1) / VJP_TY;
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
  const T* Yp = (const T*)Y;
  const T* bp = (const T*)c->b;
  const T* kp = (const T*)Kin;
#define SGN_VJP(BX, BY)                                                                                       \
  hipLaunchKernelGGL((sgn::vjp_kernel<T, BX, BY, ROLE, VJP_TY>), grid, block, 0, s, c->gc, Yp, bp, kp, (T*)Qb, \
                     (T*)Kout, (T*)Acc, (T*)Bb, (T)a_in, (T)cq, (T)cy)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (bx == 0 && by == 0) SGN_VJP(0, 0);
  else if (bx == 0 && by == 1) SGN_VJP(0, 1);
  else if (bx == 1 && by == 0) SGN_VJP(1, 0);
  else SGN_VJP(1, 1);
#undef SGN_VJP
  return hipGetLastError();
}

template <int ROLE>
hipError_t launch_vjp(const sgn_ctx* c, hipStream_t s, const void* Y, const void* Kin, void* Qb, void* Kout,
                      void* Acc, void* Bb, double a_in, double cq, double cy) {
  if (c->p.dtype == SGN_F64) return launch_vjp_t<double, ROLE>(c, s, Y, Kin, Qb, Kout, Acc, Bb, a_in, cq, cy);
  return launch_vjp_t<float, ROLE>(c, s, Y, Kin, Qb, Kout, Acc, Bb, a_in, cq, cy);
}

template <typename T, int PAIR, int TX>
hipError_t launch_vjp_pair_t(const sgn_ctx* c, hipStream_t s, const void* YA, const void* YB, const void* KinA,
                             const void* Qb, void* QbOut, void* Kout, void* Acc, void* Bb, double aA, double cqA,
                             double cyA, double cqB, double cyB) {
  constexpr int TY = sgn::VjpGeom<TX>::TY;
  const int ntx = (c->p.nx + TX - 1) / TX;
  const int nty = (c->p.ny + TY - 1) / TY;
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
#define SGN_VJPP(BX, BY)                                                                                         \
  hipLaunchKernelGGL((sgn::vjp_pair_kernel<T, BX, BY, PAIR, TX>), grid, block, 0, s, c->gc, (const T*)YA,        \
                     (const T*)YB, (const T*)c->b, (const T*)KinA, (const T*)Qb, (T*)QbOut, (T*)Kout, (T*)Acc,   \
                     (T*)Bb, (T)aA, (T)cqA, (T)cyA, (T)cqB, (T)cyB)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (bx == 0 && by == 0) SGN_VJPP(0, 0);
  else if (bx == 0 && by == 1) SGN_VJPP(0, 1);
  else if (bx == 1 && by == 0) SGN_VJPP(1, 0);
  else SGN_VJPP(1, 1);
#undef SGN_VJPP
  return hipGetLastError();
}

// Two reverse stages in one launch (sgn::vjp_pair_kernel), on 64 x 8 tiles
// when the step kernel runs 64 x 8 tiles, on 32 x 16 tiles otherwise.
template <int PAIR>
hipError_t launch_vjp_pair(const sgn_ctx* c, hipStream_t s, const void* YA, const void* YB, const void* KinA,
                           const void* Qb, void* QbOut, void* Kout, void* Acc, void* Bb, double aA, double cqA,
                           double cyA, double cqB, double cyB) {
  if (c->p.dtype == SGN_F64) {
    if (c->step_tile != 8)
      return launch_vjp_pair_t<double, PAIR, 32>(c, s, YA, YB, KinA, Qb, QbOut, Kout, Acc, Bb, aA, cqA, cyA, cqB, cyB);
    return launch_vjp_pair_t<double, PAIR, 64>(c, s, YA, YB, KinA, Qb, QbOut, Kout, Acc, Bb, aA, cqA, cyA, cqB, cyB);
  }
  if (c->step_tile != 8)
    return launch_vjp_pair_t<float, PAIR, 32>(c, s, YA, YB, KinA, Qb, QbOut, Kout, Acc, Bb, aA, cqA, cyA, cqB, cyB);
  return launch_vjp_pair_t<float, PAIR, 64>(c, s, YA, YB, KinA, Qb, QbOut, Kout, Acc, Bb, aA, cqA, cyA, cqB, cyB);
}

size_t state_bytes(const sgn_ctx* c) { return 5 * c->N * c->esize; }
void* slot(void* base, size_t i, const sgn_ctx* c) { return (char*)base + i * state_bytes(c); }

// Cotangent buffers of one step VJP (kb_a, kb_b, accb).
sgn_status ensure_vjp_buffers(sgn_ctx* c) {
  auto& a = c->adj;
  if (a.kb_a) return SGN_OK;
  if (hipMalloc(&a.kb_a, state_bytes(c)) != hipSuccess || hipMalloc(&a.kb_b, state_bytes(c)) != hipSuccess ||
      hipMalloc(&a.accb, state_bytes(c)) != hipSuccess) {
    (void)hipGetLastError();
    sgn_host::free_adjoint(c);
    return fail(c, SGN_E_ALLOC, "adjoint buffers");
  }
  return SGN_OK;
}

sgn_status ensure_stage_slots(sgn_ctx* c, size_t slots) {
  auto& a = c->adj;
  if (a.stage_slots >= slots) return SGN_OK;
  if (a.stages) (void)hipFree(a.stages);
  a.stages = nullptr;
  a.stage_slots = 0;
  if (hipMalloc(&a.stages, slots * state_bytes(c)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SGN_E_ALLOC, "adjoint stage storage (" + std::to_string(slots) + " states)");
  }
  a.stage_slots = slots;
  return SGN_OK;
}

template <typename T, int PAIR, int TY>
hipError_t launch_pair_save_t(const sgn_ctx* c, hipStream_t s, const void* Yin, const void* qn, void* acc,
                              void* yb, void* ysave, void* qout, double c1_acc, double c1_y, double c2_acc,
                              double c2_y) {
  const int ntx = (c->p.nx + sgn::TILE_X - 1) / sgn::TILE_X;
  const int nty = (c->p.ny + TY - 1) / TY;
  const dim3 grid((unsigned)(ntx * nty)), block(sgn::STAGE_THREADS);
#define SGN_PS(BX, BY)                                                                                         \
  hipLaunchKernelGGL((sgn::pair_save_kernel<T, BX, BY, PAIR, TY>), grid, block, 0, s, c->gc, (const T*)Yin,      \
                     (const T*)c->b, (const T*)qn, (T*)acc, (T*)yb, (T*)ysave, (T*)qout, (T)c1_acc, (T)c1_y, \
                     (T)c2_acc, (T)c2_y, c->flag)
  const int bx = c->p.bc_x, by = c->p.bc_y;
  if (bx == 0 && by == 0) SGN_PS(0, 0);
  else if (bx == 0 && by == 1) SGN_PS(0, 1);
  else if (bx == 1 && by == 0) SGN_PS(1, 0);
  else SGN_PS(1, 1);
#undef SGN_PS
  return hipGetLastError();
}

template <int PAIR>
hipError_t launch_pair_save(const sgn_ctx* c, hipStream_t s, const void* Yin, const void* qn, void* acc, void* yb,
                            void* ysave, void* qout, double c1_acc, double c1_y, double c2_acc, double c2_y) {
  if (c->p.dtype == SGN_F64) {
    if (c->tile_y == 16)
      return launch_pair_save_t<double, PAIR, 16>(c, s, Yin, qn, acc, yb, ysave, qout, c1_acc, c1_y, c2_acc, c2_y);
    return launch_pair_save_t<double, PAIR, 8>(c, s, Yin, qn, acc, yb, ysave, qout, c1_acc, c1_y, c2_acc, c2_y);
  }
  if (c->tile_y == 16)
    return launch_pair_save_t<float, PAIR, 16>(c, s, Yin, qn, acc, yb, ysave, qout, c1_acc, c1_y, c2_acc, c2_y);
  return launch_pair_save_t<float, PAIR, 8>(c, s, Yin, qn, acc, yb, ysave, qout, c1_acc, c1_y, c2_acc, c2_y);
}

// Forward RK4 step from `qn` into `qout`, keeping the stage states Y2, Y3, Y4
// in `ys` (three consecutive state slots).  On the pair path:
//   pair 1: k1 = f(qn), Y2 = qn + dt/2 k1 (saved), k2 = f(Y2), acc, Y3 = qn + dt/2 k2
//   pair 2: k3 = f(Y3), Y4 = qn + dt k3 (saved), k4 = f(Y4), qout = acc + dt/3 k3 + dt/6 k4
// (47 values of traffic per node); otherwise the step kernel writes the stage
// states as it forms them (26 values).  Both give the same values bit for bit.
hipError_t forward_step_keep(const sgn_ctx* c, hipStream_t s, const void* qn, void* ys, void* qout, double dt) {
  if (c->step_path != SGN_PATH_PAIRS) return sgn_host::enqueue_step_into(c, s, qn, qout, dt, 0.0, ys);
  void* y2 = slot(ys, 0, c);
  void* y3 = slot(ys, 1, c);
  void* y4 = slot(ys, 2, c);
  hipError_t e = launch_pair_save<1>(c, s, qn, nullptr, c->acc, y3, y2, nullptr, dt / 6.0, dt / 2.0, dt / 3.0,
                                     dt / 2.0);
  if (e) return e;
  return launch_pair_save<2>(c, s, y3, qn, c->acc, nullptr, y4, qout, dt / 3.0, dt, dt / 6.0, 0.0);
}

// One RK4 step of a rollout from `cur` into `oth`: the pair kernels on the pair
// path, the step kernel otherwise.
hipError_t rollout_step(const sgn_ctx* c, hipStream_t s, void* cur, void* oth, double dt) {
  if (c->step_path == SGN_PATH_PAIRS) return sgn_host::enqueue_pair_step(c, s, cur, oth, dt, 0.0);
  return sgn_host::enqueue_step_into(c, s, cur, oth, dt, 0.0, nullptr);
}

// Reverse of one RK4 step whose stage states are Y1 = qn and ys = (Y2, Y3, Y4).
// qbar: cotangent of q_{n+1} on entry; the cotangent of q_n goes to *qbar_out:
// qbar itself on the pair and four-stage paths (four role kernels, qbar
// updated in place), the context's kb_b on the fused path (two launches of the
// two-stage kernel, whose second one cannot write the qbar it reads on the
// rings of its tiles).  bbar accumulates.
hipError_t reverse_step(const sgn_ctx* c, hipStream_t s, const void* qn, const void* ys, void* qbar, void* bbar,
                        double dt, void** qbar_out) {
  const auto& a = c->adj;
  const void* y2 = slot((void*)ys, 0, c);
  const void* y3 = slot((void*)ys, 1, c);
  const void* y4 = slot((void*)ys, 2, c);
  hipError_t e;
  if (c->step_path == SGN_PATH_FUSED) {
    // S4 + S3: kb4 = dt/6 qb, kb3 = dt/3 qb + dt Yb4 (LDS); kb2 = dt/3 qb + dt/2 Yb3, acc = Yb4 + Yb3
    if ((e = launch_vjp_pair<2>(c, s, y4, y3, qbar, qbar, nullptr, a.kb_a, a.accb, bbar, dt / 6.0, dt / 3.0, dt,
                                dt / 3.0, dt / 2.0)))
      return e;
    // S2 + S1: kb1 = dt/6 qb + dt/2 Yb2 (LDS); qb_n = qb + (acc + Yb2) + Yb1
    *qbar_out = a.kb_b;
    return launch_vjp_pair<1>(c, s, y2, qn, a.kb_a, qbar, a.kb_b, nullptr, a.accb, bbar, 1.0, dt / 6.0, dt / 2.0,
                              0.0, 0.0);
  }
  *qbar_out = qbar;
  // kb4 = dt/6 qb ; next kb3 = dt/3 qb + dt Yb4
  if ((e = launch_vjp<sgn::VJP_S4>(c, s, y4, qbar, qbar, a.kb_a, a.accb, bbar, dt / 6.0, dt / 3.0, dt))) return e;
  // kb2 = dt/3 qb + dt/2 Yb3
  if ((e = launch_vjp<sgn::VJP_S3>(c, s, y3, a.kb_a, qbar, a.kb_b, a.accb, bbar, 1.0, dt / 3.0, dt / 2.0))) return e;
  // kb1 = dt/6 qb + dt/2 Yb2
  if ((e = launch_vjp<sgn::VJP_S2>(c, s, y2, a.kb_b, qbar, a.kb_a, a.accb, bbar, 1.0, dt / 6.0, dt / 2.0))) return e;
  // qb_n = qb + Yb4 + Yb3 + Yb2 + Yb1
  return launch_vjp<sgn::VJP_S1>(c, s, qn, a.kb_a, qbar, nullptr, a.accb, bbar, 1.0, 0.0, 0.0);
}

// h = zeta0 - b, u = v = w = 0, eta = h (w is then set by the initialization kernel).
template <typename T>
__global__ __launch_bounds__(256) void surface_to_state(const T* __restrict__ zeta0, const T* __restrict__ b,
                                                        T* __restrict__ q, size_t N) {
  const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  const T h = zeta0[k] - b[k];
  q[k] = h;
  q[N + k] = T(0);
  q[2 * N + k] = T(0);
  q[3 * N + k] = T(0);
  q[4 * N + k] = h;
}

// zeta = h + b at the gauges, one row of the series.  Also the misfit against a
// target row and the loss increment.  One block; thread t handles gauges t,
// t + 256, ... and the loss increment is summed in a fixed tree order, so the
// result is deterministic.
// Gauge indices come from the caller: an index outside [0, N) is skipped and
// raises FLAG_BADINDEX (reported as SGN_E_ARG by the next synchronizing call).
constexpr int GAUGE_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(GAUGE_THREADS) void gauge_record(const T* __restrict__ q, const T* __restrict__ b,
                                                              const int64_t* __restrict__ idx, int ng, size_t N,
                                                              double* __restrict__ series,
                                                              const double* __restrict__ target,
                                                              double* __restrict__ misfit, double* __restrict__ loss,
                                                              int* __restrict__ flag) {
  __shared__ double part[GAUGE_THREADS];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int g = t; g < ng; g += GAUGE_THREADS) {
    const int64_t k = idx[g];
    if (k < 0 || (size_t)k >= N) {
      atomicOr(flag, sgn::FLAG_BADINDEX);
      if (series) series[g] = 0.0;
      if (target) misfit[g] = 0.0;
      continue;
    }
    const double z = (double)q[k] + (double)b[k];
    if (series) series[g] = z;
    if (target) {
      const double m = z - target[g];
      misfit[g] = m;
      acc += 0.5 * m * m;
    }
  }
  if (!loss) return;
  part[t] = acc;
  __syncthreads();
  for (int w = GAUGE_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) *loss += part[0];
}

// Adjoint seed of one misfit row: qbar_h += m and bbar += m at the gauges.
// One thread per gauge; a node carrying several gauges is updated by the
// thread of its first gauge, which adds their misfits in gauge order.
template <typename T>
__global__ __launch_bounds__(GAUGE_THREADS) void gauge_seed(const int64_t* __restrict__ idx, int ng, size_t N,
                                                            const double* __restrict__ misfit, T* __restrict__ qbar,
                                                            T* __restrict__ bbar) {
  const int g = blockIdx.x * GAUGE_THREADS + threadIdx.x;
  if (g >= ng) return;
  const int64_t k = idx[g];
  if (k < 0 || (size_t)k >= N) return;  // flagged by gauge_record
  for (int e = 0; e < g; ++e)
    if (idx[e] == k) return;
  T qa = qbar[k], ba = bbar[k];
  for (int e = g; e < ng; ++e) {
    if (idx[e] != k) continue;
    qa += T(misfit[e]);
    ba += T(misfit[e]);
  }
  qbar[k] = qa;
  bbar[k] = ba;
}

// grad_zeta0 = hbar0 = qbar_h + qbar_eta; grad_b = bbar - hbar0 (h0 = zeta0 - b,
// eta0 = h0; with u0 = v0 = 0 the initialized w0 depends on neither).
template <typename T>
__global__ __launch_bounds__(256) void init_reverse(const T* __restrict__ qbar, const T* bbar,
                                                    T* __restrict__ gz, T* gb, size_t N) {
  const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  const T h0b = qbar[k] + qbar[4 * N + k];
  gz[k] = h0b;
  gb[k] = bbar[k] - h0b;
}

hipError_t launch_surface(const sgn_ctx* c, const void* zeta0, void* q) {
  const dim3 grid((unsigned)((c->N + 255) / 256)), block(256);
  if (c->p.dtype == SGN_F64)
    hipLaunchKernelGGL(surface_to_state<double>, grid, block, 0, c->stream, (const double*)zeta0, (const double*)c->b,
                       (double*)q, c->N);
  else
    hipLaunchKernelGGL(surface_to_state<float>, grid, block, 0, c->stream, (const float*)zeta0, (const float*)c->b,
                       (float*)q, c->N);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  const dim3 g2((c->p.nx + 63) / 64, (c->p.ny + 3) / 4);
  if (c->p.dtype == SGN_F64)
    hipLaunchKernelGGL(sgn::init_aux_kernel<double>, g2, block, 0, c->stream, c->gc, (double*)q, (const double*)c->b);
  else
    hipLaunchKernelGGL(sgn::init_aux_kernel<float>, g2, block, 0, c->stream, c->gc, (float*)q, (const float*)c->b);
  return hipGetLastError();
}

hipError_t launch_record(const sgn_ctx* c, const void* q, const int64_t* idx, int ng, double* series,
                         const double* target, double* misfit, double* loss) {
  if (c->p.dtype == SGN_F64)
    hipLaunchKernelGGL(gauge_record<double>, dim3(1), dim3(GAUGE_THREADS), 0, c->stream, (const double*)q, (const double*)c->b, idx,
                       ng, c->N, series, target, misfit, loss, c->flag);
  else
    hipLaunchKernelGGL(gauge_record<float>, dim3(1), dim3(GAUGE_THREADS), 0, c->stream, (const float*)q, (const float*)c->b, idx,
                       ng, c->N, series, target, misfit, loss, c->flag);
  return hipGetLastError();
}

sgn_status gauge_args(sgn_ctx* c, const void* zeta0, int64_t nsteps, double dt, const int64_t* idx, int32_t ng) {
  sgn_status st = sgn_host::check_ctx(c, true);
  if (st) return st;
  if (!zeta0 || !idx) return fail(c, SGN_E_ARG, "zeta0 or gauge indices NULL");
  if (ng <= 0 || ng > 4096) return fail(c, SGN_E_ARG, "need 1..4096 gauges");
  if (nsteps <= 0) return fail(c, SGN_E_ARG, "nsteps must be > 0");
  if (!(std::isfinite(dt) && dt > 0)) return fail(c, SGN_E_ARG, "dt must be finite and > 0");
  if (c->p.source != SGN_SRC_NONE) return fail(c, SGN_E_UNSUPPORTED, "rollouts are defined without source terms");
  return SGN_OK;
}

}  // namespace

namespace sgn_host {

void free_adjoint(sgn_ctx* c) {
  auto& a = c->adj;
  for (void* p : {a.kb_a, a.kb_b, a.accb, a.qbar, a.state, a.stages, a.ckpt})
    if (p) (void)hipFree(p);
  if (a.misfit) (void)hipFree(a.misfit);
  if (a.loss) (void)hipFree(a.loss);
  a = AdjointBuffers{};
}

}  // namespace sgn_host

extern "C" {

sgn_status sgn_rhs_vjp(sgn_ctx* c, const void* q, const void* a, void* qbar, void* bbar) {
  sgn_status st = sgn_host::check_ctx(c, true);
  if (st) return st;
  if (!q || !a || !qbar || !bbar) return fail(c, SGN_E_ARG, "NULL argument");
  if (c->p.source != SGN_SRC_NONE) return fail(c, SGN_E_UNSUPPORTED, "the VJP is defined without source terms");
  HIPCHK(c, launch_vjp<sgn::VJP_PLAIN>(c, c->stream, q, a, nullptr, qbar, nullptr, bbar, 1.0, 0.0, 0.0));
  return SGN_OK;
}

sgn_status sgn_step_vjp(sgn_ctx* c, const void* q_n, double dt, void* qbar, void* bbar) {
  sgn_status st = sgn_host::check_ctx(c, true);
  if (st) return st;
  if (!q_n || !qbar || !bbar) return fail(c, SGN_E_ARG, "NULL argument");
  if (!(std::isfinite(dt) && dt > 0)) return fail(c, SGN_E_ARG, "dt must be finite and > 0");
  if (c->p.source != SGN_SRC_NONE) return fail(c, SGN_E_UNSUPPORTED, "the VJP is defined without source terms");
  if ((st = ensure_vjp_buffers(c)) || (st = ensure_stage_slots(c, 4))) return st;
  void* ys = c->adj.stages;
  void* qnext = slot(c->adj.stages, 3, c);
  HIPCHK(c, forward_step_keep(c, c->stream, q_n, ys, qnext, dt));
  void* out = nullptr;
  HIPCHK(c, reverse_step(c, c->stream, q_n, ys, qbar, bbar, dt, &out));
  if (out != qbar) HIPCHK(c, hipMemcpyAsync(qbar, out, state_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  return SGN_OK;
}

sgn_status sgn_gauge_series(sgn_ctx* c, const void* zeta0, int64_t nsteps, double dt, const int64_t* gauge_idx,
                            int32_t ngauges, double* series) {
  sgn_status st = gauge_args(c, zeta0, nsteps, dt, gauge_idx, ngauges);
  if (st) return st;
  if (!series) return fail(c, SGN_E_ARG, "series is NULL");
  auto& a = c->adj;
  if (!a.state && hipMalloc(&a.state, state_bytes(c)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SGN_E_ALLOC, "rollout state");
  }
  HIPCHK(c, launch_surface(c, zeta0, a.state));
  void* cur = a.state;
  void* oth = c->acc;
  for (int64_t n = 1; n <= nsteps; ++n) {
    HIPCHK(c, rollout_step(c, c->stream, cur, oth, dt));
    std::swap(cur, oth);
    HIPCHK(c, launch_record(c, cur, gauge_idx, ngauges, series + (n - 1) * ngauges, nullptr, nullptr, nullptr));
  }
  return sgn_host::sync_results(c, 0);
}

sgn_status sgn_gauge_loss_grad(sgn_ctx* c, const void* zeta0, int64_t nsteps, double dt, const int64_t* gauge_idx,
                               int32_t ngauges, const double* target, int64_t checkpoint_every, double* loss,
                               void* grad_zeta0, void* grad_b) {
  sgn_status st = gauge_args(c, zeta0, nsteps, dt, gauge_idx, ngauges);
  if (st) return st;
  if (!target || !loss || !grad_zeta0 || !grad_b) return fail(c, SGN_E_ARG, "NULL argument");
  const size_t sb = state_bytes(c);
  // The last F steps keep their states and stage states from the forward
  // rollout (4F+1 states within the SGN_OPT_ADJOINT_STORE budget); the first
  // T0 = nsteps - F are checkpointed every K steps and recomputed segment by
  // segment in the reverse sweep.
  const int64_t budget_states = c->adj_store_bytes / (int64_t)sb;
  const int64_t F = budget_states >= 5 ? std::min<int64_t>(nsteps, (budget_states - 1) / 4) : 0;
  const int64_t T0 = nsteps - F;
  int64_t K = 1, nseg = 0;
  if (T0 > 0) {
    K = checkpoint_every > 0 ? checkpoint_every : (int64_t)std::ceil(std::sqrt((double)T0));
    K = std::max<int64_t>(1, std::min<int64_t>(K, T0));
    nseg = (T0 + K - 1) / K;
  }
  const size_t slots = (size_t)std::max<int64_t>(T0 > 0 ? 4 * K + 1 : 0, F > 0 ? 4 * F + 1 : 0);
  auto& a = c->adj;
  if ((st = ensure_vjp_buffers(c)) || (st = ensure_stage_slots(c, slots))) return st;
  bool ok = true;
  if (!a.state) ok = ok && hipMalloc(&a.state, sb) == hipSuccess;
  if (!a.qbar) ok = ok && hipMalloc(&a.qbar, sb) == hipSuccess;
  if (a.ckpt_slots < (size_t)nseg) {
    if (a.ckpt) (void)hipFree(a.ckpt);
    a.ckpt = nullptr;
    a.ckpt_slots = 0;
    ok = ok && hipMalloc(&a.ckpt, (size_t)nseg * sb) == hipSuccess;
    if (ok) a.ckpt_slots = (size_t)nseg;
  }
  const size_t mlen = (size_t)nsteps * (size_t)ngauges;
  if (a.misfit_len < mlen) {
    if (a.misfit) (void)hipFree(a.misfit);
    a.misfit = nullptr;
    a.misfit_len = 0;
    ok = ok && hipMalloc((void**)&a.misfit, mlen * sizeof(double)) == hipSuccess;
    if (ok) a.misfit_len = mlen;
  }
  if (!a.loss) ok = ok && hipMalloc((void**)&a.loss, sizeof(double)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return fail(c, SGN_E_ALLOC, "adjoint rollout storage");
  }
  hipStream_t s = c->stream;
  // 1. forward rollout: checkpoints every K steps over the first T0 steps, then
  //    the last F steps keeping every state and stage state (slot layout of a
  //    segment: states 0..F at slots [0, F], stage triples from slot F+1);
  //    misfits and loss throughout
  HIPCHK(c, hipMemsetAsync(a.loss, 0, sizeof(double), s));
  HIPCHK(c, launch_surface(c, zeta0, a.state));
  void* cur = a.state;
  void* oth = c->acc;
  for (int64_t n = 0; n < nsteps; ++n) {
    if (n < T0) {
      if (n % K == 0) HIPCHK(c, hipMemcpyAsync(slot(a.ckpt, (size_t)(n / K), c), cur, sb, hipMemcpyDeviceToDevice, s));
      HIPCHK(c, rollout_step(c, s, cur, oth, dt));
      std::swap(cur, oth);
    } else {
      const int64_t k = n - T0;
      if (k == 0) HIPCHK(c, hipMemcpyAsync(slot(a.stages, 0, c), cur, sb, hipMemcpyDeviceToDevice, s));
      HIPCHK(c, forward_step_keep(c, s, slot(a.stages, (size_t)k, c), slot(a.stages, (size_t)(F + 1 + 3 * k), c),
                                  slot(a.stages, (size_t)(k + 1), c), dt));
      cur = slot(a.stages, (size_t)(k + 1), c);
    }
    HIPCHK(c, launch_record(c, cur, gauge_idx, ngauges, nullptr, target + n * ngauges, a.misfit + n * ngauges, a.loss));
  }
  // 2. reverse sweep: the kept steps, then one segment at a time (recompute
  //    the segment keeping every state and stage state, then reverse its steps)
  HIPCHK(c, hipMemsetAsync(a.qbar, 0, sb, s));
  HIPCHK(c, hipMemsetAsync(grad_b, 0, c->N * c->esize, s));
  // reverse of step n = n0 + k from the segment storage of length len
  const auto reverse_from_slots = [&](int64_t n0, int64_t len, int64_t k) -> sgn_status {
    const int64_t n = n0 + k;  // step n maps q_n to q_{n+1}; misfit row n belongs to q_{n+1}
    if (c->p.dtype == SGN_F64)
      hipLaunchKernelGGL(gauge_seed<double>, dim3((ngauges + GAUGE_THREADS - 1) / GAUGE_THREADS), dim3(GAUGE_THREADS),
                         0, s, gauge_idx, ngauges, c->N, a.misfit + n * ngauges, (double*)a.qbar, (double*)grad_b);
    else
      hipLaunchKernelGGL(gauge_seed<float>, dim3((ngauges + GAUGE_THREADS - 1) / GAUGE_THREADS), dim3(GAUGE_THREADS),
                         0, s, gauge_idx, ngauges, c->N, a.misfit + n * ngauges, (float*)a.qbar, (float*)grad_b);
    HIPCHK(c, hipGetLastError());
    void* out = nullptr;
    HIPCHK(c, reverse_step(c, s, slot(a.stages, (size_t)k, c), slot(a.stages, (size_t)(len + 1 + 3 * k), c), a.qbar,
                           grad_b, dt, &out));
    if (out != a.qbar) std::swap(a.qbar, a.kb_b);  // both buffers belong to the context
    return SGN_OK;
  };
  for (int64_t k = F - 1; k >= 0; --k)
    if ((st = reverse_from_slots(T0, F, k))) return st;
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t n0 = seg * K;
    const int64_t len = std::min<int64_t>(K, T0 - n0);
    HIPCHK(c, hipMemcpyAsync(slot(a.stages, 0, c), slot(a.ckpt, (size_t)seg, c), sb, hipMemcpyDeviceToDevice, s));
    for (int64_t k = 0; k < len; ++k)
      HIPCHK(c, forward_step_keep(c, s, slot(a.stages, (size_t)k, c), slot(a.stages, (size_t)(len + 1 + 3 * k), c),
                                  slot(a.stages, (size_t)(k + 1), c), dt));
    for (int64_t k = len - 1; k >= 0; --k)
      if ((st = reverse_from_slots(n0, len, k))) return st;
  }
  // 3. reverse of the initialization
  const dim3 grid((unsigned)((c->N + 255) / 256)), block(256);
  if (c->p.dtype == SGN_F64)
    hipLaunchKernelGGL(init_reverse<double>, grid, block, 0, s, (const double*)a.qbar, (const double*)grad_b,
                       (double*)grad_zeta0, (double*)grad_b, c->N);
  else
    hipLaunchKernelGGL(init_reverse<float>, grid, block, 0, s, (const float*)a.qbar, (const float*)grad_b,
                       (float*)grad_zeta0, (float*)grad_b, c->N);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->host_result, a.loss, sizeof(double), hipMemcpyDeviceToHost, s));
  if ((st = sgn_host::sync_results(c, 0))) return st;
  *loss = c->host_result[0];
  return SGN_OK;
}

}  // extern "C"
