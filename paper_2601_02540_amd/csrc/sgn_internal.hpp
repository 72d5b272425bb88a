// sgn_internal.hpp -- host-side context shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "sgn.h"
#include "sgn_common.hpp"

namespace sgn_host {

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const void* q = nullptr;
  double dt = 0.0;
  int steps = 0;
  int path = -1;
  int tile_y = 0;
  int step_tile = 0;
};

// Buffers of the discrete adjoint, allocated on first use and kept by the context.
struct AdjointBuffers {
  void* kb_a = nullptr;   // stage cotangents (ping-pong)
  void* kb_b = nullptr;
  void* accb = nullptr;   // running sum of the stage cotangents of one step
  void* qbar = nullptr;   // cotangent of the state
  void* state = nullptr;  // state of a rollout
  void* stages = nullptr; // per-step stored states of a segment: (steps+1) states and 3 stage states per step
  size_t stage_slots = 0; // number of state-sized slots in `stages`
  void* ckpt = nullptr;   // checkpoints
  size_t ckpt_slots = 0;
  double* misfit = nullptr;  // nsteps * ngauges misfits of the forward rollout
  size_t misfit_len = 0;
  double* loss = nullptr;    // device accumulator
};

// Buffers of the adaptive pair (sgn_step_adaptive), allocated on first use.
struct FsalBuffers {
  void* k[2] = {nullptr, nullptr};  // k_1 of the current step / of the next one (FSAL)
  void* e = nullptr;                // partial error estimate
  double* part = nullptr;           // per-tile sums of the scaled squares
  size_t part_cap = 0;              // doubles in part
  void* ctl = nullptr;              // run state (sgn::AdaptCtl) in device memory
  void* host_ctl = nullptr;         // pinned copy read by the host
  GraphCache graph;                 // attempts captured for replay
  double* graph_rec = nullptr;      // record pointer and capacity captured in the graph
  long long graph_rec_cap = 0;
};

}  // namespace sgn_host

struct sgn_ctx {
  sgn_params p{};
  sgn::GridConst gc{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0;
  size_t N = 0;
  size_t esize = 0;
  void* b = nullptr;
  void* acc = nullptr;
  void* ya = nullptr;
  void* yb = nullptr;
  double* partials = nullptr;
  double* tile_partials = nullptr;  // 4 doubles per step tile (the step kernel's epilogue sums)
  size_t tile_partials_cap = 0;     // doubles allocated there
  int* series_counter = nullptr;    // next slot of a recorded totals series (sgn_step_totals)
  double* result = nullptr;
  double* host_result = nullptr;
  int* flag = nullptr;
  int* host_flag = nullptr;
  bool b_set = false;
  int step_path = SGN_PATH_FUSED;
  int tile_y = 8;     // stage and pair kernels
  int step_tile = 16;  // step kernel: 16 selects 32 x 16, 8 selects 64 x 8
  sgn_host::GraphCache graphs[2];
  sgn_host::GraphCache relax_graph;   // relaxation steps (sgn_step_relaxation)
  sgn_host::GraphCache totals_graph;  // steps with recorded totals (sgn_step_totals)
  double* totals_series = nullptr;    // the series pointer captured in totals_graph
  sgn_host::AdjointBuffers adj;
  int64_t adj_store_bytes = 0;  // SGN_OPT_ADJOINT_STORE
  sgn_host::FsalBuffers fs;
  // Set only inside sgn_profile_stages: the step kernel is then launched with
  // these events bound to its own start and end.
  hipEvent_t prof_start = nullptr, prof_stop = nullptr;
  std::string err;
};

namespace sgn_host {

sgn_status fail(sgn_ctx* c, sgn_status st, const std::string& msg);
sgn_status hip_fail(sgn_ctx* c, hipError_t e, const char* what);
sgn_status sync_results(sgn_ctx* c, int nres);
sgn_status check_ctx(sgn_ctx* c, bool need_b);
void free_adjoint(sgn_ctx* c);
void free_fsal(sgn_ctx* c);
// stage kernel of the four-stage path in mode `mode` (sgn::MODE_*)
hipError_t launch_stage_mode(const sgn_ctx* c, hipStream_t s, int mode, const void* Y, const void* qn, void* acc,
                             void* out, double c_acc, double c_y, double t);
// one RK4 step on the pair path from `cur` into `oth`
hipError_t enqueue_pair_step(const sgn_ctx* c, hipStream_t s, void* cur, void* oth, double dt, double t);
// One RK4 step by the step kernel from `cur` into `oth` (distinct buffers);
// with `ysave` non-null the stage states Y2, Y3, Y4 go to three consecutive
// state slots there; with `rpart` non-null each tile's epilogue sums `epi`
// (sgn::EPI_RELAX: relaxation sums at gam = 1; sgn::EPI_TOTALS: mass and
// energy of the new state) go to rpart[4 tile ..] (step_tiles(c) tiles).
// Neither with source terms, and not both.
hipError_t enqueue_step_into(const sgn_ctx* c, hipStream_t s, const void* cur, void* oth, double dt, double t,
                             void* ysave, double* rpart = nullptr, int epi = 0);
// Number of tiles of the step kernel in the current tile shape.
int step_tiles(const sgn_ctx* c);
// Makes c->tile_partials hold the epilogue sums of either tile shape
// (synchronizes and drops the graphs that captured an older buffer).
sgn_status ensure_tile_partials(sgn_ctx* c);
// Validation of sgn_params (the rules of sgn_create; failures leave their
// message for sgn_last_error(NULL)) and the grid constants the kernels take.
sgn_status check_params(const sgn_params* p);
sgn::GridConst grid_const(const sgn_params& p);

}  // namespace sgn_host

#define SGN_HIPCHK(c, expr)                                                \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) return sgn_host::hip_fail((c), e_, #expr);       \
  } while (0)
