// sgn_batch.hip -- C ABI of the ensemble solver (sgn_batch_* in include/sgn.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "sgn.h"
#include "sgn_batch.hpp"
#include "sgn_reduce.hpp"

namespace {

thread_local std::string g_batch_create_error;

constexpr int BATCH_GRAPH_DOUBLE_STEPS = 4;  // 8 RK4 steps per graph replay

}  // namespace

struct sgn_batch {
  int n = 0;
  int dtype = SGN_F64;
  size_t esize = 8;
  std::vector<sgn_params> params;
  std::vector<sgn::GridConst> gcs;
  std::vector<size_t> offs;  // first node of each instance in the packed scratch
  size_t total = 0;          // sum of nx*ny
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  void* b_all = nullptr;
  void* acc_all = nullptr;
  void* yb_all = nullptr;
  sgn::InstDesc* d_desc = nullptr;
  sgn::InstDesc* h_desc = nullptr;  // pinned staging
  int* d_work = nullptr;
  int nwork = 0;
  int work_key = 0;  // path and tile height the work list was built for
  int* d_flags = nullptr;
  int* h_flags = nullptr;
  double* d_partials = nullptr;
  double* d_results = nullptr;
  double* h_results = nullptr;
  std::vector<void*> q;
  std::vector<double> dt;
  std::vector<char> b_set;
  bool q_set = false;
  bool desc_dirty = true;
  int path = SGN_PATH_FUSED;
  int tile_y = 24;  // tile height; step tiles 64 x 8, 32 x 16 or 32 x 24, pair tiles 64 x 8 or 64 x 16
  int blocks_per_cu = 0;  // one workgroup per tile
  int num_cus = 256;
  hipGraphExec_t gexec = nullptr;
  int g_key = 0, g_bpc = 0;
  std::string err;
};

namespace {

sgn_status bfail(sgn_batch* b, sgn_status st, const std::string& msg) {
  if (b)
    b->err = msg;
  else
    g_batch_create_error = msg;
  return st;
}

sgn_status bhip(sgn_batch* b, hipError_t e, const char* what) {
  return bfail(b, SGN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define BCHK(b, expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return bhip((b), e_, #expr);  \
  } while (0)

double spacing(int n, double lo, double hi, int bc) { return bc == SGN_PERIODIC ? (hi - lo) / n : (hi - lo) / (n - 1); }

void drop_graph(sgn_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
}

int work_key(const sgn_batch* b) { return b->path * 100 + b->tile_y; }

int tile_width(const sgn_batch* b) {
  return b->path == SGN_PATH_FUSED ? (b->tile_y == 8 ? sgn::StepGeom<8>::TX : sgn::StepGeom<16>::TX) : sgn::TILE_X;
}

// (Re)build the work list and descriptors for the current path and tile height.
sgn_status build_work(sgn_batch* b) {
  if (b->work_key == work_key(b) && b->d_work) return SGN_OK;
  std::vector<int> work;
  const int tw = tile_width(b);
  for (int i = 0; i < b->n; ++i) {
    sgn::InstDesc& d = b->h_desc[i];
    d.ntx = (b->params[i].nx + tw - 1) / tw;
    d.nty = (b->params[i].ny + b->tile_y - 1) / b->tile_y;
    d.tile_base = (int)work.size();
    for (int t = 0; t < d.ntx * d.nty; ++t) work.push_back(i);
  }
  if (b->d_work) (void)hipFree(b->d_work);
  b->d_work = nullptr;
  BCHK(b, hipMalloc((void**)&b->d_work, work.size() * sizeof(int)));
  BCHK(b, hipMemcpy(b->d_work, work.data(), work.size() * sizeof(int), hipMemcpyHostToDevice));
  b->nwork = (int)work.size();
  b->work_key = work_key(b);
  b->desc_dirty = true;
  drop_graph(b);
  return SGN_OK;
}

sgn_status push_desc(sgn_batch* b) {
  if (!b->desc_dirty) return SGN_OK;
  // The pinned staging copy may still be read by an earlier async copy.
  BCHK(b, hipStreamSynchronize(b->stream));
  for (int i = 0; i < b->n; ++i) {
    b->h_desc[i].q = b->q[i];
    b->h_desc[i].dt = b->dt[i];
  }
  BCHK(b, hipMemcpyAsync(b->d_desc, b->h_desc, b->n * sizeof(sgn::InstDesc), hipMemcpyHostToDevice, b->stream));
  b->desc_dirty = false;
  return SGN_OK;
}

// Persistent grid: blocks_per_cu workgroups per CU, a multiple of 8 (one range
// of the work list per XCD), no more than the work items.
int persistent_grid(const sgn_batch* b, int bpc) {
  int grid = b->num_cus * bpc;
  grid = (grid + 7) / 8 * 8;
  const int maxgrid = (b->nwork + 7) / 8 * 8;
  return std::max(8, std::min(grid, maxgrid));
}

// blocks_per_cu 0 selects one workgroup per work item, else a persistent grid.
template <typename T, int PAIR, int TY>
void launch_batch_pair_k(const sgn_batch* b, hipStream_t s, int parity, int bpc) {
  if (bpc == 0)
    hipLaunchKernelGGL((sgn::batch_pair_kernel<T, PAIR, TY, false>), dim3(b->nwork), dim3(sgn::STAGE_THREADS), 0, s,
                       b->d_desc, b->d_work, b->nwork, parity, b->d_flags);
  else
    hipLaunchKernelGGL((sgn::batch_pair_kernel<T, PAIR, TY, true>), dim3(persistent_grid(b, bpc)),
                       dim3(sgn::STAGE_THREADS), 0, s, b->d_desc, b->d_work, b->nwork, parity, b->d_flags);
}

template <typename T, int TY>
hipError_t launch_batch_pair_t(const sgn_batch* b, hipStream_t s, int pair, int parity, int bpc) {
  if (pair == 1)
    launch_batch_pair_k<T, 1, TY>(b, s, parity, bpc);
  else
    launch_batch_pair_k<T, 2, TY>(b, s, parity, bpc);
  return hipGetLastError();
}

hipError_t launch_batch_pair(const sgn_batch* b, hipStream_t s, int pair, int parity) {
  if (b->dtype == SGN_F64)
    return b->tile_y == 16 ? launch_batch_pair_t<double, 16>(b, s, pair, parity, b->blocks_per_cu)
                           : launch_batch_pair_t<double, 8>(b, s, pair, parity, b->blocks_per_cu);
  return b->tile_y == 16 ? launch_batch_pair_t<float, 16>(b, s, pair, parity, b->blocks_per_cu)
                         : launch_batch_pair_t<float, 8>(b, s, pair, parity, b->blocks_per_cu);
}

template <typename T, int TY>
hipError_t launch_batch_step_t(const sgn_batch* b, hipStream_t s, int parity, int bpc) {
  if (TY == 24 || bpc == 0) {  // one workgroup per 32 x 24 tile: no persistent instance of that shape
    hipLaunchKernelGGL((sgn::batch_step_kernel<T, TY, false>), dim3(b->nwork), dim3(sgn::STAGE_THREADS), 0, s,
                       b->d_desc, b->d_work, b->nwork, parity, b->d_flags);
  } else if constexpr (TY != 24) {
    hipLaunchKernelGGL((sgn::batch_step_kernel<T, TY, true>), dim3(persistent_grid(b, bpc)), dim3(sgn::STAGE_THREADS),
                       0, s, b->d_desc, b->d_work, b->nwork, parity, b->d_flags);
  }
  return hipGetLastError();
}

// One RK4 step of every instance from the buffer selected by parity into the other.
hipError_t enqueue_batch_step(const sgn_batch* b, hipStream_t s, int parity) {
  if (b->path == SGN_PATH_FUSED) {
    if (b->dtype == SGN_F64)
      return b->tile_y == 24   ? launch_batch_step_t<double, 24>(b, s, parity, b->blocks_per_cu)
             : b->tile_y == 16 ? launch_batch_step_t<double, 16>(b, s, parity, b->blocks_per_cu)
                               : launch_batch_step_t<double, 8>(b, s, parity, b->blocks_per_cu);
    return b->tile_y == 24   ? launch_batch_step_t<float, 24>(b, s, parity, b->blocks_per_cu)
           : b->tile_y == 16 ? launch_batch_step_t<float, 16>(b, s, parity, b->blocks_per_cu)
                             : launch_batch_step_t<float, 8>(b, s, parity, b->blocks_per_cu);
  }
  hipError_t e = launch_batch_pair(b, s, 1, parity);
  if (e) return e;
  return launch_batch_pair(b, s, 2, parity);
}

sgn_status ready(sgn_batch* b, bool need_q) {
  if (!b) return SGN_E_ARG;
  for (int i = 0; i < b->n; ++i)
    if (!b->b_set[i]) return bfail(b, SGN_E_STATE, "bathymetry of instance " + std::to_string(i) + " not set");
  if (need_q && !b->q_set) return bfail(b, SGN_E_STATE, "states not set (call sgn_batch_set_states)");
  return SGN_OK;
}

sgn_status sync_flags(sgn_batch* b, int32_t* first_bad) {
  BCHK(b, hipMemcpyAsync(b->h_flags, b->d_flags, b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  int bad = -1, f = 0;
  for (int i = 0; i < b->n; ++i)
    if (b->h_flags[i]) {
      bad = i;
      f = b->h_flags[i];
      break;
    }
  if (first_bad) *first_bad = bad;
  if (bad >= 0) {
    BCHK(b, hipMemsetAsync(b->d_flags, 0, b->n * sizeof(int), b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    if (f & sgn::FLAG_NONFINITE) return bfail(b, SGN_E_NONFINITE, "instance " + std::to_string(bad) + " produced a non-finite value");
    return bfail(b, SGN_E_NONPOS_DEPTH, "instance " + std::to_string(bad) + " produced h <= 0");
  }
  return SGN_OK;
}

}  // namespace

extern "C" {

const char* sgn_batch_last_error(const sgn_batch* b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

sgn_status sgn_batch_create(int32_t n, const sgn_params* params, void* stream, sgn_batch** out) {
  if (!out) return bfail(nullptr, SGN_E_ARG, "out is NULL");
  *out = nullptr;
  if (n <= 0 || !params) return bfail(nullptr, SGN_E_ARG, "need n > 0 instances and their params");
  const int dtype = params[0].dtype;
  if (dtype != SGN_F64 && dtype != SGN_F32) return bfail(nullptr, SGN_E_ARG, "unknown dtype");
  sgn_batch* b = new sgn_batch();
  b->n = n;
  b->dtype = dtype;
  b->esize = dtype == SGN_F64 ? sizeof(double) : sizeof(float);
  b->tile_y = 24;
  b->stream = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    const sgn_params& p = params[i];
    std::string tag = "instance " + std::to_string(i) + ": ";
    sgn_status st = SGN_OK;
    std::string msg;
    if (p.dtype != dtype) { st = SGN_E_ARG; msg = "all instances must share one dtype"; }
    else if (p.source != SGN_SRC_NONE) { st = SGN_E_UNSUPPORTED; msg = "source terms are not supported in a batch"; }
    else if (p.nx < 4 || p.ny < 4) { st = SGN_E_SHAPE; msg = "each axis needs at least 4 nodes"; }
    else if (!(std::isfinite(p.xmin) && std::isfinite(p.xmax) && p.xmax > p.xmin && std::isfinite(p.ymin) &&
               std::isfinite(p.ymax) && p.ymax > p.ymin)) { st = SGN_E_SHAPE; msg = "bad domain"; }
    else if ((p.bc_x != 0 && p.bc_x != 1) || (p.bc_y != 0 && p.bc_y != 1)) { st = SGN_E_ARG; msg = "unknown boundary type"; }
    else if (!(std::isfinite(p.g) && p.g > 0) || !(std::isfinite(p.lambda) && p.lambda >= 0)) { st = SGN_E_ARG; msg = "bad g or lambda"; }
    if (st) {
      delete b;
      return bfail(nullptr, st, tag + msg);
    }
    b->params.push_back(p);
    sgn::GridConst gc{};
    gc.nx = p.nx;
    gc.ny = p.ny;
    gc.bc_x = p.bc_x;
    gc.bc_y = p.bc_y;
    gc.dx = spacing(p.nx, p.xmin, p.xmax, p.bc_x);
    gc.dy = spacing(p.ny, p.ymin, p.ymax, p.bc_y);
    gc.inv2dx = 1.0 / (2.0 * gc.dx);
    gc.inv2dy = 1.0 / (2.0 * gc.dy);
    gc.invdx = 1.0 / gc.dx;
    gc.invdy = 1.0 / gc.dy;
    gc.xmin = p.xmin;
    gc.ymin = p.ymin;
    gc.g = p.g;
    gc.lam = p.lambda;
    b->gcs.push_back(gc);
    b->offs.push_back(b->total);
    b->total += (size_t)p.nx * (size_t)p.ny;
  }
  b->q.assign(n, nullptr);
  b->dt.assign(n, 0.0);
  b->b_set.assign(n, 0);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete b;
    return bfail(nullptr, SGN_E_HIP, "cannot query the device");
  }
  const size_t plane = b->total * b->esize;
  bool ok = hipMalloc(&b->b_all, plane) == hipSuccess && hipMalloc(&b->acc_all, 5 * plane) == hipSuccess &&
            hipMalloc(&b->yb_all, 5 * plane) == hipSuccess &&
            hipMalloc((void**)&b->d_desc, n * sizeof(sgn::InstDesc)) == hipSuccess &&
            hipHostMalloc((void**)&b->h_desc, n * sizeof(sgn::InstDesc), hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void**)&b->d_flags, n * sizeof(int)) == hipSuccess &&
            hipHostMalloc((void**)&b->h_flags, n * sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void**)&b->d_partials, (size_t)n * 4 * sgn::RED_MAX_BLOCKS * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&b->d_results, (size_t)n * 2 * sizeof(double)) == hipSuccess &&
            hipHostMalloc((void**)&b->h_results, (size_t)n * 2 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
            hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    sgn_batch_destroy(b);
    return bfail(nullptr, SGN_E_ALLOC, "device allocation failed");
  }
  for (int i = 0; i < n; ++i) {
    sgn::InstDesc& d = b->h_desc[i];
    d = sgn::InstDesc{};
    d.gc = b->gcs[i];
    d.acc = (char*)b->acc_all + 5 * b->offs[i] * b->esize;
    d.yb = (char*)b->yb_all + 5 * b->offs[i] * b->esize;
    d.b = (char*)b->b_all + b->offs[i] * b->esize;
  }
  sgn_status st = build_work(b);
  if (st == SGN_OK && (hipMemsetAsync(b->d_flags, 0, n * sizeof(int), b->stream) != hipSuccess ||
                       hipStreamSynchronize(b->stream) != hipSuccess))
    st = SGN_E_HIP;
  if (st) {
    std::string m = b->err;
    sgn_batch_destroy(b);
    return bfail(nullptr, st, m.empty() ? "initialization failed" : m);
  }
  *out = b;
  return SGN_OK;
}

sgn_status sgn_batch_destroy(sgn_batch* b) {
  if (!b) return SGN_OK;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->b_all) (void)hipFree(b->b_all);
  if (b->acc_all) (void)hipFree(b->acc_all);
  if (b->yb_all) (void)hipFree(b->yb_all);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->d_flags) (void)hipFree(b->d_flags);
  if (b->h_flags) (void)hipHostFree(b->h_flags);
  if (b->d_partials) (void)hipFree(b->d_partials);
  if (b->d_results) (void)hipFree(b->d_results);
  if (b->h_results) (void)hipHostFree(b->h_results);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return SGN_OK;
}

sgn_status sgn_batch_set_bathymetry(sgn_batch* b, int32_t i, const void* bath) {
  if (!b) return SGN_E_ARG;
  if (i < 0 || i >= b->n || !bath) return bfail(b, SGN_E_ARG, "bad instance index or NULL b");
  const size_t N = (size_t)b->params[i].nx * b->params[i].ny;
  BCHK(b, hipMemcpyAsync((char*)b->b_all + b->offs[i] * b->esize, bath, N * b->esize, hipMemcpyDeviceToDevice, b->stream));
  b->b_set[i] = 1;
  return SGN_OK;
}

sgn_status sgn_batch_set_states(sgn_batch* b, void* const* q) {
  if (!b) return SGN_E_ARG;
  if (!q) return bfail(b, SGN_E_ARG, "q is NULL");
  for (int i = 0; i < b->n; ++i) {
    if (!q[i]) return bfail(b, SGN_E_ARG, "state pointer " + std::to_string(i) + " is NULL");
    if (b->q[i] != q[i]) {
      b->q[i] = q[i];
      b->desc_dirty = true;
      drop_graph(b);
    }
  }
  b->q_set = true;
  return SGN_OK;
}

sgn_status sgn_batch_init_aux(sgn_batch* b) {
  sgn_status st = ready(b, true);
  if (st) return st;
  for (int i = 0; i < b->n; ++i) {
    const sgn::GridConst& gc = b->gcs[i];
    const dim3 grid((gc.nx + 63) / 64, (gc.ny + 3) / 4), block(256);
    const void* bp = (char*)b->b_all + b->offs[i] * b->esize;
    if (b->dtype == SGN_F64)
      hipLaunchKernelGGL(sgn::init_aux_kernel<double>, grid, block, 0, b->stream, gc, (double*)b->q[i], (const double*)bp);
    else
      hipLaunchKernelGGL(sgn::init_aux_kernel<float>, grid, block, 0, b->stream, gc, (float*)b->q[i], (const float*)bp);
    BCHK(b, hipGetLastError());
  }
  return SGN_OK;
}

sgn_status sgn_batch_step(sgn_batch* b, const double* dt, int64_t nsteps) {
  sgn_status st = ready(b, true);
  if (st) return st;
  if (!dt) return bfail(b, SGN_E_ARG, "dt is NULL");
  if (nsteps < 0) return bfail(b, SGN_E_ARG, "nsteps must be >= 0");
  for (int i = 0; i < b->n; ++i) {
    if (!(std::isfinite(dt[i]) && dt[i] > 0)) return bfail(b, SGN_E_ARG, "dt of instance " + std::to_string(i) + " must be finite and > 0");
    if (b->dt[i] != dt[i]) {
      b->dt[i] = dt[i];
      b->desc_dirty = true;
    }
  }
  if (nsteps == 0) return SGN_OK;
  if ((st = build_work(b))) return st;
  if ((st = push_desc(b))) return st;
  int64_t left = nsteps;
  const int64_t per_graph = 2 * BATCH_GRAPH_DOUBLE_STEPS;
  if (left >= per_graph) {
    if (!b->gexec || b->g_key != work_key(b) || b->g_bpc != b->blocks_per_cu) {
      drop_graph(b);
      BCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = hipSuccess;
      for (int k = 0; k < BATCH_GRAPH_DOUBLE_STEPS && le == hipSuccess; ++k) {
        le = enqueue_batch_step(b, b->cap_stream, 0);
        if (le == hipSuccess) le = enqueue_batch_step(b, b->cap_stream, 1);
      }
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(b->cap_stream, &graph);
      if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return bhip(b, le, "batch launch during capture");
      }
      if (ce != hipSuccess) return bhip(b, ce, "hipStreamEndCapture");
      hipError_t ie = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        b->gexec = nullptr;
        return bhip(b, ie, "hipGraphInstantiate");
      }
      b->g_key = work_key(b);
      b->g_bpc = b->blocks_per_cu;
    }
    for (; left >= per_graph; left -= per_graph) BCHK(b, hipGraphLaunch(b->gexec, b->stream));
  }
  for (; left >= 2; left -= 2) {
    BCHK(b, enqueue_batch_step(b, b->stream, 0));
    BCHK(b, enqueue_batch_step(b, b->stream, 1));
  }
  if (left == 1) {
    // The last step lands in the scratch buffer; copy every state back.
    BCHK(b, enqueue_batch_step(b, b->stream, 0));
    for (int i = 0; i < b->n; ++i) {
      const size_t bytes = 5 * (size_t)b->params[i].nx * b->params[i].ny * b->esize;
      BCHK(b, hipMemcpyAsync(b->q[i], b->h_desc[i].acc, bytes, hipMemcpyDeviceToDevice, b->stream));
    }
  }
  return SGN_OK;
}

sgn_status sgn_batch_mass_energy(sgn_batch* b, double* mass, double* energy) {
  sgn_status st = ready(b, true);
  if (st) return st;
  for (int i = 0; i < b->n; ++i) {
    const sgn::GridConst& gc = b->gcs[i];
    const int nb = std::min(gc.ny, sgn::RED_MAX_BLOCKS);
    double* part = b->d_partials + (size_t)i * 4 * sgn::RED_MAX_BLOCKS;
    const void* bp = (char*)b->b_all + b->offs[i] * b->esize;
    if (b->dtype == SGN_F64)
      hipLaunchKernelGGL((sgn::totals_partial<double, 0>), dim3(nb), dim3(sgn::RED_THREADS), 0, b->stream, gc,
                         (const double*)b->q[i], (const double*)bp, (const double*)nullptr, part);
    else
      hipLaunchKernelGGL((sgn::totals_partial<float, 0>), dim3(nb), dim3(sgn::RED_THREADS), 0, b->stream, gc,
                         (const float*)b->q[i], (const float*)bp, (const float*)nullptr, part);
    hipLaunchKernelGGL(sgn::totals_final, dim3(1), dim3(sgn::RED_THREADS), 0, b->stream, part, nb, b->d_results + 2 * i);
    BCHK(b, hipGetLastError());
  }
  BCHK(b, hipMemcpyAsync(b->h_results, b->d_results, b->n * 2 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  if ((st = sync_flags(b, nullptr))) return st;
  for (int i = 0; i < b->n; ++i) {
    if (mass) mass[i] = b->h_results[2 * i];
    if (energy) energy[i] = b->h_results[2 * i + 1];
  }
  return SGN_OK;
}

sgn_status sgn_batch_cfl_dt(sgn_batch* b, double cfl, double* dt) {
  sgn_status st = ready(b, true);
  if (st) return st;
  if (!dt || !(std::isfinite(cfl) && cfl > 0)) return bfail(b, SGN_E_ARG, "bad cfl or NULL dt");
  for (int i = 0; i < b->n; ++i) {
    const sgn::GridConst& gc = b->gcs[i];
    const int nb = std::min(gc.ny, sgn::RED_MAX_BLOCKS);
    double* part = b->d_partials + (size_t)i * 4 * sgn::RED_MAX_BLOCKS;
    if (b->dtype == SGN_F64)
      hipLaunchKernelGGL(sgn::speed_partial<double>, dim3(nb), dim3(sgn::RED_THREADS), 0, b->stream, gc,
                         (const double*)b->q[i], part);
    else
      hipLaunchKernelGGL(sgn::speed_partial<float>, dim3(nb), dim3(sgn::RED_THREADS), 0, b->stream, gc,
                         (const float*)b->q[i], part);
    hipLaunchKernelGGL(sgn::speed_final, dim3(1), dim3(sgn::RED_THREADS), 0, b->stream, part, nb, b->d_results + i);
    BCHK(b, hipGetLastError());
  }
  BCHK(b, hipMemcpyAsync(b->h_results, b->d_results, b->n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  if ((st = sync_flags(b, nullptr))) return st;
  for (int i = 0; i < b->n; ++i) {
    const double m = b->h_results[i];
    if (!(std::isfinite(m) && m > 0)) return bfail(b, SGN_E_NONFINITE, "speed of instance " + std::to_string(i) + " is not finite and positive");
    dt[i] = cfl / m;
  }
  return SGN_OK;
}

sgn_status sgn_batch_set_step_path(sgn_batch* b, int32_t path) {
  if (!b) return SGN_E_ARG;
  if (path != SGN_PATH_FUSED && path != SGN_PATH_PAIRS)
    return bfail(b, SGN_E_UNSUPPORTED, "a batch steps on the fused or the pair path");
  b->path = path;
  b->tile_y = path == SGN_PATH_PAIRS ? (b->dtype == SGN_F64 ? 8 : 16) : 24;  // measured best on MI355X
  drop_graph(b);
  return build_work(b);
}

sgn_status sgn_batch_set_tiling(sgn_batch* b, int32_t tile_y, int32_t blocks_per_cu) {
  if (!b) return SGN_E_ARG;
  if (!(tile_y == 8 || tile_y == 16 || (tile_y == 24 && b->path == SGN_PATH_FUSED)))
    return bfail(b, SGN_E_UNSUPPORTED, "tile height must be 8 or 16 (or 24 on the fused path)");
  if (tile_y == 24 && blocks_per_cu != 0)
    return bfail(b, SGN_E_UNSUPPORTED, "32 x 24 step tiles run one workgroup per tile (blocks_per_cu 0)");
  if (blocks_per_cu < 0 || blocks_per_cu > 16) return bfail(b, SGN_E_ARG, "blocks per CU must be in [0, 16]");
  b->tile_y = tile_y;
  b->blocks_per_cu = blocks_per_cu;
  drop_graph(b);
  return build_work(b);
}

sgn_status sgn_batch_autotune(sgn_batch* b, const double* dt, int32_t* tile_y, int32_t* blocks_per_cu, double* ms) {
  sgn_status st = ready(b, true);
  if (st) return st;
  if (!dt) return bfail(b, SGN_E_ARG, "dt is NULL");
  for (int i = 0; i < b->n; ++i) {
    if (!(std::isfinite(dt[i]) && dt[i] > 0)) return bfail(b, SGN_E_ARG, "bad dt");
    if (b->dt[i] != dt[i]) {
      b->dt[i] = dt[i];
      b->desc_dirty = true;
    }
  }
  // Candidates are timed on one step from q into the scratch buffer (parity 0),
  // which reads the states but never writes them.
  const int tys[3] = {8, 16, 24};
  const int bpcs[7] = {0, 1, 2, 3, 4, 5, 6};
  double best = 1e300;
  int best_ty = b->tile_y, best_bpc = b->blocks_per_cu;
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0));
  BCHK(b, hipEventCreate(&e1));
  for (int ty : tys) {
    if (ty == 24 && b->path != SGN_PATH_FUSED) continue;
    b->tile_y = ty;
    if ((st = build_work(b)) || (st = push_desc(b))) break;
    for (int bpc : bpcs) {
      if (ty == 24 && bpc != 0) continue;  // one workgroup per 32 x 24 tile
      b->blocks_per_cu = bpc;
      hipError_t e = enqueue_batch_step(b, b->stream, 0);  // warm-up
      if (!e) e = hipEventRecord(e0, b->stream);
      for (int r = 0; r < 3 && !e; ++r) e = enqueue_batch_step(b, b->stream, 0);
      if (!e) e = hipEventRecord(e1, b->stream);
      if (!e) e = hipEventSynchronize(e1);
      float t = 0.f;
      if (!e) e = hipEventElapsedTime(&t, e0, e1);
      if (e) {
        st = bhip(b, e, "autotune");
        break;
      }
      if (t < best) {
        best = t;
        best_ty = ty;
        best_bpc = bpc;
      }
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  b->tile_y = best_ty;
  b->blocks_per_cu = best_bpc;
  drop_graph(b);
  if ((st = build_work(b)) || (st = push_desc(b))) return st;
  if (tile_y) *tile_y = best_ty;
  if (blocks_per_cu) *blocks_per_cu = best_bpc;
  if (ms) *ms = best / 3.0;
  return sync_flags(b, nullptr);
}

sgn_status sgn_batch_check(sgn_batch* b, int32_t* first_bad) {
  if (!b) return SGN_E_ARG;
  return sync_flags(b, first_bad);
}

sgn_status sgn_batch_total_nodes(const sgn_batch* b, int64_t* nodes) {
  if (!b || !nodes) return SGN_E_ARG;
  *nodes = (int64_t)b->total;
  return SGN_OK;
}

}  // extern "C"
