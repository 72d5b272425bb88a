// sgn_noalloc.hip -- totals without a context and without any allocation.
//
// sgn_mass_energy_noalloc runs the same two kernels as sgn_mass_energy
// (per-block compensated partial sums, then one block that merges them in
// block order), so it forms the same bits.  Its partial sums live in a
// file-scope device array instead of a context's buffer.  Each device holds its
// own copy of that array (it comes with the library's code object); host code
// never uses the array's name as an address: the device address is looked up
// once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sgn_internal.hpp"
#include "sgn_reduce.hpp"

// Room for the partial sums of one totals pass: at most RED_MAX_BLOCKS blocks
// (one per grid row up to that many; more rows are strided over the blocks),
// four doubles each -- 32 KiB per device, for every grid size.
constexpr int SCRATCH_DOUBLES = 4 * sgn::RED_MAX_BLOCKS;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
sgn_status device_scratch(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return sgn_host::hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return sgn_host::fail(nullptr, SGN_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch[dev];
  return SGN_OK;
}

template <typename T>
hipError_t launch(const sgn::GridConst& gc, const void* q, const void* b, double* part, int nb, double* out,
                  hipStream_t s) {
  hipLaunchKernelGGL((sgn::totals_partial<T, 0>), dim3(nb), dim3(sgn::RED_THREADS), 0, s, gc, (const T*)q,
                     (const T*)b, (const T*)nullptr, part);
  hipLaunchKernelGGL(sgn::totals_final, dim3(1), dim3(sgn::RED_THREADS), 0, s, part, nb, out);
  return hipGetLastError();
}

}  // namespace

extern "C" sgn_status sgn_mass_energy_noalloc(const sgn_params* p, const void* q, const void* b, void* stream,
                                              double* out) {
  sgn_status st = sgn_host::check_params(p);
  if (st) return st;
  if (!q || !b || !out) return sgn_host::fail(nullptr, SGN_E_ARG, "q, b or out is NULL");
  const int nb = p->ny < sgn::RED_MAX_BLOCKS ? p->ny : sgn::RED_MAX_BLOCKS;
  if (4 * nb > SCRATCH_DOUBLES)  // cannot happen: nb <= RED_MAX_BLOCKS
    return sgn_host::fail(nullptr, SGN_E_SHAPE, "more partial sums than the static scratch holds");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sgn_host::hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return sgn_host::fail(nullptr, SGN_E_UNSUPPORTED, "device index above 63");
  double* part = nullptr;
  if ((st = device_scratch(dev, &part))) return st;
  const sgn::GridConst gc = sgn_host::grid_const(*p);
  e = p->dtype == SGN_F64 ? launch<double>(gc, q, b, part, nb, out, (hipStream_t)stream)
                          : launch<float>(gc, q, b, part, nb, out, (hipStream_t)stream);
  if (e != hipSuccess) return sgn_host::hip_fail(nullptr, e, "totals launch");
  return SGN_OK;
}
