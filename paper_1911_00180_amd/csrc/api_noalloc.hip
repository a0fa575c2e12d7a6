// C-ABI of libwormlbm.so (declared in include/wormlbm.h): the totals readout
// for callers that cannot allocate.
//
// wlbm_read_totals keeps the float64 block partials of its reduction in the
// lattice's workspace and waits for the stream to hand the totals to the
// host.  wlbm_read_totals_noalloc runs the same kernels with the partials in
// a fixed device array of this library (`scratch`, one copy per GPU, held
// until the process ends) and writes the totals to a device buffer of the
// caller, so the call allocates nothing, never waits on the host, and can be
// recorded into a HIP graph.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "api_internal.hpp"

namespace wlbm {
namespace {

// Block partials of one reduction: at most kScratchBlocks blocks, three
// float64 sums each (24 KiB).  The reduction grid is capped at this many
// blocks and grid-strides over the cells, so every lattice fits.
constexpr int kScratchBlocks = 1024;
__device__ __align__(256) double scratch[3 * kScratchBlocks];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch;   // per device ordinal: the address of `scratch` there

}  // namespace

// Look up (once per device) the address of this GPU's copy of `scratch`.
// Called at lattice creation with the lattice's device; host code uses only
// the address returned here, never the array's name.
wlbm_status noalloc_setup(int device) {
  if (device < 0) return fail(WLBM_EINVAL, "invalid device %d", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (size_t(device) < g_scratch.size() && g_scratch[size_t(device)]) return WLBM_OK;
  int prev = -1;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != device) HIP_TRY(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess || !p)
    return fail(WLBM_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                hipGetErrorString(e));
  if (g_scratch.size() <= size_t(device)) g_scratch.resize(size_t(device) + 1, nullptr);
  g_scratch[size_t(device)] = static_cast<double*>(p);
  return WLBM_OK;
}

}  // namespace wlbm

using namespace wlbm;

extern "C" {

wlbm_status wlbm_read_totals_noalloc(wlbm_lattice* l, double* d_totals) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_totals) return fail(WLBM_EINVAL, "totals buffer is NULL");
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (size_t(l->device) < g_scratch.size()) part = g_scratch[size_t(l->device)];
  }
  if (!part)
    return fail(WLBM_ESTATE, "no scratch address for device %d (set up at wlbm_create)",
                l->device);
  HIP_TRY(launch_totals(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]), l->ptr(l->c.sxtab),
                        l->ptr(l->c.sytab), part, kScratchBlocks, d_totals, l->stream));
  return WLBM_OK;
}

}  // extern "C"
