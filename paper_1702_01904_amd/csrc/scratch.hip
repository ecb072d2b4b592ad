// prism_probe_outputs_noalloc: the probe step for callers that cannot
// allocate device memory, with its scratch in a library-held device array.
//
// The array lives in the library's code object, so every GPU the library
// runs on holds its own copy from module load until the process ends. In
// host code the array's name is a host-side stand-in, never passed to a
// kernel or a copy: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current (the entry point's first
// call on it), and only that address reaches the kernels, as the workspace
// of prism_probe_outputs.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "host_util.hpp"
#include "prism.h"

namespace {

static __device__ __align__(256) unsigned char scratch[PRISM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> that device's copy

// Address of the current device's copy of the array (looked up once per
// device, then cached).
hipError_t scratch_address(void** ptr) {
  *ptr = nullptr;
  int dev = -1;
  if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)); e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

}  // namespace

extern "C" int prism_probe_outputs_noalloc(prism_plan* plan, int f, double alpha_max_mrad,
                                           const void* smatrix_dev, size_t smatrix_bytes,
                                           const double* probe_xy_dev, int n_probes,
                                           const prism_optics* optics,
                                           const prism_detector* detector, double* out_dev,
                                           void* stream) {
  // the probe step's minimum workspace must fit the array; decided on the
  // host before the device is touched
  size_t pref = 0, minimum = 0;
  if (int r = prism_probe_workspace_bytes(plan, f, alpha_max_mrad, optics, &pref, &minimum))
    return r;
  if (minimum > (size_t)PRISM_NOALLOC_SCRATCH_BYTES)
    return prism::set_error(
        PRISM_ENOSPACE, "probe step needs " + std::to_string(minimum) +
                            " bytes of scratch, more than the library-held " +
                            std::to_string((size_t)PRISM_NOALLOC_SCRATCH_BYTES) +
                            " (call prism_probe_outputs with a workspace)");
  void* ws = nullptr;
  if (hipError_t e = scratch_address(&ws); e != hipSuccess)
    return prism::set_error(PRISM_EHIP,
                            std::string("library scratch address: ") + hipGetErrorString(e));
  return prism_probe_outputs(plan, f, alpha_max_mrad, smatrix_dev, smatrix_bytes, probe_xy_dev,
                             n_probes, optics, detector, out_dev, ws,
                             (size_t)PRISM_NOALLOC_SCRATCH_BYTES, stream);
}
