// noalloc.hip -- plan execution from a library-owned static device buffer,
// for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The buffer is one file-scope device array per GPU (the runtime gives each
// device its own copy when it loads the library's code there).  Host code
// never uses the array's name as an address: on the first call on a device,
// with that device current, its address is looked up with
// hipGetSymbolAddress and kept per device, and that address is what the
// kernels receive.  Every plan path writes each workspace byte it reads
// before reading it, so nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "comet.h"

namespace comet {
comet_status_t api_fail(comet_status_t code, const std::string &msg);
}

namespace {

__device__ __align__(256) static char scratch[COMET_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> address of that device's copy of `scratch`

comet_status_t scratch_for(int device, void **ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *ptr = it->second;
    return COMET_OK;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return comet::api_fail(COMET_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  *ptr = p;
  return COMET_OK;
}

}  // namespace

extern "C" comet_status_t comet_plan_execute_noalloc(comet_plan_t plan, double alpha, const void *A, const void *B,
                                                     double beta, void *C, void *stream) {
  if (!plan) return comet::api_fail(COMET_ERR_NULL_POINTER, "plan is NULL");
  size_t need = 0;
  comet_status_t rc = comet_plan_workspace_size(plan, &need);
  if (rc != COMET_OK) return rc;
  if (need > size_t(COMET_NOALLOC_SCRATCH_BYTES))
    return comet::api_fail(COMET_ERR_WORKSPACE,
                           "comet_plan_execute_noalloc: the plan needs " + std::to_string(need) +
                               " workspace bytes, more than the static buffer's " +
                               std::to_string(size_t(COMET_NOALLOC_SCRATCH_BYTES)));
  int device = 0;
  const hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return comet::api_fail(COMET_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  void *ws = nullptr;
  if (need > 0) {
    rc = scratch_for(device, &ws);
    if (rc != COMET_OK) return rc;
  }
  return comet_plan_execute(plan, alpha, A, B, beta, C, ws, need > 0 ? size_t(COMET_NOALLOC_SCRATCH_BYTES) : 0,
                            stream);
}
