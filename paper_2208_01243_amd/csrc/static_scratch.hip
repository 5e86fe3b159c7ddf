// The fixed device array behind aim_align_batch_static, the entry point for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, at its own address, from the moment this code object is
// loaded on it until the process ends.  In host code the array's name is
// only a host-side stand-in, so host code never passes it (or takes its
// address) anywhere: static_scratch_address() asks the runtime for the
// current device's copy once per device, checks the result, and every later
// use -- kernel arguments, fills -- goes through that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "aim_internal.h"

static __device__ __align__(256) uint8_t scratch[aim::STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES];
}  // namespace

namespace aim {

hipError_t static_scratch_address(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace aim
