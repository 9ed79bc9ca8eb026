// fl_apply_noalloc (include/fl.h): the product y = A u for callers that
// cannot allocate device memory, with the transform intermediates in a fixed
// area of the library instead of the handle's workspace.
//
// The area is a file-scope __device__ array, so every device that loads the
// library's code object holds one copy of it, at an address of its own, until
// the process ends.  In host code the array's name is only a stand-in for the
// symbol: its device address comes from hipGetSymbolAddress, looked up once
// per device with that device current and kept here, and only that address
// is ever handed to kernels.  Every call on a device shares its copy: calls
// that overlap on one device race, and the area keeps whatever the last call
// left (the passes write every intermediate they read, so nothing needs
// clearing).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <unordered_map>

#include "../../include/fl.h"
#include "fl_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(FL_NOALLOC_SCRATCH_MIB) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::unordered_map<int, void*> g_scratch_addr;   // device ordinal -> its copy

// Address of the current device's copy; `dev` is the current device.
void* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    throw fl::Error(FL_E_DEVICE, std::string("hipGetSymbolAddress of the fixed scratch area: ") +
                                     hipGetErrorString(e));
  }
  g_scratch_addr.emplace(dev, ptr);
  return ptr;
}

}  // namespace

extern "C" fl_status fl_apply_noalloc(fl_op A, const void* u, void* y, int nrhs, int fp32,
                                      void* stream) {
  return (fl_status)fl::apply_in_area(A, u, y, nrhs, fp32, stream, &scratch_on, kScratchBytes);
}
