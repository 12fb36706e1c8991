// The library's own workspace for callers that cannot allocate device memory
// (mdd_stoch_grad_noalloc): one file-scope device array per GPU, looked up once per
// device with hipGetSymbolAddress.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol); kernels receive the
// per-device pointer, as they receive a caller's workspace.
#include <mutex>

#include "mdd_internal.h"

namespace mdd {
namespace {

constexpr size_t STATIC_WS_BYTES = MDD_NOALLOC_WORKSPACE_BYTES;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

}  // namespace

size_t static_workspace_bytes() { return STATIC_WS_BYTES; }

hipError_t static_workspace(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // looked up with its device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) return hipErrorInvalidValue;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace mdd
