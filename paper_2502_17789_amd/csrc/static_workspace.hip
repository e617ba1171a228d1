// Library-owned subgrid workspace of aidg_execute_static: a file-scope device array,
// one copy on every device the library runs on, held until the process ends.  Its
// device address is looked up once per device (with that device current) and cached;
// host code uses only that address, never the array's name (which on the host is a
// stand-in symbol, not device memory).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "aidg_internal.h"

namespace aidg {
namespace {

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

}  // namespace

void* static_workspace(int device, std::string* err) {
  static std::mutex mu;
  static std::map<int, void*> ptrs;
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptrs.find(device);
  if (it != ptrs.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    *err = std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e);
    return nullptr;
  }
  ptrs[device] = ptr;
  return ptr;
}

}  // namespace aidg
