// Static device scratch for the entry points that allocate nothing.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy (kScratchBytes) until the process ends.  In host code its name
// is a host-side stand-in, not a device address, so host code never passes it
// to a kernel or a copy: scratch_address() looks up this device's copy once
// per device (hipGetSymbolAddress with that device current) and every user
// takes that address.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "hgf_internal.h"
#include "hgf_kernels.h"

namespace hgf {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* scratch_address() {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> its copy of `scratch`
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    fail(HGF_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
  }
  addr[dev] = p;
  return p;
}

}  // namespace hgf
