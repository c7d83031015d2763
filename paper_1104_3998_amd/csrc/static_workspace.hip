// static_workspace.hip -- pic_init_static: pic_init for callers that cannot allocate device
// memory.  The simulation's workspace is a library-owned device array of fixed size
// instead of one the caller passes in.
//
// `scratch` is a file-scope device array: each GPU the library runs on holds its own copy
// (at its own address) from the moment the code object is loaded there until the process
// ends.  In host code the name `scratch` is only a host-side stand-in for the symbol, not a
// device address, so the array is reached through the address hipGetSymbolAddress gives
// for the current device, looked up once per device and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_common.h"

namespace {

constexpr size_t kStaticBytes = static_cast<size_t>(PIC_STATIC_WORKSPACE_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (looked up on the first call on a device).
int scratch_address(int dev, void** out, std::string* why) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return PIC_ERR_DEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PIC_OK;
}

}  // namespace

extern "C" int pic_init_static(const pic_config* cfgs, int n_discharges, void* hip_stream,
                               pic_sim** out) {
  if (!out) return PIC_ERR_ARG;
  *out = nullptr;
  size_t need = 0;
  int rc = pic_workspace_bytes(cfgs, n_discharges, &need);
  if (rc != PIC_OK) return rc;  // pic_last_error(NULL) says why
  if (need > kStaticBytes) {
    fspic::set_init_error("pic_init_static: these discharges need " + std::to_string(need) +
                          " bytes of workspace, the static workspace holds " +
                          std::to_string(kStaticBytes) + "; use pic_init with a workspace");
    return PIC_ERR_WORKSPACE;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fspic::set_init_error("pic_init_static: no current HIP device");
    return PIC_ERR_DEVICE;
  }
  void* ws = nullptr;
  std::string why;
  rc = scratch_address(dev, &ws, &why);
  if (rc != PIC_OK) {
    fspic::set_init_error(why);
    return rc;
  }
  // pic_init clears the part of the workspace the simulation uses before anything reads it
  return pic_init(cfgs, n_discharges, ws, kStaticBytes, hip_stream, out);
}
