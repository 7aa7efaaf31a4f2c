// Allocation-free form of hddm_apply_precond, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation).  The box solutions between the local sweeps and
// the sum, which hddm_apply_precond keeps in the caller's work buffer, live
// here in a fixed device array of this library.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hddm_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// One copy per device, held until the process ends.  Its host-side name is
// not a device address: kernels get the address that hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (looked up once per device, with that
// device current); nullptr and a message on failure.
void* scratch_on(int dev, std::string& err) {
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipSetDevice(dev);
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

hddm_status hddm_apply_precond_noalloc(hddm_ctx* c, const void* r, void* z, void* stream) {
  if (!c) return hddm::set_error(HDDM_EINVAL, "null context");
  const size_t need = hddm::single_x_bytes(c);
  if (need > kScratchBytes)
    return hddm::set_error(
        HDDM_EINVAL, ("box solutions need " + std::to_string(need) +
                      " bytes; the allocation-free form holds at most " +
                      std::to_string(kScratchBytes))
                         .c_str());
  std::string err;
  void* ws = scratch_on(hddm::ctx_device(c), err);
  if (!ws) return hddm::set_error(HDDM_EDEVICE, err.c_str());
  return hddm::apply_precond_ws(c, r, z, ws, kScratchBytes, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
