// Allocation-free phase-field relaxation (Sec. II.B, Eq. 15): the
// relaxation of dpd_phi_relax with its ping-pong buffer and residual word in
// a file-scope device array (`scratch`) instead of a caller-provided
// workspace.  For callers that cannot allocate device memory: code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc.
//
// Each GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never passes the array's name to a kernel (in
// host code it is a stand-in symbol, not a device address): the device
// address comes from hipGetSymbolAddress, once per device, on the first call
// on that device, and is kept per device.  Every call on one GPU shares that
// GPU's array; calls that overlap on one GPU (two streams, two threads) race
// on it.  The residual word is cleared by a fill kernel in every call that
// asks for it; the grid part needs no clearing (each step writes every node).
#include <hip/hip_runtime.h>

#include <mutex>

#include "dpd.h"
#include "kernels.h"

namespace {

// 64 MiB of grid values plus 256 bytes for the residual word: float32 grids
// up to 16,777,216 nodes (256^3), float64 grids up to 8,388,608 nodes.
constexpr size_t kScratchGridBytes = (size_t)64 << 20;
constexpr size_t kScratchBytes = kScratchGridBytes + 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device), or nullptr with the message recorded.
void *scratch_on_current_device(int *code) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *code = dpd::fail_global(DPD_E_DEVICE, "dpd_phi_relax_static: no usable HIP device");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *code = dpd::fail_global(DPD_E_DEVICE,
                               "dpd_phi_relax_static: hipGetSymbolAddress of the scratch array "
                               "failed");
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int dpd_phi_relax_static(void *phi, int32_t dtype, const int32_t n[3], const double h[3],
                         double eps, double dtau, int32_t iters, double *residual,
                         void *hip_stream) {
  const int chk = dpd::phi_relax_check(phi, dtype, n, h, eps, dtau, iters);
  if (chk) return chk;
  const size_t nodes = (size_t)n[0] * (size_t)n[1] * (size_t)n[2];
  if (nodes > kScratchGridBytes / (size_t)dtype)
    return dpd::fail_global(DPD_E_INVAL,
                            "dpd_phi_relax_static: grid larger than the static scratch "
                            "(64 MiB: at most 16777216 float32 or 8388608 float64 nodes); "
                            "use dpd_phi_relax with a workspace");
  int code = DPD_OK;
  void *work = scratch_on_current_device(&code);
  if (!work) return code;
  return dpd::phi_relax_run(phi, work, dtype, n, h, eps, dtau, iters, residual, hip_stream);
}

}  // extern "C"
