// Allocation-free preconditioner entry point.
//
// paradiag_apply_precond_static runs the same kernels as paradiag_apply_precond,
// but its two spectral buffers (the Step-(a) output, the x-transformed copy and
// the Step-(b) result) live in a file-scope device array instead of the bound
// workspace.  The array is part of the library's code object: every device the
// library runs on holds its own copy from module load until the process ends.
//
// The array's name is only a host-side stand-in for the device symbol; kernels
// receive the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device on the first call there.

#include "internal.h"

namespace pd {
namespace {

constexpr size_t kScratchBytes = PD_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of this device's array (nullptr and the message set on failure).
void* scratch_address() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { set_error(std::string("hipGetDevice: ") + hipGetErrorString(e)); return nullptr; }
  if (dev < 0 || dev >= kMaxDevices) { set_error("device index beyond the static scratch table"); return nullptr; }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return nullptr;
    }
    g_addr[dev] = p;
  }
  return g_addr[dev];
}

}  // namespace
}  // namespace pd

extern "C" paradiag_status paradiag_apply_precond_static(paradiag_plan plan, const double* r, double* z,
                                                         void* stream) {
  char* base = static_cast<char*>(pd::scratch_address());
  if (!base) return PD_ERR_HIP;
  // two equal halves, each 256-byte aligned (kScratchBytes is a multiple of 512)
  const size_t half = pd::kScratchBytes / 2;
  return pd::apply_precond_into(plan, r, z, base, base + half, half, (hipStream_t)stream);
}
