// dft3d_execute_noalloc: dft3d_execute for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  The passes are the plan's own; only
// the workspace differs: it is `scratch`, a static device array that every
// GPU the library runs on holds until the process ends, instead of a buffer
// the plan allocates or the caller binds.
#include <mutex>

#include "../../include/dft3d.h"
#include "internal.h"

namespace {

// Largest workspace the entry point serves: 2^24 complex64 points, i.e.
// transforms of up to 256^3 points on the schedules that need a workspace.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

// The array itself.  In host code `scratch` names a host-side stand-in, not
// the device memory: host code uses only the address hipGetSymbolAddress
// returns for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

// The device address of `scratch` on device `dev` (current), looked up once
// per device on the first call there.
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return DFT3D_ERR_HIP;
    }
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return DFT3D_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" int dft3d_execute_noalloc(dft3d_plan_t p, const void* in, void* out, int sign,
                                     void* stream) {
  using namespace dft3d;
  if (!p || !in || !out || (sign != -1 && sign != 1)) return DFT3D_ERR_INVALID_ARG;
  int st = check_device(p);
  if (st != DFT3D_OK) return st;
  if (p->device < 0 || p->device >= kMaxDevices) return DFT3D_ERR_INVALID_ARG;
  const size_t bytes = (size_t)(p->n[0] * p->n[1] * p->n[2]) * sizeof(float2);
  if (overlap(in, out, bytes)) return DFT3D_ERR_INVALID_ARG;
  if (p->ws_need > kScratchBytes) return DFT3D_ERR_WORKSPACE_TOO_SMALL;
  void* ws = nullptr;
  if (p->ws_need > 0) {
    st = scratch_address(p->device, &ws);
    if (st != DFT3D_OK) return st;
  }
  // Every pass that reads the workspace reads what an earlier pass of the
  // same call wrote there, so the previous call's contents never matter and
  // nothing is cleared.
  return execute_passes(p, in, out, sign, static_cast<hipStream_t>(stream), ws);
}
