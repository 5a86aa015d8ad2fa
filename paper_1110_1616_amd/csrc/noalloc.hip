// The allocation-free advance: amr_advance_patches for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).  The scratch that the existing
// entry point takes as its workspace argument -- the face-flux arrays the
// flux kernel writes and the update kernel reads, and the coarse/fine
// registers -- lives here in a file-scope device array of fixed size, one
// copy per device, held until the process ends.
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

static __device__ __align__(256) unsigned char scratch[int64_t(256) << 20];

namespace {

static_assert(sizeof(scratch) == (int64_t(256) << 20), "scratch size");
constexpr int64_t kScratchBytes = int64_t(256) << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

// Device address of `scratch` on each device (resolved once per device with
// that device current; the array's name is not a device address in host
// code).
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

namespace amrrt {

void scratch_init_device(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(AMR_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error(AMR_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
  g_scratch_ptr[device] = ptr;
}

}  // namespace amrrt

extern "C" {

amr_status amr_advance_patches_noalloc(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset,
                                       int32_t band, const amr_state* U_a, const amr_state* U_b, uint32_t parity,
                                       const double* dt0, void* stream) {
  try {
    if (!h || !U_a || !U_b || !dt0) throw Error(AMR_EINVAL, "null argument");
    if (h->workspace_bytes > kScratchBytes)
      throw Error(AMR_EINVAL, "the hierarchy needs " + std::to_string(h->workspace_bytes) +
                                  " bytes of workspace; the allocation-free advance holds at most " +
                                  std::to_string(kScratchBytes) + " (use amr_advance_patches)");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != h->device) throw Error(AMR_EINVAL, "the current device is not the one the hierarchy was created on");
    void* ws = nullptr;
    {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      ws = g_scratch_ptr[dev];
    }
    if (!ws) throw Error(AMR_EHIP, "scratch array not resolved on this device");
    // event timing would create events: it is off for this call
    const bool timing = h->timing;
    h->timing = false;
    try {
      advance_patches(h, cycle, grid_subset, nsubset, band, U_a, U_b, parity, dt0, ws, (hipStream_t)stream);
    } catch (...) {
      h->timing = timing;
      throw;
    }
    h->timing = timing;
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

}  // extern "C"
