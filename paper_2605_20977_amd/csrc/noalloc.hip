// The encode form without any allocation: its workspace is a static device
// array of the library (one per GPU, held until the process ends) instead
// of caller memory. For callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops).
//
// Host code never uses the array's name as an address (on the host it is
// only a stand-in symbol): the device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/pswa.h"
#include "runtime.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal; null until looked up

// Device address of this device's scratch array (nullptr on error).
void* scratch_on_current_device(pswa_status* st) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0) {
    *st = pswa::fail(PSWA_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *st = pswa::fail(PSWA_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                       hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t pswa_noalloc_scratch_bytes(void) { return kScratchBytes; }

pswa_status pswa_encode_params_noalloc(const pswa_model* model, const pswa_frame_desc* frame,
                                       const int32_t* d_latents, const int32_t* d_hyper,
                                       const int32_t* d_prev, float* d_mean, float* d_scale,
                                       float* d_bits, int32_t* d_cdf_center,
                                       uint16_t* d_cdf_index, double* h_total_bits,
                                       void* stream) {
  if (!model) return pswa::fail(PSWA_E_ARG, "model is null");
  const size_t need = pswa_encode_workspace_bytes(model, frame);
  if (need == 0) return pswa::fail(PSWA_E_SHAPE, "invalid frame for this model");
  if (need > kScratchBytes)
    return pswa::fail(PSWA_E_UNSUPPORTED,
                      "frame needs %zu bytes of workspace, the static scratch holds %zu",
                      need, kScratchBytes);
  pswa_status st = PSWA_OK;
  void* ws = scratch_on_current_device(&st);
  if (!ws) return st;
  return pswa::encode_into(model, frame, d_latents, d_hyper, d_prev, d_mean, d_scale, d_bits,
                           d_cdf_center, d_cdf_index, h_total_bits, ws, kScratchBytes, stream);
}

}  // extern "C"
