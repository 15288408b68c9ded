// Host side of the persistent wavefront decode: instance choice, launch
// limits and launch. The kernel itself (one object per instance) is in
// persistent_kernel.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_ops.h"
#include "mfma_ops.h"
#include "network.h"
#include "persistent.h"

namespace pswa {

using namespace dev;

#define PSWA_DECLARE(P_, D_, R_) PSWA_PERSISTENT_GETTER(P_, D_, R_);
PSWA_PERSISTENT_INSTANCES(PSWA_DECLARE)
#undef PSWA_DECLARE

namespace {

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

size_t persistent_args_lds_offset(const NetDims& x, int prec, int rtile) {
  size_t b = x.cycle ? attn_lds_bytes(x.dh) : attn_stage_lds_bytes(x.dh, prec != 0);
  for (int K : {x.F, x.d, x.C}) {
    size_t g = prec ? qgemm_lds_bytes(K, prec, rtile) : gemm_lds_bytes(K);
    if (prec && rtile == 16 && K <= kWideMaxK) g = std::max(g, qgemm_lds_bytes(K, prec, kMBqWide));
    b = b > g ? b : g;
  }
  return (b + 255) & ~size_t(255);
}

size_t persistent_lds_bytes(const NetDims& x, int prec, int rtile) {
  return persistent_args_lds_offset(x, prec, rtile) + step_args_bytes(x.L, ct_phases(x));
}

// The instance for a model: projection arithmetic, head size and (for
// BF16/FP8) the row-tile height; FP32 has one row tile.
const void* persistent_fn(int prec, int dh, int rtile) {
  if (prec == PSWA_PREC_F32) rtile = 32;
#define PSWA_PICK(P_, D_, R_) \
  if (prec == P_ && dh == D_ && rtile == R_) return pswa_persistent_kernel_##P_##_##D_##_##R_();
  PSWA_PERSISTENT_INSTANCES(PSWA_PICK)
#undef PSWA_PICK
  return nullptr;
}

int persistent_max_grid(const NetDims& x, int prec, int rtile) {
  const void* fn = persistent_fn(prec, x.dh, rtile);
  if (!fn || !allow_big_lds(fn)) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads,
                                                   persistent_lds_bytes(x, prec, rtile)) !=
      hipSuccess)
    return 0;
  return cus * per_cu;
}

void zero_ints(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

void launch_persistent(const PersistArgs& P, const NetDims& x, int prec, int rtile, int grid,
                       hipStream_t s) {
  const void* fn = persistent_fn(prec, x.dh, rtile);
  if (!fn) return;  // head sizes and tile heights are checked by the callers
  static const bool attr = [] {
    bool ok = true;
    for (int p = 0; p < 3; ++p)
      for (int d : {16, 32, 48, 64})
        for (int r : {16, 32})
          if (const void* f = persistent_fn(p, d, r)) ok = allow_big_lds(f) && ok;
    return ok;
  }();
  (void)attr;
  const int rt = prec ? rtile : kMBq;
  PersistArgs Q = P;
  Q.args_lds_off = int(persistent_args_lds_offset(x, prec, rt));
  void* args[] = {&Q};
  (void)hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, persistent_lds_bytes(x, prec, rt),
                        s);
}

}  // namespace pswa
