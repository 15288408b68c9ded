// Persistent wavefront decode: one launch walks every diagonal of a batch of
// frames (of any sizes, I and P mixed). At global step t the rows are the
// union over frames of their diagonal t; each phase of the network (see
// network.h) is spread over the grid's blocks as GEMM tiles or attention
// items, and blocks meet at a grid barrier between dependent phases.
//
// The barrier is a monotonic arrival counter in device memory: a block's
// leader adds one arrival with release semantics (publishing the block's
// writes) and spins with acquire loads, a bounded number of times, until
// every block has arrived. Its cost grows with the number of blocks (about
// 1 us at 16 blocks and 10 us at 256 on MI355X), so the grid is kept small
// and tuned. If the
// bound is ever exceeded (a block that is not co-resident, say), the leader
// raises the abort flag; every block leaves at its next barrier, so the
// kernel always drains and the host reports the abort.
#include <hip/hip_runtime.h>

#include "device_ops.h"
#include "mfma_ops.h"
#include "network.h"
#include "persistent.h"

namespace pswa {

using namespace dev;

namespace {

__device__ bool grid_barrier(unsigned* bar, unsigned& target, int* abort_flag, long spin_limit) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    target += gridDim.x;
    // release: this block's writes become visible before its arrival counts
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    long spins = 0;
    // acquire: once every arrival is seen, every block's writes are visible
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (++spins > spin_limit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

template <int AK, bool RMS, int EPI>
__device__ void gemm_phase(const GemmArgs& a, float4* smem4, float* rstd) {
  __shared__ float rmul[kMBq];
  if (a.prec != PSWA_PREC_F32) {
    const int ct = qgemm_col_tiles(a.N, EPI), rt = qgemm_row_tiles(a.M);
    for (int t = blockIdx.x; t < ct * rt; t += gridDim.x)
      gemm_tile_q_any<AK, RMS, EPI>(a, t % ct, t / ct, reinterpret_cast<uint8_t*>(smem4), rstd,
                                    rmul);
    return;
  }
  const int ct = gemm_col_tiles(a.N, EPI), rt = gemm_row_tiles(a.M);
  for (int t = blockIdx.x; t < ct * rt; t += gridDim.x)
    gemm_tile_any<AK, RMS, EPI>(a, t % ct, t / ct, smem4, rstd);
}

__device__ void attn_phase(const AttnArgs& a, float* smem) {
  const int groups = (a.M * a.heads + kWaves - 1) / kWaves;
  for (int g = blockIdx.x; g < groups; g += gridDim.x)
    attn_item_any(a, g * kWaves + (threadIdx.x >> 6), true, smem);
}

__device__ void symbol_phase(const PassCtx& c, int C) {
  const long n = (long)c.M * C;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    gather_item(c.ysrc, c.src_compact, c.gpos, C, c.ydec, i);
    bits_item(c.gpos, C, c.ydec, c.mean, c.scale, c.bits, i);
  }
}

__global__ void __launch_bounds__(kThreads) k_persistent(PersistArgs P) {
  extern __shared__ float4 smem4[];
  __shared__ float rstd[kMBq];
  float* smem = reinterpret_cast<float*>(smem4);
  const NetDims& x = P.x;
  const DevWeights& w = P.w;
  unsigned target = 0;
#define PSWA_SYNC                                                        \
  if (!grid_barrier(P.bar, target, P.abort_flag, P.spin_limit)) return;

  for (int t = 0; t < P.T; ++t) {
    PassCtx c = P.c;
    const int r0 = P.row_start[t];
    c.M = P.row_start[t + 1] - r0;
    if (c.M == 0) continue;  // same for every block
    c.gpos = P.gpos_all + r0;
    c.fid = P.fid_all + r0;

    gemm_phase<A_FLOAT, true, EPI_STORE>(args_acc_q(x, w, c), smem4, rstd);
    PSWA_SYNC
    attn_phase(args_acc_attn(x, w, c), smem);
    PSWA_SYNC
    gemm_phase<A_FLOAT, false, EPI_RESID>(args_acc_o(x, w, c), smem4, rstd);
    PSWA_SYNC
    for (int l = 0; l < x.L; ++l) {
      gemm_phase<A_FLOAT, true, EPI_QKV>(args_qkv(x, w, c, l), smem4, rstd);
      PSWA_SYNC
      attn_phase(args_attn(x, w, c, l), smem);
      PSWA_SYNC
      gemm_phase<A_FLOAT, false, EPI_RESID>(args_o(x, w, c, l), smem4, rstd);
      PSWA_SYNC
      gemm_phase<A_FLOAT, true, EPI_SWIGLU>(args_gateup(x, w, c, l), smem4, rstd);
      PSWA_SYNC
      gemm_phase<A_FLOAT, false, EPI_RESID>(args_down(x, w, c, l), smem4, rstd);
      PSWA_SYNC
    }
    gemm_phase<A_FLOAT, true, EPI_SILU>(args_head1(x, w, c), smem4, rstd);
    PSWA_SYNC
    gemm_phase<A_FLOAT, false, EPI_HEAD>(args_head2(x, w, c), smem4, rstd);
    PSWA_SYNC
    symbol_phase(c, x.C);
    PSWA_SYNC
    gemm_phase<A_INT, false, EPI_STORE>(args_embed(x, w, c), smem4, rstd);
    PSWA_SYNC
    gemm_phase<A_FLOAT, true, EPI_STORE>(args_acc_kv(x, w, c), smem4, rstd);
    PSWA_SYNC
  }
#undef PSWA_SYNC
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

size_t persistent_lds_bytes(const NetDims& x, int prec) {
  size_t b = attn_lds_bytes(x.dh);
  for (int K : {x.F, x.d, x.C}) {
    const size_t g = prec ? qgemm_lds_bytes(K, prec) : gemm_lds_bytes(K);
    b = b > g ? b : g;
  }
  return b;
}

int persistent_max_grid(const NetDims& x, int prec) {
  static const bool attr = allow_big_lds(reinterpret_cast<const void*>(&k_persistent));
  (void)attr;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kThreads,
                                                   persistent_lds_bytes(x, prec)) != hipSuccess)
    return 0;
  return cus * per_cu;
}

void zero_ints(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

void launch_persistent(const PersistArgs& P, int grid, hipStream_t s) {
  static const bool attr = allow_big_lds(reinterpret_cast<const void*>(&k_persistent));
  (void)attr;
  hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(kThreads), persistent_lds_bytes(P.x, P.w.prec),
                     s, P);
}

}  // namespace pswa
